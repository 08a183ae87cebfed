// vp_sample_fp32neu.hip -- instantiations of the fused sampling kernel: single-precision map and integrand, compensated single-precision sums, D = 1..16.
#include "vp_sample.hpp"

namespace vp {

SampleEntry sample_entry_fp32neu(int kind, int dim, bool map_lds)
{
    SampleEntry e = {nullptr, nullptr, 0};
    if (kind == K_GAUSS_MIX) {
        switch (dim) {
        case 1: e = map_lds ? make_entry<1, P_FP32_NEUMAIER, true, K_GAUSS_MIX>() : make_entry<1, P_FP32_NEUMAIER, false, K_GAUSS_MIX>(); break;
        case 2: e = map_lds ? make_entry<2, P_FP32_NEUMAIER, true, K_GAUSS_MIX>() : make_entry<2, P_FP32_NEUMAIER, false, K_GAUSS_MIX>(); break;
        case 3: e = map_lds ? make_entry<3, P_FP32_NEUMAIER, true, K_GAUSS_MIX>() : make_entry<3, P_FP32_NEUMAIER, false, K_GAUSS_MIX>(); break;
        case 4: e = map_lds ? make_entry<4, P_FP32_NEUMAIER, true, K_GAUSS_MIX>() : make_entry<4, P_FP32_NEUMAIER, false, K_GAUSS_MIX>(); break;
        case 5: e = map_lds ? make_entry<5, P_FP32_NEUMAIER, true, K_GAUSS_MIX>() : make_entry<5, P_FP32_NEUMAIER, false, K_GAUSS_MIX>(); break;
        case 6: e = map_lds ? make_entry<6, P_FP32_NEUMAIER, true, K_GAUSS_MIX>() : make_entry<6, P_FP32_NEUMAIER, false, K_GAUSS_MIX>(); break;
        case 7: e = map_lds ? make_entry<7, P_FP32_NEUMAIER, true, K_GAUSS_MIX>() : make_entry<7, P_FP32_NEUMAIER, false, K_GAUSS_MIX>(); break;
        case 8: e = map_lds ? make_entry<8, P_FP32_NEUMAIER, true, K_GAUSS_MIX>() : make_entry<8, P_FP32_NEUMAIER, false, K_GAUSS_MIX>(); break;
        case 9: e = map_lds ? make_entry<9, P_FP32_NEUMAIER, true, K_GAUSS_MIX>() : make_entry<9, P_FP32_NEUMAIER, false, K_GAUSS_MIX>(); break;
        case 10: e = map_lds ? make_entry<10, P_FP32_NEUMAIER, true, K_GAUSS_MIX>() : make_entry<10, P_FP32_NEUMAIER, false, K_GAUSS_MIX>(); break;
        case 11: e = map_lds ? make_entry<11, P_FP32_NEUMAIER, true, K_GAUSS_MIX>() : make_entry<11, P_FP32_NEUMAIER, false, K_GAUSS_MIX>(); break;
        case 12: e = map_lds ? make_entry<12, P_FP32_NEUMAIER, true, K_GAUSS_MIX>() : make_entry<12, P_FP32_NEUMAIER, false, K_GAUSS_MIX>(); break;
        case 13: e = map_lds ? make_entry<13, P_FP32_NEUMAIER, true, K_GAUSS_MIX>() : make_entry<13, P_FP32_NEUMAIER, false, K_GAUSS_MIX>(); break;
        case 14: e = map_lds ? make_entry<14, P_FP32_NEUMAIER, true, K_GAUSS_MIX>() : make_entry<14, P_FP32_NEUMAIER, false, K_GAUSS_MIX>(); break;
        case 15: e = map_lds ? make_entry<15, P_FP32_NEUMAIER, true, K_GAUSS_MIX>() : make_entry<15, P_FP32_NEUMAIER, false, K_GAUSS_MIX>(); break;
        case 16: e = map_lds ? make_entry<16, P_FP32_NEUMAIER, true, K_GAUSS_MIX>() : make_entry<16, P_FP32_NEUMAIER, false, K_GAUSS_MIX>(); break;
        default: break;
        }
    } else {
        switch (dim) {
        case 1: if (!map_lds) e = make_entry<1, P_FP32_NEUMAIER, false, 0>(); break;
        case 2: if (!map_lds) e = make_entry<2, P_FP32_NEUMAIER, false, 0>(); break;
        case 3: if (!map_lds) e = make_entry<3, P_FP32_NEUMAIER, false, 0>(); break;
        case 4: if (!map_lds) e = make_entry<4, P_FP32_NEUMAIER, false, 0>(); break;
        case 5: if (!map_lds) e = make_entry<5, P_FP32_NEUMAIER, false, 0>(); break;
        case 6: if (!map_lds) e = make_entry<6, P_FP32_NEUMAIER, false, 0>(); break;
        case 7: if (!map_lds) e = make_entry<7, P_FP32_NEUMAIER, false, 0>(); break;
        case 8: if (!map_lds) e = make_entry<8, P_FP32_NEUMAIER, false, 0>(); break;
        case 9: if (!map_lds) e = make_entry<9, P_FP32_NEUMAIER, false, 0>(); break;
        case 10: if (!map_lds) e = make_entry<10, P_FP32_NEUMAIER, false, 0>(); break;
        case 11: if (!map_lds) e = make_entry<11, P_FP32_NEUMAIER, false, 0>(); break;
        case 12: if (!map_lds) e = make_entry<12, P_FP32_NEUMAIER, false, 0>(); break;
        case 13: if (!map_lds) e = make_entry<13, P_FP32_NEUMAIER, false, 0>(); break;
        case 14: if (!map_lds) e = make_entry<14, P_FP32_NEUMAIER, false, 0>(); break;
        case 15: if (!map_lds) e = make_entry<15, P_FP32_NEUMAIER, false, 0>(); break;
        case 16: if (!map_lds) e = make_entry<16, P_FP32_NEUMAIER, false, 0>(); break;
        default: break;
        }
    }
    return e;
}

}  // namespace vp

// vp_sample_fp32neu_gauss_k1.hip -- instantiations of the fused sampling kernel: single-precision map and integrand, compensated single-precision sums, Gaussian mixture of 1 term, D = 1..16.
// Written by gen_instances.py.
#include "vp_sample.hpp"

namespace vp {

SampleEntry sample_entry_fp32neu_gauss_k1(int dim, int map, bool rec)
{
    SampleEntry e = {nullptr, nullptr, 0};
    switch (dim) {
    case 1: e = entry_for_global_lds_only<1, P_FP32_NEUMAIER, K_GAUSS_MIX, 1>(map, rec); break;
    case 2: e = entry_for_global_lds_only<2, P_FP32_NEUMAIER, K_GAUSS_MIX, 1>(map, rec); break;
    case 3: e = entry_for_global_lds_only<3, P_FP32_NEUMAIER, K_GAUSS_MIX, 1>(map, rec); break;
    case 4: e = entry_for_global_lds_only<4, P_FP32_NEUMAIER, K_GAUSS_MIX, 1>(map, rec); break;
    case 5: e = entry_for_global_lds_only<5, P_FP32_NEUMAIER, K_GAUSS_MIX, 1>(map, rec); break;
    case 6: e = entry_for_global_lds_only<6, P_FP32_NEUMAIER, K_GAUSS_MIX, 1>(map, rec); break;
    case 7: e = entry_for_global_lds_only<7, P_FP32_NEUMAIER, K_GAUSS_MIX, 1>(map, rec); break;
    case 8: e = entry_for_global_lds_only<8, P_FP32_NEUMAIER, K_GAUSS_MIX, 1>(map, rec); break;
    case 9: e = entry_for_global_lds_only<9, P_FP32_NEUMAIER, K_GAUSS_MIX, 1>(map, rec); break;
    case 10: e = entry_for_global_lds_only<10, P_FP32_NEUMAIER, K_GAUSS_MIX, 1>(map, rec); break;
    case 11: e = entry_for_global_lds_only<11, P_FP32_NEUMAIER, K_GAUSS_MIX, 1>(map, rec); break;
    case 12: e = entry_for_global_lds_only<12, P_FP32_NEUMAIER, K_GAUSS_MIX, 1>(map, rec); break;
    case 13: e = entry_for_global_lds_only<13, P_FP32_NEUMAIER, K_GAUSS_MIX, 1>(map, rec); break;
    case 14: e = entry_for_global_lds_only<14, P_FP32_NEUMAIER, K_GAUSS_MIX, 1>(map, rec); break;
    case 15: e = entry_for_global_lds_only<15, P_FP32_NEUMAIER, K_GAUSS_MIX, 1>(map, rec); break;
    case 16: e = entry_for_global_lds_only<16, P_FP32_NEUMAIER, K_GAUSS_MIX, 1>(map, rec); break;
    default: break;
    }
    return e;
}

}  // namespace vp

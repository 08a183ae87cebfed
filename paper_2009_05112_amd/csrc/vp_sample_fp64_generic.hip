// vp_sample_fp64_generic.hip -- instantiations of the fused sampling kernel: double precision, any integrand kind, D = 1..24.
#include "vp_sample.hpp"

namespace vp {

SampleEntry sample_entry_fp64_generic(int dim, bool map_lds)
{
    SampleEntry e = {nullptr, nullptr, 0};
    switch (dim) {
    case 1: if (!map_lds) e = make_entry<1, P_FP64, false, 0>(); break;
    case 2: if (!map_lds) e = make_entry<2, P_FP64, false, 0>(); break;
    case 3: if (!map_lds) e = make_entry<3, P_FP64, false, 0>(); break;
    case 4: if (!map_lds) e = make_entry<4, P_FP64, false, 0>(); break;
    case 5: if (!map_lds) e = make_entry<5, P_FP64, false, 0>(); break;
    case 6: if (!map_lds) e = make_entry<6, P_FP64, false, 0>(); break;
    case 7: if (!map_lds) e = make_entry<7, P_FP64, false, 0>(); break;
    case 8: if (!map_lds) e = make_entry<8, P_FP64, false, 0>(); break;
    case 9: if (!map_lds) e = make_entry<9, P_FP64, false, 0>(); break;
    case 10: if (!map_lds) e = make_entry<10, P_FP64, false, 0>(); break;
    case 11: if (!map_lds) e = make_entry<11, P_FP64, false, 0>(); break;
    case 12: if (!map_lds) e = make_entry<12, P_FP64, false, 0>(); break;
    case 13: if (!map_lds) e = make_entry<13, P_FP64, false, 0>(); break;
    case 14: if (!map_lds) e = make_entry<14, P_FP64, false, 0>(); break;
    case 15: if (!map_lds) e = make_entry<15, P_FP64, false, 0>(); break;
    case 16: if (!map_lds) e = make_entry<16, P_FP64, false, 0>(); break;
    case 17: if (!map_lds) e = make_entry<17, P_FP64, false, 0>(); break;
    case 18: if (!map_lds) e = make_entry<18, P_FP64, false, 0>(); break;
    case 19: if (!map_lds) e = make_entry<19, P_FP64, false, 0>(); break;
    case 20: if (!map_lds) e = make_entry<20, P_FP64, false, 0>(); break;
    case 21: if (!map_lds) e = make_entry<21, P_FP64, false, 0>(); break;
    case 22: if (!map_lds) e = make_entry<22, P_FP64, false, 0>(); break;
    case 23: if (!map_lds) e = make_entry<23, P_FP64, false, 0>(); break;
    case 24: if (!map_lds) e = make_entry<24, P_FP64, false, 0>(); break;
    default: break;
    }
    return e;
}

}  // namespace vp

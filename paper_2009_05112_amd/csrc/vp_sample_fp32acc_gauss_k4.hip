// vp_sample_fp32acc_gauss_k4.hip -- instantiations of the fused sampling kernel: single-precision map and integrand, double sums, Gaussian mixture of 4 terms, D = 1..16.
// Written by gen_instances.py.
#include "vp_sample.hpp"

namespace vp {

SampleEntry sample_entry_fp32acc_gauss_k4(int dim, int map, bool rec)
{
    SampleEntry e = {nullptr, nullptr, 0};
    switch (dim) {
    case 1: e = entry_for<1, P_FP32_ACC64, K_GAUSS_MIX, 4>(map, rec); break;
    case 2: e = entry_for<2, P_FP32_ACC64, K_GAUSS_MIX, 4>(map, rec); break;
    case 3: e = entry_for<3, P_FP32_ACC64, K_GAUSS_MIX, 4>(map, rec); break;
    case 4: e = entry_for<4, P_FP32_ACC64, K_GAUSS_MIX, 4>(map, rec); break;
    case 5: e = entry_for<5, P_FP32_ACC64, K_GAUSS_MIX, 4>(map, rec); break;
    case 6: e = entry_for<6, P_FP32_ACC64, K_GAUSS_MIX, 4>(map, rec); break;
    case 7: e = entry_for<7, P_FP32_ACC64, K_GAUSS_MIX, 4>(map, rec); break;
    case 8: e = entry_for<8, P_FP32_ACC64, K_GAUSS_MIX, 4>(map, rec); break;
    case 9: e = entry_for<9, P_FP32_ACC64, K_GAUSS_MIX, 4>(map, rec); break;
    case 10: e = entry_for<10, P_FP32_ACC64, K_GAUSS_MIX, 4>(map, rec); break;
    case 11: e = entry_for<11, P_FP32_ACC64, K_GAUSS_MIX, 4>(map, rec); break;
    case 12: e = entry_for<12, P_FP32_ACC64, K_GAUSS_MIX, 4>(map, rec); break;
    case 13: e = entry_for<13, P_FP32_ACC64, K_GAUSS_MIX, 4>(map, rec); break;
    case 14: e = entry_for<14, P_FP32_ACC64, K_GAUSS_MIX, 4>(map, rec); break;
    case 15: e = entry_for<15, P_FP32_ACC64, K_GAUSS_MIX, 4>(map, rec); break;
    case 16: e = entry_for<16, P_FP32_ACC64, K_GAUSS_MIX, 4>(map, rec); break;
    default: break;
    }
    return e;
}

}  // namespace vp

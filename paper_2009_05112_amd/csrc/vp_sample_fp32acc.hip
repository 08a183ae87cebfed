// vp_sample_fp32acc.hip -- instantiations of the fused sampling kernel, single-precision map and integrand with double sums, D = 1..16.
#include "vp_sample.hpp"

namespace vp {

namespace {
template <int D, bool MAPLDS>
int occ(int block, size_t lds)
{
    int n = 0;
    (void)hipFuncSetAttribute((const void*)k_sample<D, P_FP32_ACC64, MAPLDS>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_sample<D, P_FP32_ACC64, MAPLDS>, block, lds) !=
        hipSuccess)
        return 0;
    return n;
}
}  // namespace

SampleEntry sample_entry_fp32acc(int dim, bool map_lds)
{
    SampleEntry e = {nullptr, nullptr};
    switch (dim) {
    case 1:
        e.launch = map_lds ? launch_sample<1, P_FP32_ACC64, true> : launch_sample<1, P_FP32_ACC64, false>;
        e.occupancy = map_lds ? occ<1, true> : occ<1, false>;
        break;
    case 2:
        e.launch = map_lds ? launch_sample<2, P_FP32_ACC64, true> : launch_sample<2, P_FP32_ACC64, false>;
        e.occupancy = map_lds ? occ<2, true> : occ<2, false>;
        break;
    case 3:
        e.launch = map_lds ? launch_sample<3, P_FP32_ACC64, true> : launch_sample<3, P_FP32_ACC64, false>;
        e.occupancy = map_lds ? occ<3, true> : occ<3, false>;
        break;
    case 4:
        e.launch = map_lds ? launch_sample<4, P_FP32_ACC64, true> : launch_sample<4, P_FP32_ACC64, false>;
        e.occupancy = map_lds ? occ<4, true> : occ<4, false>;
        break;
    case 5:
        e.launch = map_lds ? launch_sample<5, P_FP32_ACC64, true> : launch_sample<5, P_FP32_ACC64, false>;
        e.occupancy = map_lds ? occ<5, true> : occ<5, false>;
        break;
    case 6:
        e.launch = map_lds ? launch_sample<6, P_FP32_ACC64, true> : launch_sample<6, P_FP32_ACC64, false>;
        e.occupancy = map_lds ? occ<6, true> : occ<6, false>;
        break;
    case 7:
        e.launch = map_lds ? launch_sample<7, P_FP32_ACC64, true> : launch_sample<7, P_FP32_ACC64, false>;
        e.occupancy = map_lds ? occ<7, true> : occ<7, false>;
        break;
    case 8:
        e.launch = map_lds ? launch_sample<8, P_FP32_ACC64, true> : launch_sample<8, P_FP32_ACC64, false>;
        e.occupancy = map_lds ? occ<8, true> : occ<8, false>;
        break;
    case 9:
        e.launch = map_lds ? launch_sample<9, P_FP32_ACC64, true> : launch_sample<9, P_FP32_ACC64, false>;
        e.occupancy = map_lds ? occ<9, true> : occ<9, false>;
        break;
    case 10:
        e.launch = map_lds ? launch_sample<10, P_FP32_ACC64, true> : launch_sample<10, P_FP32_ACC64, false>;
        e.occupancy = map_lds ? occ<10, true> : occ<10, false>;
        break;
    case 11:
        e.launch = map_lds ? launch_sample<11, P_FP32_ACC64, true> : launch_sample<11, P_FP32_ACC64, false>;
        e.occupancy = map_lds ? occ<11, true> : occ<11, false>;
        break;
    case 12:
        e.launch = map_lds ? launch_sample<12, P_FP32_ACC64, true> : launch_sample<12, P_FP32_ACC64, false>;
        e.occupancy = map_lds ? occ<12, true> : occ<12, false>;
        break;
    case 13:
        e.launch = map_lds ? launch_sample<13, P_FP32_ACC64, true> : launch_sample<13, P_FP32_ACC64, false>;
        e.occupancy = map_lds ? occ<13, true> : occ<13, false>;
        break;
    case 14:
        e.launch = map_lds ? launch_sample<14, P_FP32_ACC64, true> : launch_sample<14, P_FP32_ACC64, false>;
        e.occupancy = map_lds ? occ<14, true> : occ<14, false>;
        break;
    case 15:
        e.launch = map_lds ? launch_sample<15, P_FP32_ACC64, true> : launch_sample<15, P_FP32_ACC64, false>;
        e.occupancy = map_lds ? occ<15, true> : occ<15, false>;
        break;
    case 16:
        e.launch = map_lds ? launch_sample<16, P_FP32_ACC64, true> : launch_sample<16, P_FP32_ACC64, false>;
        e.occupancy = map_lds ? occ<16, true> : occ<16, false>;
        break;
    default:
        break;
    }
    return e;
}

}  // namespace vp

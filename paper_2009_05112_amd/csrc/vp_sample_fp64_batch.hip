// vp_sample_fp64_batch.hip -- instantiations of the fused sampling kernel: double precision, batched integrand (accumulation of the user's values), D = 1..24.
// Written by gen_instances.py.
#include "vp_sample.hpp"

namespace vp {

SampleEntry sample_entry_fp64_batch_gen(int dim, int map)
{
    SampleEntry e = {nullptr, nullptr, 0};
    switch (dim) {
    case 1: e = map == MAP_LDS ? make_entry<1, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<1, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 2: e = map == MAP_LDS ? make_entry<2, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<2, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 3: e = map == MAP_LDS ? make_entry<3, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<3, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 4: e = map == MAP_LDS ? make_entry<4, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<4, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 5: e = map == MAP_LDS ? make_entry<5, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<5, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 6: e = map == MAP_LDS ? make_entry<6, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<6, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 7: e = map == MAP_LDS ? make_entry<7, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<7, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 8: e = map == MAP_LDS ? make_entry<8, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<8, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 9: e = map == MAP_LDS ? make_entry<9, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<9, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 10: e = map == MAP_LDS ? make_entry<10, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<10, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 11: e = map == MAP_LDS ? make_entry<11, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<11, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 12: e = map == MAP_LDS ? make_entry<12, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<12, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 13: e = map == MAP_LDS ? make_entry<13, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<13, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 14: e = map == MAP_LDS ? make_entry<14, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<14, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 15: e = map == MAP_LDS ? make_entry<15, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<15, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 16: e = map == MAP_LDS ? make_entry<16, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<16, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 17: e = map == MAP_LDS ? make_entry<17, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<17, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 18: e = map == MAP_LDS ? make_entry<18, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<18, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 19: e = map == MAP_LDS ? make_entry<19, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<19, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 20: e = map == MAP_LDS ? make_entry<20, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<20, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 21: e = map == MAP_LDS ? make_entry<21, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<21, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 22: e = map == MAP_LDS ? make_entry<22, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<22, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 23: e = map == MAP_LDS ? make_entry<23, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<23, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    case 24: e = map == MAP_LDS ? make_entry<24, P_FP64, MAP_LDS, K_BATCH_GEN, false, 0>() : make_entry<24, P_FP64, MAP_GLOBAL, K_BATCH_GEN, false, 0>(); break;
    default: break;
    }
    return e;
}

SampleEntry sample_entry_fp64_batch_acc(int dim, int map, bool rec)
{
    SampleEntry e = {nullptr, nullptr, 0};
    switch (dim) {
    case 1: e = entry_for_global<1, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 2: e = entry_for_global<2, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 3: e = entry_for_global<3, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 4: e = entry_for_global<4, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 5: e = entry_for_global<5, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 6: e = entry_for_global<6, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 7: e = entry_for_global<7, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 8: e = entry_for_global<8, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 9: e = entry_for_global<9, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 10: e = entry_for_global<10, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 11: e = entry_for_global<11, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 12: e = entry_for_global<12, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 13: e = entry_for_global<13, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 14: e = entry_for_global<14, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 15: e = entry_for_global<15, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 16: e = entry_for_global<16, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 17: e = entry_for_global<17, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 18: e = entry_for_global<18, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 19: e = entry_for_global<19, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 20: e = entry_for_global<20, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 21: e = entry_for_global<21, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 22: e = entry_for_global<22, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 23: e = entry_for_global<23, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    case 24: e = entry_for_global<24, P_FP64, K_BATCH_ACC, 0>(map, rec); break;
    default: break;
    }
    return e;
}

}  // namespace vp

// vp_internal.hpp -- types shared by the library's kernels and host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vp {

constexpr int kWave = 64;
constexpr int kMaxTerms = 4;
constexpr int kMaxDim = 24;       // FP64 sampling path
constexpr int kMaxDimSplit = 16;  // FP32 sampling paths
constexpr int kMaxNg = 4096;      // refinement keeps one axis in LDS

enum Prec { P_FP64 = 0, P_FP32_ACC64 = 1, P_FP32_NEUMAIER = 2 };
// Where the sampling kernel reads the vegas map: all of it from global memory
// (buffer loads), all of it staged in LDS, or the kMapInnerAxes innermost axes
// staged in LDS and the others from global memory.  The innermost axes are
// the ones whose increments the lanes of a wave scatter over the whole axis
// (consecutive hypercubes differ in their last digits).
enum MapPlace { MAP_GLOBAL = 0, MAP_LDS = 1, MAP_INNER = 2 };
constexpr int kMapInnerAxes = 2;
enum Kind { K_GAUSS_MIX = 1, K_CORR_GAUSS = 2, K_EXP_ABS = 3, K_CONST = 4, K_AFFINE = 5, K_BALLS = 6, K_BATCH = 100 };
// Sampling-kernel modes of a batched integrand: generate the sample points,
// then accumulate the values the user's function wrote.
enum BatchMode { K_BATCH_GEN = 101, K_BATCH_ACC = 102 };

// Sampling workgroup size (one workgroup per CU holds the LDS training data):
// the largest of 1024 / 768 / 512 threads whose register budget (128 / 168 /
// 256 VGPRs) holds the kernel body without spilling, i.e. four, three or two
// waves per SIMD.
constexpr int sample_block(int prec, int kind, int dim, bool map_lds, bool rec = false)
{
    if (prec == 0) {
        // the batched integrand's modes hold little state: the accumulate mode
        // (training data in LDS, one workgroup per CU) takes four waves per
        // SIMD, the generate mode with the map in LDS three (one workgroup per
        // CU: its registers allow five waves per SIMD, not the six of two
        // workgroups, and capped to fit two it ran no faster)
        if (kind == K_BATCH_ACC) return 1024;
        if (kind == K_BATCH_GEN) return map_lds || dim > 16 ? 768 : 1024;
        if (kind != K_GAUSS_MIX) return 512;
        if (dim == 8) return map_lds || rec ? 768 : 1024;
        if (dim < 8) return 1024;
        return dim <= 12 || (dim <= 15 && !rec) ? 768 : 512;
    }
    return dim <= 12 ? 1024 : 768;
}


// Integrand coefficients, in device memory; every lane reads the same
// addresses, so the compiler turns the reads into scalar loads.
struct IntegrandDev {
    int32_t kind, dim, n_terms, pad;
    double scale;
    double coefs[kMaxTerms];
    double amps[kMaxTerms];
    double rad2[kMaxTerms];                 // balls: coefs[k]^2
    double centers[kMaxTerms * kMaxDim + 1];
    double chol[kMaxDim * kMaxDim];
    float scale32;
    float coefs32[kMaxTerms];
    float amps32[kMaxTerms];
    float rad2_32[kMaxTerms];
    float centers32[kMaxTerms * kMaxDim + 1];
    float chol32[kMaxDim * kMaxDim];
};

// Partial sums of the hypercubes a wave's sample range starts and ends in;
// h < 0 marks an empty record.
struct EdgeRec {
    int64_t h;
    double s1, s2;
};

// Sample offsets are kept as offsets within blocks of kOffsTile hypercubes
// plus one base per block: offset(h) = loc[h] + base[h / kOffsTile]; the
// entry for h = n_hc is N_tot.
constexpr int kOffsTile = 4096;
static_assert((kOffsTile & (kOffsTile - 1)) == 0, "block index by a shift");

// Pointers into device (global) memory.  Accesses through them compile to
// global loads and stores, which count only against the vector-memory
// counter; through generic pointers they become flat accesses, and waiting
// for one of those also waits for every LDS operation the wave has in
// flight (the sampler's training-data atomics).
#define VP_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ VP_GLOBAL T* global_ptr(T* p)
{
    return (VP_GLOBAL T*)p;
}

__device__ __forceinline__ int64_t gofs(const int64_t* __restrict__ loc, const int64_t* __restrict__ base,
                                        int64_t h)
{
    return global_ptr(loc)[h] + global_ptr(base)[(uint64_t)h / kOffsTile];
}

// Position of sample pos in the point buffers of a batched integrand.  The
// samples are taken in aligned groups of 64 x 16; within a whole group the
// sample at offset r goes to (r mod 16) * 64 + r / 16, so that when the lanes
// of a wave each walk 16 consecutive samples, they touch consecutive
// addresses.  Defined on absolute positions, so every kernel and launch shape
// agrees; the last, partial group keeps its order.
constexpr int kBatchGroup = kWave * 16;
__device__ __forceinline__ int64_t batch_pos(int64_t pos, int64_t n_tot)
{
    const int64_t base = pos & ~(int64_t)(kBatchGroup - 1);
    if (base + kBatchGroup > n_tot) return pos;
    const int r = (int)(pos - base);
    return base + (int64_t)(r & 15) * kWave + (r >> 4);
}


// Per-sample dump of one iteration (vp_debug_dump): samples [first, first +
// count) of the iteration whose Philox index is `it`, as structure of arrays
// of `count` entries (x and idx: [dim][count]); count == 0 is off.
struct DumpArgs {
    int64_t* h;
    int32_t* j;
    int32_t* idx;
    double* x;
    double* jac;
    double* fx;
    int64_t first, count;
    uint32_t it;
    uint32_t pad;
};

struct SampleArgs {
    const double* map;      // [dim][n_g + 1]
    const float* map32;     // FP32 copy (split paths)
    const int64_t* offs;    // [n_hc + 1] offsets within blocks (see gofs)
    const int64_t* obase;   // per-block bases
    double* S1;             // [n_hc]
    double* S2;             // [n_hc]
    double* hist_part;      // [n_part][2][dim * n_g] per-workgroup training data
    // training records for the axes not privatised in LDS (dim * n_g too large),
    // per sample position: the value added to the numerator, the sample's n_h,
    // and the increment index of each such axis ([dim - hist_axes][rec_stride])
    double* rec_h;
    uint32_t* rec_n;        // = rec_h + rec_stride (as bytes: 8 rec_stride further)
    uint16_t* rec_bin;      // = rec_n + rec_stride
    int64_t rec_stride;     // a multiple of 64
    // batched integrand: x [dim][N_tot] (structure of arrays, packed to the
    // iteration's N_tot), J and f [cap], increment indices [dim][cap]
    double* bx;
    double* bj;
    const double* bf;
    uint16_t* bidx;
    int64_t bcap;
    EdgeRec* edges;         // [2 * n_waves]
    unsigned long long* nonfinite;
    const IntegrandDev* f;
    const void* fc;         // integrand constants in the sampler's layout (double, or float on the split paths)
    int64_t n_hc;
    int32_t n_g, n_st;
    double R;               // n_g / n_st
    float R32;
    double R53;             // R 2^-53 and R32 2^-24 (the packed form of k + u)
    float R32s;
    uint32_t key0, key1, it;
    int32_t hist_mode;      // 0 weighted, 1 literal
    int32_t hist_axes;      // training data of axes [0, hist_axes) privatised in LDS
    int32_t map_lds;        // map placement (MapPlace)
    int32_t chunk;          // samples per lane per tile
    // split precisions: the weight plane of the LDS training data is an
    // unsigned 64-bit fixed-point sum, each weight (1/n_h, or 1 in the literal
    // mode) rounded to a multiple of 1/wscale (see fixed_weight_scale)
    double wscale, wscale_inv;
    DumpArgs dump;          // per-sample dump (debugging and parity tests)
};

// Scalars every iteration kernel may need about one request (the single
// problem of the library's problem calls is a batch of one request).
struct DevState;
struct ReqArgs {
    SampleArgs s;           // sampling kernel; s.it is advanced on the device
    int32_t* n_h;
    int64_t* offs;
    int64_t* bsum;
    double* S1;
    double* S2;
    double* dh;
    double* H;
    double* W;
    double* hist_part;      // [n_part][2][dim * n_g]: bins of LDS axes have grid partials,
                            // bins of record axes have rec_chunks partials
    EdgeRec* edges;
    double* est_part;
    double* hist_I;
    double* hist_V;
    DevState* st;
    double* map;
    float* map32;
    int64_t n_hc;
    int64_t n_waves;
    int32_t dim, n_g;
    double omega, omega2, alpha, beta, n_ev;
    int32_t plus2, n_discard;
    int32_t n_adapt;        // > 0: iterations with s.it >= n_adapt neither reallocate nor refine
    int32_t average;        // 0 inverse-variance weighted, 1 unweighted combination
    int32_t slot;           // history slot of the current iteration (advanced on the device)
    int32_t grid;           // sampling workgroups
    int32_t est_blocks;     // workgroups of the estimate and reallocation passes
    int32_t hist_axes;      // axes privatised in the sampling kernel's LDS (the rest: records)
    int32_t rec_chunks;     // records: sample chunks, each one partial
    int32_t rec_slices;     // records: axis slices per chunk
    int32_t rec_axes;       // records: axes per slice (the last may hold fewer)
    int32_t checks;         // 1: run the invariant checks (k_check) every iteration
    int32_t det;            // 1: training records binned by one wave per workgroup
    const double* bounds;   // [2][dim]: lower, upper (device)
};

// One batched launch over n requests: request r's argument record is
// *reqs[r] (device pointers) and it owns workgroups [bbase[r], bbase[r + 1]).
struct LaunchSet {
    ReqArgs* const* reqs;
    const int32_t* bbase;
    int32_t n;
};

__device__ __forceinline__ int find_req(const int32_t* __restrict__ bbase, int n, int b)
{
    int lo = 0, hi = n - 1;  // largest r with bbase[r] <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bbase[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

#define VP_REQ_PROLOGUE(L)                                             \
    const int req_r_ = find_req((L).bbase, (L).n, (int)blockIdx.x);    \
    ReqArgs& q = *(L).reqs[req_r_];                                    \
    const int bid = (int)blockIdx.x - (L).bbase[req_r_];               \
    const int nblk = (L).bbase[req_r_ + 1] - (L).bbase[req_r_];        \
    (void)bid;                                                         \
    (void)nblk

typedef void (*SampleLauncher)(const LaunchSet& L, int grid, int block, size_t lds, hipStream_t s);
typedef int (*SampleOccupancy)(int block, size_t lds);
struct SampleEntry {
    SampleLauncher launch;
    SampleOccupancy occupancy;  // resident workgroups per CU at this block size and LDS
    int block;                  // workgroup size the kernel is built for
};

// Specialised kernel for (precision, integrand kind and terms, dim, map
// placement, training records), or an entry with launch == nullptr when none
// is built.
SampleEntry sample_entry(int prec, int kind, int n_terms, int dim, int map, bool rec, bool mix = false);
#define VP_DECL_GAUSS(tag)                                          \
    SampleEntry sample_entry_##tag##_gauss_k1(int dim, int map, bool rec); \
    SampleEntry sample_entry_##tag##_gauss_k2(int dim, int map, bool rec); \
    SampleEntry sample_entry_##tag##_gauss_k3(int dim, int map, bool rec); \
    SampleEntry sample_entry_##tag##_gauss_k4(int dim, int map, bool rec);
VP_DECL_GAUSS(fp64)
VP_DECL_GAUSS(fp32acc)
VP_DECL_GAUSS(fp32neu)
#undef VP_DECL_GAUSS
SampleEntry sample_entry_fp64_corr(int dim, int map, bool rec);
SampleEntry sample_entry_fp64_generic(int dim, int map, bool rec);
SampleEntry sample_entry_fp32acc_generic(int dim, int map, bool rec);
SampleEntry sample_entry_fp64_batch_gen(int dim, int map);
SampleEntry sample_entry_fp64_batch_acc(int dim, int map, bool rec);
SampleEntry sample_entry_fp32neu_generic(int dim, int map, bool rec);
// mixed stratification (per-axis counts): generic kinds and batched integrands
SampleEntry sample_entry_fp64_generic_mix(int dim, int map, bool rec);
SampleEntry sample_entry_fp32acc_generic_mix(int dim, int map, bool rec);
SampleEntry sample_entry_fp32neu_generic_mix(int dim, int map, bool rec);
SampleEntry sample_entry_fp64_batch_gen_mix(int dim, int map);
SampleEntry sample_entry_fp64_batch_acc_mix(int dim, int map, bool rec);

// sampling kernels' LDS needs (bytes) for histogram and map
inline size_t hist_lds_bytes(int dim, int n_g) { return (size_t)dim * n_g * 2 * sizeof(double); }
// Workgroup size of the records-to-histogram pass.
constexpr int kRecBlock = 1024;
__host__ __device__ constexpr int map_staged_axes(int map, int dim)
{
    return map == MAP_LDS ? dim : (map == MAP_INNER ? kMapInnerAxes : 0);
}
inline size_t map_lds_bytes(int prec, int dim, int n_g, int map)
{
    return (size_t)map_staged_axes(map, dim) * (n_g + 1) * (prec == P_FP64 ? sizeof(double) : sizeof(float));
}

// Integrand constants in the layout the sampling kernel reads (see
// vp_sample.hpp): elements (double on the FP64 path, float otherwise).  They
// are built on the host; kernels that stage them in LDS put them after the
// training data and the map.  The stratification of every axis follows the
// integrand's constants: R_mu = N_g / N_st^mu, then N_st^mu (exact as values
// of either type), read by the kernels of mixed stratification.
constexpr int kFcHead = 16;
__host__ __device__ constexpr int fc_strat_offset(int kind, int dim)
{
    return kFcHead + 4 * dim + (kind == K_CORR_GAUSS ? dim * dim : 0);
}
__host__ __device__ constexpr int fc_count(int kind, int dim)
{
    return fc_strat_offset(kind, dim) + 2 * dim;
}
__host__ __device__ constexpr size_t fc_lds_bytes(int prec, int kind, int dim)
{
    return (size_t)fc_count(kind, dim) * (prec == P_FP64 ? sizeof(double) : sizeof(float));
}
// Byte offset of the constants: after the training data and the staged
// axes of the map (map: a MapPlace), rounded up to 16 bytes.
__host__ __device__ constexpr size_t fc_lds_offset(size_t hist_bytes, int map, int prec, int dim, int n_g)
{
    return (hist_bytes + (size_t)map_staged_axes(map, dim) * (n_g + 1) * (prec == P_FP64 ? 8 : 4) + 15) / 16 * 16;
}

}  // namespace vp

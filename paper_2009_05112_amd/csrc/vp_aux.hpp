// vp_aux.hpp -- launchers of the per-hypercube and per-increment kernels.
#pragma once

#include "vp_internal.hpp"

namespace vp {

constexpr int kScanBlock = 256;
constexpr int kScanPer = 16;
constexpr int kScanTile = kScanBlock * kScanPer;
static_assert(kScanTile == kOffsTile, "scan tile and offset blocks must agree");
constexpr int kRedBlock = 256;
// Training-data reduction: kHistBlock threads per workgroup, split into G
// thread groups that each sum every G-th partial of kHistBlock / G values; G
// grows with the number of partials (up to 16, for about 16 partials per
// group), so that few partials do not leave most threads idle.
constexpr int kHistBlock = 256;
__host__ __device__ inline int hist_groups(int n_part)
{
    int g = 1;
    while (g < 16 && g * 16 < n_part) g <<= 1;
    return g;
}
// Rows of values per workgroup: about 16 partials summed per thread in all.
__host__ __device__ inline int hist_values(int n_part)
{
    const int per = (n_part + hist_groups(n_part) - 1) / hist_groups(n_part);
    int v = 1;
    while (v < 8 && v * 2 * per <= 16) v <<= 1;
    return v;
}
constexpr int kRedMaxGrid = 4096;
// Invariant-check findings (the public VP_CHECK_* bits).
enum CheckBits { CHECK_MAP_ORDER = 1, CHECK_MAP_ENDS = 2, CHECK_NH_MIN = 4, CHECK_NH_SUM = 8 };
// Invariant checks: kCheckBlock threads, up to kCheckMaxGrid workgroups per request.
constexpr int kCheckBlock = 256;
constexpr int kCheckMaxGrid = 1024;
inline int check_blocks(int64_t n_hc, int64_t n_map)
{
    const int64_t n = n_hc > n_map ? n_hc : n_map;
    const int64_t g = (n + 4 * kCheckBlock - 1) / (4 * kCheckBlock);
    return (int)(g < 1 ? 1 : (g > kCheckMaxGrid ? kCheckMaxGrid : g));
}
// Deterministic training records: one wave per binning workgroup.
constexpr int kRecDetBlock = 64;
// Records each thread of the binning pass loads before adding them.
constexpr int kRecUnroll = 4;
constexpr int kRefineBlock = 256;
constexpr int kFixBlock = 1024;  // edge fix-up: one workgroup per request
// Requests with at most kFixSmallRecs edge records (most served requests)
// take a workgroup of kFixSmallBlock threads instead: many then fit on a CU
// at once, where the full workgroup left most of its threads idle.
constexpr int kFixSmallBlock = 256;
constexpr int kFixSmallRecs = 2048;  // kFixSmallBlock x the records a thread holds

// Device-resident scalars of one problem.
struct DevState {
    double sumd;                 // sum of d_h of the last iteration
    double mean, sdev, chi2;     // combined estimate
    int64_t n_evals;             // samples drawn over all iterations
    int32_t n_iter_done;
    int32_t dof;
    unsigned long long ties;     // near-ties in reallocation
    unsigned long long nonfinite;
    // device-side invariant checks (k_check): bits seen so far, the iteration
    // of the first violation (-1: none), and the running state of the
    // current check launch (reset by its last workgroup)
    unsigned int check_flags;
    int32_t check_it;
    unsigned long long check_sum;
    unsigned int check_pending;
    unsigned int check_ticket;
};

inline int64_t scan_blocks(int64_t n_hc) { return (n_hc + kScanTile - 1) / kScanTile; }

// Initial device state of a problem: the uniform map over [lower, upper]
// (FP64 and its FP32 copy), the uniform allocation n0, zero sums.
struct InitArgs {
    const double* bounds;  // [2][dim]: lower, upper
    // when head_src is set, the kernel also copies head_bytes (a multiple of
    // 8) from head_src (host memory the device can read) to head_dst, and
    // bounds points into head_src
    const char* head_src;
    char* head_dst;
    int64_t head_bytes;
    double* map;
    float* map32;
    int32_t* n_h;
    double *S1, *S2, *H, *W;
    int64_t n_hc, nbins;
    int32_t dim, n_g, n0;
};
void launch_init(const InitArgs& a, hipStream_t s);
// The initialisation of n problems in one launch; table: n InitArgs in memory
// the device reads (entries with n_hc < 0 are skipped).
void launch_init_batch(const InitArgs* table, int n, hipStream_t s);
// Copies the estimate scalars of n problems into host-visible memory.
void launch_gather_states(DevState* const* states, int n, DevState* out, hipStream_t s);
void launch_fill_f64(double* x, int64_t n, double v, hipStream_t s);

// Training data of a preconditioned map from given points (x: [dim][n],
// f: [n]) under the current map, added into H and W (zeroed by the caller).
struct TrainArgs {
    const double* x;        // coordinate mu of point s at x[mu * x_mu + s * x_s]
    const double* f;
    const double* map;
    double* H;
    double* W;
    int64_t n;
    int64_t x_mu, x_s;      // [dim][n]: (n, 1); [n][dim]: (1, dim)
    int32_t dim, n_g;
};
void launch_train_hist(const TrainArgs& a, hipStream_t s);
// Vector-valued batched integrands: per-iteration estimates I_a and
// covariance C_ab of every component from the point buffers, and their
// combination over iterations.
constexpr int kMaxOut = 16;
constexpr int kVecBlock = 256;
constexpr int kVecMaxGrid = 1024;
constexpr int kVecHistory = 4096;
struct VecArgs {
    const double* jac;     // [cap] J of every sample (batch positions)
    const double* f;       // [n_out][n_tot] the user's values
    const int64_t* offs;   // hypercube offsets (see gofs)
    const int64_t* obase;
    double* part;          // [n_pairs + n_out][grid] partial sums
    double* hist_I;        // [kVecHistory][n_out]
    double* hist_C;        // [kVecHistory][n_out][n_out]
    double* out;           // mean [n_out], cov [n_out][n_out], chi2, dof
    int64_t n_hc, cap;
    double scale, omega, omega2;
    int32_t n_out, grid, slot, n_discard, average;
};
__host__ __device__ inline int vec_pairs(int n_out) { return n_out * (n_out + 1) / 2; }
int vec_grid(int64_t n_hc);
void launch_vec(const VecArgs& a, hipStream_t s);

// The refinement of every axis (one workgroup per axis) of the requests of L.
void launch_refine(const LaunchSet& L, int blocks, int max_ng, hipStream_t s);
void launch_fill_i32(int32_t* x, int64_t n, int32_t v, hipStream_t s);
int est_grid(int64_t n_hc);

constexpr int kMaxGroups = 64;

// Sampling launch of one group of requests sharing a kernel instantiation.
struct SampleGroup {
    SampleEntry entry;
    LaunchSet L;
    int blocks;
    size_t lds;
};

// Every launch of one batched iteration over a set of requests: the launch
// sets share the request table and differ in their workgroup counts.
struct IterPlan {
    LaunchSet scan_local, one, hist, rec, rec_det, fixup, fixup_s, est, refine, check;
    int n_scan_local, n_one, n_hist, n_rec, n_rec_det, n_fixup, n_fixup_s, n_est, n_refine, n_check;
    size_t rec_lds;  // dynamic LDS of the records-to-histogram pass
    SampleGroup groups[kMaxGroups];
    int n_groups;
    int max_ng;
};

// One-time per-device set-up of the auxiliary kernels (dynamic LDS limits,
// lds_max: the device's LDS per workgroup); done when a context is created,
// so enqueue_iteration makes no such call and can be captured into a graph.
hipError_t aux_init(size_t lds_max);
// Streams beside the main one on which the sampling launches of different
// kernel groups run side by side: they fork from the main stream and join it
// again through events, so the iteration can also be captured into a graph
// (as parallel branches).
constexpr int kMaxSide = 3;
struct SideStreams {
    int n = 0;
    hipStream_t st[kMaxSide] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kMaxSide] = {};
};
// Enqueues one iteration of every request of the plan; when given, the two
// events bracket the sampling launches, and side streams take some of them.
void enqueue_iteration(const IterPlan& P, hipStream_t s, hipEvent_t sample_begin, hipEvent_t sample_end,
                       const SideStreams* side = nullptr);
// The parts of an iteration before the sampling launches (allocation scan,
// then the invariant checks of the requests that asked for them)
// and after them (training data, estimate, reallocation, refinement).  With a
// side stream, the tail's two independent chains run side by side: training
// data and map refinement on the first side stream, edge fix-up, estimate and
// reallocation on s; both join before the iteration counters advance.
void enqueue_head(const IterPlan& P, hipStream_t s);
void enqueue_tail(const IterPlan& P, hipStream_t s, const SideStreams* side = nullptr);

}  // namespace vp

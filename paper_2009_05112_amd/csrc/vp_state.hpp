// vp_state.hpp -- host-side objects of the library (context, problem) and
// the internal calls the serving loop shares with the problem calls.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/vegasp.h"
#include "vp_aux.hpp"
#include "vp_internal.hpp"
#include "vp_plan.hpp"
#include "vp_pool.hpp"

using vp::DevState;
using vp::EdgeRec;
using vp::IntegrandDev;
using vp::IterPlan;
using vp::PlanBuilder;
using vp::ReqArgs;
using vp::SampleEntry;

// A context lives until its handle and every problem created on it are
// destroyed, whatever the order of the destroy calls.
struct vp_ctx {
    int device;
    hipStream_t stream;
    bool own_stream;
    int n_cu;
    size_t lds_max;
    int refs;
    // one side stream (forked from and joined to `stream` with events) on
    // which an iteration's map refinement chain runs beside its estimate and
    // reallocation chain; n = 0 when it could not be created
    vp::SideStreams side;
};

inline void ctx_release(vp_ctx* c)
{
    if (--c->refs > 0) return;
    (void)hipSetDevice(c->device);
    if (c->own_stream) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipStreamDestroy(c->stream);
    }
    for (int i = 0; i < c->side.n; ++i) {
        (void)hipStreamSynchronize(c->side.st[i]);
        (void)hipStreamDestroy(c->side.st[i]);
        (void)hipEventDestroy(c->side.join[i]);
    }
    if (c->side.fork) (void)hipEventDestroy(c->side.fork);
    delete c;
}

struct vp_problem {
    vp_ctx* ctx;
    vp_params P;
    std::vector<double> lower, upper;
    const double* bounds_d = nullptr;  // [2][dim] lower, upper in device memory
    std::vector<int32_t> nst_ax;  // stratifications of every axis
    int n_out = 1;               // components of a vector-valued batched integrand
    int vec_grid = 0;
    double* vI = nullptr;        // [kVecHistory][n_out] per-iteration estimates
    double* vC = nullptr;        // [kVecHistory][n_out][n_out] their covariances
    double* vpart = nullptr;     // partial sums of the vector estimate
    double* vout = nullptr;      // combined mean, covariance, chi^2, dof
    IntegrandDev fh;
    int32_t n_st;
    int64_t n_hc;
    double omega, omega2, R;
    int32_t it;  // iteration index of the next iteration
    int32_t slot;  // history slot of the next iteration
    // device state: every buffer lives in one allocation
    char* arena = nullptr;
    size_t arena_bytes = 0;
    vp::DevicePool* pool = nullptr;  // owner of the allocation, or none (own hipMalloc)
    std::vector<char> staging;  // host image of the allocation's head (initial copy)
    IntegrandDev* f_d = nullptr;
    const void* fc = nullptr;  // integrand constants in the sampler's layout
    double* map = nullptr;
    float* map32 = nullptr;
    int32_t* n_h = nullptr;
    int64_t* offs = nullptr;
    int64_t* bsum = nullptr;
    double* S1 = nullptr;
    double* S2 = nullptr;
    double* dh = nullptr;
    double* H = nullptr;
    double* W = nullptr;
    double* hist_part = nullptr;
    double* rec_h = nullptr;
    uint32_t* rec_n = nullptr;
    uint16_t* rec_bin = nullptr;
    int64_t rec_stride = 0;
    int32_t rec_chunks = 0, rec_slices = 0, rec_axes = 0;
    // batched integrand (VP_F_BATCH)
    double* bx = nullptr;
    double* bj = nullptr;
    double* bf = nullptr;
    uint16_t* bidx = nullptr;
    int64_t bcap = 0;
    SampleEntry gen_entry = {nullptr, nullptr, 0};
    size_t gen_lds = 0;
    int gen_grid = 0;
    PlanBuilder gen_planner;  // launch table of the generate mode
    IterPlan gen_plan;
    bool gen_plan_built = false;
    vp_batch_fn batch_fn = nullptr;
    void* batch_user = nullptr;
    EdgeRec* edges = nullptr;
    double* est_part = nullptr;
    double* hist_I = nullptr;
    double* hist_V = nullptr;
    DevState* st = nullptr;
    ReqArgs req;                 // host copy of the argument record
    ReqArgs* d_req = nullptr;    // device table of one record
    PlanBuilder planner;         // single-problem plan, built on the first vp_iterate
    IterPlan plan;
    bool plan_built = false;
    // sampling launch
    SampleEntry entry;
    int block, grid, chunk;
    int hist_axes, map_lds;
    size_t lds;
    int64_t n_waves;
    int32_t hist_cap;            // capacity of the estimate history
    // per-sample dump (vp_debug_dump): its own allocation
    char* dump_mem = nullptr;
    size_t dump_bytes = 0;
    vp::DumpArgs dump = {};
    // profiling
    bool prof = false;
    std::vector<hipEvent_t> ev_pending;  // pairs: k1 start, k1 end, it start, it end
    std::vector<hipEvent_t> ev_free;
    double t_sample_ms = 0.0, t_iter_ms = 0.0;
    int64_t n_sample = 0, n_iter = 0;
};


namespace vp {

vp_status fail(vp_status s, const char* fmt, ...);
vp_status validate(const vp_params* P, const vp_integrand* f);
// samples_per_wg > 0 sizes the sampling grid to about that many samples per
// workgroup (serving: many requests share the GPU); 0 fills the GPU.
// pool: the state is carved from the pool (a server's) instead of its own
// hipMalloc, and its initialisation is queued on the context's stream without
// waiting for it.
// init_out (pool only): the initialisation kernel's arguments are returned
// there instead of launched, so that a caller admitting many problems can
// initialise them all with one launch (launch_init_batch).
vp_status problem_create(vp_ctx* ctx, const vp_params* P, const vp_integrand* f, int64_t samples_per_wg,
                         DevicePool* pool, vp_problem** out, InitArgs* init_out = nullptr);
// Device bytes problem_create would allocate for these parameters.
vp_status problem_bytes(vp_ctx* ctx, const vp_params* P, const vp_integrand* f, int64_t samples_per_wg,
                        size_t* bytes);
void problem_free(vp_problem* p);
// Largest initial image (the records problem_create writes first) of any
// problem: what a request's admission stages in host memory at most.
size_t problem_head_bytes_max();
// The caller's view of a problem's estimate scalars; VP_ERR_NUMERIC (result
// still filled) when non-finite integrand values were seen.
vp_status result_from_state(const DevState& st, vp_result* out);

}  // namespace vp

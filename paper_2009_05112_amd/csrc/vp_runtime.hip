// vp_runtime.hip -- host runtime and C ABI of the vegas+ library (vegasp.h).
//
// A problem owns its device state: the vegas map (FP64 and an FP32 copy),
// the allocation n_h, the sample offsets, per-hypercube sums, training data,
// estimate history and a few device scalars.  vp_iterate enqueues the
// kernels of each iteration on the context stream without host round trips:
// the sampling kernel reads the number of samples from device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "vp_state.hpp"
#include "vp_trace.hpp"

using namespace vp;

static constexpr int64_t kMaxDump = (int64_t)1 << 24;

// The static device workspace of vp_map_train_noalloc: every device the
// library runs on holds one copy until the process ends.  Host code never
// uses the array's name as an address: vp_ctx_create looks up each device's
// copy once, with that device current, and keeps the address per device.
static constexpr size_t kScratchBytes = (size_t)32 << 20;
static constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static void* g_scratch[kMaxDevices];
static std::mutex g_scratch_mu;

// Address of this device's workspace (the device is current).
static hipError_t scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[device]) return hipSuccess;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = ptr;
    return hipSuccess;
}

namespace {
thread_local std::string g_err;
}

vp_status vp::fail(vp_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

namespace {

#define VP_HIP(call)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(e_ == hipErrorOutOfMemory ? VP_ERR_OOM : VP_ERR_DEVICE, "%s: %s (%s:%d)", \
                        #call, hipGetErrorString(e_), __FILE__, __LINE__);                      \
    } while (0)

constexpr int kMaxHistory = 65536;
constexpr uint32_t kStateMagic = 0x56504C53u;  // "SLPV"

}  // namespace

// ---------------------------------------------------------------- helpers
SampleEntry vp::sample_entry(int prec, int kind, int n_terms, int dim, int map, bool rec, bool mix)
{
    if (mix) {
        // per-axis stratification: the generic kernels (constants in LDS)
        typedef SampleEntry (*Table)(int, int, bool);
        static const Table generic_mix[3] = {sample_entry_fp64_generic_mix, sample_entry_fp32acc_generic_mix,
                                             sample_entry_fp32neu_generic_mix};
        if (prec < 0 || prec > 2) return SampleEntry{nullptr, nullptr, 0};
        if (kind == K_BATCH)
            return prec == P_FP64 ? sample_entry_fp64_batch_acc_mix(dim, map, rec) : SampleEntry{nullptr, nullptr, 0};
        return generic_mix[prec](dim, map, rec);
    }
    typedef SampleEntry (*Table)(int, int, bool);
    static const Table gauss[3][4] = {
        {sample_entry_fp64_gauss_k1, sample_entry_fp64_gauss_k2, sample_entry_fp64_gauss_k3, sample_entry_fp64_gauss_k4},
        {sample_entry_fp32acc_gauss_k1, sample_entry_fp32acc_gauss_k2, sample_entry_fp32acc_gauss_k3,
         sample_entry_fp32acc_gauss_k4},
        {sample_entry_fp32neu_gauss_k1, sample_entry_fp32neu_gauss_k2, sample_entry_fp32neu_gauss_k3,
         sample_entry_fp32neu_gauss_k4}};
    static const Table generic[3] = {sample_entry_fp64_generic, sample_entry_fp32acc_generic,
                                     sample_entry_fp32neu_generic};
    SampleEntry e = {nullptr, nullptr, 0};
    if (prec < 0 || prec > 2) return e;
    if (kind == K_BATCH) return prec == P_FP64 ? sample_entry_fp64_batch_acc(dim, map, rec) : e;
    if (kind == K_GAUSS_MIX && n_terms >= 1 && n_terms <= kMaxTerms) e = gauss[prec][n_terms - 1](dim, map, rec);
    else if (kind == K_CORR_GAUSS && prec == P_FP64) e = sample_entry_fp64_corr(dim, map, rec);
    if (!e.launch) e = generic[prec](dim, map, rec);
    return e;
}

static int32_t nst_rule(int32_t dim, int64_t n_ev)
{
    // largest n >= 1 with 4 n^dim <= n_ev (Sec. 3, Eq. Nst_vegasp)
    auto ok = [&](int64_t n) {
        int64_t acc = 4;
        if (acc > n_ev) return false;
        for (int d = 0; d < dim; ++d) {
            if (acc > n_ev / n) return false;
            acc *= n;
        }
        return acc <= n_ev;
    };
    int64_t n = 1;
    while (ok(n + 1)) ++n;
    return (int32_t)n;
}

static bool pow_le(int64_t n, int dim, int64_t mult, int64_t limit)
{
    int64_t acc = mult;
    for (int d = 0; d < dim; ++d) {
        if (acc > limit / n) return false;
        acc *= n;
    }
    return acc <= limit;
}

// mult * prod(counts) <= limit, without overflow
static bool prod_le(const int32_t* counts, int dim, int64_t mult, int64_t limit)
{
    int64_t acc = mult;
    if (acc > limit) return false;
    for (int d = 0; d < dim; ++d) {
        if (acc > limit / counts[d]) return false;
        acc *= counts[d];
    }
    return acc <= limit;
}

// Stratifications of every axis (Sec. 3 and Sec. 4): the user's per-axis
// counts; or N_st + 1 on the first d axes and N_st on the rest, d the largest
// that leaves 4 samples per hypercube on average; or N_st on every axis.
static void strat_counts(const vp_params* P, int32_t* out)
{
    const int D = P->dim;
    if (P->n_st_axes) {
        for (int d = 0; d < D; ++d) out[d] = P->n_st_axes[d];
        return;
    }
    const int32_t n = P->n_st > 0 ? P->n_st : nst_rule(D, P->n_ev);
    for (int d = 0; d < D; ++d) out[d] = n;
    if (P->strat != VP_STRAT_MIXED) return;
    for (int d = 0; d < D; ++d) {
        out[d] = n + 1;
        if (!prod_le(out, D, 4, P->n_ev)) {
            out[d] = n;
            break;
        }
    }
}

vp_status vp::validate(const vp_params* P, const vp_integrand* f)
{
    if (!P || !f) return fail(VP_ERR_INVALID_ARG, "params and integrand are required");
    const int maxd = P->precision == VP_FP64 ? kMaxDim : kMaxDimSplit;
    if (P->precision < 0 || P->precision > 2) return fail(VP_ERR_INVALID_ARG, "unknown precision %d", P->precision);
    if (P->dim < 1 || P->dim > maxd)
        return fail(VP_ERR_INVALID_ARG, "dim %d outside 1..%d for this precision", P->dim, maxd);
    if (P->n_ev < 4 || P->n_ev > 2147483647LL) return fail(VP_ERR_INVALID_ARG, "n_ev %lld outside 4..2^31-1", (long long)P->n_ev);
    if (P->n_g < 1 || P->n_g > kMaxNg) return fail(VP_ERR_INVALID_ARG, "n_g %d outside 1..%d", P->n_g, kMaxNg);
    if (!(P->alpha >= 0.0) || !std::isfinite(P->alpha)) return fail(VP_ERR_INVALID_ARG, "alpha must be >= 0");
    if (!(P->beta >= 0.0) || !std::isfinite(P->beta)) return fail(VP_ERR_INVALID_ARG, "beta must be >= 0");
    if (P->n_iter < 0) return fail(VP_ERR_INVALID_ARG, "n_iter must be >= 0");
    if (P->hist_mode != VP_HIST_WEIGHTED && P->hist_mode != VP_HIST_LITERAL)
        return fail(VP_ERR_INVALID_ARG, "unknown hist_mode %d", P->hist_mode);
    if (P->n_st < 0) return fail(VP_ERR_INVALID_ARG, "n_st must be >= 0");
    if (P->n_adapt < 0) return fail(VP_ERR_INVALID_ARG, "n_adapt must be >= 0");
    if (P->strat != VP_STRAT_UNIFORM && P->strat != VP_STRAT_MIXED)
        return fail(VP_ERR_INVALID_ARG, "unknown strat %d", P->strat);
    if (P->strat == VP_STRAT_MIXED && P->n_st > 0 && !P->n_st_axes)
        return fail(VP_ERR_INVALID_ARG, "the mixed rule takes N_st from n_ev: n_st must be 0");
    if (P->n_st_axes) {
        for (int d = 0; d < P->dim; ++d)
            if (P->n_st_axes[d] < 1) return fail(VP_ERR_INVALID_ARG, "n_st_axes[%d] = %d < 1", d, P->n_st_axes[d]);
        if (!prod_le(P->n_st_axes, P->dim, 2, P->n_ev))
            return fail(VP_ERR_INVALID_ARG, "n_st_axes leave fewer than 2 samples per hypercube");
        if (!prod_le(P->n_st_axes, P->dim, 1, 2147483647LL))
            return fail(VP_ERR_INVALID_ARG, "n_st_axes give 2^31 or more hypercubes");
    }
    if (P->average != VP_AVG_WEIGHTED && P->average != VP_AVG_UNWEIGHTED)
        return fail(VP_ERR_INVALID_ARG, "unknown average %d", P->average);
    if (P->n_st > 0 && !pow_le(P->n_st, P->dim, 2, P->n_ev))
        return fail(VP_ERR_INVALID_ARG, "n_st %d leaves fewer than 2 samples per hypercube", P->n_st);
    if (P->lower && P->upper)
        for (int d = 0; d < P->dim; ++d)
            if (!(P->lower[d] < P->upper[d])) return fail(VP_ERR_INVALID_ARG, "lower[%d] >= upper[%d]", d, d);
    if ((P->lower == nullptr) != (P->upper == nullptr))
        return fail(VP_ERR_INVALID_ARG, "lower and upper must be given together");
    if (f->dim != P->dim) return fail(VP_ERR_INVALID_ARG, "integrand dim %d != problem dim %d", f->dim, P->dim);
    switch (f->kind) {
    case VP_F_GAUSS_MIX:
    case VP_F_EXP_ABS:
    case VP_F_BALLS:
        if (f->n_terms < 1 || f->n_terms > kMaxTerms)
            return fail(VP_ERR_INVALID_ARG, "n_terms %d outside 1..%d", f->n_terms, kMaxTerms);
        if (!f->centers || !f->coefs || !f->amps) return fail(VP_ERR_INVALID_ARG, "centers, coefs, amps required");
        break;
    case VP_F_CORR_GAUSS:
        if (!f->centers || !f->chol) return fail(VP_ERR_INVALID_ARG, "centers and chol required");
        break;
    case VP_F_AFFINE:
        if (!f->centers) return fail(VP_ERR_INVALID_ARG, "centers (affine coefficients) required");
        break;
    case VP_F_CONST:
        break;
    case VP_F_BATCH:
        if (!f->fn) return fail(VP_ERR_INVALID_ARG, "a batched integrand needs fn");
        if (f->n_out < 0 || f->n_out > kMaxOut)
            return fail(VP_ERR_INVALID_ARG, "n_out %d outside 0..%d", f->n_out, kMaxOut);
        if (P->precision != VP_FP64) return fail(VP_ERR_INVALID_ARG, "batched integrands are double precision only");
        break;
    default:
        return fail(VP_ERR_INVALID_ARG, "unknown integrand kind %d", f->kind);
    }
    if (f->kind != VP_F_BATCH && f->n_out > 1)
        return fail(VP_ERR_INVALID_ARG, "vector-valued integrands (n_out > 1) are batched integrands");
    if (P->flags & ~(VP_FLAG_CHECKS | VP_FLAG_DETERMINISTIC))
        return fail(VP_ERR_INVALID_ARG, "unknown flags 0x%x", (unsigned)P->flags);
    if ((P->flags & VP_FLAG_DETERMINISTIC) && P->precision == VP_FP32_NEUMAIER)
        return fail(VP_ERR_INVALID_ARG, "the deterministic mode is not available with compensated sums");
    if ((P->flags & VP_FLAG_DETERMINISTIC) && f->kind == VP_F_BATCH)
        return fail(VP_ERR_INVALID_ARG, "the deterministic mode is not available with batched integrands");
    return VP_OK;
}

static void fill_integrand(IntegrandDev& d, const vp_integrand* f)
{
    memset(&d, 0, sizeof d);
    d.kind = f->kind;
    d.dim = f->dim;
    d.n_terms = f->n_terms;
    d.scale = f->scale;
    const int D = f->dim;
    int K = 0;
    if (f->kind == VP_F_GAUSS_MIX || f->kind == VP_F_EXP_ABS || f->kind == VP_F_BALLS) {
        K = f->n_terms;
        for (int k = 0; k < K; ++k) {
            d.coefs[k] = f->coefs[k];
            d.amps[k] = f->amps[k];
            d.rad2[k] = f->coefs[k] * f->coefs[k];
            for (int m = 0; m < D; ++m) d.centers[k * D + m] = f->centers[k * D + m];
        }
    } else if (f->kind == VP_F_CORR_GAUSS) {
        for (int m = 0; m < D; ++m) d.centers[m] = f->centers[m];
        for (int i = 0; i < D * D; ++i) d.chol[i] = f->chol[i];
    } else if (f->kind == VP_F_AFFINE) {
        for (int m = 0; m <= D; ++m) d.centers[m] = f->centers[m];
    }
    d.scale32 = (float)d.scale;
    for (int k = 0; k < kMaxTerms; ++k) {
        d.coefs32[k] = (float)d.coefs[k];
        d.amps32[k] = (float)d.amps[k];
        d.rad2_32[k] = d.coefs32[k] * d.coefs32[k];
    }
    for (int i = 0; i < kMaxTerms * kMaxDim + 1; ++i) d.centers32[i] = (float)d.centers[i];
    for (int i = 0; i < kMaxDim * kMaxDim; ++i) d.chol32[i] = (float)d.chol[i];
}

void vp::problem_free(vp_problem* p)
{
    if (!p) return;
    vp_ctx* ctx = p->ctx;
    if (p->pool) {
        // before any iteration ran, the initial copy from the staging image
        // may still be queued
        if (p->slot == 0 && !p->staging.empty()) (void)hipStreamSynchronize(ctx->stream);
        p->pool->release(p->arena);
    } else {
        (void)hipFree(p->arena);
    }
    if (p->dump_mem) (void)hipFree(p->dump_mem);
    for (auto e : p->ev_pending) (void)hipEventDestroy(e);
    for (auto e : p->ev_free) (void)hipEventDestroy(e);
    delete p;
    if (ctx) ctx_release(ctx);
}

static hipEvent_t take_event(vp_problem* p)
{
    if (!p->ev_free.empty()) {
        hipEvent_t e = p->ev_free.back();
        p->ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

static vp_status drain_events(vp_problem* p)
{
    for (size_t i = 0; i + 3 < p->ev_pending.size(); i += 4) {
        float a = 0.f, b = 0.f;
        VP_HIP(hipEventSynchronize(p->ev_pending[i + 3]));
        VP_HIP(hipEventElapsedTime(&a, p->ev_pending[i], p->ev_pending[i + 1]));
        VP_HIP(hipEventElapsedTime(&b, p->ev_pending[i + 2], p->ev_pending[i + 3]));
        p->t_sample_ms += a;
        p->t_iter_ms += b;
        p->n_sample += 1;
        p->n_iter += 1;
    }
    for (auto e : p->ev_pending) p->ev_free.push_back(e);
    p->ev_pending.clear();
    return VP_OK;
}

// Scale of the fixed-point weight plane of the split precisions' LDS
// training data: a weight w (1/n_h, or 1 in the literal mode) is added as
// rint(w 2^F).  A bin gathers at most one unit of weight from each hypercube
// whose slab on its axis contains it, so at most H = max over the axes of
// N_hc / N_st^mu units; F = 62 - ceil(log2 H) keeps every sum (with the
// rounding excess, at most half a step per sample) below 2^63.  The rounding
// error of a bin is at most half a step per sample, (N_tot / N_hc) 2^-(F+1) of
// an axis's total weight N_hc over all bins: below 2^-29 for every accepted
// problem.  The literal mode adds whole counts (F = 0): exact.
static void fixed_weight_scale(const vp_problem* p, double* scale, double* inv)
{
    int F = 0;
    if (p->P.hist_mode == VP_HIST_WEIGHTED) {
        int64_t most = 1;
        for (int32_t n : p->nst_ax) most = std::max<int64_t>(most, p->n_hc / n);
        int bits = 0;
        while (bits < 62 && ((int64_t)1 << bits) < most) ++bits;
        F = 62 - bits;
    }
    *scale = std::ldexp(1.0, F);
    *inv = std::ldexp(1.0, -F);
}

// Argument record of a problem for the batched kernels.
static void fill_req(vp_problem* p)
{
    const vp_params& P = p->P;
    ReqArgs& q = p->req;
    memset(&q, 0, sizeof q);
    SampleArgs& a = q.s;
    a.map = p->map;
    a.map32 = p->map32;
    a.offs = p->offs;
    a.obase = p->bsum;
    a.S1 = p->S1;
    a.S2 = p->S2;
    a.hist_part = p->hist_part;
    a.rec_h = p->rec_h;
    a.rec_n = p->rec_n;
    a.rec_bin = p->rec_bin;
    a.rec_stride = p->rec_stride;
    a.bx = p->bx;
    a.bj = p->bj;
    a.bf = p->bf;
    a.bidx = p->bidx;
    a.bcap = p->bcap;
    a.edges = p->edges;
    a.nonfinite = &p->st->nonfinite;
    a.f = p->f_d;
    a.fc = p->fc;
    a.n_hc = p->n_hc;
    a.n_g = P.n_g;
    a.n_st = p->n_st;
    a.R = p->R;
    a.R32 = (float)P.n_g / (float)p->n_st;
    a.R53 = std::ldexp(a.R, -53);
    a.R32s = std::ldexp(a.R32, -24);
    a.key0 = (uint32_t)(P.seed & 0xffffffffu);
    a.key1 = (uint32_t)(P.seed >> 32);
    a.it = (uint32_t)p->it;
    a.hist_mode = P.hist_mode;
    a.hist_axes = p->hist_axes;
    a.map_lds = p->map_lds;
    a.chunk = p->chunk;
    fixed_weight_scale(p, &a.wscale, &a.wscale_inv);
    q.n_h = p->n_h;
    q.offs = p->offs;
    q.bsum = p->bsum;
    q.S1 = p->S1;
    q.S2 = p->S2;
    q.dh = p->dh;
    q.H = p->H;
    q.W = p->W;
    q.hist_part = p->hist_part;
    q.edges = p->edges;
    q.est_part = p->est_part;
    q.hist_I = p->hist_I;
    q.hist_V = p->hist_V;
    q.st = p->st;
    q.map = p->map;
    q.map32 = p->map32;
    q.n_hc = p->n_hc;
    q.n_waves = p->n_waves;
    q.dim = P.dim;
    q.n_g = P.n_g;
    q.omega = p->omega;
    q.omega2 = p->omega2;
    q.alpha = P.alpha;
    q.beta = P.beta;
    q.n_ev = (double)P.n_ev;
    q.plus2 = P.realloc_plus2;
    q.n_discard = P.n_discard;
    q.n_adapt = P.n_adapt;
    q.average = P.average;
    q.slot = p->slot;
    q.grid = p->grid;
    q.est_blocks = est_grid(p->n_hc);
    q.hist_axes = p->hist_axes;
    q.rec_chunks = p->rec_chunks;
    q.rec_slices = p->rec_slices;
    q.rec_axes = p->rec_axes;
    q.checks = (P.flags & VP_FLAG_CHECKS) ? 1 : 0;
    q.det = (P.flags & VP_FLAG_DETERMINISTIC) ? 1 : 0;
    q.bounds = p->bounds_d;
}

// Writes the device copies of the iteration counters.
static hipError_t push_counters(vp_problem* p)
{
    uint32_t it = (uint32_t)p->it;
    int32_t slot = p->slot;
    hipError_t e = hipMemcpy((char*)p->d_req + offsetof(ReqArgs, s) + offsetof(SampleArgs, it), &it,
                             sizeof it, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy((char*)p->d_req + offsetof(ReqArgs, slot), &slot, sizeof slot, hipMemcpyHostToDevice);
    return e;
}

// ---------------------------------------------------------------- C ABI
extern "C" {

const char* vp_status_string(vp_status s)
{
    switch (s) {
    case VP_OK: return "ok";
    case VP_ERR_INVALID_ARG: return "invalid argument";
    case VP_ERR_OOM: return "out of memory";
    case VP_ERR_DEVICE: return "device error";
    case VP_ERR_NUMERIC: return "non-finite integrand values";
    case VP_ERR_NOT_READY: return "not ready";
    case VP_ERR_CANCELLED: return "cancelled";
    case VP_ERR_STATE: return "invalid state";
    case VP_ERR_INVARIANT: return "invariant violated";
    }
    return "unknown status";
}

const char* vp_last_error(void) { return g_err.c_str(); }

vp_status vp_ctx_create(int device, void* hip_stream, vp_ctx** out)
{
    if (!out) return fail(VP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    VP_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(VP_ERR_INVALID_ARG, "device %d not in 0..%d", device, n - 1);
    VP_HIP(hipSetDevice(device));
    vp_ctx* c = new vp_ctx();
    c->device = device;
    c->refs = 1;
    c->own_stream = (hip_stream == nullptr);
    if (c->own_stream) {
        hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete c;
            return fail(VP_ERR_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
        }
    } else {
        c->stream = (hipStream_t)hip_stream;
    }
    int cu = 0, lds = 0;
    (void)hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device);
    (void)hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    c->n_cu = cu > 0 ? cu : 1;
    c->lds_max = lds > 0 ? (size_t)lds : 65536;
    {
        hipError_t e = scratch_init(device);
        if (e != hipSuccess) {
            if (c->own_stream) (void)hipStreamDestroy(c->stream);
            delete c;
            return fail(VP_ERR_DEVICE, "workspace address on device %d: %s", device, hipGetErrorString(e));
        }
    }
    {
        hipError_t e = aux_init(c->lds_max);
        if (e != hipSuccess) {
            if (c->own_stream) (void)hipStreamDestroy(c->stream);
            delete c;
            return fail(VP_ERR_DEVICE, "configuring kernels: %s", hipGetErrorString(e));
        }
    }
    // the side stream of the iteration tail (optional: without it the tail
    // runs in one stream)
    if (hipEventCreateWithFlags(&c->side.fork, hipEventDisableTiming) == hipSuccess) {
        if (hipStreamCreateWithFlags(&c->side.st[0], hipStreamNonBlocking) == hipSuccess) {
            if (hipEventCreateWithFlags(&c->side.join[0], hipEventDisableTiming) == hipSuccess) c->side.n = 1;
            else (void)hipStreamDestroy(c->side.st[0]);
        }
    } else {
        c->side.fork = nullptr;
    }
    *out = c;
    return VP_OK;
}

vp_status vp_ctx_destroy(vp_ctx* c)
{
    if (!c) return VP_OK;
    ctx_release(c);
    return VP_OK;
}

vp_status vp_ctx_info(vp_ctx* c, int32_t* n_cu, int64_t* lds)
{
    if (!c) return fail(VP_ERR_INVALID_ARG, "ctx is NULL");
    if (n_cu) *n_cu = c->n_cu;
    if (lds) *lds = (int64_t)c->lds_max;
    return VP_OK;
}

}  // extern "C"

// Derived sizes and the sampling launch shape of a problem.
struct Shape {
    int32_t n_st;           // axis 0
    int32_t nst_ax[kMaxDim];
    bool mix;               // counts differ between axes
    int64_t n_hc;
    int hist_axes, map_lds;
    SampleEntry entry;
    int block, chunk, grid;
    size_t lds;
    int64_t n_waves;
    int32_t hist_cap;
    int64_t rec_stride;  // records path: sample positions held (0: LDS path)
    int32_t rec_chunks, rec_slices, rec_axes;
    // batched integrand: the generate-mode kernel, its LDS, and the sample
    // capacity of the point buffers (0: not batched)
    SampleEntry gen_entry;
    size_t gen_lds;
    int gen_grid;  // its own grid: it holds no training data, so many workgroups fit per CU
    int64_t bcap;
    int n_out;     // components of the integrand (1: scalar)
    int vec_grid;  // vector estimates: workgroups per pair of components
};

// The integrand constants in the sampling kernel's layout (fc_count elements:
// scale, affine constant, coefficients, amplitudes, radii^2, the K centres of
// each axis side by side, the Cholesky factor), as double on the FP64 path and
// as float on the split paths.
static void write_constants(const IntegrandDev& f, int prec, int D, int n_g, const int32_t* nst_ax, char* out)
{
    const int n = fc_count(f.kind, D);
    const int so = fc_strat_offset(f.kind, D);
    const bool gauss_like = f.kind == VP_F_GAUSS_MIX || f.kind == VP_F_EXP_ABS || f.kind == VP_F_BALLS;
    for (int i = 0; i < n; ++i) {
        double v = 0.0;
        float v32 = 0.0f;
        if (i == 0) {
            v = f.scale;
            v32 = f.scale32;
        } else if (i == 1) {
            if (f.kind == VP_F_AFFINE) {
                v = f.centers[0];
                v32 = f.centers32[0];
            }
        } else if (i >= 4 && i < kFcHead) {
            const int k = i & 3;
            const double* src = i < 8 ? f.coefs : (i < 12 ? f.amps : f.rad2);
            const float* src32 = i < 8 ? f.coefs32 : (i < 12 ? f.amps32 : f.rad2_32);
            v = src[k];
            v32 = src32[k];
        } else if (i >= kFcHead && i < kFcHead + 4 * D) {
            const int mu = (i - kFcHead) >> 2, k = (i - kFcHead) & 3;
            int c = -1;
            if (gauss_like && k < f.n_terms) c = k * D + mu;
            else if (f.kind == VP_F_CORR_GAUSS && k == 0) c = mu;
            else if (f.kind == VP_F_AFFINE && k == 0) c = mu + 1;
            if (c >= 0) {
                v = f.centers[c];
                v32 = f.centers32[c];
            }
        } else if (i >= so + D) {
            v = (double)nst_ax[i - so - D];
            v32 = (float)nst_ax[i - so - D];
        } else if (i >= so) {
            // R_mu as the uniform path computes R (double) and R32 (float)
            v = (double)n_g / (double)nst_ax[i - so];
            v32 = (float)n_g / (float)nst_ax[i - so];
        } else if (i >= kFcHead + 4 * D) {
            v = f.chol[i - kFcHead - 4 * D];
            v32 = f.chol32[i - kFcHead - 4 * D];
        }
        if (prec == VP_FP64) memcpy(out + i * sizeof(double), &v, sizeof v);
        else memcpy(out + i * sizeof(float), &v32, sizeof v32);
    }
}

// Resident sampling workgroups per CU; the query (and the kernel attribute it
// sets) is made once per device, kernel, block size and LDS size.
static int cached_occupancy(int device, const SampleEntry& e, int block, size_t lds)
{
    static std::mutex mu;
    static std::map<std::tuple<int, void*, int, size_t>, int> cache;
    const auto key = std::make_tuple(device, (void*)e.launch, block, lds);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    const int occ = e.occupancy(block, lds);
    cache[key] = occ;
    return occ;
}

static vp_status compute_shape(vp_ctx* ctx, const vp_params* P, const vp_integrand* f, int64_t samples_per_wg,
                               Shape* sh)
{
    const int D = P->dim, NG = P->n_g;
    strat_counts(P, sh->nst_ax);
    sh->n_st = sh->nst_ax[0];
    sh->mix = false;
    int64_t nhc = 1;
    for (int d = 0; d < D; ++d) {
        nhc *= sh->nst_ax[d];
        if (sh->nst_ax[d] != sh->n_st) sh->mix = true;
    }
    sh->n_hc = nhc;
    const int prec = P->precision;
    // the sampling kernels join a digit and the random bits of its axis in
    // one 32-bit word at these dimensions (uniform counts only); validation
    // already keeps N_st^D <= n_ev / 2 < 2^30, which bounds the digits
    if (!sh->mix && ((prec == VP_FP64 && D >= 6 && sh->n_st > 32) || (prec != VP_FP64 && D >= 4 && sh->n_st > 256)))
        return fail(VP_ERR_INVALID_ARG, "n_st %d too large for dim %d", sh->n_st, D);
    // training data: as many axes as fit privatised in LDS beside the
    // integrand constants, the rest as records
    const size_t fcb = fc_lds_bytes(prec, f->kind, D) + 16;
    const bool det = (P->flags & VP_FLAG_DETERMINISTIC) != 0;
    int fit = std::max<int>(1, (int)((ctx->lds_max - fcb) / (2 * sizeof(double) * (size_t)NG)));
    // deterministic mode: every axis as records, binned in slices of at most
    // two axes (small workgroups of one wave, several per CU)
    if (det) fit = std::min(fit, 2);
    sh->hist_axes = det ? 0 : std::min(D, fit);
    if (prec == VP_FP32_NEUMAIER && sh->hist_axes < D)
        return fail(VP_ERR_INVALID_ARG, "compensated sums need dim * n_g * 16 <= %zu bytes of LDS", ctx->lds_max);
    const size_t hb = hist_lds_bytes(sh->hist_axes, NG);
    const bool batch = f->kind == VP_F_BATCH;
    const bool rec = sh->hist_axes < D;
    // Map placement.  Double precision: the whole map in LDS when it fits
    // beside the training data, else its innermost axes when they fit, else
    // global memory.  The split precisions stage only the innermost axes (the
    // ones whose increments the lanes of a wave scatter over the whole axis;
    // the outer axes' reads fall in a few cache lines per wave and stay with
    // the vector-memory path, which keeps them out of the LDS queue of the
    // training-data atomics).  The accumulate mode of a batched integrand
    // reads no map.
    sh->map_lds = MAP_GLOBAL;
    if (!batch && !rec && prec == VP_FP64) {
        if (hb + map_lds_bytes(prec, D, NG, MAP_LDS) + fcb <= ctx->lds_max) sh->map_lds = MAP_LDS;
        else if (D > kMapInnerAxes && hb + map_lds_bytes(prec, D, NG, MAP_INNER) + fcb <= ctx->lds_max)
            sh->map_lds = MAP_INNER;
    } else if (!batch && !rec && D > kMapInnerAxes &&
               hb + map_lds_bytes(prec, D, NG, MAP_INNER) + fcb <= ctx->lds_max) {
        sh->map_lds = MAP_INNER;
    }
    sh->entry = sample_entry(prec, f->kind, f->n_terms, D, sh->map_lds, rec, sh->mix);
    if (!sh->entry.launch && sh->map_lds != MAP_GLOBAL) {
        sh->map_lds = MAP_GLOBAL;
        sh->entry = sample_entry(prec, f->kind, f->n_terms, D, MAP_GLOBAL, rec, sh->mix);
    }
    if (!sh->entry.launch) return fail(VP_ERR_INVALID_ARG, "no sampling kernel for dim %d", D);
    sh->block = sh->entry.block;
    sh->lds = fc_lds_offset(hb, sh->map_lds, prec, D, NG) + fc_lds_bytes(prec, f->kind, D);
    sh->chunk = 16;
    int occ = cached_occupancy(ctx->device, sh->entry, sh->block, sh->lds);
    if (occ < 1) occ = 1;
    const int64_t n_tot_max = P->n_ev + 2 * nhc;
    sh->bcap = 0;
    sh->n_out = f->n_out > 1 ? f->n_out : 1;
    sh->vec_grid = sh->n_out > 1 ? vec_grid(nhc) : 0;
    sh->gen_lds = 0;
    sh->gen_grid = 0;
    sh->gen_entry = SampleEntry{nullptr, nullptr, 0};
    if (batch) {
        // the generate mode holds no training data: its map goes to LDS whenever it fits
        const int gmap = map_lds_bytes(VP_FP64, D, NG, MAP_LDS) + fcb <= ctx->lds_max ? MAP_LDS : MAP_GLOBAL;
        sh->gen_entry = sh->mix ? sample_entry_fp64_batch_gen_mix(D, gmap) : sample_entry_fp64_batch_gen(D, gmap);
        if (!sh->gen_entry.launch) return fail(VP_ERR_INVALID_ARG, "no batched-integrand kernel for dim %d", D);
        sh->gen_lds = fc_lds_offset(0, gmap, VP_FP64, D, NG) + fc_lds_bytes(VP_FP64, VP_F_BATCH, D);
        const int gocc = std::max(1, cached_occupancy(ctx->device, sh->gen_entry, sh->gen_entry.block, sh->gen_lds));
        const int64_t gwpb = sh->gen_entry.block / kWave;
        const int64_t guseful = std::max<int64_t>(1, n_tot_max / ((int64_t)kWave * 16));
        sh->gen_grid = (int)std::max<int64_t>(
            1, std::min<int64_t>((int64_t)ctx->n_cu * gocc, (guseful + gwpb - 1) / gwpb));
        sh->bcap = (n_tot_max + 63) / 64 * 64;
    }
    const int64_t waves_per_block = sh->block / kWave;
    const int64_t useful_waves = std::max<int64_t>(1, n_tot_max / ((int64_t)kWave * sh->chunk));
    int64_t grid = (int64_t)ctx->n_cu * occ;
    grid = std::min<int64_t>(grid, (useful_waves + waves_per_block - 1) / waves_per_block);
    if (samples_per_wg > 0) grid = std::min<int64_t>(grid, (n_tot_max + samples_per_wg - 1) / samples_per_wg);
    sh->grid = (int)std::max<int64_t>(1, grid);
    sh->n_waves = (int64_t)sh->grid * waves_per_block;
    sh->hist_cap = samples_per_wg > 0 ? std::max<int32_t>(1, P->n_iter) : kMaxHistory;
    sh->rec_stride = 0;
    sh->rec_chunks = sh->rec_slices = sh->rec_axes = 0;
    if (sh->hist_axes < D) {
        // axis slices of the remaining axes whose two planes fit in LDS,
        // balanced; chunks of at least 64 Ki samples, about two workgroups per
        // CU over all slices
        const int rem = D - sh->hist_axes;
        sh->rec_slices = (rem + fit - 1) / fit;
        sh->rec_axes = (rem + sh->rec_slices - 1) / sh->rec_slices;
        const int64_t per_cu = det ? 16 : 2;
        const int64_t want = (per_cu * (int64_t)ctx->n_cu + sh->rec_slices - 1) / sh->rec_slices;
        sh->rec_chunks = (int32_t)std::max<int64_t>(1, std::min<int64_t>(want, (n_tot_max + 65535) / 65536));
        // a multiple of 64, so that the three record arrays (8-, 4- and 2-byte
        // elements) follow each other exactly at 256-byte boundaries
        sh->rec_stride = (n_tot_max + 63) / 64 * 64;
    }
    return VP_OK;
}

// Byte offsets of a problem's device buffers inside its one allocation.  The
// records the host writes at creation (integrand, scalars, argument record,
// map bounds) come first, so one copy initialises them.
struct Layout {
    size_t f_d, st, d_req, bounds, fc, head_end, map, map32;
    size_t n_h, offs, bsum, S1, S2, dh, H, W, hist, edges, est_part, hist_I, hist_V, rec_h, rec_n, rec_bin;
    size_t bx, bj, bf, bidx;
    size_t vI, vC, vpart, vout, total;
};

static Layout layout_of(const vp_params* P, const Shape& sh)
{
    const int64_t D = P->dim, NG = P->n_g, nhc = sh.n_hc, nbins = D * NG;
    Layout L;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t o = at;
        at += (bytes + 255) & ~(size_t)255;
        return o;
    };
    L.f_d = take(sizeof(IntegrandDev));
    L.st = take(sizeof(DevState));
    L.d_req = take(sizeof(ReqArgs));
    L.bounds = take((size_t)2 * D * sizeof(double));
    L.fc = take(fc_lds_bytes(VP_FP64, VP_F_CORR_GAUSS, (int)D));
    L.head_end = at;
    L.map = take((size_t)D * (NG + 1) * sizeof(double));
    L.map32 = take((size_t)D * (NG + 1) * sizeof(float));
    L.n_h = take((size_t)nhc * sizeof(int32_t));
    L.offs = take((size_t)(nhc + 1) * sizeof(int64_t));
    L.bsum = take((size_t)(scan_blocks(nhc) + 1) * sizeof(int64_t));
    L.S1 = take((size_t)nhc * sizeof(double));
    L.S2 = take((size_t)nhc * sizeof(double));
    L.dh = take((size_t)nhc * sizeof(double));
    L.H = take((size_t)nbins * sizeof(double));
    L.W = take((size_t)nbins * sizeof(double));
    L.hist = take((size_t)std::max(sh.grid, sh.rec_chunks) * 2 * nbins * sizeof(double));
    L.edges = take((size_t)2 * sh.n_waves * sizeof(EdgeRec));
    L.est_part = take((size_t)3 * est_grid(nhc) * sizeof(double));
    L.hist_I = take((size_t)sh.hist_cap * sizeof(double));
    L.hist_V = take((size_t)sh.hist_cap * sizeof(double));
    // records: values, counts and bins contiguous (the sampling kernel derives
    // the second and third array from the first)
    L.rec_h = take((size_t)sh.rec_stride * sizeof(double));
    L.rec_n = take((size_t)sh.rec_stride * sizeof(uint32_t));
    L.rec_bin = take((size_t)sh.rec_stride * (D - sh.hist_axes) * sizeof(uint16_t));
    // batched integrand: points, J, f and increment indices
    L.bx = take((size_t)sh.bcap * D * sizeof(double));
    L.bj = take((size_t)sh.bcap * sizeof(double));
    L.bf = take((size_t)sh.bcap * sh.n_out * sizeof(double));
    L.bidx = take((size_t)sh.bcap * ((D + 7) / 8) * 8 * sizeof(uint16_t));
    // vector-valued integrand: per-iteration estimates and covariances,
    // partial sums, combined result
    const size_t M = sh.n_out > 1 ? (size_t)sh.n_out : 0;
    L.vI = take((size_t)kVecHistory * M * sizeof(double));
    L.vC = take((size_t)kVecHistory * M * M * sizeof(double));
    L.vpart = take((size_t)(M * (M + 1) / 2 + M) * sh.vec_grid * sizeof(double));
    L.vout = take((M ? M + M * M + 2 : 0) * sizeof(double));
    L.total = at;
    return L;
}

size_t vp::problem_head_bytes_max()
{
    // the head (integrand, state, argument record, bounds, constants) grows
    // with the dimension only
    vp_params P;
    memset(&P, 0, sizeof P);
    P.dim = kMaxDim;
    P.n_g = 1;
    Shape sh;
    memset(&sh, 0, sizeof sh);
    return layout_of(&P, sh).head_end;
}

vp_status vp::problem_bytes(vp_ctx* ctx, const vp_params* P, const vp_integrand* f, int64_t samples_per_wg,
                            size_t* bytes)
{
    vp_status s = validate(P, f);
    if (s != VP_OK) return s;
    Shape sh;
    s = compute_shape(ctx, P, f, samples_per_wg, &sh);
    if (s != VP_OK) return s;
    const size_t b = layout_of(P, sh).total;
    *bytes = b;
    return VP_OK;
}


vp_status vp::problem_create(vp_ctx* ctx, const vp_params* P, const vp_integrand* f, int64_t samples_per_wg,
                             DevicePool* pool, vp_problem** out, InitArgs* init_out)
{
    if (init_out && !pool) return fail(VP_ERR_INVALID_ARG, "a deferred initialisation needs a pool");
    if (!ctx || !out) return fail(VP_ERR_INVALID_ARG, "ctx and out are required");
    *out = nullptr;
    vp_status s = validate(P, f);
    if (s != VP_OK) return s;
    Shape sh;
    s = compute_shape(ctx, P, f, samples_per_wg, &sh);
    if (s != VP_OK) return s;
    VP_HIP(hipSetDevice(ctx->device));
    vp_problem* p = new vp_problem();
    p->ctx = ctx;
    ctx->refs += 1;
    p->P = *P;
    const int D = P->dim, NG = P->n_g;
    p->lower.assign(D, 0.0);
    p->upper.assign(D, 1.0);
    if (P->lower)
        for (int d = 0; d < D; ++d) {
            p->lower[d] = P->lower[d];
            p->upper[d] = P->upper[d];
        }
    p->P.lower = p->lower.data();
    p->P.upper = p->upper.data();
    fill_integrand(p->fh, f);
    p->n_st = sh.n_st;
    p->nst_ax.assign(sh.nst_ax, sh.nst_ax + D);
    p->P.n_st_axes = p->nst_ax.data();
    const int64_t nhc = sh.n_hc;
    p->n_hc = nhc;
    p->omega = 1.0 / (double)nhc;
    p->omega2 = p->omega * p->omega;
    p->R = (double)NG / (double)p->n_st;
    p->it = 0;
    p->slot = 0;
    p->hist_axes = sh.hist_axes;
    p->map_lds = sh.map_lds;
    p->entry = sh.entry;
    p->block = sh.block;
    p->lds = sh.lds;
    p->chunk = sh.chunk;
    p->grid = sh.grid;
    p->n_waves = sh.n_waves;
    p->hist_cap = sh.hist_cap;

    // device state: one allocation per problem
    const int64_t nbins = (int64_t)D * NG;
    const Layout lay = layout_of(P, sh);
    hipError_t e = hipSuccess;
    if (pool) {
        p->arena = pool->alloc(lay.total);
        if (p->arena) p->pool = pool;
        else e = hipErrorOutOfMemory;
    } else {
        e = hipMalloc((void**)&p->arena, lay.total);
    }
    if (e != hipSuccess) {
        p->arena = nullptr;
        problem_free(p);
        return fail(e == hipErrorOutOfMemory ? VP_ERR_OOM : VP_ERR_DEVICE, "allocating %zu bytes of problem state: %s",
                    lay.total, hipGetErrorString(e));
    }
    p->arena_bytes = lay.total;
    char* base = p->arena;
    p->f_d = (IntegrandDev*)(base + lay.f_d);
    p->fc = base + lay.fc;
    p->st = (DevState*)(base + lay.st);
    p->d_req = (ReqArgs*)(base + lay.d_req);
    p->map = (double*)(base + lay.map);
    p->map32 = (float*)(base + lay.map32);
    p->n_h = (int32_t*)(base + lay.n_h);
    p->offs = (int64_t*)(base + lay.offs);
    p->bsum = (int64_t*)(base + lay.bsum);
    p->S1 = (double*)(base + lay.S1);
    p->S2 = (double*)(base + lay.S2);
    p->dh = (double*)(base + lay.dh);
    p->H = (double*)(base + lay.H);
    p->W = (double*)(base + lay.W);
    p->hist_part = (double*)(base + lay.hist);
    p->rec_stride = sh.rec_stride;
    p->rec_chunks = sh.rec_chunks;
    p->rec_slices = sh.rec_slices;
    p->rec_axes = sh.rec_axes;
    p->rec_h = sh.rec_stride ? (double*)(base + lay.rec_h) : nullptr;
    p->rec_n = sh.rec_stride ? (uint32_t*)(base + lay.rec_n) : nullptr;
    p->rec_bin = sh.rec_stride ? (uint16_t*)(base + lay.rec_bin) : nullptr;
    p->bcap = sh.bcap;
    p->bx = sh.bcap ? (double*)(base + lay.bx) : nullptr;
    p->bj = sh.bcap ? (double*)(base + lay.bj) : nullptr;
    p->bf = sh.bcap ? (double*)(base + lay.bf) : nullptr;
    p->bidx = sh.bcap ? (uint16_t*)(base + lay.bidx) : nullptr;
    p->gen_entry = sh.gen_entry;
    p->gen_lds = sh.gen_lds;
    p->gen_grid = sh.gen_grid;
    p->n_out = sh.n_out;
    p->vec_grid = sh.vec_grid;
    p->vI = sh.n_out > 1 ? (double*)(base + lay.vI) : nullptr;
    p->vC = sh.n_out > 1 ? (double*)(base + lay.vC) : nullptr;
    p->vpart = sh.n_out > 1 ? (double*)(base + lay.vpart) : nullptr;
    p->vout = sh.n_out > 1 ? (double*)(base + lay.vout) : nullptr;
    p->batch_fn = f->kind == VP_F_BATCH ? f->fn : nullptr;
    p->batch_user = f->kind == VP_F_BATCH ? f->user : nullptr;
    p->edges = (EdgeRec*)(base + lay.edges);
    p->est_part = (double*)(base + lay.est_part);
    p->hist_I = (double*)(base + lay.hist_I);
    p->hist_V = (double*)(base + lay.hist_V);
    // the head of the allocation (integrand, scalars, argument record, map
    // bounds) is staged on the host and copied at once; the initial map
    // (Sec. 2.3: a uniform grid), the uniform allocation and the zero sums are
    // written by one kernel
    // (a served request's image goes to the pool's pinned staging memory,
    // else to a host vector kept with the problem)
    const char* head_dev = nullptr;
    char* head = pool ? pool->stage(lay.head_end, &head_dev) : nullptr;
    if (head) {
        memset(head, 0, lay.head_end);
    } else {
        p->staging.assign(lay.head_end, 0);
        head = p->staging.data();
    }
    memcpy(head + lay.f_d, &p->fh, sizeof(IntegrandDev));
    DevState st0;
    memset(&st0, 0, sizeof st0);
    st0.check_it = -1;
    memcpy(head + lay.st, &st0, sizeof st0);
    p->bounds_d = (const double*)(base + lay.bounds);
    fill_req(p);
    memcpy(head + lay.d_req, &p->req, sizeof(ReqArgs));
    memcpy(head + lay.bounds, p->lower.data(), D * sizeof(double));
    memcpy(head + lay.bounds + D * sizeof(double), p->upper.data(), D * sizeof(double));
    write_constants(p->fh, P->precision, D, NG, sh.nst_ax, head + lay.fc);
    hipStream_t sm = ctx->stream;
    int64_t n0 = P->n_ev / nhc;
    if (n0 < 2) n0 = 2;
    // a pinned image is read by the initialisation kernel itself (one launch
    // per request instead of a copy and a launch)
    if (!head_dev) e = hipMemcpyAsync(p->arena, head, lay.head_end, hipMemcpyHostToDevice, sm);
    if (e == hipSuccess) {
        InitArgs ia;
        ia.head_src = head_dev;
        ia.head_dst = head_dev ? p->arena : nullptr;
        ia.head_bytes = head_dev ? (int64_t)lay.head_end : 0;
        ia.bounds = (const double*)(head_dev ? head_dev + lay.bounds : base + lay.bounds);
        ia.map = p->map;
        ia.map32 = p->map32;
        ia.n_h = p->n_h;
        ia.S1 = p->S1;
        ia.S2 = p->S2;
        ia.H = p->H;
        ia.W = p->W;
        ia.n_hc = nhc;
        ia.nbins = nbins;
        ia.dim = D;
        ia.n_g = NG;
        ia.n0 = (int32_t)n0;
        if (init_out && head_dev) {
            *init_out = ia;
        } else {
            if (init_out) init_out->n_hc = -1;  // initialised here (no pinned image)
            launch_init(ia, sm);
            e = hipGetLastError();
        }
    }
    // stream-ordered creation leaves the initialisation queued before the
    // request's first kernels on the same stream (the staging copy lives in
    // the problem until it is freed)
    if (e == hipSuccess && !pool) e = hipStreamSynchronize(sm);
    if (e != hipSuccess) {
        problem_free(p);
        return fail(VP_ERR_DEVICE, "initialising problem state: %s", hipGetErrorString(e));
    }
    *out = p;
    return VP_OK;
}

vp_status vp::result_from_state(const DevState& st, vp_result* out)
{
    out->mean = st.mean;
    out->sdev = st.sdev;
    out->chi2 = st.chi2;
    out->dof = st.dof;
    out->n_iter_done = st.n_iter_done;
    out->n_evals = st.n_evals;
    out->n_near_ties = (int64_t)st.ties;
    out->n_nonfinite = (int64_t)st.nonfinite;
    if (st.check_flags)
        return fail(VP_ERR_INVARIANT, "device checks found broken invariants (flags 0x%x, first at iteration %d)",
                    st.check_flags, st.check_it);
    if (st.nonfinite) return fail(VP_ERR_NUMERIC, "%llu non-finite integrand values", st.nonfinite);
    return VP_OK;
}

// One iteration with a batched integrand (Sec. 1: the integrand is evaluated
// on batches of points): the allocation scan, the generate-mode sampler
// writing the iteration's points, the user's function on the library's
// stream, the accumulate-mode sampler, then the same passes as the fused path.
// The host reads N_tot (one synchronisation) to tell the function how many
// points there are.
static vp_status iterate_batch(vp_problem* p, int32_t n_iter)
{
    hipStream_t s = p->ctx->stream;
    const SampleGroup& g = p->plan.groups[0];
    if (!p->gen_plan_built) {
        // the generate mode's own launch table: the same argument record, its
        // own grid (the kernel partitions the samples by its launch's blocks
        // and writes no per-workgroup state)
        ReqArgs gq = p->req;
        gq.grid = p->gen_grid;
        std::vector<PlanReq> pr = {{&gq, p->d_req, p->gen_entry, p->gen_lds}};
        VP_HIP(p->gen_planner.build(pr, &p->gen_plan));
        p->gen_plan_built = true;
    }
    const SampleGroup& gg = p->gen_plan.groups[0];
    const int64_t* total = p->bsum + scan_blocks(p->n_hc);
    for (int32_t r = 0; r < n_iter; ++r) {
        hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
        if (p->prof) {
            e0 = take_event(p), e1 = take_event(p), e2 = take_event(p), e3 = take_event(p);
            VP_HIP(hipEventRecord(e2, s));
        }
        enqueue_head(p->plan, s);
        if (e0) VP_HIP(hipEventRecord(e0, s));
        p->gen_entry.launch(gg.L, gg.blocks, p->gen_entry.block, p->gen_lds, s);
        int64_t n_tot = 0;
        VP_HIP(hipMemcpyAsync(&n_tot, total, sizeof n_tot, hipMemcpyDeviceToHost, s));
        VP_HIP(hipStreamSynchronize(s));
        const int rc = p->batch_fn(p->batch_user, (void*)s, n_tot, p->P.dim, p->bx, p->bf);
        if (rc != 0) return fail(VP_ERR_DEVICE, "the batched integrand returned %d", rc);
        g.entry.launch(g.L, g.blocks, g.entry.block, g.lds, s);
        if (e1) VP_HIP(hipEventRecord(e1, s));
        if (p->n_out > 1) {
            VecArgs va;
            va.jac = p->bj;
            va.f = p->bf;
            va.offs = p->offs;
            va.obase = p->bsum;
            va.part = p->vpart;
            va.hist_I = p->vI;
            va.hist_C = p->vC;
            va.out = p->vout;
            va.n_hc = p->n_hc;
            va.cap = p->bcap;
            va.scale = p->fh.scale;
            va.omega = p->omega;
            va.omega2 = p->omega2;
            va.n_out = p->n_out;
            va.grid = p->vec_grid;
            va.slot = p->slot;
            va.n_discard = p->P.n_discard;
            va.average = p->P.average;
            launch_vec(va, s);
        }
        enqueue_tail(p->plan, s);
        if (e3) {
            VP_HIP(hipEventRecord(e3, s));
            p->ev_pending.push_back(e0);
            p->ev_pending.push_back(e1);
            p->ev_pending.push_back(e2);
            p->ev_pending.push_back(e3);
        }
        VP_HIP(hipGetLastError());
        p->it += 1;
        p->slot += 1;
    }
    return VP_OK;
}

extern "C" {

vp_status vp_problem_create(vp_ctx* ctx, const vp_params* P, const vp_integrand* f, vp_problem** out)
{
    TraceRange tr("vp_problem_create");
    return problem_create(ctx, P, f, 0, nullptr, out);
}

vp_status vp_problem_destroy(vp_problem* p)
{
    if (!p) return VP_OK;
    (void)hipSetDevice(p->ctx->device);
    (void)hipStreamSynchronize(p->ctx->stream);
    problem_free(p);
    return VP_OK;
}

vp_status vp_problem_info(vp_problem* p, int32_t* n_st, int64_t* n_hc)
{
    if (!p) return fail(VP_ERR_INVALID_ARG, "problem is NULL");
    if (n_st) *n_st = p->n_st;
    if (n_hc) *n_hc = p->n_hc;
    return VP_OK;
}

vp_status vp_problem_layout(vp_problem* p, int32_t* map_place, int32_t* hist_axes)
{
    if (!p) return fail(VP_ERR_INVALID_ARG, "problem is NULL");
    static_assert(VP_MAP_GLOBAL == MAP_GLOBAL && VP_MAP_LDS == MAP_LDS && VP_MAP_INNER == MAP_INNER,
                  "map placements of the header and the kernels agree");
    if (map_place) *map_place = p->map_lds;
    if (hist_axes) *hist_axes = p->hist_axes;
    return VP_OK;
}

vp_status vp_problem_strat(vp_problem* p, int32_t* n_st_axes)
{
    if (!p || !n_st_axes) return fail(VP_ERR_INVALID_ARG, "problem and n_st_axes are required");
    for (size_t d = 0; d < p->nst_ax.size(); ++d) n_st_axes[d] = p->nst_ax[d];
    return VP_OK;
}

vp_status vp_iterate(vp_problem* p, int32_t n_iter)
{
    TraceRange tr("vp_iterate");
    if (!p || n_iter < 0) return fail(VP_ERR_INVALID_ARG, "problem is NULL or n_iter < 0");
    if (p->slot + n_iter > p->hist_cap) return fail(VP_ERR_STATE, "more than %d iterations", p->hist_cap);
    if (p->n_out > 1 && p->slot + n_iter > kVecHistory)
        return fail(VP_ERR_STATE, "more than %d iterations of a vector-valued integrand", kVecHistory);
    VP_HIP(hipSetDevice(p->ctx->device));
    hipStream_t s = p->ctx->stream;
    if (!p->plan_built) {
        std::vector<PlanReq> pr = {{&p->req, p->d_req, p->entry, p->lds}};
        VP_HIP(p->planner.build(pr, &p->plan));
        p->plan_built = true;
    }
    if (p->batch_fn) return iterate_batch(p, n_iter);
    for (int32_t r = 0; r < n_iter; ++r) {
        TraceRange tri("vegas+ iteration: enqueue");
        if (p->prof) {
            hipEvent_t e0 = take_event(p), e1 = take_event(p), e2 = take_event(p), e3 = take_event(p);
            VP_HIP(hipEventRecord(e2, s));
            enqueue_iteration(p->plan, s, e0, e1, &p->ctx->side);
            VP_HIP(hipEventRecord(e3, s));
            p->ev_pending.push_back(e0);
            p->ev_pending.push_back(e1);
            p->ev_pending.push_back(e2);
            p->ev_pending.push_back(e3);
        } else {
            enqueue_iteration(p->plan, s, nullptr, nullptr, &p->ctx->side);
        }
        VP_HIP(hipGetLastError());
        p->it += 1;
        p->slot += 1;
    }
    return VP_OK;
}

vp_status vp_sync(vp_problem* p)
{
    if (!p) return fail(VP_ERR_INVALID_ARG, "problem is NULL");
    VP_HIP(hipStreamSynchronize(p->ctx->stream));
    return VP_OK;
}

vp_status vp_result_get(vp_problem* p, vp_result* out, double* I_j, double* sig_j, double* V_j, int32_t cap)
{
    TraceRange tr("vp_result_get");
    if (!p || !out) return fail(VP_ERR_INVALID_ARG, "problem and out are required");
    VP_HIP(hipStreamSynchronize(p->ctx->stream));
    DevState st;
    VP_HIP(hipMemcpy(&st, p->st, sizeof st, hipMemcpyDeviceToHost));
    const int32_t n = std::min<int32_t>(cap, st.n_iter_done);
    if (I_j && n > 0) VP_HIP(hipMemcpy(I_j, p->hist_I, sizeof(double) * n, hipMemcpyDeviceToHost));
    if ((V_j || sig_j) && n > 0) {
        std::vector<double> v(n);
        VP_HIP(hipMemcpy(v.data(), p->hist_V, sizeof(double) * n, hipMemcpyDeviceToHost));
        for (int32_t i = 0; i < n; ++i) {
            if (V_j) V_j[i] = v[i];
            if (sig_j) sig_j[i] = std::sqrt(v[i]);
        }
    }
    return result_from_state(st, out);
}

vp_status vp_check_get(vp_problem* p, uint32_t* flags, int32_t* first_it)
{
    if (!p) return fail(VP_ERR_INVALID_ARG, "problem is NULL");
    if (!(p->P.flags & VP_FLAG_CHECKS)) return fail(VP_ERR_STATE, "the problem was created without VP_FLAG_CHECKS");
    static_assert(VP_CHECK_MAP_ORDER == CHECK_MAP_ORDER && VP_CHECK_MAP_ENDS == CHECK_MAP_ENDS &&
                      VP_CHECK_NH_MIN == CHECK_NH_MIN && VP_CHECK_NH_SUM == CHECK_NH_SUM,
                  "check bits of the header and the kernels agree");
    VP_HIP(hipSetDevice(p->ctx->device));
    VP_HIP(hipStreamSynchronize(p->ctx->stream));
    DevState st;
    VP_HIP(hipMemcpy(&st, p->st, sizeof st, hipMemcpyDeviceToHost));
    if (flags) *flags = st.check_flags;
    if (first_it) *first_it = st.check_it;
    return VP_OK;
}

vp_status vp_map_get(vp_problem* p, double* map)
{
    if (!p || !map) return fail(VP_ERR_INVALID_ARG, "problem and map are required");
    VP_HIP(hipStreamSynchronize(p->ctx->stream));
    VP_HIP(hipMemcpy(map, p->map, sizeof(double) * p->P.dim * (p->P.n_g + 1), hipMemcpyDeviceToHost));
    return VP_OK;
}

vp_status vp_map_set(vp_problem* p, const double* map)
{
    if (!p || !map) return fail(VP_ERR_INVALID_ARG, "problem and map are required");
    const int D = p->P.dim, NG = p->P.n_g;
    std::vector<float> m32((size_t)D * (NG + 1));
    for (int d = 0; d < D; ++d)
        for (int i = 0; i <= NG; ++i) {
            const double v = map[(size_t)d * (NG + 1) + i];
            if (!std::isfinite(v)) return fail(VP_ERR_INVALID_ARG, "map has a non-finite point");
            if (i > 0 && v < map[(size_t)d * (NG + 1) + i - 1])
                return fail(VP_ERR_INVALID_ARG, "map axis %d decreases at %d", d, i);
            m32[(size_t)d * (NG + 1) + i] = (float)v;
        }
    VP_HIP(hipStreamSynchronize(p->ctx->stream));
    VP_HIP(hipMemcpy(p->map, map, sizeof(double) * m32.size(), hipMemcpyHostToDevice));
    VP_HIP(hipMemcpy(p->map32, m32.data(), sizeof(float) * m32.size(), hipMemcpyHostToDevice));
    return VP_OK;
}

vp_status vp_alloc_get(vp_problem* p, int32_t* n_h)
{
    if (!p || !n_h) return fail(VP_ERR_INVALID_ARG, "problem and n_h are required");
    VP_HIP(hipStreamSynchronize(p->ctx->stream));
    VP_HIP(hipMemcpy(n_h, p->n_h, sizeof(int32_t) * p->n_hc, hipMemcpyDeviceToHost));
    return VP_OK;
}

vp_status vp_alloc_set(vp_problem* p, const int32_t* n_h)
{
    if (!p || !n_h) return fail(VP_ERR_INVALID_ARG, "problem and n_h are required");
    int64_t tot = 0;
    for (int64_t h = 0; h < p->n_hc; ++h) {
        if (n_h[h] < 2) return fail(VP_ERR_INVALID_ARG, "n_h[%lld] = %d < 2", (long long)h, n_h[h]);
        tot += n_h[h];
    }
    // the reallocation rule never exceeds N_ev + 2 N_hc; the sampling grid and
    // the training-record buffers are sized for that
    const int64_t cap = p->P.n_ev + 2 * p->n_hc;
    if (tot > cap)
        return fail(VP_ERR_INVALID_ARG, "allocation of %lld samples exceeds n_ev + 2 n_hc = %lld", (long long)tot,
                    (long long)cap);
    VP_HIP(hipStreamSynchronize(p->ctx->stream));
    VP_HIP(hipMemcpy(p->n_h, n_h, sizeof(int32_t) * p->n_hc, hipMemcpyHostToDevice));
    return VP_OK;
}

vp_status vp_iteration_get(vp_problem* p, int32_t* it)
{
    if (!p || !it) return fail(VP_ERR_INVALID_ARG, "problem and it are required");
    *it = p->it;
    return VP_OK;
}

vp_status vp_iteration_set(vp_problem* p, int32_t it)
{
    if (!p || it < 0) return fail(VP_ERR_INVALID_ARG, "problem is NULL or it < 0");
    VP_HIP(hipStreamSynchronize(p->ctx->stream));
    p->it = it;
    VP_HIP(push_counters(p));
    return VP_OK;
}

vp_status vp_accum_get(vp_problem* p, double* S1, double* S2, double* H, double* W)
{
    if (!p) return fail(VP_ERR_INVALID_ARG, "problem is NULL");
    VP_HIP(hipStreamSynchronize(p->ctx->stream));
    const size_t nb = (size_t)p->P.dim * p->P.n_g;
    if (S1) VP_HIP(hipMemcpy(S1, p->S1, sizeof(double) * p->n_hc, hipMemcpyDeviceToHost));
    if (S2) VP_HIP(hipMemcpy(S2, p->S2, sizeof(double) * p->n_hc, hipMemcpyDeviceToHost));
    if (H) VP_HIP(hipMemcpy(H, p->H, sizeof(double) * nb, hipMemcpyDeviceToHost));
    if (W) VP_HIP(hipMemcpy(W, p->W, sizeof(double) * nb, hipMemcpyDeviceToHost));
    return VP_OK;
}

// Per-sample dump: the next iteration's sampling kernel writes samples
// [first, first + count) through a second copy of its sample walk, taken only
// by tiles that hold such samples.
vp_status vp_debug_dump(vp_problem* p, int64_t first, int64_t count)
{
    if (!p || first < 0 || count < 0 || count > kMaxDump)
        return fail(VP_ERR_INVALID_ARG, "problem is NULL, first < 0 or count outside [0, %lld]", (long long)kMaxDump);
    if (p->batch_fn) return fail(VP_ERR_STATE, "the per-sample dump is not available for batched integrands");
    VP_HIP(hipSetDevice(p->ctx->device));
    VP_HIP(hipStreamSynchronize(p->ctx->stream));
    const int D = p->P.dim;
    const size_t need = (size_t)count * (sizeof(int64_t) + sizeof(int32_t) * (1 + D) + sizeof(double) * (D + 2));
    if (count > 0 && need > p->dump_bytes) {
        if (p->dump_mem) VP_HIP(hipFree(p->dump_mem));
        p->dump_mem = nullptr;
        p->dump_bytes = 0;
        if (hipMalloc((void**)&p->dump_mem, need) != hipSuccess) {
            p->dump_mem = nullptr;
            return fail(VP_ERR_OOM, "dump of %lld samples", (long long)count);
        }
        p->dump_bytes = need;
    }
    DumpArgs d = {};
    if (count > 0) {
        char* b = p->dump_mem;
        d.h = reinterpret_cast<int64_t*>(b);
        d.x = reinterpret_cast<double*>(b + (size_t)count * 8);
        d.jac = d.x + (size_t)count * D;
        d.fx = d.jac + count;
        d.j = reinterpret_cast<int32_t*>(d.fx + count);
        d.idx = d.j + count;
        d.first = first;
        d.count = count;
        d.it = (uint32_t)p->it;
        // entries the iteration does not reach keep h = -1
        VP_HIP(hipMemset(d.h, 0xff, (size_t)count * sizeof(int64_t)));
    }
    p->dump = d;
    p->req.s.dump = d;
    VP_HIP(hipMemcpy((char*)p->d_req + offsetof(ReqArgs, s) + offsetof(SampleArgs, dump), &d, sizeof d,
                     hipMemcpyHostToDevice));
    return VP_OK;
}

vp_status vp_debug_dump_get(vp_problem* p, int64_t* n_out, int64_t* h, int32_t* j, int32_t* idx, double* x,
                            double* jac, double* fx)
{
    if (!p || !n_out) return fail(VP_ERR_INVALID_ARG, "problem and n_out are required");
    if (p->dump.count == 0) return fail(VP_ERR_STATE, "no dump is armed");
    VP_HIP(hipSetDevice(p->ctx->device));
    VP_HIP(hipStreamSynchronize(p->ctx->stream));
    if (p->it <= (int32_t)p->dump.it) return fail(VP_ERR_STATE, "the dumped iteration has not run");
    const int64_t c = p->dump.count;
    const int D = p->P.dim;
    std::vector<int64_t> hh((size_t)c);
    VP_HIP(hipMemcpy(hh.data(), p->dump.h, sizeof(int64_t) * c, hipMemcpyDeviceToHost));
    int64_t n = 0;
    while (n < c && hh[(size_t)n] >= 0) ++n;
    *n_out = n;
    // the arrays are [count] and [dim][count] on the device; the caller's are
    // [n] and [dim][n]
    if (h) memcpy(h, hh.data(), sizeof(int64_t) * n);
    if (j && n) VP_HIP(hipMemcpy(j, p->dump.j, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    if (jac && n) VP_HIP(hipMemcpy(jac, p->dump.jac, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (fx && n) VP_HIP(hipMemcpy(fx, p->dump.fx, sizeof(double) * n, hipMemcpyDeviceToHost));
    for (int d = 0; d < D && n; ++d) {
        if (idx) VP_HIP(hipMemcpy(idx + (size_t)d * n, p->dump.idx + (size_t)d * c, sizeof(int32_t) * n,
                                  hipMemcpyDeviceToHost));
        if (x) VP_HIP(hipMemcpy(x + (size_t)d * n, p->dump.x + (size_t)d * c, sizeof(double) * n,
                                hipMemcpyDeviceToHost));
    }
    return VP_OK;
}

vp_status vp_result_vec_get(vp_problem* p, double* mean, double* cov, double* chi2, int32_t* dof, double* I_j,
                            double* C_j, int32_t cap)
{
    if (!p || cap < 0) return fail(VP_ERR_INVALID_ARG, "problem is NULL or cap < 0");
    const int m = p->n_out;
    if (m <= 1) {
        // a scalar problem: its result as a vector of one component
        vp_result r;
        vp_status st = vp_result_get(p, &r, I_j, nullptr, C_j, cap);
        if (st != VP_OK && st != VP_ERR_NUMERIC) return st;
        if (mean) mean[0] = r.mean;
        if (cov) cov[0] = r.sdev * r.sdev;
        if (chi2) *chi2 = r.chi2;
        if (dof) *dof = r.dof;
        return st;
    }
    VP_HIP(hipSetDevice(p->ctx->device));
    VP_HIP(hipStreamSynchronize(p->ctx->stream));
    std::vector<double> out((size_t)m + m * m + 2);
    const int done = p->slot;
    if (done > 0) {
        VP_HIP(hipMemcpy(out.data(), p->vout, out.size() * sizeof(double), hipMemcpyDeviceToHost));
    } else {
        for (auto& v : out) v = std::nan("");
        out[(size_t)m + m * m + 1] = 0.0;
    }
    if (mean) memcpy(mean, out.data(), sizeof(double) * m);
    if (cov) memcpy(cov, out.data() + m, sizeof(double) * m * m);
    if (chi2) *chi2 = out[(size_t)m + m * m];
    if (dof) *dof = (int32_t)out[(size_t)m + m * m + 1];
    const int n = std::min(cap, done);
    if (I_j && n > 0) VP_HIP(hipMemcpy(I_j, p->vI, sizeof(double) * n * m, hipMemcpyDeviceToHost));
    if (C_j && n > 0) VP_HIP(hipMemcpy(C_j, p->vC, sizeof(double) * n * m * m, hipMemcpyDeviceToHost));
    return VP_OK;
}

// Arguments of the map training calls: points inside the box, finite values.
static vp_status check_training(vp_problem* p, int64_t n, const double* x, const double* f, int32_t n_iter,
                                double alpha)
{
    if (!p || n < 1 || !x || !f || n_iter < 0)
        return fail(VP_ERR_INVALID_ARG, "problem, n >= 1 points, x, f and n_iter >= 0 are required");
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(VP_ERR_INVALID_ARG, "alpha must be >= 0");
    const int D = p->P.dim;
    for (int64_t s = 0; s < n; ++s) {
        if (!std::isfinite(f[s])) return fail(VP_ERR_INVALID_ARG, "f[%lld] is not finite", (long long)s);
        for (int mu = 0; mu < D; ++mu) {
            const double v = x[s * D + mu];
            if (!(v >= p->lower[mu] && v <= p->upper[mu]))
                return fail(VP_ERR_INVALID_ARG, "point %lld lies outside the box on axis %d", (long long)s, mu);
        }
    }
    return VP_OK;
}

vp_status vp_map_train(vp_problem* p, int64_t n, const double* x, const double* f, int32_t n_iter, double alpha)
{
    const vp_status st = check_training(p, n, x, f, n_iter, alpha);
    if (st != VP_OK) return st;
    const int D = p->P.dim, NG = p->P.n_g;
    if (n_iter == 0) return VP_OK;
    VP_HIP(hipSetDevice(p->ctx->device));
    hipStream_t sm = p->ctx->stream;
    // one device buffer: points as [dim][n], values, and a one-request launch
    // set whose record carries the training damping (and no frozen phase)
    const size_t xb = sizeof(double) * (size_t)n * D, fb = sizeof(double) * (size_t)n;
    const size_t qo = (xb + fb + 255) / 256 * 256, to = qo + (sizeof(ReqArgs) + 255) / 256 * 256;
    const size_t total = to + 64;
    std::vector<char> h(total, 0);
    double* hx = reinterpret_cast<double*>(h.data());
    for (int64_t s = 0; s < n; ++s)
        for (int mu = 0; mu < D; ++mu) hx[(size_t)mu * n + s] = x[s * D + mu];
    memcpy(h.data() + xb, f, fb);
    ReqArgs q = p->req;
    q.alpha = alpha;
    q.n_adapt = 0;
    memcpy(h.data() + qo, &q, sizeof q);
    char* d = nullptr;
    VP_HIP(hipMalloc((void**)&d, total));
    ReqArgs* dq = reinterpret_cast<ReqArgs*>(d + qo);
    memcpy(h.data() + to, &dq, sizeof dq);
    const int32_t bb[2] = {0, D};
    memcpy(h.data() + to + 16, bb, sizeof bb);
    hipError_t e = hipMemcpyAsync(d, h.data(), total, hipMemcpyHostToDevice, sm);
    TrainArgs ta;
    ta.x = reinterpret_cast<const double*>(d);
    ta.f = reinterpret_cast<const double*>(d + xb);
    ta.map = p->map;
    ta.H = p->H;
    ta.W = p->W;
    ta.n = n;
    ta.x_mu = n;
    ta.x_s = 1;
    ta.dim = D;
    ta.n_g = NG;
    LaunchSet L;
    L.reqs = reinterpret_cast<ReqArgs* const*>(d + to);
    L.bbase = reinterpret_cast<const int32_t*>(d + to + 16);
    L.n = 1;
    for (int it = 0; it < n_iter && e == hipSuccess; ++it) {
        launch_fill_f64(p->H, (int64_t)D * NG, 0.0, sm);
        launch_fill_f64(p->W, (int64_t)D * NG, 0.0, sm);
        launch_train_hist(ta, sm);
        launch_refine(L, D, NG, sm);
        e = hipGetLastError();
    }
    const hipError_t e2 = hipStreamSynchronize(sm);
    (void)hipFree(d);
    if (e != hipSuccess || e2 != hipSuccess)
        return fail(VP_ERR_DEVICE, "map training: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    return VP_OK;
}

// The training call that allocates nothing: the points, their values, the
// record with the training damping and its launch table are staged in the
// library's static device workspace instead of a buffer allocated per call.
vp_status vp_map_train_noalloc(vp_problem* p, int64_t n, const double* x, const double* f, int32_t n_iter,
                               double alpha)
{
    const vp_status st = check_training(p, n, x, f, n_iter, alpha);
    if (st != VP_OK) return st;
    const int D = p->P.dim, NG = p->P.n_g;
    // workspace layout: x as [n][dim] (the caller's order), f [n], the record,
    // the launch table (request pointer, block bases)
    const size_t xb = sizeof(double) * (size_t)n * D, fb = sizeof(double) * (size_t)n;
    const size_t qo = (xb + fb + 255) / 256 * 256, to = qo + (sizeof(ReqArgs) + 255) / 256 * 256;
    const size_t total = to + 64;
    if (n > (int64_t)(kScratchBytes / 8) || total > kScratchBytes)
        return fail(VP_ERR_INVALID_ARG,
                    "%lld points of dimension %d need %zu bytes of workspace; the limit is %zu bytes "
                    "(vp_map_train has none)", (long long)n, D, total, kScratchBytes);
    if (n_iter == 0) return VP_OK;
    const int dev = p->ctx->device;
    if (dev < 0 || dev >= kMaxDevices || !g_scratch[dev])
        return fail(VP_ERR_STATE, "no workspace address for device %d", dev);
    VP_HIP(hipSetDevice(dev));
    hipStream_t sm = p->ctx->stream;
    char* d = static_cast<char*>(g_scratch[dev]);
    ReqArgs q = p->req;
    q.alpha = alpha;
    q.n_adapt = 0;
    ReqArgs* dq = reinterpret_cast<ReqArgs*>(d + qo);
    struct {
        ReqArgs* req;
        int32_t pad[2];
        int32_t bb[2];
    } table = {dq, {0, 0}, {0, D}};
    static_assert(offsetof(decltype(table), bb) == 16, "block bases at offset 16 of the launch table");
    // earlier work on the stream may still read the workspace
    VP_HIP(hipStreamSynchronize(sm));
    hipError_t e = hipMemcpyAsync(d, x, xb, hipMemcpyHostToDevice, sm);
    if (e == hipSuccess) e = hipMemcpyAsync(d + xb, f, fb, hipMemcpyHostToDevice, sm);
    if (e == hipSuccess) e = hipMemcpyAsync(d + qo, &q, sizeof q, hipMemcpyHostToDevice, sm);
    if (e == hipSuccess) e = hipMemcpyAsync(d + to, &table, sizeof table, hipMemcpyHostToDevice, sm);
    TrainArgs ta;
    ta.x = reinterpret_cast<const double*>(d);
    ta.f = reinterpret_cast<const double*>(d + xb);
    ta.map = p->map;
    ta.H = p->H;
    ta.W = p->W;
    ta.n = n;
    ta.x_mu = 1;
    ta.x_s = D;
    ta.dim = D;
    ta.n_g = NG;
    LaunchSet L;
    L.reqs = reinterpret_cast<ReqArgs* const*>(d + to);
    L.bbase = reinterpret_cast<const int32_t*>(d + to + 16);
    L.n = 1;
    for (int it = 0; it < n_iter && e == hipSuccess; ++it) {
        launch_fill_f64(p->H, (int64_t)D * NG, 0.0, sm);
        launch_fill_f64(p->W, (int64_t)D * NG, 0.0, sm);
        launch_train_hist(ta, sm);
        launch_refine(L, D, NG, sm);
        e = hipGetLastError();
    }
    // the copies read q, table and the caller's arrays until they complete
    const hipError_t e2 = hipStreamSynchronize(sm);
    if (e != hipSuccess || e2 != hipSuccess)
        return fail(VP_ERR_DEVICE, "map training: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    return VP_OK;
}

struct StateHeader {
    uint32_t magic, version;
    int32_t dim, n_g;
    int64_t n_hc;
    int32_t it, slot;
    int64_t n_evals;
    uint64_t ties;
};

vp_status vp_state_export(vp_problem* p, void* buf, size_t* size)
{
    if (!p || !size) return fail(VP_ERR_INVALID_ARG, "problem and size are required");
    const size_t nm = (size_t)p->P.dim * (p->P.n_g + 1);
    const size_t need = sizeof(StateHeader) + nm * sizeof(double) + (size_t)p->n_hc * sizeof(int32_t) +
                        2 * (size_t)p->slot * sizeof(double);
    if (!buf) {
        *size = need;
        return VP_OK;
    }
    if (*size < need) return fail(VP_ERR_INVALID_ARG, "buffer of %zu bytes, need %zu", *size, need);
    VP_HIP(hipStreamSynchronize(p->ctx->stream));
    DevState st;
    VP_HIP(hipMemcpy(&st, p->st, sizeof st, hipMemcpyDeviceToHost));
    StateHeader hd = {kStateMagic, 1, p->P.dim, p->P.n_g, p->n_hc, p->it, p->slot, st.n_evals, st.ties};
    char* b = (char*)buf;
    memcpy(b, &hd, sizeof hd);
    b += sizeof hd;
    VP_HIP(hipMemcpy(b, p->map, nm * sizeof(double), hipMemcpyDeviceToHost));
    b += nm * sizeof(double);
    VP_HIP(hipMemcpy(b, p->n_h, (size_t)p->n_hc * sizeof(int32_t), hipMemcpyDeviceToHost));
    b += (size_t)p->n_hc * sizeof(int32_t);
    if (p->slot > 0) {
        VP_HIP(hipMemcpy(b, p->hist_I, (size_t)p->slot * sizeof(double), hipMemcpyDeviceToHost));
        b += (size_t)p->slot * sizeof(double);
        VP_HIP(hipMemcpy(b, p->hist_V, (size_t)p->slot * sizeof(double), hipMemcpyDeviceToHost));
    }
    *size = need;
    return VP_OK;
}

vp_status vp_state_import(vp_problem* p, const void* buf, size_t size)
{
    if (!p || !buf) return fail(VP_ERR_INVALID_ARG, "problem and buf are required");
    StateHeader hd;
    if (size < sizeof hd) return fail(VP_ERR_INVALID_ARG, "state blob too small");
    memcpy(&hd, buf, sizeof hd);
    if (hd.magic != kStateMagic || hd.version != 1) return fail(VP_ERR_INVALID_ARG, "not a state blob");
    if (hd.dim != p->P.dim || hd.n_g != p->P.n_g || hd.n_hc != p->n_hc)
        return fail(VP_ERR_INVALID_ARG, "state shape (dim %d, n_g %d, n_hc %lld) does not match the problem",
                    hd.dim, hd.n_g, (long long)hd.n_hc);
    if (hd.slot < 0 || hd.slot > p->hist_cap || hd.it < 0) return fail(VP_ERR_INVALID_ARG, "bad iteration counters");
    const size_t nm = (size_t)p->P.dim * (p->P.n_g + 1);
    const size_t need = sizeof hd + nm * sizeof(double) + (size_t)p->n_hc * sizeof(int32_t) +
                        2 * (size_t)hd.slot * sizeof(double);
    if (size != need) return fail(VP_ERR_INVALID_ARG, "state blob of %zu bytes, expected %zu", size, need);
    const char* b = (const char*)buf + sizeof hd;
    vp_status s = vp_map_set(p, (const double*)b);
    if (s != VP_OK) return s;
    b += nm * sizeof(double);
    s = vp_alloc_set(p, (const int32_t*)b);
    if (s != VP_OK) return s;
    b += (size_t)p->n_hc * sizeof(int32_t);
    if (hd.slot > 0) {
        VP_HIP(hipMemcpy(p->hist_I, b, (size_t)hd.slot * sizeof(double), hipMemcpyHostToDevice));
        b += (size_t)hd.slot * sizeof(double);
        VP_HIP(hipMemcpy(p->hist_V, b, (size_t)hd.slot * sizeof(double), hipMemcpyHostToDevice));
    }
    DevState st;
    VP_HIP(hipMemcpy(&st, p->st, sizeof st, hipMemcpyDeviceToHost));
    st.n_evals = hd.n_evals;
    st.ties = hd.ties;
    st.n_iter_done = hd.slot;
    VP_HIP(hipMemcpy(p->st, &st, sizeof st, hipMemcpyHostToDevice));
    p->it = hd.it;
    p->slot = hd.slot;
    VP_HIP(push_counters(p));
    return VP_OK;
}

vp_status vp_profile_enable(vp_problem* p, int32_t on)
{
    if (!p) return fail(VP_ERR_INVALID_ARG, "problem is NULL");
    vp_status s = drain_events(p);
    if (s != VP_OK) return s;
    p->prof = on != 0;
    p->t_sample_ms = p->t_iter_ms = 0.0;
    p->n_sample = p->n_iter = 0;
    return VP_OK;
}

vp_status vp_kernel_time(vp_problem* p, int32_t which, double* total_ms, int64_t* launches)
{
    if (!p || which < 0 || which > 1) return fail(VP_ERR_INVALID_ARG, "problem is NULL or which not in 0..1");
    vp_status s = drain_events(p);
    if (s != VP_OK) return s;
    if (total_ms) *total_ms = which == 0 ? p->t_sample_ms : p->t_iter_ms;
    if (launches) *launches = which == 0 ? p->n_sample : p->n_iter;
    return VP_OK;
}

vp_status vp_integrate(vp_ctx* ctx, const vp_params* P, const vp_integrand* f, vp_result* out)
{
    TraceRange tr("vp_integrate");
    if (!out) return fail(VP_ERR_INVALID_ARG, "out is NULL");
    vp_problem* p = nullptr;
    vp_status s = vp_problem_create(ctx, P, f, &p);
    if (s != VP_OK) return s;
    s = vp_iterate(p, P->n_iter);
    if (s == VP_OK) s = vp_result_get(p, out, nullptr, nullptr, nullptr, 0);
    vp_problem_destroy(p);
    return s;
}

}  // extern "C"

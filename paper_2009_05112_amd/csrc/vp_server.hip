// vp_server.hip -- continuous-batching server for many vegas+ integrations.
//
// The scheduler thread owns the GPU work.  Each loop turn:
//  1. admits queued requests in arrival order while the device-memory budget
//     and the slot count allow (a request's footprint is known before it is
//     created), creating their device state on the server's stream;
//  2. if the set of active requests changed, builds the batched iteration
//     plan (one launch per kernel for all requests, one sampling launch per
//     kernel instantiation) and drops the captured graph;
//  3. enqueues one step -- one iteration of every active request -- replaying
//     the step's captured HIP graph when the set is unchanged (the per-request
//     Philox iteration and history slot live in device memory and are
//     advanced by the step itself, so a replay is the next iteration), and
//     behind it the gather of the estimates of the requests that this step
//     finishes;
//  4. waits for the previous turn's step and retires the requests it
//     finished (or that were cancelled): copies their result, frees their
//     memory, wakes waiters.
// A step therefore always has the next one queued behind it while the host
// admits, plans and retires: the GPU does not wait for the scheduler.
// Requests submitted while a step runs are admitted at the next turn, so the
// GPU work of new and old requests overlaps in the same launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <optional>
#include <thread>
#include <unordered_map>
#include <vector>

#include "vp_state.hpp"
#include "vp_trace.hpp"

using namespace vp;

namespace {

// Sampling workgroups of a served request hold about this many samples (one
// tile of 16 per lane for 1024 threads): small requests still spread over
// many CUs (a step's launches are short), while the per-workgroup LDS set-up
// and the flush of its training-data partials stay a few percent of the work.
constexpr int64_t kServeSamplesPerWG = 16384;
// A plan is captured into a graph once it has run this many steps unchanged
// (the sets of a stream of arrivals often change after a few steps, and a
// capture costs the host as much as tens of direct launches).
constexpr int64_t kCaptureAfter = 3;
// Requests admitted per scheduler turn: a large batch arriving at once starts
// on the GPU after the first share is set up, and the rest are set up while
// the steps run (4096 requests of the served-batch workload: 0.334 s makespan
// admitted at once, 0.320 s by 1024 per turn).
constexpr int kAdmitPerTurn = 1024;

enum ReqState { R_PENDING = 0, R_ACTIVE = 1, R_DONE = 2, R_CANCELLED = 3, R_FAILED = 4 };

struct ServedReq {
    uint64_t ticket = 0;
    vp_params P;
    std::vector<double> lower, upper;
    std::vector<int32_t> nst_ax;
    vp_integrand f;
    std::vector<double> centers, coefs, amps, chol;
    size_t bytes = 0;
    int state = R_PENDING;
    bool cancel = false;
    double t_submit = -1, t_admit = -1, t_finish = -1;
    vp_problem* prob = nullptr;
    int iters_left = 0;
    vp_result res;
    vp_status status = VP_OK;
    std::string err;
};

}  // namespace

struct vp_server {
    vp_ctx* ctx = nullptr;  // own stream on the caller's device
    size_t budget = 0;
    int max_slots = 0;
    bool graphs = true;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<ServedReq*> pending;
    std::vector<ServedReq*> active;  // scheduler thread only
    std::unordered_map<uint64_t, ServedReq*> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread th;
    size_t mem_used = 0, mem_peak = 0;
    vp_server_stats st;  // guarded by mu
    struct {
        int64_t steps = 0, graph_launches = 0, graph_captures = 0;
        double t_admit = 0, t_plan = 0, t_step = 0, t_retire = 0;
    } ss;  // the scheduler's own counters, published into st under mu
    // two plan builders used in turn: a new plan's launch tables are written
    // while the step of the previous plan may still be running
    PlanBuilder planner[2];
    int pb = 0;
    IterPlan plan;
    DevicePool pool;  // device memory of admitted requests
    bool plan_valid = false;
    int64_t plan_steps = 0;  // steps run with the current plan
    hipGraphExec_t gexec = nullptr;
    std::vector<hipGraphExec_t> dead_graphs;  // destroyed once the step that used them is complete
    // the step in flight: its completion event (recorded behind the gather of
    // the estimates of the requests it finishes), those requests, and the
    // cancelled requests that it still touches
    bool inflight = false;
    int64_t turn = 0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    std::vector<ServedReq*> fin_inflight, drop_inflight;
    SideStreams side;  // sampling launches of different kernel groups side by side
    std::chrono::steady_clock::time_point t0;
    // gather of finished requests' estimates: pointers and results, host
    // (pinned) and device copies, max_slots entries each, for each of the two
    // steps that can be queued at once
    DevState** h_ptrs[2] = {nullptr, nullptr};
    DevState* h_out[2] = {nullptr, nullptr};
    DevState** d_ptrs[2] = {nullptr, nullptr};
    DevState* d_out[2] = {nullptr, nullptr};

    double tsec(std::chrono::steady_clock::time_point a) const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count();
    }

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

static void copy_request(ServedReq* r, const vp_params* P, const vp_integrand* f)
{
    r->P = *P;
    if (P->lower) {
        r->lower.assign(P->lower, P->lower + P->dim);
        r->upper.assign(P->upper, P->upper + P->dim);
        r->P.lower = r->lower.data();
        r->P.upper = r->upper.data();
    }
    if (P->n_st_axes) {
        r->nst_ax.assign(P->n_st_axes, P->n_st_axes + P->dim);
        r->P.n_st_axes = r->nst_ax.data();
    }
    r->f = *f;
    const int D = f->dim, K = f->n_terms;
    auto cp = [](std::vector<double>& dst, const double* src, size_t n) -> const double* {
        if (!src) return nullptr;
        dst.assign(src, src + n);
        return dst.data();
    };
    size_t nc = 0;
    if (f->kind == VP_F_GAUSS_MIX || f->kind == VP_F_EXP_ABS || f->kind == VP_F_BALLS) nc = (size_t)K * D;
    else if (f->kind == VP_F_CORR_GAUSS) nc = D;
    else if (f->kind == VP_F_AFFINE) nc = D + 1;
    r->f.centers = cp(r->centers, f->centers, nc);
    const size_t nk = (f->kind == VP_F_GAUSS_MIX || f->kind == VP_F_EXP_ABS || f->kind == VP_F_BALLS) ? K : 0;
    r->f.coefs = cp(r->coefs, f->coefs, nk);
    r->f.amps = cp(r->amps, f->amps, nk);
    r->f.chol = f->kind == VP_F_CORR_GAUSS ? cp(r->chol, f->chol, (size_t)D * D) : nullptr;
}

static void free_gather(vp_server* s)
{
    for (int b = 0; b < 2; ++b) {
        (void)hipHostFree(s->h_ptrs[b]);
        (void)hipHostFree(s->h_out[b]);
        (void)hipFree(s->d_ptrs[b]);
        (void)hipFree(s->d_out[b]);
        s->h_ptrs[b] = nullptr;
        s->h_out[b] = nullptr;
        s->d_ptrs[b] = nullptr;
        s->d_out[b] = nullptr;
        if (s->ev[b]) (void)hipEventDestroy(s->ev[b]);
        s->ev[b] = nullptr;
    }
}

// Side streams for the sampling launches (default priority, like the main
// stream); without them the launches run one after another.
static void make_side(vp_server* s)
{
    SideStreams& d = s->side;
    d.n = 0;
    if (hipEventCreateWithFlags(&d.fork, hipEventDisableTiming) != hipSuccess) {
        d.fork = nullptr;
        return;
    }
    for (int i = 0; i < kMaxSide; ++i) {
        if (hipStreamCreateWithFlags(&d.st[i], hipStreamNonBlocking) != hipSuccess) break;
        if (hipEventCreateWithFlags(&d.join[i], hipEventDisableTiming) != hipSuccess) {
            (void)hipStreamDestroy(d.st[i]);
            break;
        }
        d.n = i + 1;
    }
}

static void free_side(vp_server* s)
{
    SideStreams& d = s->side;
    for (int i = 0; i < d.n; ++i) {
        (void)hipStreamSynchronize(d.st[i]);
        (void)hipStreamDestroy(d.st[i]);
        (void)hipEventDestroy(d.join[i]);
    }
    if (d.fork) (void)hipEventDestroy(d.fork);
    d = SideStreams();
}

// The current graph may still be replayed by the step in flight: it is
// destroyed once that step is complete.
static void drop_graph(vp_server* s)
{
    if (s->gexec) {
        s->dead_graphs.push_back(s->gexec);
        s->gexec = nullptr;
    }
}

static void destroy_dead_graphs(vp_server* s)
{
    for (hipGraphExec_t g : s->dead_graphs) (void)hipGraphExecDestroy(g);
    s->dead_graphs.clear();
}

// Enqueues one step without waiting for it; returns false on a launch error.
// A plan is launched directly on its first kCaptureAfter steps and captured
// into a graph after them, so sets of requests that change every few steps
// pay no capture.
static bool enqueue_step(vp_server* s)
{
    hipStream_t st = s->ctx->stream;
    if (s->graphs && s->plan_steps >= kCaptureAfter) {
        if (!s->gexec) {
            const auto t0 = std::chrono::steady_clock::now();
            hipGraph_t g = nullptr;
            if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
            enqueue_iteration(s->plan, st, nullptr, nullptr, &s->side);
            if (hipStreamEndCapture(st, &g) != hipSuccess) return false;
            hipError_t e = hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                s->gexec = nullptr;
                return false;
            }
            s->ss.graph_captures += 1;
            s->ss.t_plan += s->tsec(t0);
        }
        if (hipGraphLaunch(s->gexec, st) != hipSuccess) return false;
        s->ss.graph_launches += 1;
        s->plan_steps += 1;
        return true;
    }
    enqueue_iteration(s->plan, st, nullptr, nullptr, &s->side);
    if (hipGetLastError() != hipSuccess) return false;
    s->plan_steps += 1;
    return true;
}

static void retire(vp_server* s, ServedReq* r, int state)
{
    if (r->prob) {
        problem_free(r->prob);
        r->prob = nullptr;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->mem_used -= r->bytes;
    r->state = state;
    r->t_finish = s->now();
    if (state == R_DONE) {
        s->st.completed += 1;
        s->st.samples += r->res.n_evals;
    } else if (state == R_CANCELLED) {
        s->st.cancelled += 1;
    } else {
        s->st.failed += 1;
    }
    s->cv_done.notify_all();
}

// Fails every request the scheduler holds after a device error, once the
// stream has drained.
static void fail_all(vp_server* s, const char* why)
{
    (void)hipStreamSynchronize(s->ctx->stream);
    std::vector<ServedReq*> all = s->active;
    all.insert(all.end(), s->fin_inflight.begin(), s->fin_inflight.end());
    for (ServedReq* r : all) {
        r->status = VP_ERR_DEVICE;
        r->err = why;
        retire(s, r, R_FAILED);
    }
    for (ServedReq* r : s->drop_inflight) retire(s, r, R_CANCELLED);
    s->active.clear();
    s->fin_inflight.clear();
    s->drop_inflight.clear();
    s->inflight = false;
    drop_graph(s);
    destroy_dead_graphs(s);
    s->plan_valid = false;
}

// Waits for the step in flight and retires what it finished: the requests
// whose last iteration it ran (their estimates were gathered behind it) and
// the cancelled requests it still touched.  Returns false on a device error.
static bool complete_inflight(vp_server* s)
{
    if (!s->inflight) return true;
    const int b = (int)((s->turn - 1) & 1);
    const auto t0 = std::chrono::steady_clock::now();
    const bool ok = hipEventSynchronize(s->ev[b]) == hipSuccess;
    s->ss.t_step += s->tsec(t0);
    s->inflight = false;
    if (!ok) return false;
    const auto t_ret = std::chrono::steady_clock::now();
    destroy_dead_graphs(s);
    // the admissions staged before that step have been read by now
    s->pool.reset_stage(b);
    for (size_t i = 0; i < s->fin_inflight.size(); ++i) {
        ServedReq* r = s->fin_inflight[i];
        r->status = result_from_state(s->h_out[b][i], &r->res);
        if (r->status != VP_OK) r->err = vp_last_error();
        retire(s, r, r->status == VP_OK || r->status == VP_ERR_NUMERIC ? R_DONE : R_FAILED);
    }
    for (ServedReq* r : s->drop_inflight) retire(s, r, R_CANCELLED);
    s->fin_inflight.clear();
    s->drop_inflight.clear();
    s->ss.t_retire += s->tsec(t_ret);
    return true;
}

static void publish_stats(vp_server* s)
{
    std::lock_guard<std::mutex> lk(s->mu);
    s->st.steps = s->ss.steps;
    s->st.graph_launches = s->ss.graph_launches;
    s->st.graph_captures = s->ss.graph_captures;
    s->st.t_admit = s->ss.t_admit;
    s->st.t_plan = s->ss.t_plan;
    s->st.t_step = s->ss.t_step;
    s->st.t_retire = s->ss.t_retire;
}

static void scheduler(vp_server* s)
{
    (void)hipSetDevice(s->ctx->device);
    for (;;) {
        std::vector<ServedReq*> admit;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                while (!s->pending.empty() && (int)(s->active.size() + admit.size()) < s->max_slots &&
                       (int)admit.size() < kAdmitPerTurn) {
                    ServedReq* r = s->pending.front();
                    if (r->cancel) {
                        s->pending.pop_front();
                        r->state = R_CANCELLED;
                        r->t_finish = s->now();
                        s->st.cancelled += 1;
                        s->cv_done.notify_all();
                        continue;
                    }
                    if (s->mem_used + r->bytes > s->budget) break;  // wait for memory
                    s->pending.pop_front();
                    s->mem_used += r->bytes;
                    s->mem_peak = std::max(s->mem_peak, s->mem_used);
                    r->state = R_ACTIVE;
                    r->t_admit = s->now();
                    admit.push_back(r);
                }
                if (!s->active.empty() || !admit.empty() || s->inflight) break;
                if (s->stop) return;
                s->cv_work.wait(lk);
            }
        }
        const int b = (int)(s->turn & 1);  // buffers of the step this turn enqueues
        bool changed = false;
        const auto t_adm = std::chrono::steady_clock::now();
        std::optional<TraceRange> tr_adm;
        if (!admit.empty()) tr_adm.emplace("vp_server: admit");
        // initial images of this turn's admissions go to staging set b (the
        // other set may still be read by the step in flight)
        s->pool.select_stage(b);
        std::vector<InitArgs> inits;
        inits.reserve(admit.size());
        for (ServedReq* r : admit) {
            InitArgs ia;
            vp_status st = problem_create(s->ctx, &r->P, &r->f, kServeSamplesPerWG, &s->pool, &r->prob, &ia);
            if (st != VP_OK) {
                r->status = st;
                r->err = vp_last_error();
                retire(s, r, R_FAILED);
                continue;
            }
            inits.push_back(ia);
            r->iters_left = r->P.n_iter;
            s->active.push_back(r);
            changed = true;
        }
        if (!inits.empty()) {
            // one launch initialises every admitted request (its table sits
            // in the same pinned staging memory as their images)
            const char* tdev = nullptr;
            char* th = s->pool.stage(sizeof(InitArgs) * inits.size(), &tdev);
            if (th) {
                memcpy(th, inits.data(), sizeof(InitArgs) * inits.size());
                launch_init_batch(reinterpret_cast<const InitArgs*>(tdev), (int)inits.size(), s->ctx->stream);
            } else {
                for (const InitArgs& ia : inits)
                    if (ia.n_hc >= 0) launch_init(ia, s->ctx->stream);
            }
            if (hipGetLastError() != hipSuccess) {
                fail_all(s, "initialising admitted requests failed");
                publish_stats(s);
                continue;
            }
        }
        if (!admit.empty()) s->ss.t_admit += s->tsec(t_adm);
        tr_adm.reset();
        // cancellations of active requests, and requests with nothing to do;
        // a request the step in flight still runs is freed once it is done
        for (size_t i = 0; i < s->active.size();) {
            ServedReq* r = s->active[i];
            bool cancel;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                cancel = r->cancel;
            }
            if (cancel || r->iters_left <= 0) {
                s->active.erase(s->active.begin() + i);
                changed = true;
                if (!cancel) {
                    r->status = vp_result_get(r->prob, &r->res, nullptr, nullptr, nullptr, 0);
                    retire(s, r, R_DONE);
                } else if (r->prob && r->prob->slot > 0 && s->inflight) {
                    s->drop_inflight.push_back(r);
                } else {
                    retire(s, r, R_CANCELLED);
                }
            } else {
                ++i;
            }
        }
        bool ok = true;
        const bool stepping = !s->active.empty();
        if (stepping) {
            if (changed || !s->plan_valid) {
                TraceRange tr_plan("vp_server: plan");
                const auto t_pl = std::chrono::steady_clock::now();
                std::vector<PlanReq> pr;
                pr.reserve(s->active.size());
                for (ServedReq* r : s->active)
                    pr.push_back({&r->prob->req, r->prob->d_req, r->prob->entry, r->prob->lds});
                drop_graph(s);
                s->plan_steps = 0;
                // the other builder: the step in flight reads the current one's tables
                s->pb ^= 1;
                s->plan_valid = s->planner[s->pb].build(pr, &s->plan) == hipSuccess;
                s->ss.t_plan += s->tsec(t_pl);
                if (!s->plan_valid) {
                    fail_all(s, "building the batched plan failed");
                    publish_stats(s);
                    continue;
                }
                std::lock_guard<std::mutex> lk(s->mu);
                s->st.peak_active = std::max<int32_t>(s->st.peak_active, (int32_t)s->active.size());
            }
            {
                TraceRange tr_step("vp_server: step");
                ok = enqueue_step(s);
            }
            s->ss.steps += 1;
        }
        // the previous step (queued ahead of this one) completes meanwhile
        if (ok) {
            TraceRange tr_ret("vp_server: wait and retire");
            ok = complete_inflight(s);
        }
        if (!ok) {
            fail_all(s, "device error during a batched step");
            publish_stats(s);
            continue;
        }
        if (stepping) {
            // bookkeeping of the step just enqueued; the requests it finishes
            // have their estimates gathered behind it
            std::vector<ServedReq*> keep;
            keep.reserve(s->active.size());
            for (ServedReq* r : s->active) {
                r->prob->it += 1;
                r->prob->slot += 1;
                r->iters_left -= 1;
                (r->iters_left <= 0 ? s->fin_inflight : keep).push_back(r);
            }
            s->active.swap(keep);
            hipStream_t st = s->ctx->stream;
            const int n = (int)s->fin_inflight.size();
            bool got = true;
            if (n > 0) {
                for (int i = 0; i < n; ++i) s->h_ptrs[b][i] = s->fin_inflight[i]->prob->st;
                got = hipMemcpyAsync(s->d_ptrs[b], s->h_ptrs[b], n * sizeof(DevState*), hipMemcpyHostToDevice, st) ==
                      hipSuccess;
                if (got) {
                    launch_gather_states(s->d_ptrs[b], n, s->d_out[b], st);
                    got = hipGetLastError() == hipSuccess &&
                          hipMemcpyAsync(s->h_out[b], s->d_out[b], n * sizeof(DevState), hipMemcpyDeviceToHost, st) ==
                              hipSuccess;
                }
                s->plan_valid = false;  // the next step runs without them
            }
            got = got && hipEventRecord(s->ev[b], st) == hipSuccess;
            s->inflight = true;
            s->turn += 1;
            if (!got) {
                fail_all(s, "reading the estimates failed");
                publish_stats(s);
                continue;
            }
        }
        publish_stats(s);
    }
}

extern "C" {

vp_status vp_server_create(vp_ctx* ctx, size_t mem_budget_bytes, int32_t max_slots, int32_t flags,
                           vp_server** out)
{
    if (!ctx || !out || max_slots < 1) return fail(VP_ERR_INVALID_ARG, "ctx, out and max_slots >= 1 are required");
    *out = nullptr;
    vp_ctx* own = nullptr;
    vp_status st = vp_ctx_create(ctx->device, nullptr, &own);
    if (st != VP_OK) return st;
    if (mem_budget_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            vp_ctx_destroy(own);
            return fail(VP_ERR_DEVICE, "hipMemGetInfo failed");
        }
        mem_budget_bytes = fr / 4 * 3;
    }
    vp_server* s = new vp_server();
    s->ctx = own;
    (void)hipSetDevice(own->device);
    bool got = true;
    for (int b = 0; b < 2 && got; ++b)
        got = hipHostMalloc((void**)&s->h_ptrs[b], sizeof(DevState*) * max_slots, 0) == hipSuccess &&
              hipHostMalloc((void**)&s->h_out[b], sizeof(DevState) * max_slots, 0) == hipSuccess &&
              hipMalloc((void**)&s->d_ptrs[b], sizeof(DevState*) * max_slots) == hipSuccess &&
              hipMalloc((void**)&s->d_out[b], sizeof(DevState) * max_slots) == hipSuccess &&
              hipEventCreateWithFlags(&s->ev[b], hipEventDisableTiming) == hipSuccess;
    if (!got) {
        free_gather(s);
        vp_ctx_destroy(own);
        delete s;
        return fail(VP_ERR_OOM, "allocating the server's result buffers");
    }
    (void)hipSetDevice(own->device);
    make_side(s);
    s->budget = mem_budget_bytes;
    // slabs of at most 1 GiB and a quarter of the budget
    s->pool.set_slab_bytes(std::min<size_t>(size_t(1) << 30, mem_budget_bytes / 4));
    s->max_slots = max_slots;
    // set-up that would otherwise fall into the first turns: the plan tables
    // of both builders for max_slots requests (at most 16384, about 2 MB
    // each), and pinned staging for one turn's admissions (their initial
    // images and the table of their initialisation); either may fail, and a
    // turn then allocates what it needs itself
    (void)s->planner[0].reserve(std::min(max_slots, 16384));
    (void)s->planner[1].reserve(std::min(max_slots, 16384));
    (void)hipGetLastError();
    (void)s->pool.reserve_stage((size_t)std::min(max_slots, kAdmitPerTurn) *
                                (problem_head_bytes_max() + sizeof(InitArgs)));
    s->graphs = (flags & VP_SERVER_NO_GRAPH) == 0;
    memset(&s->st, 0, sizeof s->st);
    s->t0 = std::chrono::steady_clock::now();
    s->th = std::thread(scheduler, s);
    *out = s;
    return VP_OK;
}

vp_status vp_server_submit(vp_server* s, const vp_params* P, const vp_integrand* f, uint64_t* ticket)
{
    if (!s || !ticket) return fail(VP_ERR_INVALID_ARG, "server and ticket are required");
    vp_status st = validate(P, f);
    if (st != VP_OK) return st;
    if (f->kind == VP_F_BATCH)
        return fail(VP_ERR_INVALID_ARG, "batched integrands call host code between kernels and are not servable");
    size_t bytes = 0;
    st = problem_bytes(s->ctx, P, f, kServeSamplesPerWG, &bytes);
    if (st != VP_OK) return st;
    if (bytes > s->budget)
        return fail(VP_ERR_OOM, "request needs %zu device bytes, the budget is %zu", bytes, s->budget);
    ServedReq* r = new ServedReq();
    copy_request(r, P, f);
    r->bytes = bytes;
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    r->t_submit = s->now();
    s->all[r->ticket] = r;
    s->pending.push_back(r);
    s->cv_work.notify_one();
    *ticket = r->ticket;
    return VP_OK;
}

vp_status vp_server_submit_many(vp_server* s, int32_t n, const vp_params* P, const vp_integrand* f,
                                uint64_t* tickets)
{
    if (!s || n < 0 || (n > 0 && (!P || !f || !tickets)))
        return fail(VP_ERR_INVALID_ARG, "server, n >= 0 and the three arrays are required");
    std::vector<ServedReq*> made;
    made.reserve(n);
    auto drop = [&]() {
        for (ServedReq* r : made) delete r;
    };
    for (int32_t i = 0; i < n; ++i) {
        vp_status st = validate(&P[i], &f[i]);
        if (st == VP_OK && f[i].kind == VP_F_BATCH)
            st = fail(VP_ERR_INVALID_ARG, "batched integrands call host code between kernels and are not servable");
        size_t bytes = 0;
        if (st == VP_OK) st = problem_bytes(s->ctx, &P[i], &f[i], kServeSamplesPerWG, &bytes);
        if (st == VP_OK && bytes > s->budget)
            st = fail(VP_ERR_OOM, "request needs %zu device bytes, the budget is %zu", bytes, s->budget);
        if (st != VP_OK) {
            drop();
            return fail(st, "request %d of %d: %s", i, n, vp_last_error());
        }
        ServedReq* r = new ServedReq();
        copy_request(r, &P[i], &f[i]);
        r->bytes = bytes;
        made.push_back(r);
    }
    std::lock_guard<std::mutex> lk(s->mu);
    const double t = s->now();
    for (int32_t i = 0; i < n; ++i) {
        ServedReq* r = made[i];
        r->ticket = s->next_ticket++;
        r->t_submit = t;
        s->all[r->ticket] = r;
        s->pending.push_back(r);
        tickets[i] = r->ticket;
    }
    if (n > 0) s->cv_work.notify_one();
    return VP_OK;
}

vp_status vp_server_request_bytes(vp_server* s, const vp_params* P, const vp_integrand* f, size_t* bytes)
{
    if (!s || !bytes) return fail(VP_ERR_INVALID_ARG, "server and bytes are required");
    vp_status st = validate(P, f);
    if (st != VP_OK) return st;
    return problem_bytes(s->ctx, P, f, kServeSamplesPerWG, bytes);
}

static vp_status result_of(ServedReq* r, vp_result* out)
{
    if (r->state == R_CANCELLED) return fail(VP_ERR_CANCELLED, "request %llu was cancelled", (unsigned long long)r->ticket);
    if (r->state == R_FAILED) return fail(r->status, "request %llu failed: %s", (unsigned long long)r->ticket, r->err.c_str());
    if (r->state != R_DONE) return fail(VP_ERR_NOT_READY, "request %llu is not finished", (unsigned long long)r->ticket);
    if (out) *out = r->res;
    if (r->status != VP_OK) return fail(r->status, "request %llu: %s", (unsigned long long)r->ticket, r->err.c_str());
    return VP_OK;
}

vp_status vp_server_poll(vp_server* s, uint64_t ticket, vp_result* out)
{
    if (!s) return fail(VP_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(VP_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    return result_of(it->second, out);
}

vp_status vp_server_wait(vp_server* s, uint64_t ticket, vp_result* out)
{
    if (!s) return fail(VP_ERR_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(VP_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    ServedReq* r = it->second;
    s->cv_done.wait(lk, [&] { return r->state >= R_DONE; });
    return result_of(r, out);
}

vp_status vp_server_times(vp_server* s, uint64_t ticket, double* t_submit, double* t_admit, double* t_finish)
{
    if (!s) return fail(VP_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(VP_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    if (t_submit) *t_submit = it->second->t_submit;
    if (t_admit) *t_admit = it->second->t_admit;
    if (t_finish) *t_finish = it->second->t_finish;
    return VP_OK;
}

vp_status vp_server_now(vp_server* s, double* t)
{
    if (!s || !t) return fail(VP_ERR_INVALID_ARG, "server and t are required");
    *t = s->now();
    return VP_OK;
}

vp_status vp_server_cancel(vp_server* s, uint64_t ticket)
{
    if (!s) return fail(VP_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(VP_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    ServedReq* r = it->second;
    if (r->state >= R_DONE) return VP_OK;
    r->cancel = true;
    if (r->state == R_PENDING) {
        auto pit = std::find(s->pending.begin(), s->pending.end(), r);
        if (pit != s->pending.end()) s->pending.erase(pit);
        r->state = R_CANCELLED;
        r->t_finish = s->now();
        s->st.cancelled += 1;
        s->cv_done.notify_all();
    }
    s->cv_work.notify_one();
    return VP_OK;
}

vp_status vp_server_stats_get(vp_server* s, vp_server_stats* out)
{
    if (!s || !out) return fail(VP_ERR_INVALID_ARG, "server and out are required");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    out->pending = (int32_t)s->pending.size();
    int32_t act = 0;
    for (auto& kv : s->all)
        if (kv.second->state == R_ACTIVE) ++act;
    out->active = act;
    out->mem_in_use = (int64_t)s->mem_used;
    out->mem_peak = (int64_t)s->mem_peak;
    return VP_OK;
}

vp_status vp_server_destroy(vp_server* s)
{
    if (!s) return VP_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto& kv : s->all)
            if (kv.second->state < R_DONE) kv.second->cancel = true;
        for (ServedReq* r : s->pending) {
            r->state = R_CANCELLED;
            r->t_finish = s->now();
        }
        s->pending.clear();
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    (void)hipStreamSynchronize(s->ctx->stream);
    drop_graph(s);
    destroy_dead_graphs(s);
    for (auto& kv : s->all) {
        if (kv.second->prob) problem_free(kv.second->prob);
        delete kv.second;
    }
    (void)hipStreamSynchronize(s->ctx->stream);
    free_side(s);
    s->pool.release_all();
    free_gather(s);
    vp_ctx_destroy(s->ctx);
    delete s;
    return VP_OK;
}

}  // extern "C"

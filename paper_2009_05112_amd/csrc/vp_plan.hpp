// vp_plan.hpp -- host-side construction of a batched iteration (IterPlan).
//
// Given the requests of one step (their device argument records in a table
// and host copies of the same records), the builder computes every launch's
// workgroup count per request, the block-base prefix arrays that map a
// workgroup to its request, and the sampling groups (requests that share a
// kernel instantiation), and uploads the integer arrays in one copy.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "vp_aux.hpp"
#include "vp_internal.hpp"

namespace vp {

struct PlanReq {
    const ReqArgs* host;  // host copy of the request's argument record
    ReqArgs* dev;         // the same record in device memory
    SampleEntry entry;    // sampling kernel of the request
    size_t lds;           // dynamic LDS of that kernel for this request
};

class PlanBuilder {
public:
    ~PlanBuilder() { (void)hipFree(dev_); }

    // Device memory for the tables of up to n requests, allocated ahead of
    // the first build (hipFree of an outgrown table waits for the device, so
    // a builder that grows while a step runs would stall the host until it
    // ends).  Per request: two pointer words and one base in each of the ten
    // per-request sets and in the sampling groups; per set and group: one
    // alignment word and the final base.
    hipError_t reserve(int n)
    {
        const size_t words = 33 * (size_t)n + 2 * (10 + (size_t)kMaxGroups) + 16;
        const size_t bytes = words * sizeof(int32_t);
        if (bytes <= cap_) return hipSuccess;
        (void)hipFree(dev_);
        dev_ = nullptr;
        cap_ = 0;
        hipError_t e = hipMalloc((void**)&dev_, bytes + 16);
        if (e != hipSuccess) return e;
        cap_ = bytes;
        host_.reserve(words);
        return hipSuccess;
    }

    // Builds the plan; the integer arrays are copied to the device before
    // returning (synchronous), so the plan may be enqueued or captured at once.
    hipError_t build(const std::vector<PlanReq>& reqs, IterPlan* out)
    {
        const int n = (int)reqs.size();
        host_.clear();
        struct Pending {
            size_t idx_off, bb_off;
            int n;
        };
        // device pointers are stored as pairs of int32 words, 8-byte aligned
        auto put_ptr = [&](const void* ptr) {
            const uint64_t v = (uint64_t)(uintptr_t)ptr;
            host_.push_back((int32_t)(uint32_t)v);
            host_.push_back((int32_t)(uint32_t)(v >> 32));
        };
        auto align8 = [&]() {
            if (host_.size() & 1) host_.push_back(0);
        };
        auto add_set = [&](auto blocks_of, int* total) {
            Pending p;
            align8();
            p.idx_off = host_.size();
            for (int r = 0; r < n; ++r) put_ptr(reqs[r].dev);
            p.bb_off = host_.size();
            int acc = 0;
            for (int r = 0; r < n; ++r) {
                host_.push_back(acc);
                acc += blocks_of(*reqs[r].host);
            }
            host_.push_back(acc);
            p.n = n;
            *total = acc;
            return p;
        };
        int n_scan = 0, n_one = 0, n_hist = 0, n_rec = 0, n_rec_det = 0, n_fix = 0, n_fix_s = 0, n_est = 0, n_ref = 0,
            n_chk = 0;
        Pending ps = add_set([](const ReqArgs& q) { return (int)scan_blocks(q.n_hc); }, &n_scan);
        Pending po = add_set([](const ReqArgs&) { return 1; }, &n_one);
        Pending ph = add_set(
            [](const ReqArgs& q) {
                const int n_max = std::max(q.grid, q.rec_chunks);
                const int tile = kHistBlock / hist_groups(n_max) * hist_values(n_max);
                return (int)((2LL * q.dim * q.n_g + tile - 1) / tile);
            },
            &n_hist);
        Pending prc = add_set(
            [](const ReqArgs& q) { return q.hist_axes < q.dim && !q.det ? q.rec_chunks * q.rec_slices : 0; }, &n_rec);
        // deterministic requests: the same binning, one wave per workgroup
        Pending prd = add_set(
            [](const ReqArgs& q) { return q.hist_axes < q.dim && q.det ? q.rec_chunks * q.rec_slices : 0; },
            &n_rec_det);
        Pending pck = add_set(
            [](const ReqArgs& q) { return q.checks ? check_blocks(q.n_hc, (int64_t)q.dim * (q.n_g + 1)) : 0; },
            &n_chk);
        // edge fix-up: one workgroup per request, a small one for requests
        // with few edge records (two per wave)
        Pending pf = add_set([](const ReqArgs& q) { return 2 * q.n_waves > kFixSmallRecs ? 1 : 0; }, &n_fix);
        Pending pfs = add_set([](const ReqArgs& q) { return 2 * q.n_waves > kFixSmallRecs ? 0 : 1; }, &n_fix_s);
        Pending pe = add_set([](const ReqArgs& q) { return q.est_blocks; }, &n_est);
        Pending pr = add_set([](const ReqArgs& q) { return q.dim; }, &n_ref);
        // sampling groups: requests with the same kernel instantiation
        std::vector<SampleLauncher> keys;
        std::vector<std::vector<int>> members;
        for (int r = 0; r < n; ++r) {
            auto it = std::find(keys.begin(), keys.end(), reqs[r].entry.launch);
            if (it == keys.end()) {
                keys.push_back(reqs[r].entry.launch);
                members.push_back({r});
            } else {
                members[it - keys.begin()].push_back(r);
            }
        }
        if ((int)keys.size() > kMaxGroups) return hipErrorInvalidValue;
        std::vector<Pending> pg(keys.size());
        std::vector<int> gblocks(keys.size());
        std::vector<size_t> glds(keys.size(), 0);
        for (size_t g = 0; g < keys.size(); ++g) {
            align8();
            pg[g].idx_off = host_.size();
            for (int r : members[g]) put_ptr(reqs[r].dev);
            pg[g].bb_off = host_.size();
            int acc = 0;
            for (int r : members[g]) {
                host_.push_back(acc);
                acc += reqs[r].host->grid;
                glds[g] = std::max(glds[g], reqs[r].lds);
            }
            host_.push_back(acc);
            pg[g].n = (int)members[g].size();
            gblocks[g] = acc;
        }
        const size_t bytes = host_.size() * sizeof(int32_t);
        if (bytes > cap_) {
            (void)hipFree(dev_);
            dev_ = nullptr;
            cap_ = 0;
            hipError_t e = hipMalloc((void**)&dev_, bytes * 2 + 16);
            if (e != hipSuccess) return e;
            cap_ = bytes * 2;
        }
        hipError_t e = hipMemcpy(dev_, host_.data(), bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) return e;
        auto mk = [&](const Pending& p) {
            LaunchSet L;
            L.reqs = reinterpret_cast<ReqArgs* const*>(dev_ + p.idx_off);
            L.bbase = dev_ + p.bb_off;
            L.n = p.n;
            return L;
        };
        out->scan_local = mk(ps);
        out->one = mk(po);
        out->hist = mk(ph);
        out->rec = mk(prc);
        out->rec_det = mk(prd);
        out->check = mk(pck);
        out->fixup = mk(pf);
        out->fixup_s = mk(pfs);
        out->est = mk(pe);
        out->refine = mk(pr);
        out->n_scan_local = n_scan;
        out->n_one = n_one;
        out->n_hist = n_hist;
        out->n_rec = n_rec;
        out->n_rec_det = n_rec_det;
        out->n_check = n_chk;
        out->n_fixup = n_fix;
        out->n_fixup_s = n_fix_s;
        out->n_est = n_est;
        out->n_refine = n_ref;
        out->n_groups = (int)keys.size();
        out->max_ng = 1;
        out->rec_lds = 0;
        for (int r = 0; r < n; ++r) {
            const ReqArgs& q = *reqs[r].host;
            out->max_ng = std::max(out->max_ng, q.n_g);
            if (q.hist_axes < q.dim)
                out->rec_lds = std::max(out->rec_lds, (size_t)2 * q.rec_axes * q.n_g * sizeof(double));
        }
        for (size_t g = 0; g < keys.size(); ++g) {
            out->groups[g].entry = reqs[members[g][0]].entry;
            out->groups[g].L = mk(pg[g]);
            out->groups[g].blocks = gblocks[g];
            out->groups[g].lds = glds[g];
        }
        return hipSuccess;
    }

private:
    std::vector<int32_t> host_;
    int32_t* dev_ = nullptr;
    size_t cap_ = 0;
};

}  // namespace vp

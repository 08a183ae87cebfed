// vp_pool.hpp -- device memory of served requests.
//
// Requests are carved out of large slabs (hipMalloc once) by first fit over
// each slab's free ranges, which are coalesced on release.  A steady stream of
// admissions and retirements therefore makes no allocation call into the HIP
// runtime.  The pool is used by one thread (the scheduler), which releases a
// request's range only once no queued or running kernel uses it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <iterator>
#include <map>
#include <vector>

namespace vp {

class DevicePool {
public:
    static constexpr size_t kAlign = 256;

    ~DevicePool() { release_all(); }

    // Slabs are this large (a request larger than a slab gets its own).
    void set_slab_bytes(size_t b) { slab_ = b > kAlign ? round_up(b) : kAlign; }

    // nullptr when the device cannot provide a new slab.
    char* alloc(size_t bytes)
    {
        bytes = round_up(bytes ? bytes : 1);
        for (Slab& s : slabs_)
            if (char* p = take(s, bytes)) return p;
        Slab s;
        s.size = bytes > slab_ ? bytes : slab_;
        if (hipMalloc((void**)&s.base, s.size) != hipSuccess) {
            // retry with an exact-size slab: the device may lack a whole slab
            s.size = bytes;
            if (hipMalloc((void**)&s.base, s.size) != hipSuccess) return nullptr;
        }
        s.free_ranges[0] = s.size;
        slabs_.push_back(s);
        return take(slabs_.back(), bytes);
    }

    void release(char* p)
    {
        if (!p) return;
        for (Slab& s : slabs_) {
            if (p < s.base || p >= s.base + s.size) continue;
            const size_t off = (size_t)(p - s.base);
            auto u = s.used.find(off);
            if (u == s.used.end()) return;
            size_t len = u->second;
            s.used.erase(u);
            size_t start = off;
            // coalesce with the free ranges on both sides
            auto nx = s.free_ranges.lower_bound(start);
            if (nx != s.free_ranges.begin()) {
                auto pv = std::prev(nx);
                if (pv->first + pv->second == start) {
                    start = pv->first;
                    len += pv->second;
                    s.free_ranges.erase(pv);
                }
            }
            nx = s.free_ranges.lower_bound(start);
            if (nx != s.free_ranges.end() && start + len == nx->first) {
                len += nx->second;
                s.free_ranges.erase(nx);
            }
            s.free_ranges[start] = len;
            return;
        }
    }

    // Frees slabs that hold no request (call with the device idle).
    void trim()
    {
        std::vector<Slab> keep;
        for (Slab& s : slabs_) {
            if (s.used.empty()) (void)hipFree(s.base);
            else keep.push_back(s);
        }
        slabs_.swap(keep);
    }

    void release_all()
    {
        for (Slab& s : slabs_) (void)hipFree(s.base);
        slabs_.clear();
        for (Stage& g : stages_) {
            for (Chunk& c : g.chunks) (void)hipHostFree(c.base);
            g = Stage();
        }
    }

    // Pinned host memory holding the initial image of admitted requests'
    // state, which the initialisation kernel reads directly (*dev: the same
    // memory's device address).  Two independent sets: images go to the set
    // chosen by select_stage(), and a set is reset (reset_stage) only once the
    // kernels reading it are complete, while the other set takes new images.
    // nullptr when no pinned memory can be had.
    void select_stage(int i) { cur_ = i & 1; }
    // Pins one chunk of at least `bytes` for each set ahead of use (a server
    // does it once, when created, rather than in its first turns).  False
    // when the memory cannot be had (the sets then grow on demand, as
    // without it).
    bool reserve_stage(size_t bytes)
    {
        for (Stage& g : stages_) {
            if (!g.chunks.empty()) continue;
            Chunk c;
            c.size = round_up(bytes > kStageChunk ? bytes : kStageChunk);
            if (hipHostMalloc((void**)&c.base, c.size, hipHostMallocDefault) != hipSuccess) return false;
            void* d = nullptr;
            if (hipHostGetDevicePointer(&d, c.base, 0) != hipSuccess) {
                (void)hipHostFree(c.base);
                return false;
            }
            c.dev = (const char*)d;
            g.chunks.push_back(c);
        }
        return true;
    }
    char* stage(size_t bytes, const char** dev)
    {
        Stage& g = stages_[cur_];
        bytes = round_up(bytes ? bytes : 1);
        while (g.chunk < g.chunks.size() && g.off + bytes > g.chunks[g.chunk].size) {
            ++g.chunk;
            g.off = 0;
        }
        if (g.chunk == g.chunks.size()) {
            Chunk c;
            c.size = bytes > kStageChunk ? bytes : kStageChunk;
            if (hipHostMalloc((void**)&c.base, c.size, hipHostMallocDefault) != hipSuccess) return nullptr;
            void* d = nullptr;
            if (hipHostGetDevicePointer(&d, c.base, 0) != hipSuccess) {
                (void)hipHostFree(c.base);
                return nullptr;
            }
            c.dev = (const char*)d;
            g.chunks.push_back(c);
            g.off = 0;
        }
        char* p = g.chunks[g.chunk].base + g.off;
        *dev = g.chunks[g.chunk].dev + g.off;
        g.off += bytes;
        return p;
    }
    bool stage_used(int i) const { return stages_[i & 1].chunk > 0 || stages_[i & 1].off > 0; }
    void reset_stage(int i)
    {
        stages_[i & 1].chunk = 0;
        stages_[i & 1].off = 0;
    }

    size_t reserved() const
    {
        size_t t = 0;
        for (const Slab& s : slabs_) t += s.size;
        return t;
    }

private:
    struct Slab {
        char* base = nullptr;
        size_t size = 0;
        std::map<size_t, size_t> free_ranges;  // offset -> length
        std::map<size_t, size_t> used;         // offset -> length
    };

    static size_t round_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

    static char* take(Slab& s, size_t bytes)
    {
        for (auto it = s.free_ranges.begin(); it != s.free_ranges.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, len = it->second;
            s.free_ranges.erase(it);
            if (len > bytes) s.free_ranges[off + bytes] = len - bytes;
            s.used[off] = bytes;
            return s.base + off;
        }
        return nullptr;
    }

    std::vector<Slab> slabs_;
    size_t slab_ = size_t(1) << 30;

    struct Chunk {
        char* base = nullptr;
        const char* dev = nullptr;
        size_t size = 0;
    };
    static constexpr size_t kStageChunk = size_t(16) << 20;
    struct Stage {
        std::vector<Chunk> chunks;
        size_t chunk = 0, off = 0;
    };
    Stage stages_[2];
    int cur_ = 0;
};

}  // namespace vp

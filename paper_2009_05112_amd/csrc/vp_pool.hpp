// vp_pool.hpp -- device memory of served requests.
//
// Requests are carved out of large slabs (hipMalloc once) by first fit over
// each slab's free ranges, which are coalesced on release.  A steady stream of
// admissions and retirements therefore makes no allocation call into the HIP
// runtime.  The pool is used by one thread (the scheduler) and only between
// steps, after the stream has been synchronised, so a released range is never
// still in use by a kernel.
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
        for (Chunk& c : chunks_) (void)hipHostFree(c.base);
        chunks_.clear();
        chunk_ = 0;
        chunk_off_ = 0;
    }

    // Pinned host memory holding the initial image of admitted requests'
    // state, which the initialisation kernel reads directly (*dev: the same
    // memory's device address).  Valid until reset_stage(), which the caller
    // invokes only with those kernels complete; nullptr when no pinned memory
    // can be had.
    char* stage(size_t bytes, const char** dev)
    {
        bytes = round_up(bytes ? bytes : 1);
        while (chunk_ < chunks_.size() && chunk_off_ + bytes > chunks_[chunk_].size) {
            ++chunk_;
            chunk_off_ = 0;
        }
        if (chunk_ == chunks_.size()) {
            Chunk c;
            c.size = bytes > kStageChunk ? bytes : kStageChunk;
            if (hipHostMalloc((void**)&c.base, c.size, hipHostMallocDefault) != hipSuccess) return nullptr;
            void* d = nullptr;
            if (hipHostGetDevicePointer(&d, c.base, 0) != hipSuccess) {
                (void)hipHostFree(c.base);
                return nullptr;
            }
            c.dev = (const char*)d;
            chunks_.push_back(c);
            chunk_off_ = 0;
        }
        char* p = chunks_[chunk_].base + chunk_off_;
        *dev = chunks_[chunk_].dev + chunk_off_;
        chunk_off_ += bytes;
        return p;
    }
    bool stage_used() const { return chunk_ > 0 || chunk_off_ > 0; }
    void reset_stage()
    {
        chunk_ = 0;
        chunk_off_ = 0;
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
    std::vector<Chunk> chunks_;
    size_t chunk_ = 0, chunk_off_ = 0;
};

}  // namespace vp

// isa_rates.hip -- issue rate of the VALU instruction kinds the sampling
// kernel is made of, and throughput of the LDS atomics its training data
// use, on the device it runs on.
//
// Each kernel runs CH independent dependency chains of one instruction kind
// per thread (REP iterations, fully unrolled over the chains), over enough
// workgroups to fill every CU several times.  The rate is reported in lane
// operations per second and as VALU slots per operation against the
// peak 256 CUs x 64 lanes x 2.4 GHz.  The loop bodies compile to the named
// instruction alone (the exp loop adds one subtract per exp, listed).
// Results are kept live so that no chain is removed; nothing is read or
// written out of bounds (one 64-byte buffer, written only when an impossible
// value appears).
//
// LDS atomics: every thread updates kAtomRep pseudo-random bins of an
// 8192-bin LDS array (the sampler's pattern: 64 lanes of a wave scattered
// over the bins), two 1024-thread workgroups per CU.  Reported as lane
// updates per second per CU and as cycles per wave-wide instruction at
// 2.4 GHz.
//
// Gathers: every thread issues kCh independent buffer loads per iteration
// (8 or 16 bytes each) at pseudo-random positions of a table of the map's
// size (8192 entries: 64 KB of doubles), the sampler's map reads from
// global memory; reported the same way.
//
//   paper_2009_05112_amd/isa_rates
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace {

constexpr int kRep = 4096;
constexpr int kCh = 8;

__global__ void k_mad_u64_u32(uint64_t* out, uint32_t seed)
{
    uint64_t c[kCh];
    for (int i = 0; i < kCh; ++i) c[i] = threadIdx.x * 2654435761u + i + seed;
    for (int r = 0; r < kRep; ++r)
#pragma unroll
        for (int i = 0; i < kCh; ++i) c[i] = (uint64_t)(uint32_t)(c[i] >> 32) * 0xD2511F53u + c[i];
    uint64_t t = 0;
    for (int i = 0; i < kCh; ++i) t ^= c[i];
    if (t == 0x123456789ull) out[0] = t;
}

__global__ void k_fma_f64(double* out, double seed)
{
    double a[kCh];
    for (int i = 0; i < kCh; ++i) a[i] = threadIdx.x * 1e-9 + i + seed;
    for (int r = 0; r < kRep; ++r)
#pragma unroll
        for (int i = 0; i < kCh; ++i) a[i] = __builtin_fma(a[i], 0.999999, 1e-7);
    double t = 0;
    for (int i = 0; i < kCh; ++i) t += a[i];
    if (t == 0.125) out[0] = t;
}

__global__ void k_fma_f32(float* out, float seed)
{
    float a[kCh];
    for (int i = 0; i < kCh; ++i) a[i] = threadIdx.x * 1e-6f + i + seed;
    for (int r = 0; r < kRep; ++r)
#pragma unroll
        for (int i = 0; i < kCh; ++i) a[i] = __builtin_fmaf(a[i], 0.999f, 1e-3f);
    float t = 0;
    for (int i = 0; i < kCh; ++i) t += a[i];
    if (t == 0.125f) out[0] = t;
}

__global__ void k_bitop3(uint32_t* out, uint32_t seed)
{
    uint32_t a[kCh];
    for (int i = 0; i < kCh; ++i) a[i] = threadIdx.x * 2654435761u + i + seed;
    for (int r = 0; r < kRep; ++r)
#pragma unroll
        for (int i = 0; i < kCh; ++i) a[i] = __builtin_amdgcn_bitop3_b32(a[i], 0x9E3779B9u, a[(i + 1) % kCh], 0x96);
    uint32_t t = 0;
    for (int i = 0; i < kCh; ++i) t ^= a[i];
    if (t == 0x12345u) out[0] = t;
}

__global__ void k_exp_f32(float* out, float seed)
{
    float a[kCh];
    for (int i = 0; i < kCh; ++i) a[i] = -(threadIdx.x & 7) * 1e-3f - i * 1e-4f + seed;
    for (int r = 0; r < kRep; ++r)
#pragma unroll
        for (int i = 0; i < kCh; ++i) a[i] = __builtin_amdgcn_exp2f(a[i]) - 1.0f;
    float t = 0;
    for (int i = 0; i < kCh; ++i) t += a[i];
    if (t == 0.125f) out[0] = t;
}

constexpr int kAtomRep = 1024;
constexpr int kBins = 8192;

__device__ __forceinline__ uint32_t lcg(uint32_t a) { return a * 1664525u + 1013904223u; }

// kind 0: ds_add_f64, 1: ds_add_f32, 2: ds_add_u32, 3: read + 64-bit compare-and-swap of a double,
// 4: ds_add_f64 with the 64 lanes of a wave inside one window of 128 bins (a new window per
// update), the pattern of the outer axes, whose increments a wave's samples share
template <int KIND>
__global__ __launch_bounds__(1024) void k_lds_atomic(double* out, uint32_t seed)
{
    __shared__ uint64_t bins[kBins];
    for (int i = threadIdx.x; i < kBins; i += blockDim.x) bins[i] = 0;
    __syncthreads();
    uint32_t a = lcg(threadIdx.x * 2654435761u + blockIdx.x * 97u + seed);
    for (int r = 0; r < kAtomRep; ++r) {
        a = lcg(a);
        uint32_t b = a >> 19;  // < kBins
        if constexpr (KIND == 4) {
            const uint32_t w = __builtin_amdgcn_readfirstlane(lcg(a ^ (uint32_t)r));
            b = ((w >> 19) & ~127u) | (a >> 25);  // window of 128 bins, < kBins
        }
        if constexpr (KIND == 0 || KIND == 4) {
            atomicAdd(reinterpret_cast<double*>(bins) + b, 1.0);
        } else if constexpr (KIND == 1) {
            atomicAdd(reinterpret_cast<float*>(bins) + b, 1.0f);
        } else if constexpr (KIND == 2) {
            atomicAdd(reinterpret_cast<uint32_t*>(bins) + b, 1u);
        } else {
            unsigned long long* w = reinterpret_cast<unsigned long long*>(bins) + b;
            unsigned long long cur = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            for (;;) {
                const unsigned long long nw = __double_as_longlong(__longlong_as_double(cur) + 1.0);
                const unsigned long long old = atomicCAS(w, cur, nw);
                if (old == cur) break;
                cur = old;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && bins[seed & (kBins - 1)] == 0x123456789ull) out[0] = 1.0;
}

template <int BYTES>
__global__ __launch_bounds__(1024) void k_gather(const double* table, double* out, uint32_t seed)
{
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)table, (short)0, kBins * 8, 0x00020000);
    uint32_t a[kCh];
    for (int i = 0; i < kCh; ++i) a[i] = lcg(threadIdx.x * 2654435761u + blockIdx.x * 97u + i * 7919u + seed);
    double acc = 0.0;
    for (int r = 0; r < kAtomRep / kCh; ++r) {
#pragma unroll
        for (int i = 0; i < kCh; ++i) {
            a[i] = lcg(a[i]);
            const uint32_t pos = (a[i] >> 19) & (kBins - 2);  // even, so a 16-byte load stays inside the table
            if constexpr (BYTES == 8) {
                const auto v = __builtin_amdgcn_raw_buffer_load_b64(rsrc, pos * 8u, 0, 0);
                acc += __builtin_bit_cast(double, ((uint64_t)(uint32_t)v[1] << 32) | (uint32_t)v[0]);
            } else {
                const auto v = __builtin_amdgcn_raw_buffer_load_b128(rsrc, pos * 8u, 0, 0);
                acc += __builtin_bit_cast(double, ((uint64_t)(uint32_t)v[1] << 32) | (uint32_t)v[0]) +
                       __builtin_bit_cast(double, ((uint64_t)(uint32_t)v[3] << 32) | (uint32_t)v[2]);
            }
        }
    }
    if (acc == 0.123) out[0] = acc;
}

template <int BYTES>
void run_gather(const char* name, double* table, double* buf, hipEvent_t e0, hipEvent_t e1)
{
    const int blocks = 256 * 2 * 4, threads = 1024;
    auto launch = [&] { hipLaunchKernelGGL(k_gather<BYTES>, dim3(blocks), dim3(threads), 0, 0, table, buf, 5u); };
    launch();
    (void)hipDeviceSynchronize();
    (void)hipEventRecord(e0);
    launch();
    (void)hipEventRecord(e1);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double lane_ops = (double)blocks * threads * (kAtomRep / kCh * kCh);
    const double per_cu = lane_ops / (ms * 1e-3) / 256.0;
    printf("%-18s %8.3f ms  %.3e lane loads/s per CU  %.1f cycles per wave instruction at 2.4 GHz\n", name, ms,
           per_cu, 2.4e9 / per_cu * 64.0);
}

template <int KIND>
void run_atomic(const char* name, double* buf, hipEvent_t e0, hipEvent_t e1)
{
    const int blocks = 256 * 2 * 4, threads = 1024;
    auto launch = [&] { hipLaunchKernelGGL(k_lds_atomic<KIND>, dim3(blocks), dim3(threads), 0, 0, buf, 5u); };
    launch();
    (void)hipDeviceSynchronize();
    (void)hipEventRecord(e0);
    launch();
    (void)hipEventRecord(e1);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double lane_ops = (double)blocks * threads * kAtomRep;
    const double per_cu = lane_ops / (ms * 1e-3) / 256.0;
    printf("%-18s %8.3f ms  %.3e lane updates/s per CU  %.1f cycles per wave instruction at 2.4 GHz\n", name, ms,
           per_cu, 2.4e9 / per_cu * 64.0);
}

template <typename F>
void run(const char* name, const char* body, F launch, double ops, hipEvent_t e0, hipEvent_t e1)
{
    launch();
    (void)hipDeviceSynchronize();
    (void)hipEventRecord(e0);
    launch();
    (void)hipEventRecord(e1);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double peak = 256.0 * 64.0 * 2.4e9;
    const double rate = ops / (ms * 1e-3);
    printf("%-14s %-34s %8.3f ms  %.3e lane-ops/s  %.3f of peak  %.2f slots/op\n", name, body, ms, rate,
           rate / peak, peak / rate);
}

}  // namespace

int main()
{
    void* buf = nullptr;
    if (hipMalloc(&buf, 64) != hipSuccess) return 1;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const int blocks = 256 * 8, threads = 256;
    const double ops = (double)blocks * threads * kRep * kCh;
    run("v_mad_u64_u32", "(mad only)", [&] {
        hipLaunchKernelGGL(k_mad_u64_u32, dim3(blocks), dim3(threads), 0, 0, (uint64_t*)buf, 1u);
    }, ops, e0, e1);
    run("v_fma_f64", "(fma only)", [&] {
        hipLaunchKernelGGL(k_fma_f64, dim3(blocks), dim3(threads), 0, 0, (double*)buf, 0.5);
    }, ops, e0, e1);
    run("v_fma_f32", "(fma only, unpacked)", [&] {
        hipLaunchKernelGGL(k_fma_f32, dim3(blocks), dim3(threads), 0, 0, (float*)buf, 0.5f);
    }, ops, e0, e1);
    run("v_bitop3_b32", "(bitop3 only)", [&] {
        hipLaunchKernelGGL(k_bitop3, dim3(blocks), dim3(threads), 0, 0, (uint32_t*)buf, 1u);
    }, ops, e0, e1);
    run("v_exp_f32", "(exp + 1 subtract per op)", [&] {
        hipLaunchKernelGGL(k_exp_f32, dim3(blocks), dim3(threads), 0, 0, (float*)buf, 0.f);
    }, ops, e0, e1);
    run_atomic<0>("ds_add_f64", (double*)buf, e0, e1);
    run_atomic<1>("ds_add_f32", (double*)buf, e0, e1);
    run_atomic<2>("ds_add_u32", (double*)buf, e0, e1);
    run_atomic<3>("ds_cmpst_rtn_b64", (double*)buf, e0, e1);
    run_atomic<4>("ds_add_f64 window", (double*)buf, e0, e1);
    void* table = nullptr;
    if (hipMalloc(&table, kBins * 8) != hipSuccess) return 1;
    (void)hipMemset(table, 0, kBins * 8);
    run_gather<8>("gather b64", (double*)table, (double*)buf, e0, e1);
    run_gather<16>("gather b128", (double*)table, (double*)buf, e0, e1);
    (void)hipFree(table);
    const hipError_t e = hipGetLastError();
    (void)hipFree(buf);
    return e == hipSuccess ? 0 : 1;
}

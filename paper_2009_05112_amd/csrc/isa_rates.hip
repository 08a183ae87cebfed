// isa_rates.hip -- issue rate of the VALU instruction kinds the sampling
// kernel is made of, on the device it runs on.
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
    const hipError_t e = hipGetLastError();
    (void)hipFree(buf);
    return e == hipSuccess ? 0 : 1;
}

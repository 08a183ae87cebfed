// vp_examples.hip -- example batched integrands (libvegasp_examples.so).
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <unordered_map>

#include "../../include/vegasp_examples.h"

namespace {

constexpr int kTerms = 4;
constexpr int kDim = 24;

// Term count of each mixture handle, on the host (the launch picks the
// kernel specialised for it without reading device memory).
std::mutex g_mu;
std::unordered_map<const void*, int32_t> g_terms;

struct GaussMix {
    int32_t dim, n_terms;
    double centers[kTerms * kDim];
    double coefs[kTerms];
    double amps[kTerms];
};

// Two points per thread (s and s + n/2 rounded up, both coalesced across the
// wave); coordinate d of point s is x[d * n + s].  The number of terms is a
// template argument, so the per-term sums stay in registers.
template <int K>
__global__ void k_gauss_mix(const GaussMix* __restrict__ g, int64_t n, const double* __restrict__ x,
                            double* __restrict__ f)
{
    const int64_t half = (n + 1) / 2;
    const int64_t s0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s0 >= half) return;
    const int64_t s1 = s0 + half;
    const bool two = s1 < n;
    const int D = g->dim;
    double q0[K], q1[K];
#pragma unroll
    for (int k = 0; k < K; ++k) q0[k] = q1[k] = 0.0;
    for (int d = 0; d < D; ++d) {
        const double xa = x[(int64_t)d * n + s0];
        const double xb = two ? x[(int64_t)d * n + s1] : 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double c = g->centers[k * D + d];
            const double ta = xa - c, tb = xb - c;
            q0[k] = fma(ta, ta, q0[k]);
            q1[k] = fma(tb, tb, q1[k]);
        }
    }
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        a0 = fma(g->amps[k], exp(-(g->coefs[k] * q0[k])), a0);
        a1 = fma(g->amps[k], exp(-(g->coefs[k] * q1[k])), a1);
    }
    f[s0] = a0;
    if (two) f[s1] = a1;
}

constexpr int kOut = 16;

struct GaussMoments {
    GaussMix g;
    int32_t n_out;
    int32_t e1[kOut], e2[kOut];  // component a: g(x) * x_e1 * x_e2 (-1: factor 1)
};

// One thread per point: the mixture g as in k_gauss_mix, then every
// component g * m_a with the monomial m_a = (x_e1 or 1) * (x_e2 or 1).
__global__ void k_gauss_moments(const GaussMoments* __restrict__ gm, int64_t n, const double* __restrict__ x,
                                double* __restrict__ f)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const GaussMix* g = &gm->g;
    const int D = g->dim, K = g->n_terms;
    double q[kTerms] = {0.0, 0.0, 0.0, 0.0};
    for (int d = 0; d < D; ++d) {
        const double xd = x[(int64_t)d * n + s];
        for (int k = 0; k < K; ++k) {
            const double t = xd - g->centers[k * D + d];
            q[k] = fma(t, t, q[k]);
        }
    }
    double acc = 0.0;
    for (int k = 0; k < K; ++k) acc = fma(g->amps[k], exp(-(g->coefs[k] * q[k])), acc);
    for (int a = 0; a < gm->n_out; ++a) {
        double m = 1.0;
        if (gm->e1[a] >= 0) m = x[(int64_t)gm->e1[a] * n + s];
        if (gm->e2[a] >= 0) m = m * x[(int64_t)gm->e2[a] * n + s];
        f[(int64_t)a * n + s] = acc * m;
    }
}

}  // namespace

extern "C" {

int vp_example_gauss_mix_user(int32_t dim, int32_t n_terms, const double* centers, const double* coefs,
                              const double* amps, void** user)
{
    if (!user || dim < 1 || dim > kDim || n_terms < 1 || n_terms > kTerms || !centers || !coefs || !amps) return 1;
    GaussMix h;
    memset(&h, 0, sizeof h);
    h.dim = dim;
    h.n_terms = n_terms;
    for (int i = 0; i < dim * n_terms; ++i) h.centers[i] = centers[i];
    for (int k = 0; k < n_terms; ++k) {
        h.coefs[k] = coefs[k];
        h.amps[k] = amps[k];
    }
    GaussMix* d = nullptr;
    if (hipMalloc((void**)&d, sizeof h) != hipSuccess) return 2;
    if (hipMemcpy(d, &h, sizeof h, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return 3;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_terms[d] = n_terms;
    }
    *user = d;
    return 0;
}

int vp_example_gauss_mix(void* user, void* hip_stream, int64_t n, int32_t dim, const double* x_soa, double* f_out)
{
    (void)dim;
    if (!user || n < 0) return 1;
    if (n == 0) return 0;
    const int block = 256;
    const int64_t grid = ((n + 1) / 2 + block - 1) / block;
    const GaussMix* g = (const GaussMix*)user;
    int32_t k = 0;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_terms.find(user);
        if (it == g_terms.end()) return 1;
        k = it->second;
    }
    const hipStream_t st = (hipStream_t)hip_stream;
    switch (k) {
    case 1: hipLaunchKernelGGL(k_gauss_mix<1>, dim3((unsigned)grid), dim3(block), 0, st, g, n, x_soa, f_out); break;
    case 2: hipLaunchKernelGGL(k_gauss_mix<2>, dim3((unsigned)grid), dim3(block), 0, st, g, n, x_soa, f_out); break;
    case 3: hipLaunchKernelGGL(k_gauss_mix<3>, dim3((unsigned)grid), dim3(block), 0, st, g, n, x_soa, f_out); break;
    default: hipLaunchKernelGGL(k_gauss_mix<4>, dim3((unsigned)grid), dim3(block), 0, st, g, n, x_soa, f_out); break;
    }
    return hipGetLastError() == hipSuccess ? 0 : 4;
}

int vp_example_gauss_moments_user(int32_t dim, int32_t n_terms, const double* centers, const double* coefs,
                                  const double* amps, int32_t n_out, const int32_t* e1, const int32_t* e2, void** user)
{
    if (!user || dim < 1 || dim > kDim || n_terms < 1 || n_terms > kTerms || !centers || !coefs || !amps ||
        n_out < 1 || n_out > kOut || !e1 || !e2)
        return 1;
    GaussMoments h;
    memset(&h, 0, sizeof h);
    h.g.dim = dim;
    h.g.n_terms = n_terms;
    for (int i = 0; i < dim * n_terms; ++i) h.g.centers[i] = centers[i];
    for (int k = 0; k < n_terms; ++k) {
        h.g.coefs[k] = coefs[k];
        h.g.amps[k] = amps[k];
    }
    h.n_out = n_out;
    for (int a = 0; a < n_out; ++a) {
        if (e1[a] < -1 || e1[a] >= dim || e2[a] < -1 || e2[a] >= dim) return 1;
        h.e1[a] = e1[a];
        h.e2[a] = e2[a];
    }
    GaussMoments* d = nullptr;
    if (hipMalloc((void**)&d, sizeof h) != hipSuccess) return 2;
    if (hipMemcpy(d, &h, sizeof h, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return 3;
    }
    *user = d;
    return 0;
}

int vp_example_gauss_moments(void* user, void* hip_stream, int64_t n, int32_t dim, const double* x_soa, double* f_out)
{
    (void)dim;
    if (!user || n < 0) return 1;
    if (n == 0) return 0;
    const int block = 256;
    const int64_t grid = (n + block - 1) / block;
    hipLaunchKernelGGL(k_gauss_moments, dim3((unsigned)grid), dim3(block), 0, (hipStream_t)hip_stream,
                       (const GaussMoments*)user, n, x_soa, f_out);
    return hipGetLastError() == hipSuccess ? 0 : 4;
}

int vp_example_failing(void* user, void* hip_stream, int64_t n, int32_t dim, const double* x_soa, double* f_out)
{
    (void)user;
    (void)hip_stream;
    (void)n;
    (void)dim;
    (void)x_soa;
    (void)f_out;
    return 7;
}

int vp_example_free_user(void* user)
{
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_terms.erase(user);
    }
    return hipFree(user) == hipSuccess ? 0 : 1;
}

}  // extern "C"

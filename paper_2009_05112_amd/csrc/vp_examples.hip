// vp_examples.hip -- example batched integrands (libvegasp_examples.so).
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/vegasp_examples.h"

namespace {

constexpr int kTerms = 4;
constexpr int kDim = 24;

struct GaussMix {
    int32_t dim, n_terms;
    double centers[kTerms * kDim];
    double coefs[kTerms];
    double amps[kTerms];
};

// One thread per point; coordinate d of point s is x[d * n + s], so the
// reads of one coordinate are coalesced across the wave.
__global__ void k_gauss_mix(const GaussMix* __restrict__ g, int64_t n, const double* __restrict__ x,
                            double* __restrict__ f)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
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
    f[s] = acc;
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
    *user = d;
    return 0;
}

int vp_example_gauss_mix(void* user, void* hip_stream, int64_t n, int32_t dim, const double* x_soa, double* f_out)
{
    (void)dim;
    if (!user || n < 0) return 1;
    if (n == 0) return 0;
    const int block = 256;
    const int64_t grid = (n + block - 1) / block;
    hipLaunchKernelGGL(k_gauss_mix, dim3((unsigned)grid), dim3(block), 0, (hipStream_t)hip_stream,
                       (const GaussMix*)user, n, x_soa, f_out);
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
    return hipFree(user) == hipSuccess ? 0 : 1;
}

}  // extern "C"

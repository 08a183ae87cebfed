/* vegasp_examples.h -- example batched integrands for VP_F_BATCH.
 *
 * libvegasp_examples.so holds ready-made vp_batch_fn functions, each with a
 * constructor for the `user` argument it expects.  They show how a batched
 * integrand is written (one kernel over the structure-of-arrays points,
 * enqueued on the library's stream) and serve the tests that compare the
 * batched path with the built-in integrands.
 *
 * Conventions as in vegasp.h: host arrays are copied; the functions return 0
 * on success.
 */
#ifndef VEGASP_EXAMPLES_H
#define VEGASP_EXAMPLES_H

#include <stdint.h>

#include "vegasp.h"

#ifdef __cplusplus
extern "C" {
#endif

/* g(x) = sum_k amps[k] exp(-coefs[k] |x - c_k|^2), c_k = centers[k*dim ..],
 * 1 <= n_terms <= 4, 1 <= dim <= 24: the same operations, in the same order,
 * as the built-in VP_F_GAUSS_MIX (the library multiplies by `scale`).
 * *user receives a device-side parameter block, freed by
 * vp_example_free_user. */
int vp_example_gauss_mix_user(int32_t dim, int32_t n_terms, const double* centers, const double* coefs,
                              const double* amps, void** user);
int vp_example_gauss_mix(void* user, void* hip_stream, int64_t n, int32_t dim, const double* x_soa,
                         double* f_out);

/* Vector-valued (n_out components, 1 <= n_out <= 16): component a is
 * g(x) m_a(x) with g the mixture above and the monomial
 * m_a = (e1[a] < 0 ? 1 : x_e1[a]) * (e2[a] < 0 ? 1 : x_e2[a]), e.g. the
 * normalisation, the means and the second moments of the density g. */
int vp_example_gauss_moments_user(int32_t dim, int32_t n_terms, const double* centers, const double* coefs,
                                  const double* amps, int32_t n_out, const int32_t* e1, const int32_t* e2,
                                  void** user);
int vp_example_gauss_moments(void* user, void* hip_stream, int64_t n, int32_t dim, const double* x_soa,
                             double* f_out);

/* Always fails (returns 7) and writes nothing: for testing error paths. */
int vp_example_failing(void* user, void* hip_stream, int64_t n, int32_t dim, const double* x_soa, double* f_out);

int vp_example_free_user(void* user);

#ifdef __cplusplus
}
#endif

#endif /* VEGASP_EXAMPLES_H */

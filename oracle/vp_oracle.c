/*
 * vp_oracle.c -- plain, slow FP64 CPU oracle for one vegas+ iteration.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the HIP library.
 *
 * Source: G. P. Lepage, "Adaptive Multidimensional Integration: VEGAS
 * Enhanced" (arXiv:2009.05112).  Every function names the passage it follows.
 * The paper leaves the random-number generator, the enumeration order of the
 * hypercubes and the rounding of each step open; the readings taken here are
 * listed in the repository's design notes and restated next to the code.
 *
 * Every floating-point operation is a single IEEE round-to-nearest operation
 * (the file is compiled with -ffp-contract=off); fused multiply-adds appear
 * only where fma() is written.
 *
 * Pins: every function is checked by the tests against what the paper and
 * the mathematics fix.  The default, weighted increment training data (the
 * sum of (J f)^2 / n_h over the sum of 1 / n_h, the reading of Sec. 2.3 under
 * a non-uniform allocation) are pinned exactly to the printed formula where
 * the two coincide (uniform allocation), and statistically elsewhere: under
 * an arbitrary allocation their ratio is an unbiased estimate of N_g times
 * the increment's integral of (J f)^2, which the allocation-independence of
 * the optimal map (Sec. 3) asks for, checked against a closed form.  The
 * printed formula itself is the literal mode.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (Salmon, Moraes, Dror and    */
/* Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3", SC'11, Sec. 3.2).     */
/* A round multiplies counter words 0 and 2 by two fixed odd constants, and  */
/* builds the next counter from the high halves xored with the other two     */
/* words and the round key, and the low halves.  The key is advanced by two  */
/* Weyl constants between rounds.  The paper fixes no generator; this one is */
/* keyed by the 64-bit seed and counted by (sample, hypercube, iteration,    */
/* block), so every sample is reproducible in isolation.                     */
/* ------------------------------------------------------------------------ */
#define OR_PHILOX_M0 0xD2511F53u
#define OR_PHILOX_M1 0xCD9E8D57u
#define OR_PHILOX_W0 0x9E3779B9u
#define OR_PHILOX_W1 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += OR_PHILOX_W0;
            k1 += OR_PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)OR_PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)OR_PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* Stratification count, Sec. 3, Eq. (Nst_vegasp): N_st = floor((N_ev/4)^(1/D)).  */
/* Taken as the largest integer n >= 1 with 4 n^D <= N_ev, found by integer */
/* search so exact powers are not lost to rounding of the real root.         */
/* Returns 1 when even n = 1 does not satisfy the bound (then there is a      */
/* single hypercube), 0 on invalid input.                                     */
/* ------------------------------------------------------------------------ */
static int or_pow_le(int64_t n, int32_t dim, int64_t limit)
{
    /* 1 if 4 * n^dim <= limit, computed without overflow */
    int64_t acc = 4;
    if (acc > limit) return 0;
    for (int32_t d = 0; d < dim; ++d) {
        if (acc > limit / n) return 0;
        acc *= n;
    }
    return acc <= limit;
}

int32_t or_nst(int32_t dim, int64_t n_ev)
{
    if (dim < 1 || n_ev < 1) return 0;
    int64_t n = 1;
    while (or_pow_le(n + 1, dim, n_ev)) ++n;
    return (int32_t)n;
}

/* Classic vegas stratification, Sec. 3, Eq. (Nst): largest n >= 1 with 2 n^D <= N_ev. */
int32_t or_nst_classic(int32_t dim, int64_t n_ev)
{
    if (dim < 1 || n_ev < 1) return 0;
    int64_t n = 1;
    for (;;) {
        int64_t m = n + 1, acc = 2;
        int ok = 1;
        for (int32_t d = 0; d < dim; ++d) {
            if (acc > n_ev / m) { ok = 0; break; }
            acc *= m;
        }
        if (!ok || acc > n_ev) break;
        n = m;
    }
    return (int32_t)n;
}

/* Mixed stratification, Sec. 4: N_st + 1 stratifications on the first d     */
/* axes and N_st on the others, with N_st from Eq. (Nst_vegasp) and d the     */
/* largest number of axes that still leaves an average of 4 samples per       */
/* hypercube, i.e. 4 (N_st + 1)^d N_st^(D - d) <= N_ev.  out[0..dim-1].       */
/* ------------------------------------------------------------------------ */
int32_t or_nst_mixed(int32_t dim, int64_t n_ev, int32_t* out)
{
    int32_t n = or_nst(dim, n_ev);
    if (n < 1) return 0;
    int32_t best = 0;
    for (int32_t d = 0; d <= dim; ++d) {
        /* 4 (n + 1)^d n^(dim - d), stopping once it passes n_ev */
        double prod = 4.0;
        int ok = 1;
        for (int32_t mu = 0; mu < dim; ++mu) {
            prod *= (mu < d) ? (double)(n + 1) : (double)n;
            if (prod > (double)n_ev) { ok = 0; break; }
        }
        if (ok) best = d;
    }
    for (int32_t mu = 0; mu < dim; ++mu) out[mu] = mu < best ? n + 1 : n;
    return best;
}

/* ------------------------------------------------------------------------ */
/* Integrands.  f(x) as the user defines it; the sampler multiplies by J.     */
/* ------------------------------------------------------------------------ */
enum {
    OR_F_GAUSS_MIX = 1,  /* scale * sum_k amp_k exp(-coef_k |x - c_k|^2)      */
    OR_F_CORR_GAUSS = 2, /* scale * exp(-1/2 |U (x - mu)|^2), U upper-tri     */
    OR_F_EXP_ABS = 3,    /* scale * sum_k amp_k exp(-coef_k |x - c_k|)        */
    OR_F_CONST = 4,      /* scale                                             */
    OR_F_AFFINE = 5,     /* scale * (a_0 + sum_d a_{d+1} x_d), a in centers   */
    OR_F_BALLS = 6       /* scale * sum_k amp_k [|x - c_k| < coef_k]          */
};

typedef struct {
    int32_t kind;
    int32_t dim;
    int32_t n_terms;
    const double* centers; /* n_terms x dim; CORR_GAUSS: mean (dim); AFFINE: dim+1 */
    const double* coefs;   /* n_terms */
    const double* amps;    /* n_terms */
    const double* chol;    /* dim x dim row-major upper-triangular U (CORR_GAUSS) */
    double scale;
} or_integrand;

double or_integrand_eval(const or_integrand* f, const double* x)
{
    const int32_t D = f->dim;
    switch (f->kind) {
    case OR_F_GAUSS_MIX: {
        double acc = 0.0;
        for (int32_t k = 0; k < f->n_terms; ++k) {
            double q = 0.0;
            for (int32_t d = 0; d < D; ++d) {
                double t = x[d] - f->centers[(int64_t)k * D + d];
                q = fma(t, t, q);
            }
            double e = exp(-(f->coefs[k] * q));
            acc = fma(f->amps[k], e, acc);
        }
        return f->scale * acc;
    }
    case OR_F_CORR_GAUSS: {
        double q = 0.0;
        for (int32_t d = 0; d < D; ++d) {
            double z = 0.0;
            for (int32_t e = d; e < D; ++e) {
                double t = x[e] - f->centers[e];
                z = fma(f->chol[(int64_t)d * D + e], t, z);
            }
            q = fma(z, z, q);
        }
        return f->scale * exp(-0.5 * q);
    }
    case OR_F_EXP_ABS: {
        double acc = 0.0;
        for (int32_t k = 0; k < f->n_terms; ++k) {
            double q = 0.0;
            for (int32_t d = 0; d < D; ++d) {
                double t = x[d] - f->centers[(int64_t)k * D + d];
                q = fma(t, t, q);
            }
            double e = exp(-(f->coefs[k] * sqrt(q)));
            acc = fma(f->amps[k], e, acc);
        }
        return f->scale * acc;
    }
    case OR_F_CONST:
        return f->scale;
    case OR_F_AFFINE: {
        double acc = f->centers[0];
        for (int32_t d = 0; d < D; ++d) acc = fma(f->centers[d + 1], x[d], acc);
        return f->scale * acc;
    }
    case OR_F_BALLS: {
        double acc = 0.0;
        for (int32_t k = 0; k < f->n_terms; ++k) {
            double q = 0.0;
            for (int32_t d = 0; d < D; ++d) {
                double t = x[d] - f->centers[(int64_t)k * D + d];
                q = fma(t, t, q);
            }
            double r2 = f->coefs[k] * f->coefs[k];
            if (q < r2) acc = acc + f->amps[k];
        }
        return f->scale * acc;
    }
    default:
        return NAN;
    }
}

/* Single-precision evaluation of the same integrands, for the precision split
 * (FP32 map and integrand).  Same operation order, float arithmetic, expf. */
float or_integrand_eval_f32(const or_integrand* f, const float* x)
{
    const int32_t D = f->dim;
    switch (f->kind) {
    case OR_F_GAUSS_MIX: {
        float acc = 0.0f;
        for (int32_t k = 0; k < f->n_terms; ++k) {
            float q = 0.0f;
            for (int32_t d = 0; d < D; ++d) {
                float t = x[d] - (float)f->centers[(int64_t)k * D + d];
                q = fmaf(t, t, q);
            }
            float e = expf(-((float)f->coefs[k] * q));
            acc = fmaf((float)f->amps[k], e, acc);
        }
        return (float)f->scale * acc;
    }
    case OR_F_CORR_GAUSS: {
        float q = 0.0f;
        for (int32_t d = 0; d < D; ++d) {
            float z = 0.0f;
            for (int32_t e = d; e < D; ++e) {
                float t = x[e] - (float)f->centers[e];
                z = fmaf((float)f->chol[(int64_t)d * D + e], t, z);
            }
            q = fmaf(z, z, q);
        }
        return (float)f->scale * expf(-0.5f * q);
    }
    case OR_F_EXP_ABS: {
        float acc = 0.0f;
        for (int32_t k = 0; k < f->n_terms; ++k) {
            float q = 0.0f;
            for (int32_t d = 0; d < D; ++d) {
                float t = x[d] - (float)f->centers[(int64_t)k * D + d];
                q = fmaf(t, t, q);
            }
            float e = expf(-((float)f->coefs[k] * sqrtf(q)));
            acc = fmaf((float)f->amps[k], e, acc);
        }
        return (float)f->scale * acc;
    }
    case OR_F_CONST:
        return (float)f->scale;
    case OR_F_AFFINE: {
        float acc = (float)f->centers[0];
        for (int32_t d = 0; d < D; ++d) acc = fmaf((float)f->centers[d + 1], x[d], acc);
        return (float)f->scale * acc;
    }
    case OR_F_BALLS: {
        float acc = 0.0f;
        for (int32_t k = 0; k < f->n_terms; ++k) {
            float q = 0.0f;
            for (int32_t d = 0; d < D; ++d) {
                float t = x[d] - (float)f->centers[(int64_t)k * D + d];
                q = fmaf(t, t, q);
            }
            float r = (float)f->coefs[k];
            if (q < r * r) acc = acc + (float)f->amps[k];
        }
        return (float)f->scale * acc;
    }
    default:
        return NAN;
    }
}

/* ------------------------------------------------------------------------ */
/* Problem description shared by the steps below.                             */
/* ------------------------------------------------------------------------ */
enum { OR_FP64 = 0, OR_FP32_ACC64 = 1, OR_FP32_NEUMAIER = 2 };
enum { OR_HIST_WEIGHTED = 0, OR_HIST_LITERAL = 1 };

typedef struct {
    int32_t dim;
    int64_t n_ev;
    int32_t n_g;
    int32_t n_st;
    double alpha;
    double beta;
    uint64_t seed;
    int32_t precision;      /* OR_FP64 / OR_FP32_ACC64 / OR_FP32_NEUMAIER */
    int32_t hist_mode;      /* OR_HIST_WEIGHTED / OR_HIST_LITERAL */
    int32_t realloc_plus2;  /* 1: n_h = floor(q) + 2 (Sec. 3, alternative rule) */
    int32_t n_adapt;        /* > 0: iterations it >= n_adapt keep map and n_h (Sec. 2.5) */
    int32_t n_st_axes[64];  /* stratifications of axis mu (Sec. 4); 0: n_st */
} or_params;

/* N_st^mu, the stratifications of axis mu */
static int32_t or_nst_axis(const or_params* p, int32_t mu)
{
    return p->n_st_axes[mu] > 0 ? p->n_st_axes[mu] : p->n_st;
}

/* Number of hypercubes, prod_mu N_st^mu (Sec. 3: N_st^D when uniform). */
int64_t or_n_hypercubes(const or_params* p)
{
    int64_t n = 1;
    for (int32_t d = 0; d < p->dim; ++d) n *= or_nst_axis(p, d);
    return n;
}

/* Initial vegas map, Sec. 2.3: a uniform grid, x_i = a + (b - a) i / N_g, with
 * the last point set to b exactly.  Layout: map[mu * (N_g + 1) + i]. */
void or_map_init(int32_t dim, int32_t n_g, const double* lower, const double* upper, double* map)
{
    for (int32_t mu = 0; mu < dim; ++mu) {
        double a = lower ? lower[mu] : 0.0;
        double b = upper ? upper[mu] : 1.0;
        double* x = map + (int64_t)mu * (n_g + 1);
        for (int32_t i = 0; i < n_g; ++i) x[i] = a + (b - a) * ((double)i / (double)n_g);
        x[n_g] = b;
    }
}

/* First allocation, Sec. 3: every hypercube gets the classic share
 * floor(N_ev / N_st^D), at least 2. */
void or_alloc_init(const or_params* p, int32_t* n_h)
{
    int64_t nhc = or_n_hypercubes(p);
    int64_t n = p->n_ev / nhc;
    if (n < 2) n = 2;
    for (int64_t h = 0; h < nhc; ++h) n_h[h] = (int32_t)n;
}

/* Neumaier's compensated summation (improved Kahan-Babuska), single precision. */
static void or_neumaier_add(float* s, float* c, float v)
{
    float t = *s + v;
    if (fabsf(*s) >= fabsf(v)) *c += (*s - t) + v;
    else *c += (v - t) + *s;
    *s = t;
}

/* Neumaier's compensated summation in double precision: the oracle takes its
 * sums (per hypercube, per increment, over hypercubes) to within about one
 * rounding of the exact sum, so that its own summation error stays far below
 * the comparison tolerance even over 1e7 terms. */
typedef struct {
    double s, c;
} or_ksum;

static void or_kadd(or_ksum* k, double v)
{
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else k->c += (v - t) + k->s;
    k->s = t;
}

static double or_kval(const or_ksum* k) { return k->s + k->c; }

/* Optional per-sample record for inspection tests. */
typedef struct {
    int64_t h;
    int32_t j;
    int32_t pad;
    double v;          /* J f */
    double jac;        /* J */
    double fx;         /* f(x) */
} or_sample_rec;

/* ------------------------------------------------------------------------ */
/* One iteration of sampling over hypercubes [h_begin, h_end).                */
/*                                                                            */
/* Sec. 2.4 (multidimensional map) and Sec. 3 (stratified sampling): in each  */
/* hypercube h with digits k_mu (axis 0 most significant), n_h points y are  */
/* drawn uniformly in the hypercube; y is mapped through the per-axis vegas  */
/* map of Sec. 2.2, Eqs. (y) and (jac): i = floor(y N_g), delta = y N_g - i,  */
/* x = x_i + Delta x_i delta, J = prod_mu N_g Delta x_i.  The sums of J f and */
/* (J f)^2 per hypercube (Sec. 3, step 2) and the per-axis, per-increment    */
/* training data d_i of Sec. 2.3 / 2.4 are accumulated.                       */
/*                                                                            */
/* Readings: y^mu = (k_mu + u) / N_st, so t = y N_g = (k_mu + u) R with       */
/* R = N_g / N_st rounded once; i = min(floor t, N_g - 1), delta = min(t - i, */
/* 1).  u takes 53 bits from two Philox words per axis: the high words of    */
/* axes 0..D-1 come first in the stream, then the low words.  The FP32 split */
/* takes u = (w >> 8) 2^-24 from the high words alone.                         */
/*                                                                            */
/* Training data.  Weighted mode: H += (J f)^2 / n_h and W += 1 / n_h, so the */
/* refinement uses d_i = H / W, the (1/n_i) sum of J^2 f^2 of Sec. 2.3 with   */
/* each sample weighted by its hypercube's share of y-space.  Literal mode:  */
/* H += (J f)^2 and W += 1, the formula as printed.                           */
/*                                                                            */
/* Outputs S1[h - h_begin], S2[h - h_begin] are written for every h in the   */
/* range; H and W (dim x n_g) are accumulated into (callers zero them).       */
/* ------------------------------------------------------------------------ */
/* One FP64 sample point from its Philox words w (Sec. 3 and Sec. 2.2): u from 53
 * bits (the high word of axis mu is word mu, its low word word D + mu),
 * t = (k_mu + u) R_mu, i = floor(t) (at most N_g - 1), delta = t - i (at most 1),
 * x = x_i + Delta x_i delta, J = prod_mu N_g Delta x_i.  Returns J. */
static double or_point64(int32_t D, int32_t NG, const double* R, const int32_t* k, const uint32_t* w,
                         const double* map, double* xs, int32_t* idx)
{
    double jac = 1.0;
    for (int32_t mu = 0; mu < D; ++mu) {
        uint64_t a = (uint64_t)(w[mu] >> 5);
        uint64_t bb = (uint64_t)(w[D + mu] >> 6);
        double u = (double)((a << 26) | bb) * 0x1p-53;
        double t = ((double)k[mu] + u) * R[mu];
        int32_t i = (int32_t)floor(t);
        if (i > NG - 1) i = NG - 1;
        double delta = t - (double)i;
        if (delta > 1.0) delta = 1.0;
        const double* xm = map + (int64_t)mu * (NG + 1);
        double dx = xm[i + 1] - xm[i];
        xs[mu] = fma(dx, delta, xm[i]);
        jac = jac * ((double)NG * dx);
        idx[mu] = i;
    }
    return jac;
}

/* The single-precision sample point of the precision split: u = (w >> 8) 2^-24
 * from the high word of each axis alone, then the steps of or_point64 in
 * float arithmetic with the map rounded to float.  Returns J. */
static float or_point32(int32_t D, int32_t NG, const float* R32, const int32_t* k, const uint32_t* w,
                        const float* map32, float* xs32, int32_t* idx)
{
    float jac = 1.0f;
    for (int32_t mu = 0; mu < D; ++mu) {
        float u = (float)(w[mu] >> 8) * 0x1p-24f;
        float t = ((float)k[mu] + u) * R32[mu];
        int32_t i = (int32_t)floorf(t);
        if (i > NG - 1) i = NG - 1;
        float delta = t - (float)i;
        if (delta > 1.0f) delta = 1.0f;
        const float* xm = map32 + (int64_t)mu * (NG + 1);
        float dx = xm[i + 1] - xm[i];
        xs32[mu] = fmaf(dx, delta, xm[i]);
        jac = jac * ((float)NG * dx);
        idx[mu] = i;
    }
    return jac;
}

int or_sample_range(const or_params* p, const or_integrand* f, const double* map,
                    const int32_t* n_h, int32_t it, int64_t h_begin, int64_t h_end,
                    double* S1, double* S2, double* H, double* W,
                    or_sample_rec* rec, int64_t rec_cap, int64_t* rec_count)
{
    const int32_t D = p->dim, NG = p->n_g;
    if (D < 1 || D > 64 || NG < 1) return -1;
    /* y^mu = (k_mu + u) / N_st^mu, so t = y^mu N_g = (k_mu + u) R_mu */
    int32_t NST[64];
    double R[64];
    float R32[64];
    for (int32_t mu = 0; mu < D; ++mu) {
        NST[mu] = or_nst_axis(p, mu);
        if (NST[mu] < 1) return -1;
        R[mu] = (double)NG / (double)NST[mu];
        R32[mu] = (float)NG / (float)NST[mu];
    }
    const uint32_t key[2] = {(uint32_t)(p->seed & 0xffffffffu), (uint32_t)(p->seed >> 32)};
    const int fp32 = (p->precision != OR_FP64);
    const int nwords = fp32 ? D : 2 * D;
    const int nblk = (nwords + 3) / 4;
    uint32_t w[4 * 33];
    int32_t k[64];
    int32_t idx[64];
    double xs[64];
    float xs32[64];
    float* map32 = NULL;
    if (fp32) {
        map32 = (float*)malloc(sizeof(float) * (size_t)D * (NG + 1));
        if (!map32) return -2;
        for (int64_t q = 0; q < (int64_t)D * (NG + 1); ++q) map32[q] = (float)map[q];
    }
    or_ksum* kH = NULL;
    or_ksum* kW = NULL;
    if (p->precision != OR_FP32_NEUMAIER) {
        kH = (or_ksum*)calloc((size_t)D * NG, sizeof(or_ksum));
        kW = (or_ksum*)calloc((size_t)D * NG, sizeof(or_ksum));
        if (!kH || !kW) {
            free(kH); free(kW); free(map32);
            return -2;
        }
    }
    float* nH = NULL;
    float* nW = NULL;
    if (p->precision == OR_FP32_NEUMAIER) {
        nH = (float*)calloc((size_t)2 * D * NG, sizeof(float));
        nW = (float*)calloc((size_t)2 * D * NG, sizeof(float));
        if (!nH || !nW) {
            free(nH); free(nW); free(map32);
            return -2;
        }
    }
    int64_t nrec = 0;

    for (int64_t h = h_begin; h < h_end; ++h) {
        /* digits of h in the mixed radix (N_st^0, ..., N_st^(D-1)), axis 0 most significant */
        int64_t rem = h;
        for (int32_t mu = D - 1; mu >= 0; --mu) {
            k[mu] = (int32_t)(rem % NST[mu]);
            rem /= NST[mu];
        }
        const int32_t n = n_h[h];
        const double inv_n = 1.0 / (double)n;
        const float inv_n32 = 1.0f / (float)n;
        or_ksum k1 = {0.0, 0.0}, k2 = {0.0, 0.0};
        double s1 = 0.0, s2 = 0.0;
        float ns1 = 0.0f, nc1 = 0.0f, ns2 = 0.0f, nc2 = 0.0f;

        for (int32_t j = 0; j < n; ++j) {
            for (int b = 0; b < nblk; ++b) {
                uint32_t ctr[4] = {(uint32_t)j, (uint32_t)h, (uint32_t)it, (uint32_t)b};
                or_philox4x32_10(ctr, key, &w[4 * b]);
            }
            double v, jac_out, f_out;
            if (!fp32) {
                double jac = or_point64(D, NG, R, k, w, map, xs, idx);
                double fx = or_integrand_eval(f, xs);
                v = jac * fx;
                jac_out = jac;
                f_out = fx;
            } else {
                float jac = or_point32(D, NG, R32, k, w, map32, xs32, idx);
                float fx = or_integrand_eval_f32(f, xs32);
                float v32 = jac * fx;
                v = (double)v32;
                jac_out = (double)jac;
                f_out = (double)fx;
                if (p->precision == OR_FP32_NEUMAIER) {
                    or_neumaier_add(&ns1, &nc1, v32);
                    or_neumaier_add(&ns2, &nc2, v32 * v32);
                }
            }
            if (p->precision != OR_FP32_NEUMAIER) {
                const double v2 = v * v;
                or_kadd(&k1, v);
                or_kadd(&k2, v2);
                for (int32_t mu = 0; mu < D; ++mu) {
                    int64_t bin = (int64_t)mu * NG + idx[mu];
                    if (p->hist_mode == OR_HIST_WEIGHTED) {
                        or_kadd(&kH[bin], v2 * inv_n);
                        or_kadd(&kW[bin], inv_n);
                    } else {
                        or_kadd(&kH[bin], v2);
                        or_kadd(&kW[bin], 1.0);
                    }
                }
            } else {
                const float v32 = (float)v;
                const float v2 = v32 * v32;
                for (int32_t mu = 0; mu < D; ++mu) {
                    int64_t bin = (int64_t)mu * NG + idx[mu];
                    if (p->hist_mode == OR_HIST_WEIGHTED) {
                        or_neumaier_add(&nH[2 * bin], &nH[2 * bin + 1], v2 * inv_n32);
                        or_neumaier_add(&nW[2 * bin], &nW[2 * bin + 1], inv_n32);
                    } else {
                        or_neumaier_add(&nH[2 * bin], &nH[2 * bin + 1], v2);
                        or_neumaier_add(&nW[2 * bin], &nW[2 * bin + 1], 1.0f);
                    }
                }
            }
            if (rec && nrec < rec_cap) {
                rec[nrec].h = h;
                rec[nrec].j = j;
                rec[nrec].pad = 0;
                rec[nrec].v = v;
                rec[nrec].jac = jac_out;
                rec[nrec].fx = f_out;
            }
            ++nrec;
        }
        if (p->precision == OR_FP32_NEUMAIER) {
            s1 = (double)ns1 + (double)nc1;
            s2 = (double)ns2 + (double)nc2;
        } else {
            s1 = or_kval(&k1);
            s2 = or_kval(&k2);
        }
        S1[h - h_begin] = s1;
        S2[h - h_begin] = s2;
    }
    if (kH) {
        for (int64_t bin = 0; bin < (int64_t)D * NG; ++bin) {
            H[bin] = H[bin] + or_kval(&kH[bin]);
            W[bin] = W[bin] + or_kval(&kW[bin]);
        }
    }
    if (nH) {
        /* compensated single-precision bins are merged in double precision */
        for (int64_t bin = 0; bin < (int64_t)D * NG; ++bin) {
            H[bin] = H[bin] + ((double)nH[2 * bin] + (double)nH[2 * bin + 1]);
            W[bin] = W[bin] + ((double)nW[2 * bin] + (double)nW[2 * bin + 1]);
        }
    }
    if (rec_count) *rec_count = nrec;
    free(kH);
    free(kW);
    free(nH);
    free(nW);
    free(map32);
    return 0;
}

/* Per-sample indices for inspection: increment index of every axis and the
 * hypercube of every sample, in (h, j) order.  idx_out is [n_samples][dim]. */
int or_sample_indices(const or_params* p, const int32_t* n_h, int32_t it, int64_t h_begin,
                      int64_t h_end, int32_t* idx_out, double* t_out, int64_t cap)
{
    const int32_t D = p->dim, NG = p->n_g;
    if (D < 1 || D > 64) return -1;
    int32_t NST[64];
    double R[64];
    float R32[64];
    for (int32_t mu = 0; mu < D; ++mu) {
        NST[mu] = or_nst_axis(p, mu);
        R[mu] = (double)NG / (double)NST[mu];
        R32[mu] = (float)NG / (float)NST[mu];
    }
    const uint32_t key[2] = {(uint32_t)(p->seed & 0xffffffffu), (uint32_t)(p->seed >> 32)};
    const int fp32 = (p->precision != OR_FP64);
    const int nblk = ((fp32 ? D : 2 * D) + 3) / 4;
    uint32_t w[4 * 33];
    int64_t s = 0;
    for (int64_t h = h_begin; h < h_end; ++h) {
        int32_t k[64];
        int64_t rem = h;
        for (int32_t mu = D - 1; mu >= 0; --mu) {
            k[mu] = (int32_t)(rem % NST[mu]);
            rem /= NST[mu];
        }
        for (int32_t j = 0; j < n_h[h]; ++j, ++s) {
            if (s >= cap) return -1;
            for (int b = 0; b < nblk; ++b) {
                uint32_t ctr[4] = {(uint32_t)j, (uint32_t)h, (uint32_t)it, (uint32_t)b};
                or_philox4x32_10(ctr, key, &w[4 * b]);
            }
            for (int32_t mu = 0; mu < D; ++mu) {
                int32_t i;
                double tt;
                if (!fp32) {
                    uint64_t a = (uint64_t)(w[mu] >> 5);
                    uint64_t bb = (uint64_t)(w[D + mu] >> 6);
                    double u = (double)((a << 26) | bb) * 0x1p-53;
                    tt = ((double)k[mu] + u) * R[mu];
                    i = (int32_t)floor(tt);
                } else {
                    float u = (float)(w[mu] >> 8) * 0x1p-24f;
                    float t32 = ((float)k[mu] + u) * R32[mu];
                    tt = (double)t32;
                    i = (int32_t)floorf(t32);
                }
                if (i > NG - 1) i = NG - 1;
                idx_out[s * D + mu] = i;
                if (t_out) t_out[s * D + mu] = tt;
            }
        }
    }
    return 0;
}

/* Every sample of hypercubes [h_begin, h_end) in (h, j) order, for per-sample
 * inspection: its hypercube h and index j, increment index and point x on
 * every axis ([n_samples][dim]), J and f(x) (split precisions: their single-
 * precision values widened).  The same steps as or_sample_range. */
int or_sample_points(const or_params* p, const or_integrand* f, const double* map, const int32_t* n_h,
                     int32_t it, int64_t h_begin, int64_t h_end, int64_t* h_out, int32_t* j_out,
                     int32_t* idx_out, double* x_out, double* jac_out, double* fx_out, int64_t cap)
{
    const int32_t D = p->dim, NG = p->n_g;
    if (D < 1 || D > 64 || NG < 1) return -1;
    int32_t NST[64];
    double R[64];
    float R32[64];
    for (int32_t mu = 0; mu < D; ++mu) {
        NST[mu] = or_nst_axis(p, mu);
        R[mu] = (double)NG / (double)NST[mu];
        R32[mu] = (float)NG / (float)NST[mu];
    }
    const uint32_t key[2] = {(uint32_t)(p->seed & 0xffffffffu), (uint32_t)(p->seed >> 32)};
    const int fp32 = (p->precision != OR_FP64);
    const int nblk = ((fp32 ? D : 2 * D) + 3) / 4;
    float* map32 = NULL;
    if (fp32) {
        map32 = (float*)malloc(sizeof(float) * (size_t)D * (NG + 1));
        if (!map32) return -2;
        for (int64_t q = 0; q < (int64_t)D * (NG + 1); ++q) map32[q] = (float)map[q];
    }
    uint32_t w[4 * 33];
    int32_t k[64], idx[64];
    double xs[64];
    float xs32[64];
    int64_t s = 0;
    for (int64_t h = h_begin; h < h_end; ++h) {
        int64_t rem = h;
        for (int32_t mu = D - 1; mu >= 0; --mu) {
            k[mu] = (int32_t)(rem % NST[mu]);
            rem /= NST[mu];
        }
        for (int32_t j = 0; j < n_h[h]; ++j, ++s) {
            if (s >= cap) {
                free(map32);
                return -1;
            }
            for (int b = 0; b < nblk; ++b) {
                uint32_t ctr[4] = {(uint32_t)j, (uint32_t)h, (uint32_t)it, (uint32_t)b};
                or_philox4x32_10(ctr, key, &w[4 * b]);
            }
            h_out[s] = h;
            j_out[s] = j;
            if (!fp32) {
                jac_out[s] = or_point64(D, NG, R, k, w, map, xs, idx);
                fx_out[s] = or_integrand_eval(f, xs);
                for (int32_t mu = 0; mu < D; ++mu) x_out[s * D + mu] = xs[mu];
            } else {
                jac_out[s] = (double)or_point32(D, NG, R32, k, w, map32, xs32, idx);
                fx_out[s] = (double)or_integrand_eval_f32(f, xs32);
                for (int32_t mu = 0; mu < D; ++mu) x_out[s * D + mu] = (double)xs32[mu];
            }
            for (int32_t mu = 0; mu < D; ++mu) idx_out[s * D + mu] = idx[mu];
        }
    }
    free(map32);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Iteration estimate, Sec. 2.1 Eqs. (MCIy), (sigest) applied per hypercube  */
/* and summed over hypercubes as in Sec. 3, Eq. (sumI):                       */
/*   I = sum_h Omega S1_h / n_h,                                              */
/*   V = sum_h max(0, Omega^2 S2_h / n_h - (Omega S1_h / n_h)^2) / (n_h - 1). */
/* Sums are compensated (see or_ksum).                                        */
/* ------------------------------------------------------------------------ */
void or_reduce(const or_params* p, const int32_t* n_h, const double* S1, const double* S2,
               double* I_out, double* V_out)
{
    const int64_t nhc = or_n_hypercubes(p);
    const double omega = 1.0 / (double)nhc;
    const double omega2 = omega * omega;
    or_ksum I = {0.0, 0.0}, V = {0.0, 0.0};
    for (int64_t h = 0; h < nhc; ++h) {
        const double n = (double)n_h[h];
        const double m = (omega * S1[h]) / n;
        double var = (omega2 * S2[h]) / n - m * m;
        if (var < 0.0) var = 0.0;
        or_kadd(&I, m);
        or_kadd(&V, var / (n - 1.0));
    }
    *I_out = or_kval(&I);
    *V_out = or_kval(&V);
}

/* ------------------------------------------------------------------------ */
/* Reallocation, Sec. 3 steps 2-4, Eqs. (dh), (nh):                           */
/*   sigma_h = sqrt(max(0, Omega^2 S2_h/n_h - (Omega S1_h/n_h)^2)),           */
/*   d_h = sigma_h^beta (d_h = 1 when beta = 0),                              */
/*   n_h' = max(2, floor(N_ev d_h / sum d)), or floor(...) + 2 in the         */
/* alternative rule.  sum d is compensated; when it is zero the allocation is  */
/* kept.  Counts near-ties |q - round q| <= 1e-9 max(1, q) at                 */
/* integers where floor(q) decides n_h (>= 3 for the max(2, .) rule, >= 1 for */
/* the +2 rule): there a last-bit difference in sum d could move n_h.         */
/* ------------------------------------------------------------------------ */
int64_t or_realloc(const or_params* p, const double* S1, const double* S2, const int32_t* n_in,
                   int32_t* n_out)
{
    const int64_t nhc = or_n_hypercubes(p);
    const double omega = 1.0 / (double)nhc;
    const double omega2 = omega * omega;
    double* dh = (double*)malloc(sizeof(double) * (size_t)nhc);
    if (!dh) return -1;
    or_ksum ksum = {0.0, 0.0};
    for (int64_t h = 0; h < nhc; ++h) {
        const double n = (double)n_in[h];
        const double m = (omega * S1[h]) / n;
        double var = (omega2 * S2[h]) / n - m * m;
        if (var < 0.0) var = 0.0;
        const double sig = sqrt(var);
        dh[h] = (p->beta == 0.0) ? 1.0 : pow(sig, p->beta);
        or_kadd(&ksum, dh[h]);
    }
    const double sum = or_kval(&ksum);
    int64_t ties = 0;
    if (!(sum > 0.0)) {
        for (int64_t h = 0; h < nhc; ++h) n_out[h] = n_in[h];
        free(dh);
        return 0;
    }
    const double nev = (double)p->n_ev;
    for (int64_t h = 0; h < nhc; ++h) {
        const double q = nev * (dh[h] / sum);
        double fl = floor(q);
        double r = nearbyint(q);
        double tol = 1e-9 * (q > 1.0 ? q : 1.0);
        /* a tie only matters where floor(q) is not hidden by the max(2, .) */
        double first_visible = p->realloc_plus2 ? 1.0 : 3.0;
        if (r >= first_visible && fabs(q - r) <= tol) ++ties;
        int64_t n = (int64_t)fl;
        if (p->realloc_plus2) n = n + 2;
        else if (n < 2) n = 2;
        if (n > 2147483647) n = 2147483647;
        n_out[h] = (int32_t)n;
    }
    free(dh);
    return ties;
}

/* ------------------------------------------------------------------------ */
/* Map refinement of one axis, Sec. 2.3.                                      */
/*  1. d_i from the training data (weighted: H/W; literal: H/count), 0 for an */
/*     increment with no samples.                                             */
/*  2. Smoothing with weights (7,1)/8, (1,6,1)/8, (1,7)/8 and normalisation   */
/*     by the raw sum of the d_i.                                             */
/*  3. Range compression d -> ((1 - d) / ln(1/d))^alpha, 0 for d = 0.         */
/*  4. Regrid: the new grid gives every new increment an equal share          */
/*     delta_d = (sum c) / N_g of the compressed values c_j, each c_j spread  */
/*     uniformly over its old increment.  So new point i is the inverse, at   */
/*     i delta_d, of the cumulative C(x) that is linear on every old          */
/*     increment with C(x_j) = c_0 + ... + c_{j-1}: in the old increment j    */
/*     with C(x_j) < i delta_d <= C(x_{j+1}),                                 */
/*       x'_i = x_j + (i delta_d - C(x_j)) / c_j (x_{j+1} - x_j).              */
/*     (The paper reaches the same points by a running walk over the c_j.)    */
/* An axis is left untouched when alpha = 0, N_g = 1, or every d_i is zero.  */
/* x: the axis's N_g + 1 grid points, replaced in place.                      */
/* work: 4 (N_g + 1) doubles.                                                 */
/* ------------------------------------------------------------------------ */
int or_refine_axis(const or_params* p, const double* H, const double* W, double* x, double* work)
{
    const int32_t NG = p->n_g;
    if (p->alpha == 0.0 || NG < 2) return 0;
    double* d = work;
    double* c = work + (NG + 1);
    double* cum = work + 2 * (NG + 1);
    double* xn = work + 3 * (NG + 1);
    or_ksum ks = {0.0, 0.0};
    for (int32_t i = 0; i < NG; ++i) {
        d[i] = (W[i] > 0.0) ? H[i] / W[i] : 0.0;
        or_kadd(&ks, d[i]);
    }
    const double s = or_kval(&ks);
    if (!(s > 0.0)) return 0;
    /* smoothing, then normalisation */
    c[0] = (7.0 * d[0] + d[1]) / 8.0;
    for (int32_t i = 1; i < NG - 1; ++i) c[i] = (d[i - 1] + 6.0 * d[i] + d[i + 1]) / 8.0;
    c[NG - 1] = (d[NG - 2] + 7.0 * d[NG - 1]) / 8.0;
    for (int32_t i = 0; i < NG; ++i) c[i] = c[i] / s;
    /* compression */
    for (int32_t i = 0; i < NG; ++i) {
        double di = c[i];
        c[i] = (di == 0.0) ? 0.0 : pow((1.0 - di) / (-log(di)), p->alpha);
    }
    /* cumulative at the old grid points, cum[j] = C(x_j) (compensated sums) */
    or_ksum kc = {0.0, 0.0};
    cum[0] = 0.0;
    for (int32_t j = 0; j < NG; ++j) {
        or_kadd(&kc, c[j]);
        cum[j + 1] = or_kval(&kc);
    }
    /* with nothing to share out (the compressed sum underflowed or is not
     * finite) the share is not positive and the axis is kept */
    const double delta_d = cum[NG] / (double)NG;
    if (!(delta_d > 0.0)) return 0;
    xn[0] = x[0];
    int32_t j = 0;
    for (int32_t i = 1; i < NG; ++i) {
        const double target = (double)i * delta_d;
        /* the old increment holding the target: cum[j] < target <= cum[j + 1] */
        while (j < NG - 1 && cum[j + 1] < target) ++j;
        double frac = (c[j] > 0.0) ? (target - cum[j]) / c[j] : 1.0;
        if (frac < 0.0) frac = 0.0;
        if (frac > 1.0) frac = 1.0;
        xn[i] = x[j] + frac * (x[j + 1] - x[j]);
    }
    for (int32_t i = 1; i < NG; ++i) x[i] = xn[i];
    return 1;
}

/* The first three refinement stages of one axis, for inspection: raw d_i,
 * smoothed-and-normalised d_i, compressed d_i (Sec. 2.3).  Returns 0 when the
 * axis would be left untouched (then the outputs are not all written). */
int or_refine_stages(const or_params* p, const double* H, const double* W, double* d_raw,
                     double* d_smooth, double* d_comp)
{
    const int32_t NG = p->n_g;
    if (NG < 2) return 0;
    or_ksum ks = {0.0, 0.0};
    for (int32_t i = 0; i < NG; ++i) {
        d_raw[i] = (W[i] > 0.0) ? H[i] / W[i] : 0.0;
        or_kadd(&ks, d_raw[i]);
    }
    const double s = or_kval(&ks);
    if (!(s > 0.0)) return 0;
    const double* d = d_raw;
    double* c = d_smooth;
    c[0] = (7.0 * d[0] + d[1]) / 8.0;
    for (int32_t i = 1; i < NG - 1; ++i) c[i] = (d[i - 1] + 6.0 * d[i] + d[i + 1]) / 8.0;
    c[NG - 1] = (d[NG - 2] + 7.0 * d[NG - 1]) / 8.0;
    for (int32_t i = 0; i < NG; ++i) c[i] = c[i] / s;
    for (int32_t i = 0; i < NG; ++i)
        d_comp[i] = (c[i] == 0.0) ? 0.0 : pow((1.0 - c[i]) / (-log(c[i])), p->alpha);
    return 1;
}

int or_refine(const or_params* p, const double* H, const double* W, double* map)
{
    const int32_t D = p->dim, NG = p->n_g;
    double* work = (double*)malloc(sizeof(double) * 4 * ((size_t)NG + 1));
    if (!work) return -1;
    for (int32_t mu = 0; mu < D; ++mu)
        or_refine_axis(p, H + (int64_t)mu * NG, W + (int64_t)mu * NG, map + (int64_t)mu * (NG + 1),
                       work);
    free(work);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Vector-valued integrands, Sec. 6: several integrals from the same samples. */
/* Component a of the integrand is g(x) m_a(x), g the (unscaled) integrand f  */
/* and m_a = (e1[a] < 0 ? 1 : x_e1[a]) (e2[a] < 0 ? 1 : x_e2[a]); the value   */
/* of a sample is v_a = J (scale (g m_a)).  Per hypercube the sums            */
/* S1_a = sum v_a and S2_ab = sum v_a v_b give                                */
/*   I_a  = sum_h Omega S1_a / n_h,                                           */
/*   C_ab = sum_h (Omega^2 S2_ab / n_h - (Omega S1_a / n_h)(Omega S1_b / n_h)) */
/*          / (n_h - 1),  diagonal terms at least 0                            */
/* (the covariance form of Eq. sigest).  FP64 only.  I_out [M], C_out [M][M]; */
/* scale_out [M] (or NULL): sum_h Omega^2 S2_aa / n_h / (n_h - 1), the size   */
/* of the terms before their cancellation.                                    */
/* ------------------------------------------------------------------------ */
int or_vec_iteration(const or_params* p, const or_integrand* f, const double* map, const int32_t* n_h,
                     int32_t it, int32_t M, const int32_t* e1, const int32_t* e2, double* I_out, double* C_out,
                     double* scale_out)
{
    const int32_t D = p->dim, NG = p->n_g;
    if (D < 1 || D > 64 || M < 1 || M > 16) return -1;
    int32_t NST[64];
    double R[64];
    for (int32_t mu = 0; mu < D; ++mu) {
        NST[mu] = or_nst_axis(p, mu);
        R[mu] = (double)NG / (double)NST[mu];
    }
    or_integrand g = *f;
    g.scale = 1.0;
    const uint32_t key[2] = {(uint32_t)(p->seed & 0xffffffffu), (uint32_t)(p->seed >> 32)};
    const int nblk = (2 * D + 3) / 4;
    const int64_t nhc = or_n_hypercubes(p);
    const double om = 1.0 / (double)nhc;
    or_ksum kI[16], kC[16 * 16], kS[16];
    memset(kI, 0, sizeof kI);
    memset(kS, 0, sizeof kS);
    memset(kC, 0, sizeof kC);
    uint32_t w[4 * 33];
    int32_t k[64], idx[64];
    double xs[64], v[16];
    for (int64_t h = 0; h < nhc; ++h) {
        int64_t rem = h;
        for (int32_t mu = D - 1; mu >= 0; --mu) {
            k[mu] = (int32_t)(rem % NST[mu]);
            rem /= NST[mu];
        }
        const int32_t n = n_h[h];
        or_ksum s1[16], s2[16 * 16];
        memset(s1, 0, sizeof s1);
        memset(s2, 0, sizeof s2);
        for (int32_t j = 0; j < n; ++j) {
            for (int b = 0; b < nblk; ++b) {
                uint32_t ctr[4] = {(uint32_t)j, (uint32_t)h, (uint32_t)it, (uint32_t)b};
                or_philox4x32_10(ctr, key, &w[4 * b]);
            }
            const double jac = or_point64(D, NG, R, k, w, map, xs, idx);
            const double gx = or_integrand_eval(&g, xs);
            for (int32_t a = 0; a < M; ++a) {
                double m = 1.0;
                if (e1[a] >= 0) m = xs[e1[a]];
                if (e2[a] >= 0) m = m * xs[e2[a]];
                v[a] = jac * (f->scale * (gx * m));
            }
            for (int32_t a = 0; a < M; ++a) {
                or_kadd(&s1[a], v[a]);
                for (int32_t b = 0; b < M; ++b) or_kadd(&s2[a * M + b], v[a] * v[b]);
            }
        }
        const double nd = (double)n;
        for (int32_t a = 0; a < M; ++a) {
            const double ma = om * or_kval(&s1[a]) / nd;
            or_kadd(&kI[a], ma);
            or_kadd(&kS[a], om * om * or_kval(&s2[a * M + a]) / nd / (nd - 1.0));
            for (int32_t b = 0; b < M; ++b) {
                const double mb = om * or_kval(&s1[b]) / nd;
                double c = (om * om * or_kval(&s2[a * M + b]) / nd - ma * mb) / (nd - 1.0);
                if (a == b && !(c > 0.0)) c = 0.0;
                or_kadd(&kC[a * M + b], c);
            }
        }
    }
    for (int32_t a = 0; a < M; ++a) {
        I_out[a] = or_kval(&kI[a]);
        if (scale_out) scale_out[a] = or_kval(&kS[a]);
        for (int32_t b = 0; b < M; ++b) C_out[a * M + b] = or_kval(&kC[a * M + b]);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Preconditioned map, Sec. 5.2: training on given samples {x, f(x)} before   */
/* integrating.  Each point's y = y(x) is found by inverting the map axis by  */
/* axis: x lies in increment i of axis mu when x_i <= x^mu (the last such i,  */
/* at most N_g - 1).  Its Jacobian J(y(x)) is the product over the axes of    */
/* N_g Delta x_i (Eq. jac).  The training data are                            */
/*   d_i^mu = (1 / n_i^mu) sum over the points in increment i of (J f)^2,     */
/* i.e. H_i = sum (J f)^2 and W_i = n_i, and the map is refined from them as  */
/* after an iteration (Sec. 2.3), with the training damping alpha.  The same  */
/* points are used again in every training pass.                              */
/* x: [n][dim] inside the map's box; fx: [n].                                 */
/* ------------------------------------------------------------------------ */
int32_t or_map_locate(const double* xm, int32_t NG, double x)
{
    for (int32_t i = NG - 1; i > 0; --i)
        if (xm[i] <= x) return i;
    return 0;
}

int or_train_hist(const or_params* p, const double* x, const double* fx, int64_t n, const double* map,
                  double* H, double* W)
{
    const int32_t D = p->dim, NG = p->n_g;
    or_ksum* kH = (or_ksum*)calloc((size_t)D * NG, sizeof(or_ksum));
    if (!kH) return -1;
    for (int64_t q = 0; q < (int64_t)D * NG; ++q) W[q] = 0.0;
    for (int64_t s = 0; s < n; ++s) {
        const double* xs = x + s * D;
        double jac = 1.0;
        for (int32_t mu = 0; mu < D; ++mu) {
            const double* xm = map + (int64_t)mu * (NG + 1);
            const int32_t i = or_map_locate(xm, NG, xs[mu]);
            jac = jac * ((double)NG * (xm[i + 1] - xm[i]));
        }
        const double v = jac * fx[s];
        const double v2 = v * v;
        for (int32_t mu = 0; mu < D; ++mu) {
            const double* xm = map + (int64_t)mu * (NG + 1);
            const int32_t i = or_map_locate(xm, NG, xs[mu]);
            or_kadd(&kH[(int64_t)mu * NG + i], v2);
            W[(int64_t)mu * NG + i] += 1.0;
        }
    }
    for (int64_t q = 0; q < (int64_t)D * NG; ++q) H[q] = or_kval(&kH[q]);
    free(kH);
    return 0;
}

int or_map_train(const or_params* p, const double* x, const double* fx, int64_t n, double* map,
                 int32_t n_iter, double alpha)
{
    const int32_t D = p->dim, NG = p->n_g;
    or_params q = *p;
    q.alpha = alpha;
    double* H = (double*)malloc(sizeof(double) * (size_t)D * NG);
    double* W = (double*)malloc(sizeof(double) * (size_t)D * NG);
    if (!H || !W) {
        free(H); free(W);
        return -1;
    }
    int rc = 0;
    for (int32_t it = 0; it < n_iter && rc == 0; ++it) {
        rc = or_train_hist(&q, x, fx, n, map, H, W);
        if (rc == 0) rc = or_refine(&q, H, W, map);
    }
    free(H); free(W);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Combining iterations, Sec. 2.5: inverse-variance weighted mean, its        */
/* standard error and chi^2 over iterations n_discard..n-1.  When any sigma_j */
/* is zero the weights are undefined: the plain mean is returned with zero    */
/* error and chi^2 = NaN.                                                     */
/* With unweighted != 0 (for iterations that no longer adapt, Sec. 2.5): the  */
/* plain mean of the I_j, and the plain mean of the sigma_j divided by the    */
/* square root of their count as its error; chi^2 about that mean.            */
/* ------------------------------------------------------------------------ */
void or_combine(const double* I, const double* sig, int32_t n, int32_t n_discard, int32_t unweighted,
                double* mean, double* sdev, double* chi2, int32_t* dof)
{
    int32_t first = n_discard < 0 ? 0 : n_discard;
    int32_t cnt = n - first;
    if (cnt <= 0) {
        *mean = NAN; *sdev = NAN; *chi2 = NAN; *dof = 0;
        return;
    }
    int zero = 0;
    for (int32_t j = first; j < n; ++j)
        if (!(sig[j] > 0.0)) zero = 1;
    *dof = cnt - 1;
    if (unweighted) {
        double s = 0.0, ss = 0.0;
        for (int32_t j = first; j < n; ++j) {
            s = s + I[j];
            ss = ss + sig[j];
        }
        double m = s / (double)cnt;
        double c2 = 0.0;
        for (int32_t j = first; j < n; ++j) {
            double r = I[j] - m;
            c2 = c2 + r * r / (sig[j] * sig[j]);
        }
        *mean = m;
        *sdev = (ss / (double)cnt) / sqrt((double)cnt);
        *chi2 = zero ? NAN : c2;
        return;
    }
    if (zero) {
        double s = 0.0;
        for (int32_t j = first; j < n; ++j) s = s + I[j];
        *mean = s / (double)cnt;
        *sdev = 0.0;
        *chi2 = NAN;
        return;
    }
    double sw = 0.0, swi = 0.0;
    for (int32_t j = first; j < n; ++j) {
        double w = 1.0 / (sig[j] * sig[j]);
        sw = sw + w;
        swi = swi + I[j] * w;
    }
    double m = swi / sw;
    double c2 = 0.0;
    for (int32_t j = first; j < n; ++j) {
        double r = I[j] - m;
        c2 = c2 + r * r / (sig[j] * sig[j]);
    }
    *mean = m;
    *sdev = 1.0 / sqrt(sw);
    *chi2 = c2;
}

/* ------------------------------------------------------------------------ */
/* One full iteration: sample every hypercube, estimate, reallocate, refine.  */
/* The two adaptations both use this iteration's samples and take effect in  */
/* the next iteration (Sec. 3, after step 4).  map and n_h are updated in    */
/* place.  S1, S2 (N_hc) and H, W (dim x N_g) receive this iteration's sums. */
/* ------------------------------------------------------------------------ */
int64_t or_iteration(const or_params* p, const or_integrand* f, double* map, int32_t* n_h,
                     int32_t it, double* S1, double* S2, double* H, double* W, double* I_out,
                     double* V_out)
{
    const int64_t nhc = or_n_hypercubes(p);
    memset(H, 0, sizeof(double) * (size_t)p->dim * p->n_g);
    memset(W, 0, sizeof(double) * (size_t)p->dim * p->n_g);
    if (or_sample_range(p, f, map, n_h, it, 0, nhc, S1, S2, H, W, NULL, 0, NULL) != 0) return -1;
    or_reduce(p, n_h, S1, S2, I_out, V_out);
    /* Sec. 2.5: once adaptation has ended (alpha = 0), the map and the
     * allocation are those of the last adapting iteration. */
    if (p->n_adapt > 0 && it >= p->n_adapt) return 0;
    int32_t* n_new = (int32_t*)malloc(sizeof(int32_t) * (size_t)nhc);
    if (!n_new) return -1;
    int64_t ties = or_realloc(p, S1, S2, n_h, n_new);
    memcpy(n_h, n_new, sizeof(int32_t) * (size_t)nhc);
    free(n_new);
    or_refine(p, H, W, map);
    return ties;
}

/* Full driver over n_iter iterations starting from the given map and
 * allocation (callers use or_map_init / or_alloc_init for a fresh start).
 * I_j and V_j (variances) of each iteration are returned; ties_total counts
 * near-ties over all reallocations, evals_total the samples drawn (the sum
 * of n_h over the iterations). */
int or_integrate(const or_params* p, const or_integrand* f, double* map, int32_t* n_h,
                 int32_t it0, int32_t n_iter, double* I_j, double* V_j, int64_t* ties_total,
                 int64_t* evals_total)
{
    const int64_t nhc = or_n_hypercubes(p);
    double* S1 = (double*)malloc(sizeof(double) * (size_t)nhc);
    double* S2 = (double*)malloc(sizeof(double) * (size_t)nhc);
    double* H = (double*)malloc(sizeof(double) * (size_t)p->dim * p->n_g);
    double* W = (double*)malloc(sizeof(double) * (size_t)p->dim * p->n_g);
    if (!S1 || !S2 || !H || !W) {
        free(S1); free(S2); free(H); free(W);
        return -1;
    }
    int64_t ties = 0, evals = 0;
    for (int32_t j = 0; j < n_iter; ++j) {
        for (int64_t h = 0; h < nhc; ++h) evals += n_h[h];
        int64_t t = or_iteration(p, f, map, n_h, it0 + j, S1, S2, H, W, &I_j[j], &V_j[j]);
        if (t < 0) { ties = -1; break; }
        ties += t;
    }
    free(S1); free(S2); free(H); free(W);
    if (ties_total) *ties_total = ties;
    if (evals_total) *evals_total = evals;
    return ties < 0 ? -1 : 0;
}

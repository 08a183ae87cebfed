// vp_sample.hpp -- the fused per-sample kernel of one vegas+ iteration.
//
// One launch draws every sample of the iteration, maps it through the vegas
// map, evaluates J f, and accumulates (a) the per-hypercube sums of J f and
// (J f)^2 (Sec. 3, step 2) and (b) the per-axis, per-increment training data
// of the map (Sec. 2.3 and 2.4).  Nothing per sample touches HBM.
//
// Work decomposition.  The samples of an iteration are numbered in hypercube
// order, s = offset(h) + j (the exclusive scan of n_h).  The launch is
// persistent: every wave owns one contiguous, equal share of the sample range
// and walks it in tiles of 64 * chunk samples, each lane taking `chunk`
// consecutive samples.  A lane finds the hypercube of its first sample with a
// wave-cooperative search over 64 offsets at a time, then walks forward.
// Runs of samples of one hypercube are summed in registers; runs that cross
// lane boundaries are joined by a segmented scan across the wave (a fixed
// shuffle tree, so the result does not depend on timing), and runs that cross
// wave boundaries are handed to a fix-up kernel as edge records.  Every
// hypercube's S1, S2 is therefore written exactly once, deterministically.
//
// Training data are privatised per workgroup in LDS (one workgroup per CU
// holds all D * N_g bins, numerators and weights in separate planes so the
// 8-byte atomics of a wave spread over every LDS bank) and written out once
// per workgroup; a second kernel reduces the per-workgroup partials in a
// fixed order.
#pragma once

#include "vp_internal.hpp"

namespace vp {

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies of counter words 0 and 2, with the high halves xored
// into words 1 and 3 and the round key, the key advanced by two Weyl
// constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t* out)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        // three-way xors as single CDNA4 bitop3 instructions (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// 1/n for a sample count n >= 1: the hardware reciprocal refined by one
// Newton step (within an ulp of the correctly rounded quotient; the weights
// 1/n_h of the training data are compared at 1e-12).
__device__ __forceinline__ double recip_count(uint32_t n)
{
    const double d = (double)n;
    const double r = __builtin_amdgcn_rcp(d);
    const double e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

// ---------------------------------------------------------------- wave helpers
__device__ __forceinline__ int64_t shfl64(int64_t v, int src)
{
    int lo = __shfl((int)(uint32_t)(uint64_t)v, src);
    int hi = __shfl((int)(uint32_t)((uint64_t)v >> 32), src);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

// Largest h with offs[h] <= s over the whole array (wave-uniform s):
// a 64-ary search, one coalesced load per level.
__device__ __forceinline__ int64_t find_hypercube(const int64_t* __restrict__ offs,
                                                  const int64_t* __restrict__ ob, int64_t n_hc,
                                                  int64_t s, int lane)
{
    int64_t lo = 0, hi = n_hc;  // offs[lo] <= s < offs[hi]
    while (hi - lo > 64) {
        const int64_t step = (hi - lo) / 64;
        const int64_t p = lo + (int64_t)(lane + 1) * step;
        const bool le = (p < hi) && (gofs(offs, ob, p) <= s);
        const int c = __popcll(__ballot(le));
        const int64_t nlo = lo + (int64_t)c * step;
        const int64_t nhi = (c < 64) ? lo + (int64_t)(c + 1) * step : hi;
        lo = nlo;
        hi = nhi < hi ? nhi : hi;
    }
    const int64_t p = lo + 1 + lane;
    const bool le = (p < hi) && (gofs(offs, ob, p) <= s);
    return lo + __popcll(__ballot(le));
}

// Per-lane hypercube of s (s >= offs[base] for every active lane): windows of
// 64 consecutive offsets, binary-searched with lane shuffles.
__device__ __forceinline__ int64_t locate(const int64_t* __restrict__ offs,
                                          const int64_t* __restrict__ ob, int64_t n_hc,
                                          int64_t base, int64_t s, bool active, int lane)
{
    int64_t res = base;
    bool done = !active;
    for (;;) {
        const int64_t p = base + 1 + lane;
        const int64_t bnd = (p <= n_hc) ? gofs(offs, ob, p) : INT64_MAX;
        int pos = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
            const int64_t b = shfl64(bnd, pos + step - 1);
            if (b <= s) pos += step;
        }
        const int64_t last = shfl64(bnd, 63);
        if (!done && last > s) {
            res = base + pos;
            done = true;
        }
        if (__all(done)) break;
        base += 64;
    }
    return res;
}

// An edge record into device memory (member by member: a global-address
// object has no implicit assignment).
__device__ __forceinline__ void put_edge(VP_GLOBAL EdgeRec* p, const EdgeRec& r)
{
    p->h = r.h;
    p->s1 = r.s1;
    p->s2 = r.s2;
}

// ---------------------------------------------------------------- run sums
// Sums of J f and (J f)^2 over a run of samples of one hypercube.
struct AccD {
    double a, b;
    __device__ void zero() { a = 0.0; b = 0.0; }
    __device__ void add(double v)
    {
        a = a + v;
        b = b + v * v;
    }
    // this := prev (+) this, prev's samples first
    __device__ void join_after(const AccD& prev)
    {
        a = prev.a + a;
        b = prev.b + b;
    }
    __device__ double sa() const { return a; }
    __device__ double sb() const { return b; }
    __device__ AccD shfl_up(int d) const
    {
        AccD r;
        r.a = __shfl_up(a, d);
        r.b = __shfl_up(b, d);
        return r;
    }
    __device__ AccD bcast(int src) const
    {
        AccD r;
        r.a = __shfl(a, src);
        r.b = __shfl(b, src);
        return r;
    }
};

// Neumaier's compensated summation in single precision.
__device__ __forceinline__ void neumaier_add(float& s, float& c, float v)
{
    const float t = s + v;
    if (fabsf(s) >= fabsf(v)) c += (s - t) + v;
    else c += (v - t) + s;
    s = t;
}

struct AccN {
    float as, ac, bs, bc;
    __device__ void zero() { as = ac = bs = bc = 0.0f; }
    __device__ void addf(float v)
    {
        neumaier_add(as, ac, v);
        neumaier_add(bs, bc, v * v);
    }
    __device__ void join_after(const AccN& prev)
    {
        float s = prev.as, c = prev.ac;
        neumaier_add(s, c, as);
        ac = c + ac;
        as = s;
        s = prev.bs;
        c = prev.bc;
        neumaier_add(s, c, bs);
        bc = c + bc;
        bs = s;
    }
    __device__ double sa() const { return (double)as + (double)ac; }
    __device__ double sb() const { return (double)bs + (double)bc; }
    __device__ AccN shfl_up(int d) const
    {
        AccN r;
        r.as = __shfl_up(as, d);
        r.ac = __shfl_up(ac, d);
        r.bs = __shfl_up(bs, d);
        r.bc = __shfl_up(bc, d);
        return r;
    }
    __device__ AccN bcast(int src) const
    {
        AccN r;
        r.as = __shfl(as, src);
        r.ac = __shfl(ac, src);
        r.bs = __shfl(bs, src);
        r.bc = __shfl(bc, src);
        return r;
    }
};

template <int PREC>
struct AccOf {
    typedef AccD type;
};
template <>
struct AccOf<P_FP32_NEUMAIER> {
    typedef AccN type;
};

// Compensated single-precision training data in LDS.  Each numerator bin is
// one 8-byte word holding the pair (sum, compensation); an update reads the
// pair, takes Neumaier's step with the new value, and stores the result with
// a 64-bit compare-and-swap, retried while another lane or wave changed the
// word in between.  (Single-precision LDS atomic adds cost about ten times a
// 64-bit integer add on this hardware.)  Each of the D updates of a sample
// reads its word and swaps at once; then the lanes whose swap lost retry.
// The weights go to the fixed-point plane by integer adds.
__device__ __forceinline__ uint64_t pack_pair(float s, float c)
{
    return ((uint64_t)__float_as_uint(c) << 32) | (uint64_t)__float_as_uint(s);
}

template <int D>
__device__ __forceinline__ void lds_neumaier_sample(uint64_t* pairs, int lbins, int n_g, const int32_t* idx,
                                                    float hh, uint64_t wq)
{
    uint64_t* addr[D];
    uint64_t cur[D];
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        const int bin = mu * n_g + idx[mu];
        addr[mu] = pairs + bin;
        atomicAdd(reinterpret_cast<unsigned long long*>(pairs + lbins + bin), (unsigned long long)wq);
    }
    // first attempt: each swap right after its read, so that the window in
    // which another lane or wave can change the word is one read's latency
    static_assert(D <= 32, "one pending bit per update");
    uint32_t pending = 0;
#pragma unroll
    for (int m = 0; m < D; ++m) {
        cur[m] = __hip_atomic_load(addr[m], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        float s = __uint_as_float((uint32_t)cur[m]);
        float c = __uint_as_float((uint32_t)(cur[m] >> 32));
        neumaier_add(s, c, hh);
        const uint64_t old = atomicCAS(reinterpret_cast<unsigned long long*>(addr[m]),
                                       (unsigned long long)cur[m], (unsigned long long)pack_pair(s, c));
        if (old != cur[m]) pending |= 1u << m;
        cur[m] = old;
    }
    // retries of the lanes whose swap lost, from the value the swap returned
    while (pending) {
#pragma unroll
        for (int m = 0; m < D; ++m) {
            if (pending & (1u << m)) {
                float s = __uint_as_float((uint32_t)cur[m]);
                float c = __uint_as_float((uint32_t)(cur[m] >> 32));
                neumaier_add(s, c, hh);
                const uint64_t old = atomicCAS(reinterpret_cast<unsigned long long*>(addr[m]),
                                               (unsigned long long)cur[m], (unsigned long long)pack_pair(s, c));
                if (old == cur[m]) pending &= ~(1u << m);
                cur[m] = old;
            }
        }
    }
}

// A weight as a multiple of 1/scale, rounded to nearest (0 <= w * scale < 2^63).
__device__ __forceinline__ uint64_t fixed_weight(double w, double scale)
{
    return (uint64_t)__builtin_rint(w * scale);
}

// ---------------------------------------------------------------- integrands
// Per-axis accumulation followed by a finish step, in the same operation
// order as the problem statement defines each integrand.
template <int D, typename T>
struct FState {
    T q[kMaxTerms];
    T lin;
    T t[D];
};

// Integrand constants in the sampler's layout, built on the host in the
// problem's device memory (SampleArgs::fc).  Layout, in units of T (double on
// the FP64 path, float on the split paths):
//   [0] scale, [1] affine constant, [4..7] coefs, [8..11] amps, [12..15] radii^2,
//   [16 + 4 mu + k] centre k of axis mu (the four terms of an axis adjacent),
//   [16 + 4 D + d D + e] Cholesky factor (correlated Gaussian only).

__device__ __forceinline__ double vexp(double x) { return exp(x); }
__device__ __forceinline__ float vexp(float x) { return expf(x); }
__device__ __forceinline__ double vsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float vsqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double vfma(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float vfma(float a, float b, float c) { return fmaf(a, b, c); }

// KT: number of terms fixed at compile time (0: the run-time K).
// FP: pointer to the constants -- LDS, or the constant address space (read
// through the scalar cache into scalar registers).
template <int D, int KT, typename T, typename FP>
__device__ __forceinline__ void f_axis(FP fc, int kind, int K, int mu, T x, FState<D, T>& st)
{
    constexpr int KN = KT ? KT : kMaxTerms;
    const auto c = fc + kFcHead + 4 * mu;
    if (kind == K_GAUSS_MIX || kind == K_EXP_ABS || kind == K_BALLS) {
        T cv[KN];
#pragma unroll
        for (int k = 0; k < KN; ++k) cv[k] = c[k];
#pragma unroll
        for (int k = 0; k < KN; ++k) {
            if (KT || k < K) {
                const T tt = x - cv[k];
                st.q[k] = vfma(tt, tt, st.q[k]);
            }
        }
    } else if (kind == K_CORR_GAUSS) {
        st.t[mu] = x - c[0];
    } else if (kind == K_AFFINE) {
        st.lin = vfma(c[0], x, st.lin);
    }
}

template <int D, int KT, typename T, typename FP>
__device__ __forceinline__ T f_finish(FP fc, int kind, int K, FState<D, T>& st)
{
    constexpr int KN = KT ? KT : kMaxTerms;
    const T scale = fc[0];
    const auto coefs = fc + 4;
    const auto amps = fc + 8;
    const auto rad2 = fc + 12;
    T acc = (T)0;
    switch (kind) {
    case K_GAUSS_MIX:
#pragma unroll
        for (int k = 0; k < KN; ++k)
            if (KT || k < K) acc = vfma(amps[k], vexp(-(coefs[k] * st.q[k])), acc);
        return scale * acc;
    case K_EXP_ABS:
#pragma unroll
        for (int k = 0; k < KN; ++k)
            if (KT || k < K) acc = vfma(amps[k], vexp(-(coefs[k] * vsqrt(st.q[k]))), acc);
        return scale * acc;
    case K_BALLS:
#pragma unroll
        for (int k = 0; k < KN; ++k)
            if ((KT || k < K) && st.q[k] < rad2[k]) acc = acc + amps[k];
        return scale * acc;
    case K_CORR_GAUSS: {
        const auto chol = fc + kFcHead + 4 * D;
        T q = (T)0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            T z = (T)0;
#pragma unroll
            for (int e = d; e < D; ++e) z = vfma(chol[d * D + e], st.t[e], z);
            q = vfma(z, z, q);
            // one row of the factor at a time: without this fence the
            // scheduler hoists the loads of every row (D^2 values) and spills
            __builtin_amdgcn_sched_barrier(0);
        }
        return scale * vexp((T)(-0.5) * q);
    }
    case K_CONST:
        return scale;
    case K_AFFINE:
        return scale * st.lin;
    default:
        return (T)__builtin_nan("");
    }
}

// ---------------------------------------------------------------- map access
// The map of one axis is x[mu][0..N_g]; a sample needs the pair (x_i, x_{i+1}).
// From LDS: two adjacent reads.  From global memory: one 16-byte (FP64) or
// 8-byte (FP32) buffer load with a 32-bit offset from a wave-uniform buffer
// resource (bounds-checked by the hardware: reads past the map return zero).
// MAPL (MapPlace) says where: all axes in global memory, all in LDS, or the
// kMapInnerAxes innermost axes in LDS (their pairs start at element
// `inner0` = (D - kMapInnerAxes) (N_g + 1) of the map) and the rest in global
// memory.  `staged` is a compile-time property of the axis.
constexpr int kBufferWord3 = 0x00020000;  // raw buffer, gfx9 family

template <int MAPL>
struct MapPair64 {
    const double* lds;
    uint32_t inner0;
    __amdgpu_buffer_rsrc_t rsrc;
    __device__ __forceinline__ void get(uint32_t pos, double& x0, double& x1, bool staged) const
    {
        if (MAPL == MAP_LDS || (MAPL == MAP_INNER && staged)) {
            const uint32_t p = MAPL == MAP_INNER ? pos - inner0 : pos;
            x0 = lds[p];
            x1 = lds[p + 1];
        } else {
            const auto v = __builtin_amdgcn_raw_buffer_load_b128(rsrc, pos * 8u, 0, 0);
            x0 = __builtin_bit_cast(double, ((uint64_t)(uint32_t)v[1] << 32) | (uint32_t)v[0]);
            x1 = __builtin_bit_cast(double, ((uint64_t)(uint32_t)v[3] << 32) | (uint32_t)v[2]);
        }
    }
};

template <int MAPL>
struct MapPair32 {
    const float* lds;
    uint32_t inner0;
    __amdgpu_buffer_rsrc_t rsrc;
    __device__ __forceinline__ void get(uint32_t pos, float& x0, float& x1, bool staged) const
    {
        if (MAPL == MAP_LDS || (MAPL == MAP_INNER && staged)) {
            const uint32_t p = MAPL == MAP_INNER ? pos - inner0 : pos;
            x0 = lds[p];
            x1 = lds[p + 1];
        } else {
            const auto v = __builtin_amdgcn_raw_buffer_load_b64(rsrc, pos * 4u, 0, 0);
            x0 = __builtin_bit_cast(float, (uint32_t)v[0]);
            x1 = __builtin_bit_cast(float, (uint32_t)v[1]);
        }
    }
};

// The per-request scalars the sample loop needs, read once before the loop.
struct SampleHot {
    uint32_t key0, key1, it;
    int32_t n_g;
    double R;
    float R32;
    double R53;
    float R32s;
    const double* Rv;    // mixed stratification: R_mu per axis (LDS)
    const float* Rv32;
};

// ---------------------------------------------------------------- one sample
// Stratified y in hypercube k (Sec. 3): y^mu = (k_mu + u) / N_st, so
// t = y N_g = (k_mu + u) R (MIX: N_st^mu and R_mu per axis, Sec. 4); vegas map (Sec. 2.2, Eqs. y and jac):
// i = floor(t) (clamped to N_g - 1), delta = t - i (clamped to 1),
// x = x_i + Delta x_i delta, J = prod_mu N_g Delta x_i.
// FP64: u from 53 bits -- the high word of axis mu is word mu of the
// stream, its low word is word D + mu.
// Packed form of k + u: where every digit is known to be small, the digit
// joins the high random bits in one 32-bit word (one funnel shift), so the
// integer k 2^53 + U (split precisions: k 2^24 + U) is rounded once on its
// conversion or fma, just as k + u is rounded in the plain form; the power
// of two moves into R.  The same t bit for bit, with three operations fewer
// per axis.  The uniform stratification keeps N_st^D <= n_ev / 2 < 2^30, so
// the digits are below 32 for D >= 6 and below 182 for D >= 4: the packed
// form is taken there (k < 32 with 27 random bits beside it in double
// precision, k < 256 with 24 in the split ones).
template <int D, bool MIX>
constexpr bool kPack64 = !MIX && D >= 6;
template <int D, bool MIX>
constexpr bool kPack32 = !MIX && D >= 4;
__device__ __forceinline__ uint32_t join_digit(int32_t k, uint32_t w, int shift)
{
    return __builtin_amdgcn_alignbit((uint32_t)k, w, (uint32_t)shift);
}
// Where the generate mode of a batched integrand puts a sample: x at
// x[mu * n + pos], J at jac[pos]; its increment indices, 16-bit, in groups of
// eight axes at idx[(pos * ceil(D / 8) + g) * 8 ..] (one 16-byte store and
// load per group; the index buffer is the library's own).
typedef uint32_t U32x4 __attribute__((ext_vector_type(4)));
struct BatchOut {
    double* x;
    double* jac;
    uint16_t* idx;
    int64_t n, cap, pos;
};

// Where a dumped sample goes (vp_debug_dump): entry `pos` of the dump's
// arrays (x and idx [dim][count]); J and f(x) are written apart.
struct DumpPos {
    const DumpArgs* d;
    int64_t pos;
};

template <int D, int MAPL, int KT, typename FP, bool GEN = false, bool MIX = false, bool DUMP = false>
__device__ __forceinline__ double sample_fp64(const SampleHot& a, const MapPair64<MAPL>& map, FP fc,
                                              uint32_t j, uint32_t h, const int32_t* k,
                                              int32_t* idx, int kind, int K, const BatchOut* out = nullptr,
                                              const DumpPos* dp = nullptr)
{
    // Axes are processed in groups of four: group g takes its high words from
    // block g and its low words from the block(s) holding words D+4g..D+4g+3,
    // each block generated right before its first use so that only a few
    // words are live at a time.
    constexpr int NG4 = (D + 3) / 4;
    const int n_g = a.n_g;
    // A wave drawing and mapping its sample (up to its map reads and the
    // per-axis sums) runs at raised priority, dropped for the integrand's
    // exponentials: among the ready waves of a SIMD, those about to issue
    // their map reads go first, so more reads are in flight while other
    // waves compute (0.5-1% on the FP64 kernel, 1.5-3% on the split ones).
    if constexpr (!GEN && !DUMP) __builtin_amdgcn_s_setprio(1);
    FState<D, double> st;
#pragma unroll
    for (int kk = 0; kk < kMaxTerms; ++kk) st.q[kk] = 0.0;
    st.lin = fc[1];
    double jac = 1.0;
    uint32_t lo_blk[4];
    int lo_have = -1;  // index of the block held in lo_blk
#pragma unroll
    for (int g = 0; g < NG4; ++g) {
        uint32_t hi_blk[4];
        philox4x32_10(j, h, a.it, (uint32_t)g, a.key0, a.key1, hi_blk);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int mu = 4 * g + r;
            if (mu >= D) break;
            const int lw = D + mu;
            const int lb = lw / 4;
            if (lb != lo_have) {
                philox4x32_10(j, h, a.it, (uint32_t)lb, a.key0, a.key1, lo_blk);
                lo_have = lb;
            }
            double t;
            if constexpr (kPack64<D, MIX>) {
                const double hk = (double)join_digit(k[mu], hi_blk[r], 5);  // k 2^27 + (w >> 5), exact
                t = fma(hk, 0x1p26, (double)(lo_blk[lw % 4] >> 6)) * a.R53;
            } else {
                const double hi = (double)(hi_blk[r] >> 5);
                const double lo = (double)(lo_blk[lw % 4] >> 6);
                const double u = fma(hi, 0x1p-27, lo * 0x1p-53);  // exact: a 53-bit integer times 2^-53
                t = ((double)k[mu] + u) * (MIX ? a.Rv[mu] : a.R);
            }
            int i = (int)t;
            i = i < n_g - 1 ? i : n_g - 1;
            double delta = t - (double)i;
            delta = delta < 1.0 ? delta : 1.0;
            double x0, x1;
            map.get((uint32_t)(mu * (n_g + 1) + i), x0, x1, mu >= D - kMapInnerAxes);
            const double dx = x1 - x0;
            const double x = fma(dx, delta, x0);
            jac = jac * ((double)n_g * dx);
            idx[mu] = i;
            if constexpr (GEN) {
                // global (not flat) stores: a flat store would also hold up
                // every later wait for the map reads from LDS
                global_ptr(out->x)[mu * out->n + out->pos] = x;
            } else {
                f_axis<D, KT, double, FP>(fc, kind, K, mu, x, st);
            }
            if constexpr (DUMP) {
                dp->d->x[mu * dp->d->count + dp->pos] = x;
                dp->d->idx[mu * dp->d->count + dp->pos] = i;
            }
        }
    }
    if constexpr (GEN) {
        global_ptr(out->jac)[out->pos] = jac;
        return 0.0;
    } else {
        if constexpr (!DUMP) __builtin_amdgcn_s_setprio(0);
        const double fx = f_finish<D, KT, double, FP>(fc, kind, K, st);
        if constexpr (DUMP) {
            dp->d->jac[dp->pos] = jac;
            dp->d->fx[dp->pos] = fx;
        }
        return jac * fx;
    }
}

// FP32 split: u = (w >> 8) 2^-24 from the high word of each axis alone.
// Early: called with (axis, increment index) as soon as an axis is mapped
// (the split precision adds its fixed-point weights there).
struct NoEarly {
    __device__ void operator()(int, int) const {}
};
template <int D, int MAPL, int KT, typename FP, bool MIX = false, bool DUMP = false, typename Early = NoEarly>
__device__ __forceinline__ float sample_fp32(const SampleHot& a, const MapPair32<MAPL>& map, FP fc,
                                             uint32_t j, uint32_t h, const int32_t* k, int32_t* idx,
                                             int kind, int K, const DumpPos* dp = nullptr, Early early = Early())
{
    constexpr int NG4 = (D + 3) / 4;
    const int n_g = a.n_g;
    // raised priority up to the integrand, as in sample_fp64
    if constexpr (!DUMP) __builtin_amdgcn_s_setprio(1);
    FState<D, float> st;
#pragma unroll
    for (int kk = 0; kk < kMaxTerms; ++kk) st.q[kk] = 0.0f;
    st.lin = fc[1];
    float jac = 1.0f;
#pragma unroll
    for (int g = 0; g < NG4; ++g) {
        uint32_t w[4];
        philox4x32_10(j, h, a.it, (uint32_t)g, a.key0, a.key1, w);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int mu = 4 * g + r;
            if (mu >= D) break;
            float t;
            if constexpr (kPack32<D, MIX>) {
                t = (float)join_digit(k[mu], w[r], 8) * a.R32s;
            } else {
                const float u = (float)(w[r] >> 8) * 0x1p-24f;
                t = ((float)k[mu] + u) * (MIX ? a.Rv32[mu] : a.R32);
            }
            int i = (int)t;
            i = i < n_g - 1 ? i : n_g - 1;
            float delta = t - (float)i;
            delta = delta < 1.0f ? delta : 1.0f;
            float x0, x1;
            map.get((uint32_t)(mu * (n_g + 1) + i), x0, x1, mu >= D - kMapInnerAxes);
            const float dx = x1 - x0;
            const float x = fmaf(dx, delta, x0);
            jac = jac * ((float)n_g * dx);
            idx[mu] = i;
            early(mu, i);
            f_axis<D, KT, float, FP>(fc, kind, K, mu, x, st);
            if constexpr (DUMP) {
                dp->d->x[mu * dp->d->count + dp->pos] = (double)x;
                dp->d->idx[mu * dp->d->count + dp->pos] = i;
            }
        }
    }
    if constexpr (!DUMP) __builtin_amdgcn_s_setprio(0);
    const float fx = f_finish<D, KT, float, FP>(fc, kind, K, st);
    if constexpr (DUMP) {
        dp->d->jac[dp->pos] = (double)jac;
        dp->d->fx[dp->pos] = (double)fx;
    }
    return jac * fx;
}

// ---------------------------------------------------------------- the kernel
// KIND fixes the integrand at compile time (K_GAUSS_MIX, K_CORR_GAUSS), or is
// 0 for the generic kernel that dispatches on the integrand's kind at run time.
// Training data of one sample: atomics into the LDS bins of the privatised
// axes, and for the other axes a record at position pos (the sample's
// position, permuted within aligned groups) -- the numerator value, n_h and
// those axes' increment indices (k_hist_records bins them in any order).  The
// three record arrays follow each other at rec (see SampleArgs).
// WFIX: the weight plane is the unsigned 64-bit fixed-point sum (weight wq);
// else a double-precision sum (weight hw).  WDONE: the weights of the LDS
// axes were added already, as each axis was mapped.
template <int D, bool REC, bool WFIX, bool WDONE = false>
__device__ __forceinline__ void put_training(double* rec, int64_t stride, int ha, double* lds_hist, int lbins, int n_g,
                                             int64_t pos, double hh, double hw, uint64_t wq, uint32_t n,
                                             const int32_t* idx)
{
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
        if (mu < ha) {
            const int bin = mu * n_g + idx[mu];
            atomicAdd(&lds_hist[bin], hh);
            if constexpr (WDONE) {
            } else if constexpr (WFIX)
                atomicAdd(reinterpret_cast<unsigned long long*>(&lds_hist[lbins + bin]), (unsigned long long)wq);
            else
                atomicAdd(&lds_hist[lbins + bin], hw);
        }
    }
    if (REC && ha < D) {
        uint32_t* rn0 = reinterpret_cast<uint32_t*>(rec + stride);
        VP_GLOBAL uint32_t* rn = global_ptr(rn0);
        VP_GLOBAL uint16_t* rb = global_ptr(reinterpret_cast<uint16_t*>(rn0 + stride));
        global_ptr(rec)[pos] = hh;
        rn[pos] = n;
#pragma unroll
        for (int mu = 0; mu < D; ++mu)
            if (mu >= ha) rb[(mu - ha) * stride + pos] = (uint16_t)idx[mu];
    }
}

// Per-sample dump (vp_debug_dump) of the samples of [s_a, s_b) that lie in
// the dumped range: each is evaluated again through the same per-sample
// function as in the walk, from its hypercube h (binary search over the
// offsets) and index j, and written with x, the increment indices, J and
// f(x).  It sets up its own copies of the map and constant accessors (the
// LDS contents are still those of the walk).
template <int D, int PREC, int MAPL, int KIND, bool REC, int KT, bool MIX>
__device__ __forceinline__ void dump_share(const SampleArgs& a, int64_t s_a, int64_t s_b, int lane,
                                        unsigned char* lds_raw)
{
    typedef typename std::conditional<PREC == P_FP64, double, float>::type MapT;
    const int n_g = a.n_g;
    const int ha = REC ? a.hist_axes : D;
    const size_t hist_bytes = (size_t)ha * n_g * 16;
    MapT* lds_map = reinterpret_cast<MapT*>(lds_raw + hist_bytes);
    const MapT* lds_fc = reinterpret_cast<const MapT*>(lds_raw + fc_lds_offset(hist_bytes, MAPL, PREC, D, n_g));
    const MapT* gmap;
    if constexpr (PREC == P_FP64) gmap = a.map;
    else gmap = a.map32;
    typedef typename std::conditional<PREC == P_FP64, MapPair64<MAPL>, MapPair32<MAPL>>::type MapAcc;
    MapAcc map;
    map.lds = lds_map;
    map.inner0 = (uint32_t)((D - kMapInnerAxes) * (n_g + 1));
    map.rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)gmap, (short)0,
                                                 (int)((size_t)D * (n_g + 1) * sizeof(MapT)), kBufferWord3);
    constexpr bool FC_SMEM = (KIND == K_GAUSS_MIX);
    typedef __attribute__((address_space(4))) const MapT ConstT;
    ConstT* fcg = (ConstT*)a.fc;
    const int kind = KIND ? KIND : a.f->kind;
    const int K = a.f->n_terms;
    SampleHot hot;
    hot.key0 = a.key0;
    hot.key1 = a.key1;
    hot.it = a.it;
    hot.n_g = n_g;
    hot.R = a.R;
    hot.R32 = a.R32;
    hot.R53 = a.R53;
    hot.R32s = a.R32s;
    const MapT* mix_r = lds_fc + fc_strat_offset(kind, D);
    const MapT* mix_n = mix_r + D;
    if constexpr (PREC == P_FP64) {
        hot.Rv = reinterpret_cast<const double*>(mix_r);
        hot.Rv32 = nullptr;
    } else {
        hot.Rv = nullptr;
        hot.Rv32 = reinterpret_cast<const float*>(mix_r);
    }
    const int64_t* offs = a.offs;
    const int64_t* ob = a.obase;
    const int64_t n_hc = a.n_hc;
    const uint32_t n_st = (uint32_t)a.n_st;
    const int64_t d0 = s_a > a.dump.first ? s_a : a.dump.first;
    const int64_t d_end = a.dump.first + a.dump.count;
    const int64_t d1 = s_b < d_end ? s_b : d_end;
    for (int64_t sd = d0 + lane; sd < d1; sd += kWave) {
        int64_t lo = 0, hi = n_hc;  // offset(lo) <= sd < offset(hi)
        while (hi - lo > 1) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (gofs(offs, ob, mid) <= sd) lo = mid;
            else hi = mid;
        }
        const uint32_t h = (uint32_t)lo;
        const uint32_t j = (uint32_t)(sd - gofs(offs, ob, lo));
        int32_t k[D], idx[D];
        uint32_t r = h;
#pragma unroll
        for (int m = D - 1; m >= 0; --m) {
            const uint32_t nm = MIX ? (uint32_t)mix_n[m] : n_st;
            k[m] = (int32_t)(r % nm);
            r /= nm;
        }
        DumpPos dp;
        dp.d = &a.dump;
        dp.pos = sd - a.dump.first;
        // constants staged in LDS read afresh for each sample (hoisted out of
        // this loop, a D x D factor would be held in registers and spilled)
        const MapT* fcl = lds_fc;
        {
            int z;
            asm volatile("s_mov_b32 %0, 0" : "=s"(z));
            fcl = lds_fc + z;
        }
        a.dump.h[dp.pos] = (int64_t)h;
        a.dump.j[dp.pos] = (int32_t)j;
        if constexpr (PREC == P_FP64) {
            if constexpr (FC_SMEM)
                (void)sample_fp64<D, MAPL, KT, ConstT*, false, false, true>(hot, map, fcg, j, h, k, idx, kind, K,
                                                                           nullptr, &dp);
            else
                (void)sample_fp64<D, MAPL, KT, const MapT*, false, MIX, true>(hot, map, fcl, j, h, k, idx, kind, K,
                                                                             nullptr, &dp);
        } else {
            if constexpr (FC_SMEM)
                (void)sample_fp32<D, MAPL, KT, ConstT*, false, true>(hot, map, fcg, j, h, k, idx, kind, K, &dp);
            else
                (void)sample_fp32<D, MAPL, KT, const MapT*, MIX, true>(hot, map, fcl, j, h, k, idx, kind, K, &dp);
        }
    }
}

// REC: some axes' training data go out as records (the bins of all D axes do
// not fit in LDS); a separate instantiation, so that the common case carries
// none of that code.
// KT: Gaussian-mixture terms fixed at compile time (0: read at run time).
// MIX: per-axis stratification counts (Sec. 4), read with R_mu from the
// constants staged in LDS; only kernels that stage them there have it.
template <int D, int PREC, int MAPL, int KIND, bool REC, int KT, bool MIX>
__global__ __launch_bounds__(sample_block(PREC, KIND, D, MAPL == MAP_LDS, REC)) void k_sample(LaunchSet L)
{
    static_assert(MAPL != MAP_INNER || D > kMapInnerAxes, "staging the innermost axes needs more axes");
    VP_REQ_PROLOGUE(L);
    // The argument record stays in memory; the fields the loop needs are read
    // into registers here, the others where they are used (a copy of the
    // whole record would hold every field in scalar registers across the loop).
    const SampleArgs& a = q.s;
    typedef typename AccOf<PREC>::type Acc;
    typedef typename std::conditional<PREC == P_FP64, double, float>::type MapT;
    extern __shared__ __align__(16) unsigned char lds_raw[];

    // modes of a batched integrand (FP64 only): GEN writes the sample points
    // and touches no sums; ACC takes v = J f from memory
    constexpr bool GEN = (KIND == K_BATCH_GEN);
    constexpr bool ACC = (KIND == K_BATCH_ACC);
    static_assert(!(GEN || ACC) || PREC == P_FP64, "batched integrands are double precision");
    const int n_g = a.n_g;
    const int nbins = D * n_g;
    const int ha = GEN ? 0 : (REC ? a.hist_axes : D);  // axes privatised in LDS
    const int lbins = ha * n_g;            // bins per LDS plane
    const size_t hist_bytes = (size_t)lbins * 16;
    double* lds_hist = reinterpret_cast<double*>(lds_raw);
    uint64_t* lds_pairs = reinterpret_cast<uint64_t*>(lds_raw);  // compensated single precision: (sum, comp) per bin
    MapT* lds_map = reinterpret_cast<MapT*>(lds_raw + hist_bytes);
    const MapT* gmap;
    if constexpr (PREC == P_FP64) gmap = a.map;
    else gmap = a.map32;

    const int kind = KIND ? KIND : a.f->kind;
    const int K = a.f->n_terms;
    MapT* lds_fc = reinterpret_cast<MapT*>(lds_raw + fc_lds_offset(hist_bytes, MAPL, PREC, D, n_g));

    for (int i = threadIdx.x; i < 2 * lbins; i += blockDim.x) lds_hist[i] = 0.0;
    // the map values to stage in LDS: kStageU loads per thread in flight
    // before their stores (the set-up is latency that nothing else on the CU
    // hides, and a served request's workgroup walks about one tile per wave)
    const uint32_t inner0 = (uint32_t)((D - kMapInnerAxes) * (n_g + 1));
    if constexpr (MAPL == MAP_LDS || MAPL == MAP_INNER) {
        constexpr int kStageU = 8;
        const int n_stage = MAPL == MAP_LDS ? D * (n_g + 1) : kMapInnerAxes * (n_g + 1);
        const VP_GLOBAL MapT* src = global_ptr(MAPL == MAP_INNER ? gmap + inner0 : gmap);
        for (int i0 = threadIdx.x; i0 < n_stage; i0 += kStageU * blockDim.x) {
            MapT v[kStageU];
#pragma unroll
            for (int u = 0; u < kStageU; ++u) {
                const int i = i0 + u * (int)blockDim.x;
                v[u] = i < n_stage ? src[i] : MapT(0);
            }
#pragma unroll
            for (int u = 0; u < kStageU; ++u) {
                const int i = i0 + u * (int)blockDim.x;
                if (i < n_stage) lds_map[i] = v[u];
            }
        }
    }
    // Gaussian-mixture constants (4 D + 16 values) are read through the
    // scalar cache at every sample, from the constant address space: the
    // VALU takes them as scalar operands, and they occupy no register across
    // the loop (held there for the whole loop, they spill).  The correlated
    // Gaussian's D x D factor and the generic kernel's constants are staged
    // in LDS.
    constexpr bool FC_SMEM = (KIND == K_GAUSS_MIX);
    static_assert(!(MIX && FC_SMEM), "mixed stratification reads its constants from LDS");
    typedef __attribute__((address_space(4))) const MapT ConstT;
    ConstT* fcg = (ConstT*)a.fc;
    if constexpr (!FC_SMEM) {
        const VP_GLOBAL MapT* src = global_ptr(reinterpret_cast<const MapT*>(a.fc));
        for (int i = threadIdx.x; i < fc_count(kind, D); i += blockDim.x) lds_fc[i] = src[i];
    }
    __syncthreads();
    typedef typename std::conditional<PREC == P_FP64, MapPair64<MAPL>, MapPair32<MAPL>>::type MapAcc;
    MapAcc map;
    map.lds = lds_map;
    map.inner0 = inner0;
    map.rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)gmap, (short)0,
                                                 (int)((size_t)D * (n_g + 1) * sizeof(MapT)), kBufferWord3);

    const int lane = threadIdx.x & (kWave - 1);
    const int waves_per_block = blockDim.x / kWave;
    // Share of the sample range: the waves of one workgroup take shares nblk
    // apart, so that the workgroup's waves work on distant hypercubes.  (The
    // waves of a workgroup share its LDS bins; waves on neighbouring
    // hypercubes update the same bins of the outer axes at the same time,
    // which the compare-and-swap of the compensated form pays for in retries.)
    // Edge records are indexed by share, so they stay in sample order.
    const int64_t wave = (int64_t)(threadIdx.x / kWave) * nblk + bid;
    const int64_t n_waves = (int64_t)nblk * waves_per_block;
    const int64_t* __restrict__ offs = a.offs;
    const int64_t* __restrict__ ob = a.obase;
    const int64_t n_hc = a.n_hc;
    const int64_t n_tot = gofs(offs, ob, n_hc);
    // the batched-integrand modes start every wave at a group boundary of the
    // point buffers (batch_pos), so that its tiles coincide with the groups
    // and each buffer row is written whole
    auto wave_start = [&](int64_t w) -> int64_t {
        const int64_t x = n_tot * w / n_waves;
        if constexpr (GEN || ACC) return w == n_waves ? n_tot : (x & ~(int64_t)(kBatchGroup - 1));
        return x;
    };
    const int64_t s_a = wave_start(wave);
    const int64_t s_b = wave_start(wave + 1);
    const int C = a.chunk;
    const uint32_t n_st = (uint32_t)a.n_st;
    const bool literal = (a.hist_mode != 0);
    const double wscale = a.wscale;
    VP_GLOBAL double* __restrict__ S1 = global_ptr(a.S1);
    VP_GLOBAL double* __restrict__ S2 = global_ptr(a.S2);
    VP_GLOBAL EdgeRec* __restrict__ edges = global_ptr(a.edges);
    double* rec = REC ? a.rec_h : nullptr;
    const int64_t rec_stride = REC ? a.rec_stride : 0;
    BatchOut bout;
    const double* bf = nullptr;
    double bscale = 0.0;
    if constexpr (GEN || ACC) {
        bout.x = a.bx;
        bout.jac = a.bj;
        bout.idx = a.bidx;
        bout.n = n_tot;
        bout.cap = a.bcap;
        bf = a.bf;
        bscale = lds_fc[0];
    }
    SampleHot hot;
    hot.key0 = a.key0;
    hot.key1 = a.key1;
    hot.it = a.it;
    hot.n_g = n_g;
    hot.R = a.R;
    hot.R32 = a.R32;
    hot.R53 = a.R53;
    hot.R32s = a.R32s;
    // mixed stratification: R_mu, then N_st^mu, after the integrand constants
    const MapT* mix_r = lds_fc + fc_strat_offset(kind, D);
    const MapT* mix_n = mix_r + D;
    if constexpr (PREC == P_FP64) {
        hot.Rv = reinterpret_cast<const double*>(mix_r);
        hot.Rv32 = nullptr;
    } else {
        hot.Rv = nullptr;
        hot.Rv32 = reinterpret_cast<const float*>(mix_r);
    }
    uint32_t bad = 0;

    if (s_a < s_b) {
        const int64_t h_a = find_hypercube(offs, ob, n_hc, s_a, lane);
        int64_t h_cur = h_a;
        Acc carry;
        carry.zero();
        bool carry_ext = true;   // the run reaching the next lane is the wave's first hypercube
        bool carry_live = true;  // an unfinished run reaches the next lane
        int64_t h_open = h_a;

        for (int64_t s0 = s_a; s0 < s_b;) {
            // A share's last tile spreads what is left over all the lanes
            // (Ct = ceil(left / 64) samples each instead of C), so that it
            // takes only the steps its fullest lane needs: a served request's
            // workgroup of 768 threads walks 1.33 tiles per wave, and its
            // second tile would otherwise run 16 steps for a third of the lanes.
            // The batched-integrand modes keep C: their shares are whole groups
            // of the point buffers.
            const int64_t left = s_b - s0;
            const int Ct = (GEN || ACC || left >= (int64_t)kWave * C) ? C : (int)((left + kWave - 1) / kWave);
            const int64_t s_l = s0 + (int64_t)lane * Ct;
            const bool active = s_l < s_b;
            const int64_t e_l = active ? (s_l + Ct < s_b ? s_l + Ct : s_b) : s_l;
            int64_t h = locate(offs, ob, n_hc, h_cur, s_l, active, lane);

            Acc run, headacc;
            run.zero();
            headacc.zero();
            bool in_head = true, head_closed = false, open_end = false;
            const int64_t head_h = h;
            int64_t h_end = h;
            if (active) {
                // Walk state in 32 bits: sample positions relative to the wave's
                // first sample s_a (N_tot < 2^32), the index j within the current
                // hypercube, and the hypercube itself (N_hc < 2^31).
                const int64_t o_cur0 = gofs(offs, ob, h);
                uint32_t hh32 = (uint32_t)h;
                uint32_t next = (uint32_t)(gofs(offs, ob, h + 1) - s_a);
                // Batched-integrand modes: the boundaries of the hypercubes the
                // lane can reach in this tile (h + 2 .. h + 1 + kPreB) are
                // loaded here, once per tile, as positions relative to s_a.
                // Loads and stores share one counter, so a boundary loaded at
                // the switch that needs it would wait there for every point
                // the generate mode stored before it (and in the accumulate
                // mode for the next sample's prefetched values).  With
                // n_h >= 2 the tile's C = 16 samples cross at most 8
                // boundaries; a lane that runs out loads the next one at its
                // switch.  The offsets' low words suffice (the walk is 32-bit),
                // and kPreB < kOffsTile, so at most two block bases occur.
                constexpr int kPreB = 8;
                uint32_t bq[kPreB];
                int nbq = 0;
                if constexpr (GEN || ACC) {
                    const VP_GLOBAL uint32_t* lo = global_ptr(reinterpret_cast<const uint32_t*>(offs));
                    const VP_GLOBAL uint32_t* bo = global_ptr(reinterpret_cast<const uint32_t*>(ob));
                    const int64_t h_lo = h + 2 < n_hc ? h + 2 : n_hc;
                    const int64_t h_hi = h + 1 + kPreB < n_hc ? h + 1 + kPreB : n_hc;
                    const int64_t blk_a = h_lo / kOffsTile;
                    const uint32_t base_a = bo[2 * blk_a], base_b = bo[2 * (h_hi / kOffsTile)];
#pragma unroll
                    for (int i = 0; i < kPreB; ++i) {
                        const int64_t hq = h + 2 + i < n_hc ? h + 2 + i : n_hc;
                        bq[i] = lo[2 * hq] + (hq / kOffsTile == blk_a ? base_a : base_b) - (uint32_t)s_a;
                    }
                    nbq = kPreB;
                }
                uint32_t j = (uint32_t)(s_l - o_cur0);
                const uint32_t s_end = (uint32_t)(e_l - s_a);
                int32_t k[D];
                {
                    uint32_t r = hh32;
#pragma unroll
                    for (int m = D - 1; m >= 0; --m) {
                        const uint32_t nm = MIX ? (uint32_t)mix_n[m] : n_st;
                        k[m] = (int32_t)(r % nm);
                        r /= nm;
                    }
                }
                uint32_t n_cur = (uint32_t)(gofs(offs, ob, h + 1) - o_cur0);
                double inv_n = recip_count(n_cur);
                float inv_n32 = 1.0f / (float)n_cur;
                // split precisions: the hypercube's weight in the fixed-point plane
                // (the double-precision 1/n_h, or the single-precision one of the
                // compensated form; 1 in the literal mode)
                auto weight_q = [&]() -> uint64_t {
                    if constexpr (PREC == P_FP64) return 0;
                    else if constexpr (PREC == P_FP32_ACC64) return fixed_weight(literal ? 1.0 : inv_n, wscale);
                    else return fixed_weight(literal ? 1.0 : (double)inv_n32, wscale);
                };
                uint64_t wq = weight_q();
                constexpr int IDXG = (D + 7) / 8;  // 16-byte groups of increment indices
                // accumulate mode: J, f and the indices of the lane's next
                // sample are loaded while the current one is added up
                double pj = 0.0, pf = 0.0;
                U32x4 pw[IDXG];
                auto acc_load = [&](uint32_t s_rel) {
                    const int64_t pos = batch_pos(s_a + (int64_t)s_rel, n_tot);
                    pj = global_ptr(bout.jac)[pos];
                    pf = global_ptr(bf)[pos];
#pragma unroll
                    for (int g = 0; g < IDXG; ++g)
                        pw[g] = *global_ptr(reinterpret_cast<const U32x4*>(bout.idx + (pos * IDXG + g) * 8));
                };
                if constexpr (ACC) acc_load((uint32_t)(s_l - s_a));
                for (uint32_t s = (uint32_t)(s_l - s_a); s < s_end; ++s, ++j) {
                    if (s == next) {
                        if (in_head) {
                            headacc = run;
                            head_closed = true;
                            in_head = false;
                        } else {
                            if constexpr (!GEN) {
                                S1[hh32] = run.sa();
                                S2[hh32] = run.sb();
                            }
                        }
                        run.zero();
                        ++hh32;
                        j = 0;
                        uint32_t nn;
                        if ((GEN || ACC) && nbq > 0) {
                            nn = bq[0];
#pragma unroll
                            for (int i = 0; i + 1 < kPreB; ++i) bq[i] = bq[i + 1];
                            --nbq;
                        } else {
                            nn = (uint32_t)(gofs(offs, ob, (int64_t)hh32 + 1) - s_a);
                        }
                        n_cur = nn - next;
                        next = nn;
                        inv_n = recip_count(n_cur);
                        inv_n32 = 1.0f / (float)n_cur;
                        wq = weight_q();
                        // next hypercube: increment the last coordinate with
                        // carry, without branches (the lanes of a wave switch
                        // hypercubes at different samples)
                        int32_t carry = 1;
#pragma unroll
                        for (int m = D - 1; m >= 0; --m) {
                            const int32_t v = k[m] + carry;
                            carry = v == (MIX ? (int32_t)mix_n[m] : (int32_t)n_st) ? 1 : 0;
                            k[m] = carry ? 0 : v;
                        }
                    }
                    int32_t idx[D];
                    // an offset the compiler cannot see through keeps the
                    // scalar loads of the constants inside the loop
                    ConstT* fcs = fcg;
                    const MapT* fcl = lds_fc;
                    {
                        int z;
                        asm volatile("s_mov_b32 %0, 0" : "=s"(z));
                        if constexpr (FC_SMEM) fcs = fcg + z;
                        // likewise the reads of constants staged in LDS (the
                        // correlated Gaussian's D x D factor would otherwise be
                        // hoisted into registers and spilled)
                        else fcl = lds_fc + z;
                    }
                    // the sample's position permuted within aligned groups: where
                    // a batched integrand's point goes, and where a training
                    // record goes (the lanes of a wave, each walking 16
                    // consecutive samples, then write consecutive addresses)
                    const int64_t bpos = batch_pos(s_a + (int64_t)s, n_tot);
                    if constexpr (GEN) {
                        bout.pos = bpos;
                        (void)sample_fp64<D, MAPL, 0, const MapT*, true, MIX>(hot, map, fcl, j, hh32, k, idx, kind, K,
                                                                           &bout);
#pragma unroll
                        for (int g = 0; g < IDXG; ++g) {
                            uint32_t w[4];
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const int m0 = 8 * g + 2 * r, m1 = m0 + 1;
                                w[r] = (m0 < D ? (uint32_t)idx[m0] : 0u) | ((m1 < D ? (uint32_t)idx[m1] : 0u) << 16);
                            }
                            U32x4* dst = reinterpret_cast<U32x4*>(bout.idx + (bpos * IDXG + g) * 8);
                            *global_ptr(dst) = U32x4{w[0], w[1], w[2], w[3]};
                        }
                    } else if constexpr (PREC == P_FP64) {
                        double v;
                        if constexpr (ACC) {
                            v = pj * (bscale * pf);
                            U32x4 cw[IDXG];
#pragma unroll
                            for (int g = 0; g < IDXG; ++g) cw[g] = pw[g];
                            if (s + 1 < s_end) acc_load(s + 1);
#pragma unroll
                            for (int g = 0; g < IDXG; ++g) {
                                const U32x4 wv = cw[g];
                                const uint32_t w[4] = {wv[0], wv[1], wv[2], wv[3]};
#pragma unroll
                                for (int r = 0; r < 4; ++r) {
                                    const int m0 = 8 * g + 2 * r, m1 = m0 + 1;
                                    if (m0 < D) idx[m0] = (int32_t)(w[r] & 0xffffu);
                                    if (m1 < D) idx[m1] = (int32_t)(w[r] >> 16);
                                }
                            }
                        } else {
                            v = (FC_SMEM ? sample_fp64<D, MAPL, KT, ConstT*>(hot, map, fcs, j, hh32, k, idx, kind, K)
                                         : sample_fp64<D, MAPL, KT, const MapT*, false, MIX>(hot, map, fcl, j, hh32, k, idx, kind, K));
                        }
                        run.add(v);
                        if (!isfinite(v)) ++bad;
                        const double v2 = v * v;
                        const double hh = literal ? v2 : v2 * inv_n;
                        const double hw = literal ? 1.0 : inv_n;
                        put_training<D, REC, false>(rec, rec_stride, ha, lds_hist, lbins, n_g, REC ? bpos : 0, hh, hw,
                                                    wq, n_cur, idx);
                    } else if constexpr (PREC == P_FP32_ACC64) {
                        // Up to D = 11 the weight (known before the integrand) goes
                        // to its bin as soon as the axis's increment is known,
                        // which spreads the sample's LDS atomics over its map
                        // phase (from D = 12 the hook's registers would spill).
                        constexpr bool WE = D <= 11;
                        auto wadd = [&](int mu, int i) {
                            if (WE && mu < ha)
                                atomicAdd(reinterpret_cast<unsigned long long*>(&lds_hist[lbins + mu * n_g + i]),
                                          (unsigned long long)wq);
                        };
                        const float v32 = (FC_SMEM ? sample_fp32<D, MAPL, KT, ConstT*, false, false>(hot, map, fcs, j, hh32, k, idx, kind, K, nullptr, wadd)
                                           : sample_fp32<D, MAPL, KT, const MapT*, MIX, false>(hot, map, fcl, j, hh32, k, idx, kind, K, nullptr, wadd));
                        const double v = (double)v32;
                        run.add(v);
                        if (!isfinite(v32)) ++bad;
                        const double v2 = v * v;
                        const double hh = literal ? v2 : v2 * inv_n;
                        const double hw = literal ? 1.0 : inv_n;
                        put_training<D, REC, true, WE>(rec, rec_stride, ha, lds_hist, lbins, n_g, REC ? bpos : 0, hh, hw,
                                                       wq, n_cur, idx);
                    } else {
                        const float v32 = (FC_SMEM ? sample_fp32<D, MAPL, KT, ConstT*>(hot, map, fcs, j, hh32, k, idx, kind, K)
                                           : sample_fp32<D, MAPL, KT, const MapT*, MIX>(hot, map, fcl, j, hh32, k, idx, kind, K));
                        run.addf(v32);
                        if (!isfinite(v32)) ++bad;
                        const float v2 = v32 * v32;
                        const float hh = literal ? v2 : v2 * inv_n32;
                        lds_neumaier_sample<D>(lds_pairs, lbins, n_g, idx, hh, wq);
                    }
                }
                if (s_end == next) {
                    // the run ends exactly at the end of this lane's samples
                    if (in_head) {
                        headacc = run;
                        head_closed = true;
                        in_head = false;
                    } else {
                        if constexpr (!GEN) {
                            S1[hh32] = run.sa();
                            S2[hh32] = run.sb();
                        }
                    }
                    run.zero();
                    h_end = (int64_t)hh32 + 1;
                } else {
                    open_end = true;
                    h_end = (int64_t)hh32;
                }
            }

            // Segmented scan of the runs that cross lane boundaries.  Lane l maps
            // the carry reaching it to the carry leaving it: a lane whose first
            // run never closes (pass-through) adds its sums to the carry; any
            // other lane starts a new carry from its open last run (or zero).
            // Inactive lanes are the identity.
            bool A = !active || !head_closed;
            Acc B = run;
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const bool Ap = __shfl_up((int)A, d) != 0;
                const Acc Bp = B.shfl_up(d);
                if (lane >= d) {
                    if (A) B.join_after(Bp);
                    A = A && Ap;
                }
            }
            // exclusive prefix for this lane
            bool Ax = __shfl_up((int)A, 1) != 0;
            Acc Bx = B.shfl_up(1);
            if (lane == 0) {
                Ax = true;
                Bx.zero();
            }
            if (active && head_closed) {
                Acc cin = Bx;
                if (Ax) cin.join_after(carry);
                const bool ext = Ax && carry_ext;
                Acc tot = headacc;
                tot.join_after(cin);
                if (ext) {
                    EdgeRec r;
                    r.h = head_h;
                    r.s1 = tot.sa();
                    r.s2 = tot.sb();
                    if constexpr (!GEN) put_edge(edges + (2 * wave), r);
                } else if constexpr (!GEN) {
                    S1[head_h] = tot.sa();
                    S2[head_h] = tot.sb();
                }
            }
            // carry into the next tile: lane 63's inclusive map applied to the carry
            const bool A63 = __shfl((int)A, kWave - 1) != 0;
            Acc B63 = B.bcast(kWave - 1);
            if (A63) B63.join_after(carry);
            carry = B63;
            carry_ext = A63 && carry_ext;
            // the last active lane decides whether a run is still open, and where
            const int64_t rem = (s_b - 1 - s0) / Ct;
            const int last_active = rem < kWave - 1 ? (int)rem : kWave - 1;
            const bool live_own = active && (!head_closed || open_end);
            carry_live = __shfl((int)live_own, last_active) != 0;
            h_open = shfl64(h_end, last_active);
            h_cur = shfl64(h_end, kWave - 1);
            s0 += (int64_t)kWave * Ct;
        }
        if (lane == 0 && !GEN) {
            EdgeRec empty;
            empty.h = -1;
            empty.s1 = 0.0;
            empty.s2 = 0.0;
            if (carry_live) {
                EdgeRec r;
                r.s1 = carry.sa();
                r.s2 = carry.sb();
                if (carry_ext) {
                    r.h = h_a;
                    put_edge(edges + (2 * wave), r);
                    put_edge(edges + (2 * wave + 1), empty);
                } else {
                    r.h = h_open;
                    put_edge(edges + (2 * wave + 1), r);
                }
            } else {
                put_edge(edges + (2 * wave + 1), empty);
            }
        }
    } else if (lane == 0 && !GEN) {
        EdgeRec empty;
        empty.h = -1;
        empty.s1 = 0.0;
        empty.s2 = 0.0;
        put_edge(edges + (2 * wave), empty);
        put_edge(edges + (2 * wave + 1), empty);
    }

    // Per-sample dump (vp_debug_dump), after the share is done.  Every value
    // it needs is read again through a pointer the compiler cannot trace to
    // the one above, so that nothing is kept live across the walk for it.
    if constexpr (!GEN && !ACC) {
        int z;
        asm volatile("s_mov_b32 %0, 0" : "=s"(z));
        const SampleArgs* ap = &a + z;
        if (ap->dump.count > 0 && ap->dump.it == ap->it)
            dump_share<D, PREC, MAPL, KIND, REC, KT, MIX>(*ap, s_a, s_b, lane, lds_raw);
    }

    // non-finite samples: one atomic per wave
    for (int d = kWave / 2; d >= 1; d >>= 1) bad += __shfl_down(bad, d);
    if (lane == 0 && bad) atomicAdd(a.nonfinite, (unsigned long long)bad);

    __syncthreads();
    // The training data to this workgroup's partial: four bins' LDS reads per
    // thread in flight before their stores.
    if constexpr (!GEN) {
        VP_GLOBAL double* out = global_ptr(a.hist_part + (size_t)bid * 2 * nbins);
        const double wsi = a.wscale_inv;
        auto bin = [&](int i, double& h, double& w) {
            if constexpr (PREC == P_FP32_NEUMAIER) {
                const uint64_t ph = lds_pairs[i];
                h = (double)__uint_as_float((uint32_t)ph) + (double)__uint_as_float((uint32_t)(ph >> 32));
                w = (double)lds_pairs[lbins + i] * wsi;
            } else if constexpr (PREC == P_FP32_ACC64) {
                h = lds_hist[i];
                w = (double)reinterpret_cast<const uint64_t*>(lds_hist)[lbins + i] * wsi;
            } else {
                h = lds_hist[i];
                w = lds_hist[lbins + i];
            }
        };
        constexpr int U = 4;
        for (int i0 = threadIdx.x; i0 < lbins; i0 += U * blockDim.x) {
            double h[U], w[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * (int)blockDim.x;
                if (i < lbins) bin(i, h[u], w[u]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * (int)blockDim.x;
                if (i < lbins) {
                    out[i] = h[u];
                    out[nbins + i] = w[u];
                }
            }
        }
    }
}

template <int D, int PREC, int MAPL, int KIND, bool REC, int KT, bool MIX>
void launch_sample(const LaunchSet& L, int grid, int block, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((k_sample<D, PREC, MAPL, KIND, REC, KT, MIX>), dim3(grid), dim3(block), lds, s, L);
}

template <int D, int PREC, int MAPL, int KIND, bool REC, int KT, bool MIX>
int sample_occupancy(int block, size_t lds)
{
    int n = 0;
    (void)hipFuncSetAttribute((const void*)k_sample<D, PREC, MAPL, KIND, REC, KT, MIX>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_sample<D, PREC, MAPL, KIND, REC, KT, MIX>, block,
                                                     lds) != hipSuccess)
        return 0;
    return n;
}

template <int D, int PREC, int MAPL, int KIND, bool REC, int KT, bool MIX = false>
SampleEntry make_entry()
{
    SampleEntry e;
    e.launch = launch_sample<D, PREC, MAPL, KIND, REC, KT, MIX>;
    e.occupancy = sample_occupancy<D, PREC, MAPL, KIND, REC, KT, MIX>;
    e.block = sample_block(PREC, KIND, D, MAPL == MAP_LDS, REC);
    return e;
}

// The instantiation for a layout (map: a MapPlace).  All training data in
// LDS, with the whole map in LDS, its innermost axes in LDS, or the map in
// global memory; or training records with the map in global memory.  The
// split precisions read the map from global memory only: their kernels are
// bound by the LDS atomics of the training data, and map reads from LDS
// would queue behind them.
constexpr SampleEntry kNoEntry = {nullptr, nullptr, 0};

template <int D, int PREC, int KIND, int KT = 0, bool MIX = false>
SampleEntry entry_for(int map, bool rec)
{
    if (rec) return map == MAP_GLOBAL ? make_entry<D, PREC, MAP_GLOBAL, KIND, true, KT, MIX>() : kNoEntry;
    if (map == MAP_GLOBAL) return make_entry<D, PREC, MAP_GLOBAL, KIND, false, KT, MIX>();
    if constexpr (PREC == P_FP64)
        if (map == MAP_LDS) return make_entry<D, PREC, MAP_LDS, KIND, false, KT, MIX>();
    if constexpr (D > kMapInnerAxes)
        if (map == MAP_INNER) return make_entry<D, PREC, MAP_INNER, KIND, false, KT, MIX>();
    return kNoEntry;
}

// The map in global memory only (kernels whose integrand constants take the
// LDS the map would use).
template <int D, int PREC, int KIND, int KT = 0, bool MIX = false>
SampleEntry entry_for_global(int map, bool rec)
{
    if (map != MAP_GLOBAL) return kNoEntry;
    return rec ? make_entry<D, PREC, MAP_GLOBAL, KIND, true, KT, MIX>() : make_entry<D, PREC, MAP_GLOBAL, KIND, false, KT, MIX>();
}

// Compensated sums need every axis's bins in LDS: no record variants.
template <int D, int PREC, int KIND, int KT = 0, bool MIX = false>
SampleEntry entry_for_global_lds_only(int map, bool rec)
{
    if (rec) return kNoEntry;
    if (map == MAP_GLOBAL) return make_entry<D, PREC, MAP_GLOBAL, KIND, false, KT, MIX>();
    if constexpr (D > kMapInnerAxes)
        if (map == MAP_INNER) return make_entry<D, PREC, MAP_INNER, KIND, false, KT, MIX>();
    return kNoEntry;
}

}  // namespace vp

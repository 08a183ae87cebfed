// vp_aux.hip -- the per-hypercube and per-increment kernels of one iteration:
// allocation scan, edge fix-up, training-data reduction, iteration estimate
// and combination, reallocation, and map refinement.
#include "vp_aux.hpp"

#include <algorithm>

namespace vp {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ int64_t wave_incl_scan(int64_t v, int lane)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int64_t lo = __shfl_up((int)(uint32_t)v, d);
        const int64_t hi = __shfl_up((int)(uint32_t)((uint64_t)v >> 32), d);
        const int64_t p = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
        if (lane >= d) v += p;
    }
    return v;
}

// Exclusive scan of one value per thread across a block of kScanBlock
// threads; returns the block total in *total.
__device__ int64_t block_excl_scan(int64_t v, int64_t* total)
{
    __shared__ int64_t wsum[kScanBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t incl = wave_incl_scan(v, lane);
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    if (w == 0) {
        int64_t x = lane < kScanBlock / kWave ? wsum[lane] : 0;
        x = wave_incl_scan(x, lane);
        if (lane < kScanBlock / kWave) wsum[lane] = x;
    }
    __syncthreads();
    const int64_t before = (w > 0 ? wsum[w - 1] : 0) + incl - v;
    *total = wsum[kScanBlock / kWave - 1];
    __syncthreads();
    return before;
}

// ---------------------------------------------------------------- allocation scan
// Sample offsets of every hypercube: offs[h] = sum_{h' < h} n_h', and
// offs[n_hc] = N_tot (the samples actually drawn this iteration, Sec. 3).
__global__ __launch_bounds__(kScanBlock) void k_scan_local(LaunchSet L)
{
    VP_REQ_PROLOGUE(L);
    const int32_t* __restrict__ n_h = q.n_h;
    const int64_t n_hc = q.n_hc;
    int64_t* __restrict__ offs = q.offs;
    int64_t* __restrict__ bsum = q.bsum;
    // each thread scans kScanPer consecutive counts.  A whole tile moves
    // through LDS so that the lanes of each 16-byte load and store touch
    // consecutive addresses (the arrays are 256-byte aligned); the last,
    // partial tile is read and written element by element.
    __shared__ int64_t stage[kScanTile];
    int32_t* const cnt = reinterpret_cast<int32_t*>(stage);
    const int64_t tile0 = (int64_t)bid * kScanTile;
    const int64_t base = tile0 + (int64_t)threadIdx.x * kScanPer;
    const bool whole = tile0 + kScanTile <= n_hc;  // uniform over the workgroup
    int64_t v[kScanPer];
    int64_t t = 0;
    if (whole) {
        const int4* __restrict__ src = reinterpret_cast<const int4*>(n_h + tile0);
#pragma unroll
        for (int i = 0; i < kScanPer / 4; ++i)
            reinterpret_cast<int4*>(cnt)[i * kScanBlock + threadIdx.x] = src[i * kScanBlock + threadIdx.x];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kScanPer; i += 4) {
            const int4 c = reinterpret_cast<const int4*>(cnt)[(threadIdx.x * kScanPer + i) / 4];
            v[i] = c.x;
            v[i + 1] = c.y;
            v[i + 2] = c.z;
            v[i + 3] = c.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kScanPer; ++i) v[i] = base + i < n_hc ? (int64_t)n_h[base + i] : 0;
    }
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) t += v[i];
    int64_t total;
    int64_t run = block_excl_scan(t, &total);  // synchronises the workgroup: the counts are read
    int64_t o[kScanPer];
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        o[i] = run;
        run += v[i];
    }
    if (whole) {
#pragma unroll
        for (int i = 0; i < kScanPer; i += 2)
            reinterpret_cast<longlong2*>(stage)[(threadIdx.x * kScanPer + i) / 2] = make_longlong2(o[i], o[i + 1]);
        __syncthreads();
        longlong2* __restrict__ dst = reinterpret_cast<longlong2*>(offs + tile0);
#pragma unroll
        for (int i = 0; i < kScanPer / 2; ++i)
            dst[i * kScanBlock + threadIdx.x] = reinterpret_cast<const longlong2*>(stage)[i * kScanBlock + threadIdx.x];
    } else {
#pragma unroll
        for (int i = 0; i < kScanPer; ++i)
            if (base + i < n_hc) offs[base + i] = o[i];
    }
    if (threadIdx.x == 0) bsum[bid] = total;
}

// Exclusive scan of the block totals by one block.  Afterwards the sample
// offset of hypercube h is loc[h] + bsum[h / kScanTile] (see gofs), and the
// entry for h = n_hc holds N_tot, the samples drawn this iteration.
__global__ __launch_bounds__(kScanBlock) void k_scan_top(LaunchSet L)
{
    VP_REQ_PROLOGUE(L);
    int64_t* __restrict__ bsum = q.bsum;
    int64_t* __restrict__ loc = q.offs;
    const int64_t n_hc = q.n_hc;
    const int64_t nb = (n_hc + kScanTile - 1) / kScanTile;
    const int64_t per = (nb + kScanBlock - 1) / kScanBlock;
    const int64_t b0 = (int64_t)threadIdx.x * per;
    int64_t t = 0;
    for (int64_t i = 0; i < per; ++i)
        if (b0 + i < nb) t += bsum[b0 + i];
    int64_t total;
    int64_t run = block_excl_scan(t, &total);
    for (int64_t i = 0; i < per; ++i) {
        if (b0 + i < nb) {
            const int64_t x = bsum[b0 + i];
            bsum[b0 + i] = run;
            run += x;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        bsum[nb] = total;
        loc[n_hc] = total - bsum[n_hc / kScanTile];
    }
}

// ---------------------------------------------------------------- edge fix-up
// Hypercubes whose samples span several waves leave one partial per wave as
// edge records (h = -1: no record), sorted by h in wave order.  One workgroup
// per request sums every run of equal h: each thread summarises a contiguous
// slice of records, a fixed-shape scan over the slices gives each thread the
// run reaching it from the left, and the thread holding a run's last record
// writes S1[h], S2[h].  The summation order depends only on the records'
// positions, never on timing.
struct RunSum {
    int64_t hf, hl;  // first and last hypercube of the slice
    double a, b;     // sums of the slice's last run
    int has;         // the slice holds a record
    int single;      // every record of the slice has the same h
};

__device__ __forceinline__ RunSum run_combine(const RunSum& x, const RunSum& y)
{
    if (!y.has) return x;
    if (!x.has) return y;
    RunSum r;
    r.has = 1;
    r.hf = x.hf;
    r.hl = y.hl;
    if (y.single && y.hf == x.hl) {
        r.a = x.a + y.a;
        r.b = x.b + y.b;
        r.single = x.single;
    } else {
        r.a = y.a;
        r.b = y.b;
        r.single = 0;
    }
    return r;
}

// Records per thread held in registers (more per thread are read twice from
// memory instead).  Eight cover the 2 x 4096 records of a full-device grid
// with 1024 threads; sixteen took the kernel to 128 registers and spilled.
constexpr int kFixPer = 8;
static_assert(kFixSmallRecs <= kFixSmallBlock * kFixPer, "small requests' records are held in registers");

__device__ __forceinline__ RunSum run_shfl(const RunSum& x, int src)
{
    RunSum r;
    r.hf = __shfl((long long)x.hf, src);
    r.hl = __shfl((long long)x.hl, src);
    r.a = __shfl(x.a, src);
    r.b = __shfl(x.b, src);
    r.has = __shfl(x.has, src);
    r.single = __shfl(x.single, src);
    return r;
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_edge_fixup(LaunchSet L)
{
    VP_REQ_PROLOGUE(L);
    __shared__ RunSum wrun[BLOCK / kWave];
    __shared__ int64_t wfirst[BLOCK / kWave];
    const EdgeRec* __restrict__ e = q.edges;
    const int64_t n_rec = 2 * q.n_waves;
    const int t = threadIdx.x;
    const int64_t per = (n_rec + BLOCK - 1) / BLOCK;
    const int64_t r0 = min(n_rec, (int64_t)t * per), r1 = min(n_rec, r0 + per);
    const bool held = per <= kFixPer;
    // the thread's records, loaded independently of each other
    EdgeRec buf[kFixPer];
    if (held) {
#pragma unroll
        for (int i = 0; i < kFixPer; ++i) {
            if (r0 + i < r1) buf[i] = e[r0 + i];
            else buf[i].h = -1;
        }
    }
    // visits the thread's records in order: from registers (unrolled, so the
    // buffer stays in registers) or from memory
    auto visit = [&](auto&& f) {
        if (held) {
#pragma unroll
            for (int i = 0; i < kFixPer; ++i) f(buf[i]);
        } else {
            for (int64_t r = r0; r < r1; ++r) f(e[r]);
        }
    };
    RunSum mine;
    mine.has = 0;
    mine.single = 1;
    mine.hf = mine.hl = -1;
    mine.a = mine.b = 0.0;
    visit([&](const EdgeRec& x) {
        const int64_t h = x.h;
        if (h < 0) return;
        if (!mine.has) {
            mine.has = 1;
            mine.hf = mine.hl = h;
            mine.a = x.s1;
            mine.b = x.s2;
        } else if (h == mine.hl) {
            mine.a = mine.a + x.s1;
            mine.b = mine.b + x.s2;
        } else {
            mine.hl = h;
            mine.a = x.s1;
            mine.b = x.s2;
            mine.single = 0;
        }
    });
    // The run reaching each thread from the left (an inclusive scan of the
    // slice summaries) and the first record to its right (a suffix scan of
    // the slices' first hypercubes, -1 for none): within each wave by
    // shuffles, across the waves through one summary per wave, in a fixed
    // shape.
    const int lane = t & (kWave - 1), w = t / kWave;
    RunSum incl = mine;
    int64_t first = mine.has ? mine.hf : -1;  // first record at or right of this thread, in the wave
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const RunSum u = run_shfl(incl, lane - d);
        if (lane >= d) incl = run_combine(u, incl);
        const int64_t f = __shfl((long long)first, lane + d);
        if (first < 0 && lane + d < kWave) first = f;
    }
    // (every lane takes part in these shuffles: a lane that has left the
    // kernel gives no value)
    const RunSum left = run_shfl(incl, lane - 1);
    int64_t next_h = __shfl((long long)first, lane + 1);
    if (lane == kWave - 1) next_h = -1;
    if (lane == kWave - 1) wrun[w] = incl;
    if (lane == 0) wfirst[w] = first;
    __syncthreads();
    if (!mine.has) return;
    RunSum carry;
    carry.has = 0;
    for (int v = 0; v < w; ++v) carry = run_combine(carry, wrun[v]);
    if (lane > 0) carry = run_combine(carry, left);
    for (int v = w + 1; v < BLOCK / kWave && next_h < 0; ++v) next_h = wfirst[v];
    const int next_has = next_h >= 0;
    double* __restrict__ S1 = q.S1;
    double* __restrict__ S2 = q.S2;
    bool open = false;
    int64_t ch = -1;
    double ca = 0.0, cb = 0.0;
    visit([&](const EdgeRec& x) {
        const int64_t h = x.h;
        if (h < 0) return;
        if (!open) {
            open = true;
            ch = h;
            if (carry.has && carry.hl == h) {
                ca = carry.a + x.s1;
                cb = carry.b + x.s2;
            } else {
                ca = x.s1;
                cb = x.s2;
            }
        } else if (h == ch) {
            ca = ca + x.s1;
            cb = cb + x.s2;
        } else {
            S1[ch] = ca;
            S2[ch] = cb;
            ch = h;
            ca = x.s1;
            cb = x.s2;
        }
    });
    if (open && !(next_has && next_h == ch)) {
        S1[ch] = ca;
        S2[ch] = cb;
    }
}

// ---------------------------------------------------------------- training data
// Sum of the per-workgroup partials; each partial holds the numerator plane
// H[nbins] followed by the weight plane W[nbins].  A workgroup takes V rows of
// kHistBlock / G consecutive values; each of its G thread groups sums every
// G-th partial (two interleaved chains), and the group sums are added in
// group order -- a fixed order, independent of timing, with G times more
// loads in flight than one thread per value.  Few partials (small served
// requests) give G = 1 and several rows per workgroup.
__global__ __launch_bounds__(kHistBlock) void k_hist_reduce(LaunchSet L)
{
    VP_REQ_PROLOGUE(L);
    const double* __restrict__ part = q.hist_part;
    const int64_t nbins = (int64_t)q.dim * q.n_g;
    const int64_t lbins = (int64_t)q.hist_axes * q.n_g;
    double* __restrict__ H = q.H;
    double* __restrict__ W = q.W;
    __shared__ double red[kHistBlock];
    const int n_max = max(q.grid, q.rec_chunks);
    const int G = hist_groups(n_max), V = hist_values(n_max);
    const int lanes = kHistBlock / G;  // values side by side; each thread takes V of them, lanes apart
    const int b = threadIdx.x % lanes, g = threadIdx.x / lanes;
    for (int v = 0; v < V; ++v) {
        const int64_t i = ((int64_t)bid * V + v) * lanes + b;
        double s = 0.0;
        if (i < 2 * nbins) {
            const int64_t j = i < nbins ? i : i - nbins;
            const int n_part = j < lbins ? q.grid : q.rec_chunks;
            double a0 = 0.0, a1 = 0.0;
            int p = g;
#pragma unroll 4
            for (; p + G < n_part; p += 2 * G) {
                a0 = a0 + part[(int64_t)p * 2 * nbins + i];
                a1 = a1 + part[(int64_t)(p + G) * 2 * nbins + i];
            }
            if (p < n_part) a0 = a0 + part[(int64_t)p * 2 * nbins + i];
            s = a0 + a1;
        }
        red[threadIdx.x] = s;
        __syncthreads();
        if (g == 0 && i < 2 * nbins) {
            double tot = red[b];
            for (int k = 1; k < G; ++k) tot = tot + red[k * lanes + b];
            if (i >= nbins) W[i - nbins] = tot;
            else H[i] = tot;
        }
        __syncthreads();
    }
}

// Training data from per-sample records, for the axes the sampling kernel
// could not privatise in LDS (D * N_g bins too many).  Workgroup (chunk c,
// slice l) bins the records of sample positions
// [c N / chunks, (c + 1) N / chunks) for the axes of slice l into
// LDS -- numerator and weight planes of rec_axes * n_g bins -- and writes them
// to partial c, which k_hist_reduce sums over chunks.  The weight is 1/n_h
// (1 for the literal form), as the sampling kernel computes it.
__global__ __launch_bounds__(kRecBlock) void k_hist_records(LaunchSet L)
{
    VP_REQ_PROLOGUE(L);
    extern __shared__ __align__(16) unsigned char lds_raw[];
    double* lh = reinterpret_cast<double*>(lds_raw);
    const int n_g = q.n_g;
    const int c = bid / q.rec_slices;
    const int l = bid - c * q.rec_slices;
    const int a0 = q.hist_axes + l * q.rec_axes;
    const int a1 = min(q.dim, a0 + q.rec_axes);
    const int nb = (a1 - a0) * n_g;
    double* lw = lh + nb;
    for (int i = threadIdx.x; i < 2 * nb; i += blockDim.x) lh[i] = 0.0;
    __syncthreads();
    const SampleArgs& a = q.s;
    const int64_t n_tot = gofs(a.offs, a.obase, q.n_hc);
    const int64_t p0 = n_tot * c / q.rec_chunks;
    const int64_t p1 = n_tot * (c + 1) / q.rec_chunks;
    const bool literal = a.hist_mode != 0;
    const double* __restrict__ rh = a.rec_h;
    const uint32_t* __restrict__ rn = a.rec_n;
    const uint16_t* __restrict__ rb = a.rec_bin;
    const int64_t stride = a.rec_stride;
    // kRecUnroll records per thread and pass: their loads are in flight
    // together (a workgroup of one wave would otherwise wait out one load
    // latency per record); the additions follow in a fixed order
    constexpr int U = kRecUnroll;
    const int64_t step = (int64_t)U * blockDim.x;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += step) {
        double hh[U], hw[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t r = p + (int64_t)u * blockDim.x;
            hh[u] = r < p1 ? rh[r] : 0.0;
            hw[u] = r < p1 ? (literal ? 1.0 : 1.0 / (double)rn[r]) : 0.0;
        }
        for (int mu = a0; mu < a1; ++mu) {
            const uint16_t* __restrict__ rbm = rb + (int64_t)(mu - q.hist_axes) * stride;
            int bin[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t r = p + (int64_t)u * blockDim.x;
                bin[u] = (mu - a0) * n_g + (r < p1 ? (int)rbm[r] : 0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (p + (int64_t)u * blockDim.x < p1) {
                    atomicAdd(&lh[bin[u]], hh[u]);
                    atomicAdd(&lw[bin[u]], hw[u]);
                }
            }
        }
    }
    __syncthreads();
    const int64_t nbins = (int64_t)q.dim * n_g;
    double* out = q.hist_part + (int64_t)c * 2 * nbins + (int64_t)a0 * n_g;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        out[i] = lh[i];
        out[nbins + i] = lw[i];
    }
}

// Threads t0, t0 + stride, ... of the initialisation of one problem.
__device__ __forceinline__ void init_problem(const InitArgs& a, int64_t t0, int64_t stride)
{
    const int64_t nm = (int64_t)a.dim * (a.n_g + 1);
    const int64_t n = max(nm, max(a.n_hc, a.nbins));
    if (a.head_src) {
        const uint64_t* __restrict__ src = reinterpret_cast<const uint64_t*>(a.head_src);
        uint64_t* __restrict__ dst = reinterpret_cast<uint64_t*>(a.head_dst);
        for (int64_t i = t0; i < a.head_bytes / 8; i += stride) dst[i] = src[i];
    }
    for (int64_t i = t0; i < n; i += stride) {
        if (i < nm) {
            const int d = (int)(i / (a.n_g + 1)), k = (int)(i - (int64_t)d * (a.n_g + 1));
            const double lo = a.bounds[d], hi = a.bounds[a.dim + d];
            const double v = k == a.n_g ? hi : lo + (hi - lo) * ((double)k / (double)a.n_g);
            a.map[i] = v;
            a.map32[i] = (float)v;
        }
        if (i < a.n_hc) {
            a.n_h[i] = a.n0;
            a.S1[i] = 0.0;
            a.S2[i] = 0.0;
        }
        if (i < a.nbins) {
            a.H[i] = 0.0;
            a.W[i] = 0.0;
        }
    }
}

__global__ void k_init(InitArgs a)
{
    init_problem(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

// Problem blockIdx.y of the table, with gridDim.x workgroups.
__global__ void k_init_batch(const InitArgs* __restrict__ table)
{
    const InitArgs a = table[blockIdx.y];
    if (a.n_hc < 0) return;
    init_problem(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

void launch_init_batch(const InitArgs* table, int n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_init_batch, dim3(8, (unsigned)n), dim3(256), 0, s, table);
}

void launch_init(const InitArgs& a, hipStream_t s)
{
    const int64_t nm = (int64_t)a.dim * (a.n_g + 1);
    const int64_t n = std::max(nm, std::max(a.n_hc, a.nbins));
    const int64_t g = std::min<int64_t>(4096, std::max<int64_t>(1, (n + 255) / 256));
    hipLaunchKernelGGL(k_init, dim3((unsigned)g), dim3(256), 0, s, a);
}

__global__ void k_gather_states(DevState* const* states, int n, DevState* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = *states[i];
}

void launch_gather_states(DevState* const* states, int n, DevState* out, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_gather_states, dim3((n + 255) / 256), dim3(256), 0, s, states, n, out);
}

__global__ void k_fill_f64(double* __restrict__ x, int64_t n, double v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

__global__ void k_fill_i32(int32_t* __restrict__ x, int64_t n, int32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

// ---------------------------------------------------------------- estimate
// Per hypercube (Sec. 2.1 Eq. sigest per hypercube, Sec. 3 step 2):
// m = Omega S1 / n, var = max(0, Omega^2 S2 / n - m^2); the iteration takes
// I = sum m and V = sum var / (n - 1); the allocation takes
// d = sqrt(var)^beta (1 when beta = 0).  For beta a multiple of 1/4 up to 1
// (the paper uses 3/4) the power is taken by square roots -- the same value
// in exact arithmetic, within two ulps of pow, at a fraction of its cost.
// quarter: 4 beta when that is 1, 2, 3 or 4; else 0 (use pow).
__device__ __forceinline__ void hypercube_terms(double s1, double s2, int32_t n_i, double omega,
                                                double omega2, double beta, int quarter, double* m_out,
                                                double* var_out, double* d_out)
{
    const double n = (double)n_i;
    const double m = (omega * s1) / n;
    double var = (omega2 * s2) / n - m * m;
    if (var < 0.0) var = 0.0;
    *m_out = m;
    *var_out = var;
    if (beta == 0.0) {
        *d_out = 1.0;
    } else if (quarter) {
        const double r1 = sqrt(var), r2 = sqrt(r1), r4 = sqrt(r2);  // sigma, sigma^(1/2), sigma^(1/4)
        *d_out = quarter == 4 ? r1 : (quarter == 3 ? r2 * r4 : (quarter == 2 ? r2 : r4));
    } else {
        *d_out = pow(sqrt(var), beta);
    }
}

__device__ __forceinline__ int beta_quarter(double beta)
{
    const double b4 = 4.0 * beta;
    return (b4 == 1.0 || b4 == 2.0 || b4 == 3.0 || b4 == 4.0) ? (int)b4 : 0;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) v = v + __shfl_down(v, d);
    return v;
}

__global__ __launch_bounds__(kRedBlock) void k_est_partial(LaunchSet L)
{
    VP_REQ_PROLOGUE(L);
    const int32_t* __restrict__ n_h = q.n_h;
    const double* __restrict__ S1 = q.S1;
    const double* __restrict__ S2 = q.S2;
    const int64_t n_hc = q.n_hc;
    const double omega = q.omega, omega2 = q.omega2, beta = q.beta;
    double* __restrict__ part = q.est_part;
    double* __restrict__ dh = q.dh;
    const int quarter = beta_quarter(beta);
    double I = 0.0, V = 0.0, Sd = 0.0;
    // hypercubes in pairs, moved by 16-byte loads and stores (the arrays are
    // 256-byte aligned); an odd last hypercube goes to the grid's first thread
    auto term = [&](double s1, double s2, int32_t n) {
        double m, var, d;
        hypercube_terms(s1, s2, n, omega, omega2, beta, quarter, &m, &var, &d);
        I = I + m;
        V = V + var / ((double)n - 1.0);
        Sd = Sd + d;
        return d;
    };
    const int64_t np = n_hc / 2;
    const int2* __restrict__ n2 = reinterpret_cast<const int2*>(n_h);
    const double2* __restrict__ a2 = reinterpret_cast<const double2*>(S1);
    const double2* __restrict__ b2 = reinterpret_cast<const double2*>(S2);
    double2* __restrict__ d2 = reinterpret_cast<double2*>(dh);
#pragma unroll 2
    for (int64_t i = (int64_t)bid * blockDim.x + threadIdx.x; i < np; i += (int64_t)nblk * blockDim.x) {
        const int2 n = n2[i];
        const double2 a = a2[i], b = b2[i];
        const double d0 = term(a.x, b.x, n.x);
        const double d1 = term(a.y, b.y, n.y);
        d2[i] = make_double2(d0, d1);
    }
    if ((n_hc & 1) && bid == 0 && threadIdx.x == 0) dh[n_hc - 1] = term(S1[n_hc - 1], S2[n_hc - 1], n_h[n_hc - 1]);
    __shared__ double red[3][kRedBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    I = wave_sum(I);
    V = wave_sum(V);
    Sd = wave_sum(Sd);
    if (lane == 0) {
        red[0][w] = I;
        red[1][w] = V;
        red[2][w] = Sd;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0, c = 0.0;
        for (int i = 0; i < kRedBlock / kWave; ++i) {
            a = a + red[0][i];
            b = b + red[1][i];
            c = c + red[2][i];
        }
        part[3 * bid + 0] = a;
        part[3 * bid + 1] = b;
        part[3 * bid + 2] = c;
    }
}

// Adaptation ends after the first n_adapt iterations (Sec. 2.5: the map and
// the allocation are frozen so that later estimates are independent of one
// another's fluctuations).
__device__ __forceinline__ bool frozen(const ReqArgs& q)
{
    return q.n_adapt > 0 && q.s.it >= (uint32_t)q.n_adapt;
}

// Totals over the partials (one block, fixed tree order), the iteration's
// record, and the combination over iterations n_discard..it (Sec. 2.5):
// inverse-variance weighted, or the unweighted mean with the mean sigma_j
// over sqrt(count) as its error.
__global__ __launch_bounds__(kRedBlock) void k_est_final(LaunchSet L)
{
    VP_REQ_PROLOGUE(L);
    const double* __restrict__ part = q.est_part;
    const int n_part = q.est_blocks;
    DevState* st = q.st;
    double* __restrict__ hist_I = q.hist_I;
    double* __restrict__ hist_V = q.hist_V;
    const int64_t* __restrict__ loc = q.offs;
    const int64_t* __restrict__ bbase = q.bsum;
    const int64_t n_hc = q.n_hc;
    const int32_t it_slot = q.slot;
    const int32_t n_discard = q.n_discard;
    // thread t sums partials t, t + blockDim, ... (coalesced reads, fixed order)
    double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll 8
    for (int p = threadIdx.x; p < n_part; p += kRedBlock) {
        a = a + part[3 * p + 0];
        b = b + part[3 * p + 1];
        c = c + part[3 * p + 2];
    }
    __shared__ double red[3][kRedBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    if (lane == 0) {
        red[0][w] = a;
        red[1][w] = b;
        red[2][w] = c;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double I = 0.0, V = 0.0, Sd = 0.0;
    for (int i = 0; i < kRedBlock / kWave; ++i) {
        I = I + red[0][i];
        V = V + red[1][i];
        Sd = Sd + red[2][i];
    }
    st->sumd = Sd;
    hist_I[it_slot] = I;
    hist_V[it_slot] = V;
    st->n_iter_done = it_slot + 1;
    st->n_evals += loc[n_hc] + bbase[n_hc / kScanTile];
    const int first = n_discard < 0 ? 0 : n_discard;
    const int n = it_slot + 1;
    const int cnt = n - first;
    if (cnt <= 0) {
        st->mean = __builtin_nan("");
        st->sdev = __builtin_nan("");
        st->chi2 = __builtin_nan("");
        st->dof = 0;
        return;
    }
    st->dof = cnt - 1;
    bool zero = false;
    for (int j = first; j < n; ++j)
        if (!(hist_V[j] > 0.0)) zero = true;
    if (q.average == 1) {
        double s = 0.0, ss = 0.0;
        for (int j = first; j < n; ++j) {
            s = s + hist_I[j];
            ss = ss + sqrt(hist_V[j]);
        }
        const double m = s / (double)cnt;
        double c2 = 0.0;
        for (int j = first; j < n; ++j) {
            const double sig = sqrt(hist_V[j]);
            const double r = hist_I[j] - m;
            c2 = c2 + r * r / (sig * sig);
        }
        st->mean = m;
        st->sdev = (ss / (double)cnt) / sqrt((double)cnt);
        st->chi2 = zero ? __builtin_nan("") : c2;
        return;
    }
    if (zero) {
        double s = 0.0;
        for (int j = first; j < n; ++j) s = s + hist_I[j];
        st->mean = s / (double)cnt;
        st->sdev = 0.0;
        st->chi2 = __builtin_nan("");
        return;
    }
    double sw = 0.0, swi = 0.0;
    for (int j = first; j < n; ++j) {
        const double sig = sqrt(hist_V[j]);
        const double w = 1.0 / (sig * sig);
        sw = sw + w;
        swi = swi + hist_I[j] * w;
    }
    const double m = swi / sw;
    double c2 = 0.0;
    for (int j = first; j < n; ++j) {
        const double sig = sqrt(hist_V[j]);
        const double r = hist_I[j] - m;
        c2 = c2 + r * r / (sig * sig);
    }
    st->mean = m;
    st->sdev = 1.0 / sqrt(sw);
    st->chi2 = c2;
}

// ---------------------------------------------------------------- reallocation
// Sec. 3 steps 3-4: n_h = max(2, floor(N_ev d_h / sum d)), or floor(.) + 2.
// Near-ties (within 1e-9 relative of an integer that decides n_h) are counted.
__global__ __launch_bounds__(kRedBlock) void k_realloc(LaunchSet L)
{
    VP_REQ_PROLOGUE(L);
    int32_t* __restrict__ n_h = q.n_h;
    const double* __restrict__ dh = q.dh;
    const int64_t n_hc = q.n_hc;
    const double n_ev = q.n_ev;
    const int32_t plus2 = q.plus2;
    const DevState* __restrict__ st = q.st;
    unsigned long long* __restrict__ ties = &q.st->ties;
    const double sumd = st->sumd;
    if (!(sumd > 0.0) || frozen(q)) return;
    unsigned long long nt = 0;
    const double first_visible = plus2 ? 1.0 : 3.0;
    auto count = [&](double d) {
        const double qv = n_ev * (d / sumd);
        const double fl = floor(qv);
        const double r = rint(qv);
        const double tol = 1e-9 * (qv > 1.0 ? qv : 1.0);
        if (r >= first_visible && fabs(qv - r) <= tol) ++nt;
        int64_t n = (int64_t)fl;
        if (plus2) n = n + 2;
        else if (n < 2) n = 2;
        if (n > 2147483647) n = 2147483647;
        return (int32_t)n;
    };
    // hypercubes in pairs (16-byte loads, 8-byte stores), as in k_est_partial
    const int64_t np = n_hc / 2;
    const double2* __restrict__ d2 = reinterpret_cast<const double2*>(dh);
    int2* __restrict__ o2 = reinterpret_cast<int2*>(n_h);
#pragma unroll 2
    for (int64_t i = (int64_t)bid * blockDim.x + threadIdx.x; i < np; i += (int64_t)nblk * blockDim.x) {
        const double2 d = d2[i];
        int2 o;
        o.x = count(d.x);
        o.y = count(d.y);
        o2[i] = o;
    }
    if ((n_hc & 1) && bid == 0 && threadIdx.x == 0) n_h[n_hc - 1] = count(dh[n_hc - 1]);
    for (int d = kWave / 2; d >= 1; d >>= 1) nt += __shfl_down(nt, d);
    if ((threadIdx.x & (kWave - 1)) == 0 && nt) atomicAdd(ties, nt);
}

// ---------------------------------------------------------------- refinement
// Double-double arithmetic (Dekker / Knuth error-free sums) for sums and
// prefix sums of non-negative terms: the refinement's sums are taken to
// within about one rounding of the exact value.
struct DD {
    double hi, lo;
};

__device__ __forceinline__ DD dd_from(double a) { return DD{a, 0.0}; }

__device__ __forceinline__ DD dd_add(DD a, DD b)
{
    const double s = a.hi + b.hi;
    const double bp = s - a.hi;
    const double e = (a.hi - (s - bp)) + (b.hi - bp);
    const double lo = e + (a.lo + b.lo);
    const double r = s + lo;
    return DD{r, lo - (r - s)};
}

__device__ __forceinline__ bool dd_ge(DD a, DD b) { return a.hi > b.hi || (a.hi == b.hi && a.lo >= b.lo); }

// a - b rounded to double
__device__ __forceinline__ double dd_sub_to_d(DD a, DD b)
{
    const double s = a.hi - b.hi;
    const double bp = s - a.hi;
    const double e = (a.hi - (s - bp)) + (-b.hi - bp);
    return s + (e + (a.lo - b.lo));
}

// Block-wide sum of per-thread double-doubles (fixed tree order); every
// thread receives the total.
__device__ DD block_dd_sum(DD v, DD* scratch)
{
    scratch[threadIdx.x] = v;
    __syncthreads();
    for (int d = kRefineBlock / 2; d >= 1; d >>= 1) {
        if ((int)threadIdx.x < d) scratch[threadIdx.x] = dd_add(scratch[threadIdx.x], scratch[threadIdx.x + d]);
        __syncthreads();
    }
    const DD t = scratch[0];
    __syncthreads();
    return t;
}

// One workgroup per axis (Sec. 2.3): d_i = H_i / W_i (0 without samples);
// smoothing (7,1)/8, (1,6,1)/8, (1,7)/8 and division by sum d_i; compression
// ((1 - d) / ln(1/d))^alpha (0 at d = 0); then the regrid that gives every new
// increment an equal share delta_d = sum c / N_g of the compressed data.  The
// regrid walk (add old increments until the running sum reaches delta_d, take
// delta_d off, interpolate inside the last increment) puts new point i in the
// first old increment j where the prefix sum C_j = c_0 + ... + c_{j-1}
// reaches i delta_d, at the fraction (C_j - i delta_d) / c_{j-1} from its top;
// here every new point finds its increment by binary search over the prefix
// sums, kept in double-double so they carry no accumulated rounding.
__global__ __launch_bounds__(kRefineBlock) void k_refine(LaunchSet L)
{
    VP_REQ_PROLOGUE(L);
    double* __restrict__ map = q.map;
    float* __restrict__ map32 = q.map32;
    const double* __restrict__ H = q.H;
    const double* __restrict__ W = q.W;
    const int n_g = q.n_g;
    const double alpha = q.alpha;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    double* x = reinterpret_cast<double*>(lds_raw);  // [n_g + 1] old grid
    double* c = x + (n_g + 1);                        // [n_g]     d, then compressed d
    double* A = c + n_g;                              // [n_g + 1] smoothed d, then prefix hi
    double* Bv = A + (n_g + 1);                       // [n_g + 1] prefix lo
    __shared__ DD scratch[kRefineBlock];
    const int mu = bid;
    const int tid = threadIdx.x;
    double* xm = map + (int64_t)mu * (n_g + 1);
    float* xm32 = map32 + (int64_t)mu * (n_g + 1);
    const double* Hm = H + (int64_t)mu * n_g;
    const double* Wm = W + (int64_t)mu * n_g;
    if (alpha == 0.0 || n_g < 2 || frozen(q)) return;

    for (int i = tid; i <= n_g; i += kRefineBlock) x[i] = xm[i];
    DD part = dd_from(0.0);
    for (int i = tid; i < n_g; i += kRefineBlock) {
        const double w = Wm[i];
        const double d = (w > 0.0) ? Hm[i] / w : 0.0;
        c[i] = d;
        part = dd_add(part, dd_from(d));
    }
    const DD sd = block_dd_sum(part, scratch);
    const double s = sd.hi + sd.lo;
    if (!(s > 0.0)) return;
    for (int i = tid; i < n_g; i += kRefineBlock) {
        double v;
        if (i == 0) v = (7.0 * c[0] + c[1]) / 8.0;
        else if (i == n_g - 1) v = (c[n_g - 2] + 7.0 * c[n_g - 1]) / 8.0;
        else v = (c[i - 1] + 6.0 * c[i] + c[i + 1]) / 8.0;
        A[i] = v / s;
    }
    __syncthreads();
    // compression, and this thread's contiguous chunk of the prefix sums
    const int per = (n_g + kRefineBlock - 1) / kRefineBlock;
    const int j0 = tid * per;
    const int j1 = (j0 + per < n_g) ? j0 + per : n_g;
    for (int i = j0; i < j1; ++i) {
        const double di = A[i];
        c[i] = (di == 0.0) ? 0.0 : pow((1.0 - di) / (-log(di)), alpha);
    }
    DD tot = dd_from(0.0);
    for (int i = j0; i < j1; ++i) tot = dd_add(tot, dd_from(c[i]));
    __syncthreads();
    // exclusive scan of the chunk totals (Hillis-Steele over the block)
    scratch[tid] = tot;
    __syncthreads();
    for (int d = 1; d < kRefineBlock; d <<= 1) {
        const DD prev = (tid >= d) ? scratch[tid - d] : dd_from(0.0);
        __syncthreads();
        if (tid >= d) scratch[tid] = dd_add(prev, scratch[tid]);
        __syncthreads();
    }
    DD run = (tid > 0) ? scratch[tid - 1] : dd_from(0.0);
    const DD csum = scratch[kRefineBlock - 1];
    __syncthreads();
    // prefix sums C_j (j = 0..n_g) into (A, Bv)
    if (tid == 0) {
        A[0] = 0.0;
        Bv[0] = 0.0;
    }
    for (int i = j0; i < j1; ++i) {
        run = dd_add(run, dd_from(c[i]));
        A[i + 1] = run.hi;
        Bv[i + 1] = run.lo;
    }
    __syncthreads();
    const double delta_d = (csum.hi + csum.lo) / (double)n_g;
    if (!(delta_d > 0.0)) return;  // nothing to share out: keep the axis
    for (int i = 1 + tid; i < n_g; i += kRefineBlock) {
        // target i * delta_d exactly as a double-double
        const double th = (double)i * delta_d;
        const DD T = DD{th, fma((double)i, delta_d, -th)};
        int lo = 1, hi = n_g + 1;  // smallest j in [1, n_g] with C_j >= T, or n_g + 1
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (dd_ge(DD{A[mid], Bv[mid]}, T)) hi = mid;
            else lo = mid + 1;
        }
        double xn;
        if (lo > n_g) {
            xn = x[n_g];
        } else {
            const double S = dd_sub_to_d(DD{A[lo], Bv[lo]}, T);
            const double frac_left = (S > 0.0) ? S / c[lo - 1] : 0.0;
            xn = x[lo] - frac_left * (x[lo] - x[lo - 1]);
        }
        xm[i] = xn;
        xm32[i] = (float)xn;
    }
}

// ---------------------------------------------------------------- map training
// Preconditioned map (Sec. 5.2): training data from given points {x, f(x)}.
// A point's increment on axis mu is the last i <= N_g - 1 with x_i <= x^mu
// (inverting the map), its Jacobian the product over the axes of
// N_g Delta x_i; it adds (J f)^2 to H and 1 to W of its increment on every
// axis, so that H_i / W_i is the mean of (J f)^2 over the points there.  One
// thread per point; x is [dim][n] or [n][dim] (strides in TrainArgs).
__device__ __forceinline__ int map_locate(const double* __restrict__ xm, int n_g, double x)
{
    int lo = 0, hi = n_g - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (xm[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_train_hist(TrainArgs a)
{
    const int n_g = a.n_g, D = a.dim;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < a.n; s += stride) {
        double jac = 1.0;
        for (int mu = 0; mu < D; ++mu) {
            const double* xm = a.map + (int64_t)mu * (n_g + 1);
            const int i = map_locate(xm, n_g, a.x[(int64_t)mu * a.x_mu + s * a.x_s]);
            jac = jac * ((double)n_g * (xm[i + 1] - xm[i]));
        }
        const double v = jac * a.f[s];
        const double v2 = v * v;
        for (int mu = 0; mu < D; ++mu) {
            const double* xm = a.map + (int64_t)mu * (n_g + 1);
            const int i = map_locate(xm, n_g, a.x[(int64_t)mu * a.x_mu + s * a.x_s]);
            atomicAdd(&a.H[(int64_t)mu * n_g + i], v2);
            atomicAdd(&a.W[(int64_t)mu * n_g + i], 1.0);
        }
    }
}

// ---------------------------------------------------------------- vector integrands
// Component pair (a, b), a <= b, of pair index p: (0,0), (0,1), .., (0,M-1),
// (1,1), ..
__device__ __forceinline__ void vec_pair(int p, int m, int& a, int& b)
{
    a = 0;
    while (p >= m - a) {
        p -= m - a;
        ++a;
    }
    b = a + p;
}

// One thread per hypercube and one grid row per pair of components: the
// hypercube's sums S1_a, S1_b, S2_ab over its samples, its covariance term
// (Omega^2 S2_ab / n - (Omega S1_a / n)(Omega S1_b / n)) / (n - 1), at least 0
// on the diagonal (the multivariable form of Eq. sigest), and on the diagonal
// its estimate term Omega S1_a / n; block sums in a fixed tree order.
__global__ __launch_bounds__(kVecBlock) void k_vec_partial(VecArgs a)
{
    const int p = blockIdx.y;
    int ia, ib;
    vec_pair(p, a.n_out, ia, ib);
    const int64_t n_tot = gofs(a.offs, a.obase, a.n_hc);
    // the user's function wrote component c of sample s at c * n_tot + s
    const double* __restrict__ fa = a.f + (int64_t)ia * n_tot;
    const double* __restrict__ fb = a.f + (int64_t)ib * n_tot;
    double c = 0.0, t = 0.0;
    for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < a.n_hc;
         h += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o0 = gofs(a.offs, a.obase, h), o1 = gofs(a.offs, a.obase, h + 1);
        double s1a = 0.0, s1b = 0.0, s2 = 0.0;
        for (int64_t s = o0; s < o1; ++s) {
            const int64_t pos = batch_pos(s, n_tot);
            const double J = a.jac[pos];
            const double va = J * (a.scale * fa[pos]);
            const double vb = J * (a.scale * fb[pos]);
            s1a = s1a + va;
            s1b = s1b + vb;
            s2 = s2 + va * vb;
        }
        const double n = (double)(o1 - o0);
        const double ma = a.omega * s1a / n, mb = a.omega * s1b / n;
        double cab = (a.omega2 * s2 / n - ma * mb) / (n - 1.0);
        if (ia == ib && !(cab > 0.0)) cab = 0.0;
        c = c + cab;
        t = t + ma;
    }
    __shared__ double red[2][kVecBlock];
    red[0][threadIdx.x] = c;
    red[1][threadIdx.x] = t;
    __syncthreads();
    for (int d = kVecBlock / 2; d >= 1; d >>= 1) {
        if ((int)threadIdx.x < d) {
            red[0][threadIdx.x] = red[0][threadIdx.x] + red[0][threadIdx.x + d];
            red[1][threadIdx.x] = red[1][threadIdx.x] + red[1][threadIdx.x + d];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.part[(int64_t)p * a.grid + blockIdx.x] = red[0][0];
        if (ia == ib) a.part[(int64_t)(vec_pairs(a.n_out) + ia) * a.grid + blockIdx.x] = red[1][0];
    }
}

// Cholesky factor of the m x m matrix A (row-major) into L; false when a
// pivot is not above 1e-14 of its diagonal entry (not positive definite to
// working precision).
__device__ bool vec_chol(const double* A, double* L, int m)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = A[i * m + j];
            for (int k = 0; k < j; ++k) s = s - L[i * m + k] * L[j * m + k];
            if (i == j) {
                if (!(s > 1e-14 * A[i * m + i])) return false;
                L[i * m + i] = sqrt(s);
            } else {
                L[i * m + j] = s / L[j * m + j];
            }
        }
    return true;
}

// A^-1 from its Cholesky factor L (columns by forward and back substitution).
__device__ void vec_inv(const double* L, double* X, double* y, int m)
{
    for (int c = 0; c < m; ++c) {
        for (int i = 0; i < m; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) s = s - L[i * m + k] * y[k];
            y[i] = s / L[i * m + i];
        }
        for (int i = m - 1; i >= 0; --i) {
            double s = y[i];
            for (int k = i + 1; k < m; ++k) s = s - L[k * m + i] * X[k * m + c];
            X[i * m + c] = s / L[i * m + i];
        }
    }
}

// d^T W d for the m x m matrix W.
__device__ double vec_quad(const double* W, const double* d, int m)
{
    double q = 0.0;
    for (int i = 0; i < m; ++i) {
        double r = 0.0;
        for (int j = 0; j < m; ++j) r = r + W[i * m + j] * d[j];
        q = q + d[i] * r;
    }
    return q;
}

// Totals of the partials (one block, fixed order), the iteration's record,
// and the combination over iterations n_discard..slot: inverse-covariance
// weighted (Sec. 2.5 for several correlated estimates) or unweighted.
__global__ __launch_bounds__(kVecBlock) void k_vec_final(VecArgs a)
{
    const int m = a.n_out, np = vec_pairs(m), nt = np + m;
    __shared__ double tot[kMaxOut * (kMaxOut + 1) / 2 + kMaxOut];
    for (int e = threadIdx.x; e < nt; e += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < a.grid; ++b) s = s + a.part[(int64_t)e * a.grid + b];
        tot[e] = s;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double* hI = a.hist_I + (int64_t)a.slot * m;
    double* hC = a.hist_C + (int64_t)a.slot * m * m;
    for (int p = 0; p < np; ++p) {
        int i, j;
        vec_pair(p, m, i, j);
        hC[i * m + j] = tot[p];
        hC[j * m + i] = tot[p];
    }
    for (int i = 0; i < m; ++i) hI[i] = tot[np + i];

    __shared__ double L[kMaxOut * kMaxOut], W[kMaxOut * kMaxOut], SW[kMaxOut * kMaxOut];
    __shared__ double SWI[kMaxOut], y[kMaxOut], d[kMaxOut];
    double* mean = a.out;
    double* cov = a.out + m;
    double* chi2 = a.out + m + m * m;
    double* dof = chi2 + 1;
    const int first = a.n_discard < 0 ? 0 : a.n_discard;
    const int cnt = a.slot + 1 - first;
    if (cnt <= 0) {
        for (int i = 0; i < m + m * m + 1; ++i) a.out[i] = __builtin_nan("");
        *dof = 0.0;
        return;
    }
    *dof = (double)((cnt - 1) * m);
    bool pd = true;
    for (int j = first; j <= a.slot && pd; ++j) pd = vec_chol(a.hist_C + (int64_t)j * m * m, L, m);
    if (a.average == 0 && pd) {
        for (int i = 0; i < m * m; ++i) SW[i] = 0.0;
        for (int i = 0; i < m; ++i) SWI[i] = 0.0;
        for (int j = first; j <= a.slot; ++j) {
            (void)vec_chol(a.hist_C + (int64_t)j * m * m, L, m);
            vec_inv(L, W, y, m);
            const double* Ij = a.hist_I + (int64_t)j * m;
            for (int r = 0; r < m; ++r) {
                double s = 0.0;
                for (int c = 0; c < m; ++c) {
                    SW[r * m + c] = SW[r * m + c] + W[r * m + c];
                    s = s + W[r * m + c] * Ij[c];
                }
                SWI[r] = SWI[r] + s;
            }
        }
        if (vec_chol(SW, L, m)) {
            vec_inv(L, cov, y, m);
            for (int r = 0; r < m; ++r) {
                double s = 0.0;
                for (int c = 0; c < m; ++c) s = s + cov[r * m + c] * SWI[c];
                mean[r] = s;
            }
        } else {
            pd = false;
        }
    }
    if (a.average != 0 || !pd) {
        for (int r = 0; r < m; ++r) {
            double s = 0.0;
            for (int j = first; j <= a.slot; ++j) s = s + a.hist_I[(int64_t)j * m + r];
            mean[r] = s / (double)cnt;
        }
        for (int e = 0; e < m * m; ++e) {
            double s = 0.0;
            for (int j = first; j <= a.slot; ++j) s = s + a.hist_C[(int64_t)j * m * m + e];
            cov[e] = s / ((double)cnt * (double)cnt);
        }
    }
    if (!pd) {
        *chi2 = __builtin_nan("");
        return;
    }
    double c2 = 0.0;
    for (int j = first; j <= a.slot; ++j) {
        (void)vec_chol(a.hist_C + (int64_t)j * m * m, L, m);
        vec_inv(L, W, y, m);
        for (int r = 0; r < m; ++r) d[r] = a.hist_I[(int64_t)j * m + r] - mean[r];
        c2 = c2 + vec_quad(W, d, m);
    }
    *chi2 = c2;
}

// ---------------------------------------------------------------- invariant checks
// The state an iteration starts from, after the allocation scan: every map
// point finite and every axis strictly increasing from the box's lower to its
// upper end (the map of Sec. 2.2), every n_h >= 2 (Sec. 3), and the scanned
// total equal to sum n_h and at most n_ev + 2 N_hc.  Workgroups OR their
// findings and add their share of sum n_h into the problem's state; the last
// one to finish compares the sum, records the findings with the iteration
// index and clears the running fields for the next launch.
__global__ __launch_bounds__(kCheckBlock) void k_check(LaunchSet L)
{
    VP_REQ_PROLOGUE(L);
    __shared__ unsigned long long wsum[kCheckBlock / kWave];
    __shared__ unsigned int wbad[kCheckBlock / kWave];
    __shared__ bool last;
    const int D = q.dim, NG = q.n_g;
    const int64_t nm = (int64_t)D * (NG + 1);
    const int64_t n = nm > q.n_hc ? nm : q.n_hc;
    const double* __restrict__ map = q.map;
    const int32_t* __restrict__ nh = q.n_h;
    unsigned int bad = 0;
    unsigned long long sum = 0;
    for (int64_t i = (int64_t)bid * blockDim.x + threadIdx.x; i < n; i += (int64_t)nblk * blockDim.x) {
        if (i < nm) {
            const int d = (int)(i / (NG + 1));
            const int k = (int)(i - (int64_t)d * (NG + 1));
            const double v = map[i];
            if (!isfinite(v) || (k > 0 && !(v > map[i - 1]))) bad |= CHECK_MAP_ORDER;
            if ((k == 0 && v != q.bounds[d]) || (k == NG && v != q.bounds[D + d])) bad |= CHECK_MAP_ENDS;
        }
        if (i < q.n_hc) {
            const int32_t c = nh[i];
            if (c < 2) bad |= CHECK_NH_MIN;
            sum += (unsigned long long)(c > 0 ? c : 0);
        }
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        sum += (unsigned long long)__shfl_xor((long long)sum, o);
        bad |= (unsigned int)__shfl_xor((int)bad, o);
    }
    if (lane == 0) {
        wsum[w] = sum;
        wbad[w] = bad;
    }
    __syncthreads();
    DevState* st = q.st;
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        unsigned int b = 0;
        for (int i = 0; i < kCheckBlock / kWave; ++i) {
            s += wsum[i];
            b |= wbad[i];
        }
        atomicAdd(&st->check_sum, s);
        if (b) atomicOr(&st->check_pending, b);
        __threadfence();
        last = atomicAdd(&st->check_ticket, 1u) == (unsigned int)nblk - 1;
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
        __threadfence();
        const unsigned long long total = atomicAdd(&st->check_sum, 0ull);
        unsigned int b = atomicOr(&st->check_pending, 0u);
        const int64_t scanned = gofs(q.offs, q.bsum, q.n_hc);
        if ((unsigned long long)scanned != total || (double)scanned > q.n_ev + 2.0 * (double)q.n_hc)
            b |= CHECK_NH_SUM;
        if (b) {
            if (st->check_flags == 0) st->check_it = q.s.it;
            st->check_flags |= b;
        }
        st->check_sum = 0;
        st->check_pending = 0;
        st->check_ticket = 0;
    }
}

// ---------------------------------------------------------------- advance
// End of an iteration: the next iteration's Philox counter and history slot.
__global__ void k_advance(LaunchSet L)
{
    VP_REQ_PROLOGUE(L);
    if (threadIdx.x == 0) {
        q.s.it += 1;
        q.slot += 1;
    }
}

// ---------------------------------------------------------------- launchers
static void launch(void (*k)(LaunchSet), const LaunchSet& L, int blocks, int threads, size_t lds,
                   hipStream_t s)
{
    if (blocks > 0) hipLaunchKernelGGL(k, dim3(blocks), dim3(threads), lds, s, L);
}

hipError_t aux_init(size_t lds_max)
{
    hipError_t e = hipFuncSetAttribute((const void*)k_refine, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)((4 * kMaxNg + 3) * sizeof(double)));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_hist_records, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds_max);
    return e;
}

void enqueue_head(const IterPlan& P, hipStream_t s)
{
    launch(k_scan_local, P.scan_local, P.n_scan_local, kScanBlock, 0, s);
    launch(k_scan_top, P.one, P.n_one, kScanBlock, 0, s);
    launch(k_check, P.check, P.n_check, kCheckBlock, 0, s);
}

void enqueue_iteration(const IterPlan& P, hipStream_t s, hipEvent_t sample_begin, hipEvent_t sample_end,
                       const SideStreams* side)
{
    enqueue_head(P, s);
    if (sample_begin) (void)hipEventRecord(sample_begin, s);
    const int ns = side ? std::min(side->n, P.n_groups - 1) : 0;
    if (ns > 0) {
        // groups go to the stream with the fewest workgroups so far, largest first
        (void)hipEventRecord(side->fork, s);
        for (int i = 0; i < ns; ++i) (void)hipStreamWaitEvent(side->st[i], side->fork, 0);
        int order[kMaxGroups];
        for (int g = 0; g < P.n_groups; ++g) order[g] = g;
        std::sort(order, order + P.n_groups, [&](int a, int b) { return P.groups[a].blocks > P.groups[b].blocks; });
        int64_t load[kMaxSide + 1] = {};
        for (int o = 0; o < P.n_groups; ++o) {
            const SampleGroup& G = P.groups[order[o]];
            int best = 0;
            for (int i = 1; i <= ns; ++i)
                if (load[i] < load[best]) best = i;
            load[best] += G.blocks;
            G.entry.launch(G.L, G.blocks, G.entry.block, G.lds, best == 0 ? s : side->st[best - 1]);
        }
        for (int i = 0; i < ns; ++i) {
            (void)hipEventRecord(side->join[i], side->st[i]);
            (void)hipStreamWaitEvent(s, side->join[i], 0);
        }
    } else {
        for (int g = 0; g < P.n_groups; ++g)
            P.groups[g].entry.launch(P.groups[g].L, P.groups[g].blocks, P.groups[g].entry.block, P.groups[g].lds, s);
    }
    if (sample_end) (void)hipEventRecord(sample_end, s);
    enqueue_tail(P, s, side);
}

void enqueue_tail(const IterPlan& P, hipStream_t s, const SideStreams* side)
{
    const size_t refine_lds = (size_t)(4 * P.max_ng + 3) * sizeof(double);
    if (side && side->n > 0) {
        hipStream_t m = side->st[0];
        (void)hipEventRecord(side->fork, s);
        (void)hipStreamWaitEvent(m, side->fork, 0);
        launch(k_hist_records, P.rec, P.n_rec, kRecBlock, P.rec_lds, m);
        launch(k_hist_records, P.rec_det, P.n_rec_det, kRecDetBlock, P.rec_lds, m);
        launch(k_hist_reduce, P.hist, P.n_hist, kHistBlock, 0, m);
        launch(k_refine, P.refine, P.n_refine, kRefineBlock, refine_lds, m);
        (void)hipEventRecord(side->join[0], m);
        launch(k_edge_fixup<kFixBlock>, P.fixup, P.n_fixup, kFixBlock, 0, s);
        launch(k_edge_fixup<kFixSmallBlock>, P.fixup_s, P.n_fixup_s, kFixSmallBlock, 0, s);
        launch(k_est_partial, P.est, P.n_est, kRedBlock, 0, s);
        launch(k_est_final, P.one, P.n_one, kRedBlock, 0, s);
        launch(k_realloc, P.est, P.n_est, kRedBlock, 0, s);
        (void)hipStreamWaitEvent(s, side->join[0], 0);
        launch(k_advance, P.one, P.n_one, 64, 0, s);
        return;
    }
    launch(k_hist_records, P.rec, P.n_rec, kRecBlock, P.rec_lds, s);
    launch(k_hist_records, P.rec_det, P.n_rec_det, kRecDetBlock, P.rec_lds, s);
    launch(k_edge_fixup<kFixBlock>, P.fixup, P.n_fixup, kFixBlock, 0, s);
    launch(k_edge_fixup<kFixSmallBlock>, P.fixup_s, P.n_fixup_s, kFixSmallBlock, 0, s);
    launch(k_hist_reduce, P.hist, P.n_hist, kHistBlock, 0, s);
    launch(k_est_partial, P.est, P.n_est, kRedBlock, 0, s);
    launch(k_est_final, P.one, P.n_one, kRedBlock, 0, s);
    launch(k_realloc, P.est, P.n_est, kRedBlock, 0, s);
    launch(k_refine, P.refine, P.n_refine, kRefineBlock, refine_lds, s);
    launch(k_advance, P.one, P.n_one, 64, 0, s);
}

void launch_fill_f64(double* x, int64_t n, double v, hipStream_t s)
{
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)g), dim3(256), 0, s, x, n, v);
}

void launch_fill_i32(int32_t* x, int64_t n, int32_t v, hipStream_t s)
{
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)g), dim3(256), 0, s, x, n, v);
}

void launch_train_hist(const TrainArgs& a, hipStream_t s)
{
    int64_t g = (a.n + 255) / 256;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_train_hist, dim3((unsigned)g), dim3(256), 0, s, a);
}

void launch_refine(const LaunchSet& L, int blocks, int max_ng, hipStream_t s)
{
    launch(k_refine, L, blocks, kRefineBlock, (size_t)(4 * max_ng + 3) * sizeof(double), s);
}

int vec_grid(int64_t n_hc)
{
    int64_t g = (n_hc + kVecBlock - 1) / kVecBlock;
    if (g > kVecMaxGrid) g = kVecMaxGrid;
    return (int)(g < 1 ? 1 : g);
}

void launch_vec(const VecArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_vec_partial, dim3((unsigned)a.grid, (unsigned)vec_pairs(a.n_out)), dim3(kVecBlock), 0, s,
                       a);
    hipLaunchKernelGGL(k_vec_final, dim3(1), dim3(kVecBlock), 0, s, a);
}

int est_grid(int64_t n_hc)
{
    // about 16 hypercubes per thread: small served requests launch few workgroups
    int64_t g = (n_hc + 16 * kRedBlock - 1) / (16 * kRedBlock);
    if (g > kRedMaxGrid) g = kRedMaxGrid;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace vp

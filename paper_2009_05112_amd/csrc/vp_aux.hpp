// vp_aux.hpp -- launchers of the per-hypercube and per-increment kernels.
#pragma once

#include "vp_internal.hpp"

namespace vp {

constexpr int kScanBlock = 1024;
constexpr int kScanPer = 4;
constexpr int kScanTile = kScanBlock * kScanPer;
static_assert(kScanTile == kOffsTile, "scan tile and offset blocks must agree");
constexpr int kRedBlock = 256;
constexpr int kRedMaxGrid = 16384;
constexpr int kRefineBlock = 256;

// Device-resident scalars of one problem.
struct DevState {
    double sumd;                 // sum of d_h of the last iteration
    double mean, sdev, chi2;     // combined estimate
    int64_t n_evals;             // samples drawn over all iterations
    int32_t n_iter_done;
    int32_t dof;
    unsigned long long ties;     // near-ties in reallocation
    unsigned long long nonfinite;
};

void launch_scan(const int32_t* n_h, int64_t n_hc, int64_t* offs, int64_t* bsum, hipStream_t s);
inline int64_t scan_blocks(int64_t n_hc) { return (n_hc + kScanTile - 1) / kScanTile; }
void launch_edge_fixup(const EdgeRec* e, int64_t n_rec, double* S1, double* S2, hipStream_t s);
void launch_hist_reduce(const double* part, int n_part, int64_t nbins, double* H, double* W,
                        hipStream_t s);
void launch_fill_f64(double* x, int64_t n, double v, hipStream_t s);
void launch_fill_i32(int32_t* x, int64_t n, int32_t v, hipStream_t s);
int est_grid(int64_t n_hc);
void launch_estimate(const int32_t* n_h, const double* S1, const double* S2, int64_t n_hc,
                     double omega, double omega2, double beta, double* part, double* dh, DevState* st,
                     double* hist_I, double* hist_V, const int64_t* loc, const int64_t* bbase,
                     int32_t it_slot, int32_t n_discard, hipStream_t s);
void launch_realloc(int32_t* n_h, const double* dh, int64_t n_hc, double n_ev, int32_t plus2,
                    const DevState* st, unsigned long long* ties, hipStream_t s);
void launch_refine(double* map, float* map32, const double* H, const double* W, int dim, int n_g,
                   double alpha, hipStream_t s);

}  // namespace vp

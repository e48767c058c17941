// Host-side launchers of the library's kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.h"

namespace gabp {

// dtype: 0 = FP32 message planes, 1 = FP64.
// rpt: rows per thread of the iteration kernel's tile (1, 2, 4 or 8); every
// choice gives bitwise-identical results.
constexpr int kRptChoices[] = {1, 2, 4, 8};
// The iteration kernels number their iterations t = *t_base + t_off (a
// device counter, so that a captured graph numbers replays correctly); flag
// receives the first diverged iteration.
hipError_t launch_iter(int dtype, int rpt, const Lattice &L, const void *m_in, void *m_out,
                       const void *adiag, const void *bw, double eta, uint32_t *flag,
                       const uint32_t *t_base, uint32_t t_off, hipStream_t s);
// Information-only iteration with precomputed edge gains (after the
// precision messages froze), the gain set-up and a bitwise-change test.
hipError_t launch_iter_theta(int dtype, int rpt, const Lattice &L, const void *m_in,
                             void *m_out, const void *gain, const void *bw, double eta,
                             uint32_t *flag, const uint32_t *t_base, uint32_t t_off,
                             hipStream_t s);
// Two information-only iterations (t+1 and t+2) per launch on 64 x th tiles
// (th = 4, 8, 16 or 32 for FP32, 4 for FP64); m_in and m_out must differ.
// Bitwise equal to two launch_iter_theta calls.
constexpr int kPairChoicesF32[] = {4, 8, 12, 16, 32};
hipError_t launch_iter_theta2(int dtype, int th, const Lattice &L, const void *m_in, void *m_out,
                              const void *gain, const void *bw, double eta, uint32_t *flag,
                              const uint32_t *t_base, uint32_t t_off, hipStream_t s);
// The same two iterations by the column-strip walker: persistent workgroups
// of rb waves march down 64-column strips in bands of rb rows (rb = 2, 4 or
// 8 for FP32, 2 for FP64).  Bitwise equal to two launch_iter_theta calls.
hipError_t launch_iter_theta2w(int dtype, int rb, const Lattice &L, const void *m_in,
                               void *m_out, const void *gain, const void *bw, double eta,
                               uint32_t *flag, const uint32_t *t_base, uint32_t t_off,
                               hipStream_t s);
// Device counter helpers for captured chunks (kernels, not memsets, so that
// they may sit in a graph): *p = v, and *p += k.
hipError_t launch_set_u32(uint32_t *p, uint32_t v, hipStream_t s);
hipError_t launch_add_u32(uint32_t *p, uint32_t k, hipStream_t s);
hipError_t launch_gain(int dtype, const Lattice &L, const void *m, const void *adiag, void *gain,
                       hipStream_t s);
// Precision-message change between buffers a and b (n elements): adds the
// number of bitwise differing elements to *count and raises *maxrel (float
// bits) to their largest relative change.  The caller zeroes both first.
hipError_t launch_prec_change(int dtype, const void *a, const void *b, int64_t n,
                              unsigned long long *count, uint32_t *maxrel, hipStream_t s);
// Marginals: bel64 != NULL selects the frozen-precision variant that reads
// the belief precisions from bel64; otherwise bel_out (may be NULL) receives
// them.
hipError_t launch_post(int dtype, const Lattice &L, const void *m, const double *adiag64,
                       const double *b64, const double *bel64, double *mu_plane, double *mean,
                       double *var, double *bel_out, hipStream_t s);
hipError_t launch_resid(const Lattice &L, const double *mu, const double *adiag64,
                        const double *b64, double *partials, int npart, double *out,
                        hipStream_t s);
hipError_t launch_abs_change(int dtype, const void *a, const void *b, int64_t n,
                             double *partials, int npart, double *out, hipStream_t s);
// Deterministic fold of point observations into FP64 node terms (obs.hip):
// p[i] += sum 1/s_k^2 and h[i] += sum y_k/s_k^2 over the observations of
// cell c, i = (c / nx) * pitch + c % nx, summed in input order.  Synchronises
// the stream (temporary sort buffers are freed before it returns).
hipError_t launch_obs_fold(int64_t n, const int64_t *cell, const double *y, const double *var,
                           double sigma2, int64_t ncells, int32_t nx, int32_t pitch,
                           double *p_plane, double *h_plane, uint32_t *err_flag, hipStream_t s);
hipError_t launch_setup(int dtype, const Lattice &L, int64_t nobs, const int64_t *cell,
                        const double *y, const double *var, double sigma2, double *adiag64,
                        double *b64, const double *prior_mean, void *adiag_w, void *b_w,
                        uint32_t *err_flag, hipStream_t s);
// Multigrid: bilinear upsampling of a coarse mean into a prediction.
hipError_t launch_upscale_prec(int dtype, const Lattice &Lc, const void *m, float scale,
                               float *pred, int nxf, int nyf, hipStream_t s);
// Multigrid: the coarse messages copied unchanged onto the fine grid.
hipError_t launch_copy_coarse(int dtype, const Lattice &Lc, const void *mc, const Lattice &Lf,
                              void *mf, hipStream_t s);
hipError_t launch_upsample_mean(const double *coarse, int nxc, int nyc, int perx, int pery,
                                float *pred, int nxf, int nyf, hipStream_t s);
// Message initialisation from a network prediction (net.hip).
hipError_t launch_warm_init(int dtype, const Lattice &L, const float *pred, int keep_prec,
                            void *m, hipStream_t s);
// Targets log(-Lam) and edge masks of the precision outputs (net.hip).
hipError_t launch_log_prec(int dtype, const Lattice &L, const void *m, float *lam, float *valid,
                           hipStream_t s);
hipError_t launch_msgs_get(int dtype, const Lattice &L, const void *m, void *prec, void *info,
                           hipStream_t s);
hipError_t launch_msgs_set(int dtype, const Lattice &L, void *m, const void *prec,
                           const void *info, hipStream_t s);

}  // namespace gabp

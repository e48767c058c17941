// Folding point observations into node terms (Section "Including
// Observations"): every observation k of cell c contributes w_k = 1/s_k^2 to
// the node precision p_c and w_k y_k to the node information h_c; several
// observations of one cell multiply their likelihoods, so their terms add.
//
// Deterministic: the observations are sorted by cell with a stable radix
// sort, and the thread that owns the first observation of a run sums the run
// in input order, starting from 0.  The node terms therefore do not depend on
// thread timing (floating-point atomics would), and equal a sequential sum in
// input order.  Shared by the lattice, batched and space-time set-up paths.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <hipcub/hipcub.hpp>

#include "internal.h"

#pragma clang fp contract(off)

namespace gabp {

namespace {

__global__ __launch_bounds__(256) void k_obs_index(int64_t n, int32_t *__restrict__ idx) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < n) idx[k] = (int32_t)k;
}

// Thread per sorted position s; the first of each run of equal cells sums
// the run.  Cell c maps to the pitched index (c / nx) * pitch + c % nx, which
// serves both the lattice (row y) and the space-time grid (row n * ny + y,
// slices pitch * ny apart).
__global__ __launch_bounds__(256) void k_obs_fold(int64_t n, const int64_t *__restrict__ cell_s,
                                                  const int32_t *__restrict__ idx_s,
                                                  const double *__restrict__ yv,
                                                  const double *__restrict__ var, double sigma2,
                                                  int64_t ncells, int32_t nx, int32_t pitch,
                                                  double *__restrict__ p_plane,
                                                  double *__restrict__ h_plane,
                                                  uint32_t *__restrict__ err_flag) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const int64_t c = cell_s[s];
    if (s > 0 && cell_s[s - 1] == c) return;
    if (c < 0 || c >= ncells) {
        *err_flag = 1u;
        return;
    }
    double p = 0.0, h = 0.0;
    for (int64_t r = s; r < n && cell_s[r] == c; ++r) {
        const int32_t k = idx_s[r];
        const double s2 = var ? var[k] : sigma2;
        const double y = yv[k];
        if (!(s2 > 0.0) || !isfinite(s2) || !isfinite(y)) {
            *err_flag = 1u;
            return;
        }
        const double w = 1.0 / s2;
        p += w;
        h += w * y;
    }
    const int64_t i = (c / nx) * (int64_t)pitch + c % nx;
    p_plane[i] += p;
    h_plane[i] += h;
}

}  // namespace

hipError_t launch_obs_fold(int64_t n, const int64_t *cell, const double *y, const double *var,
                           double sigma2, int64_t ncells, int32_t nx, int32_t pitch,
                           double *p_plane, double *h_plane, uint32_t *err_flag, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (n > INT32_MAX) return hipErrorInvalidValue;
    int64_t *cell_s = nullptr;
    int32_t *idx = nullptr, *idx_s = nullptr;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, cell, cell_s, idx,
                                                      idx_s, (int)n, 0, 64, s);
    if (e == hipSuccess) e = hipMalloc((void **)&cell_s, (size_t)n * sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc((void **)&idx, (size_t)n * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void **)&idx_s, (size_t)n * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&tmp, tmp_bytes > 0 ? tmp_bytes : 1);
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_obs_index, dim3(nb), dim3(256), 0, s, n, idx);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, cell, cell_s, idx, idx_s, (int)n,
                                               0, 64, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_obs_fold, dim3(nb), dim3(256), 0, s, n, (const int64_t *)cell_s,
                           (const int32_t *)idx_s, y, var, sigma2, ncells, nx, pitch, p_plane,
                           h_plane, err_flag);
        e = hipGetLastError();
    }
    const hipError_t es = hipStreamSynchronize(s);
    if (e == hipSuccess) e = es;
    (void)hipFree(cell_s);
    (void)hipFree(idx);
    (void)hipFree(idx_s);
    (void)hipFree(tmp);
    return e;
}

}  // namespace gabp

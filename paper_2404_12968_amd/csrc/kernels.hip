// gfx950 kernels of the lattice Gaussian belief propagation library.
//
// Message storage: two ping-pong buffers, each 2*deg planes (deg precision
// planes, then deg information planes) of the message precision T, receiver
// indexed: plane d at (x, y) is the message INTO (x, y) FROM (x, y) + off_d.
// Iteration t reads buffer (t-1)&1 and writes buffer t&1 (flooding schedule:
// every new message depends only on the previous iteration's messages).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "internal.h"
#include "lattice.h"

namespace gabp {

template <typename T>
__device__ __forceinline__ T recip(T v);
template <>
__device__ __forceinline__ float recip<float>(float v) {
    return __builtin_amdgcn_rcpf(v);  // 1 ulp; FP32 messages are checked at 1e-5
}
template <>
__device__ __forceinline__ double recip<double>(double v) {
    return 1.0 / v;  // correctly rounded: FP64 parity is checked at 1e-12
}

// --------------------------------------------------------------------------
// One flooding iteration, thread per node (the reference GPU formulation).
//
// Node i = (x, y) with incoming messages m_{k->i} (its own slots):
//   belief  Lam_i = A_ii + c sum_k Lam_{k->i},   th_i = b_i + c sum_k th_{k->i}
// and for every neighbour j = i + off_d (outgoing i -> j, stored at j in the
// opposite plane d^1):
//   cavity  Lam_c = Lam_i - Lam_{j->i},  th_c = th_i - th_{j->i}
//   new     Lam~ = -(Q_ij/c)^2 / Lam_c,  th~ = -(Q_ij/c) th_c / Lam_c
//   damped  m^t = (1 - eta) m^{t-1} + eta m~
// (Appendix "Re-weighted message updates" in information form; Section
// "Update Damping".)  A cavity precision <= 0 or a non-finite value records t
// in diverged_at; later launches then return at once, keeping that state.
//
// Every load of a node is issued before the first use so that a wave keeps
// ~50 loads in flight.  Workgroups whose 64x4 tile and its radius-2 halo lie
// inside the grid take the INTERIOR path with no neighbour tests; the others
// clamp addresses, predicate stores and wrap periodic axes.
// --------------------------------------------------------------------------
template <typename T, int ALPHA, bool INTERIOR>
__device__ __forceinline__ void iter_node(const Lattice &L, const T *__restrict__ m_in,
                                          T *__restrict__ m_out, const T *__restrict__ adiag,
                                          const T *__restrict__ bw, T eta,
                                          uint32_t *__restrict__ diverged_at, uint32_t t,
                                          int x, int y) {
    constexpr int DEG = ALPHA == 1 ? 4 : 12;
    const int64_t P = L.plane;
    const int64_t i = (int64_t)y * L.pitch + x;
    const T c = (T)L.c, inv_c = (T)L.inv_c, keep = (T)1 - eta;

    int64_t j[DEG];
    int xs[DEG], ys[DEG];
    bool ok[DEG];
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        int xn, yn;
        if (INTERIOR) {
            xn = x + dir_dx(d);
            yn = y + dir_dy(d);
            ok[d] = true;
        } else {
            ok[d] = neighbour(L, x, y, d, xn, yn);
            xn = min(max(xn, 0), L.nx - 1);
            yn = min(max(yn, 0), L.ny - 1);
        }
        xs[d] = xn;
        ys[d] = yn;
        j[d] = (int64_t)yn * L.pitch + xn;
    }
    T lam[DEG], th[DEG], ol[DEG], ot[DEG];
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        lam[d] = m_in[d * P + i];
        th[d] = m_in[(DEG + d) * P + i];
    }
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        ol[d] = m_in[(d ^ 1) * P + j[d]];
        ot[d] = m_in[(DEG + (d ^ 1)) * P + j[d]];
    }
    const T a = adiag[i];
    const T b = bw[i];
    T sl = 0, st = 0;
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        sl += lam[d];
        st += th[d];
    }
    const T bl = a + c * sl;
    const T bt = b + c * st;
    // near-neighbour coefficients need l at both ends (13-point prior)
    const T li = ALPHA == 2 ? ell<T>(L, x, y) : (T)0;
    bool bad = false;
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        T q;
        if (ALPHA == 1) {
            q = -(T)L.tau * (d < 2 ? (T)L.ihx2 : (T)L.ihy2);
        } else if (d < 4) {
            q = -(T)L.tau * (li + ell<T>(L, xs[d], ys[d])) * (d < 2 ? (T)L.ihx2 : (T)L.ihy2);
        } else if (d < 8) {
            q = d < 6 ? (T)(L.tau * L.ihx2 * L.ihx2) : (T)(L.tau * L.ihy2 * L.ihy2);
        } else {
            q = (T)(2.0 * L.tau * L.ihx2 * L.ihy2);
        }
        q *= inv_c;
        const T lc = bl - lam[d];
        const T tc = bt - th[d];
        const T r = recip<T>(lc);
        const T dl = keep * ol[d] + eta * (-(q * q) * r);
        const T dt = keep * ot[d] + eta * (-(q * tc) * r);
        if (ok[d]) {
            bad |= !(lc > (T)0) || !isfinite(dl) || !isfinite(dt);
            m_out[(d ^ 1) * P + j[d]] = dl;
            m_out[(DEG + (d ^ 1)) * P + j[d]] = dt;
        }
    }
    if (bad) *diverged_at = t;
}

template <typename T, int ALPHA>
__global__ __launch_bounds__(256) void k_iter_direct(Lattice L, const T *__restrict__ m_in,
                                                     T *__restrict__ m_out,
                                                     const T *__restrict__ adiag,
                                                     const T *__restrict__ bw, T eta,
                                                     uint32_t *__restrict__ diverged_at,
                                                     uint32_t t) {
    if (*diverged_at != 0u) return;
    const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int tx = tile % L.tiles_x, ty = tile / L.tiles_x;
    const int x = tx * 64 + (int)(threadIdx.x & 63u);
    const int y = ty * 4 + (int)(threadIdx.x >> 6);
    const bool interior = tx * 64 >= 2 && tx * 64 + 66 <= L.nx && ty * 4 >= 2 &&
                          ty * 4 + 6 <= L.ny;
    if (interior) {
        iter_node<T, ALPHA, true>(L, m_in, m_out, adiag, bw, eta, diverged_at, t, x, y);
    } else if (x < L.nx && y < L.ny) {
        iter_node<T, ALPHA, false>(L, m_in, m_out, adiag, bw, eta, diverged_at, t, x, y);
    }
}

// --------------------------------------------------------------------------
// Marginals (Compute Marginal) in FP64 from messages of precision T:
// Lam_i = A_ii + c sum Lam_{k->i}, th_i = b_i + c sum th_{k->i}; mu = th/Lam,
// var = 1/Lam.  Writes the pitched FP64 mean plane used by the residual and,
// when given, contiguous mean/var arrays.
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_post(Lattice L, const T *__restrict__ m,
                                              const double *__restrict__ adiag64,
                                              const double *__restrict__ b64,
                                              double *__restrict__ mu_plane,
                                              double *__restrict__ mean,
                                              double *__restrict__ var) {
    const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int x = (tile % L.tiles_x) * 64 + (int)(threadIdx.x & 63u);
    const int y = (tile / L.tiles_x) * 4 + (int)(threadIdx.x >> 6);
    if (x >= L.nx || y >= L.ny) return;
    const int64_t P = L.plane;
    const int64_t i = (int64_t)y * L.pitch + x;
    double sl = 0.0, st = 0.0;
    for (int d = 0; d < L.deg; ++d) {
        sl += (double)m[d * P + i];
        st += (double)m[(L.deg + d) * P + i];
    }
    const double bl = adiag64[i] + L.c * sl;
    const double bt = b64[i] + L.c * st;
    const double mu = bt / bl;
    if (mu_plane) mu_plane[i] = mu;
    const int64_t o = (int64_t)y * L.nx + x;
    if (mean) mean[o] = mu;
    if (var) var[o] = 1.0 / bl;
}

// --------------------------------------------------------------------------
// FP64 residual r = A mu - b of the posterior-mean equations, A = Q + diag(p).
// Each workgroup sums r^2 and b^2 over a fixed set of tiles in a fixed order
// (wave64 butterfly, then LDS across the four waves): deterministic partials.
// --------------------------------------------------------------------------
template <int ALPHA>
__global__ __launch_bounds__(256) void k_resid(Lattice L, const double *__restrict__ mu,
                                               const double *__restrict__ adiag64,
                                               const double *__restrict__ b64,
                                               double *__restrict__ partials, int ntiles) {
    constexpr int DEG = ALPHA == 1 ? 4 : 12;
    __shared__ double sh[2][4];
    double rr = 0.0, bb = 0.0;
    for (int tile = (int)blockIdx.x; tile < ntiles; tile += (int)gridDim.x) {
        const int x = (tile % L.tiles_x) * 64 + (int)(threadIdx.x & 63u);
        const int y = (tile / L.tiles_x) * 4 + (int)(threadIdx.x >> 6);
        if (x < L.nx && y < L.ny) {
            const int64_t i = (int64_t)y * L.pitch + x;
            double s = adiag64[i] * mu[i];
#pragma unroll
            for (int d = 0; d < DEG; ++d) {
                int xn, yn;
                if (!neighbour(L, x, y, d, xn, yn)) continue;
                s += q_off<double>(L, d, x, y, xn, yn) * mu[(int64_t)yn * L.pitch + xn];
            }
            const double r = s - b64[i];
            rr += r * r;
            bb += b64[i] * b64[i];
        }
    }
    rr = wave_sum(rr);
    bb = wave_sum(bb);
    const int w = (int)(threadIdx.x >> 6);
    if ((threadIdx.x & 63u) == 0u) {
        sh[0][w] = rr;
        sh[1][w] = bb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
        partials[2 * blockIdx.x + 1] = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
    }
}

// Sum of |a - b| over a flat range of message slots (the paper's early-stop
// statistic); zero slots contribute nothing.  Deterministic partials.
template <typename T>
__global__ __launch_bounds__(256) void k_abs_change(const T *__restrict__ a,
                                                    const T *__restrict__ b, int64_t n,
                                                    double *__restrict__ partials) {
    __shared__ double sh[4];
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += stride)
        s += fabs((double)a[k] - (double)b[k]);
    s = wave_sum(s);
    if ((threadIdx.x & 63u) == 0u) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
        partials[2 * blockIdx.x + 1] = 0.0;
    }
}

// Fixed-order reduction of npart (pairs of) partials into out[0..1].
__global__ __launch_bounds__(256) void k_reduce(const double *__restrict__ partials, int npart,
                                                double *__restrict__ out) {
    __shared__ double sh[2][4];
    double a = 0.0, b = 0.0;
    for (int k = (int)threadIdx.x; k < npart; k += 256) {
        a += partials[2 * k];
        b += partials[2 * k + 1];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = (int)(threadIdx.x >> 6);
    if ((threadIdx.x & 63u) == 0u) {
        sh[0][w] = a;
        sh[1][w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
        out[1] = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
    }
}

// --------------------------------------------------------------------------
// Problem setup (Section "Including Observations"): fold every observation
// into its cell's node terms, p_i += 1/s^2 and h_i += y/s^2, accumulated in
// the (zeroed) FP64 diagonal and information planes.  Out-of-range cells and
// non-finite or non-positive inputs set err_flag and are skipped.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_obs_scatter(Lattice L, int64_t n,
                                                     const int64_t *__restrict__ cell,
                                                     const double *__restrict__ yv,
                                                     const double *__restrict__ var,
                                                     double sigma2, double *__restrict__ adiag64,
                                                     double *__restrict__ b64,
                                                     uint32_t *__restrict__ err_flag) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const int64_t c = cell[k];
    const double s2 = var ? var[k] : sigma2;
    const double y = yv[k];
    const int64_t N = (int64_t)L.nx * L.ny;
    if (c < 0 || c >= N || !(s2 > 0.0) || !isfinite(s2) || !isfinite(y)) {
        *err_flag = 1u;
        return;
    }
    const int64_t x = c % L.nx, row = c / L.nx;
    const int64_t i = row * L.pitch + x;
    const double w = 1.0 / s2;
    atomicAdd(&adiag64[i], w);
    atomicAdd(&b64[i], w * y);
}

// A_ii = Q_ii + p_i in FP64, b_i (+ (Q f_b)_i for a prior mean f_b), and the
// copies in message precision that the iteration reads.
template <typename T>
__global__ __launch_bounds__(256) void k_node_init(Lattice L, double *__restrict__ adiag64,
                                                   double *__restrict__ b64,
                                                   const double *__restrict__ prior_mean,
                                                   T *__restrict__ adiag_w, T *__restrict__ b_w,
                                                   uint32_t *__restrict__ err_flag) {
    const int tile = (int)blockIdx.x;
    const int x = (tile % L.tiles_x) * 64 + (int)(threadIdx.x & 63u);
    const int y = (tile / L.tiles_x) * 4 + (int)(threadIdx.x >> 6);
    if (x >= L.nx || y >= L.ny) return;
    const int64_t i = (int64_t)y * L.pitch + x;
    const double a = q_diag<double>(L, x, y) + adiag64[i];
    double b = b64[i];
    if (prior_mean) {
        double s = q_diag<double>(L, x, y) * prior_mean[(int64_t)y * L.nx + x];
        for (int d = 0; d < L.deg; ++d) {
            int xn, yn;
            if (!neighbour(L, x, y, d, xn, yn)) continue;
            s += q_off<double>(L, d, x, y, xn, yn) * prior_mean[(int64_t)yn * L.nx + xn];
        }
        if (!isfinite(s)) *err_flag = 1u;
        b += s;
    }
    adiag64[i] = a;
    b64[i] = b;
    if (adiag_w) adiag_w[i] = (T)a;
    if (b_w) b_w[i] = (T)b;
}

// Checkpoint copies between the pitched message planes and a dense
// [deg][ny][nx] layout.  The set direction forces slots without a sender to 0.
template <typename T>
__global__ __launch_bounds__(256) void k_msgs_get(Lattice L, const T *__restrict__ m,
                                                  T *__restrict__ prec, T *__restrict__ info) {
    const int tile = (int)blockIdx.x;
    const int x = (tile % L.tiles_x) * 64 + (int)(threadIdx.x & 63u);
    const int y = (tile / L.tiles_x) * 4 + (int)(threadIdx.x >> 6);
    if (x >= L.nx || y >= L.ny) return;
    const int64_t i = (int64_t)y * L.pitch + x;
    const int64_t n = (int64_t)L.nx * L.ny, o = (int64_t)y * L.nx + x;
    for (int d = 0; d < L.deg; ++d) {
        if (prec) prec[d * n + o] = m[d * L.plane + i];
        if (info) info[d * n + o] = m[(L.deg + d) * L.plane + i];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_msgs_set(Lattice L, T *__restrict__ m,
                                                  const T *__restrict__ prec,
                                                  const T *__restrict__ info) {
    const int tile = (int)blockIdx.x;
    const int x = (tile % L.tiles_x) * 64 + (int)(threadIdx.x & 63u);
    const int y = (tile / L.tiles_x) * 4 + (int)(threadIdx.x >> 6);
    if (x >= L.nx || y >= L.ny) return;
    const int64_t i = (int64_t)y * L.pitch + x;
    const int64_t n = (int64_t)L.nx * L.ny, o = (int64_t)y * L.nx + x;
    for (int d = 0; d < L.deg; ++d) {
        int xn, yn;
        const bool ok = neighbour(L, x, y, d, xn, yn);
        if (prec) m[d * L.plane + i] = ok ? prec[d * n + o] : (T)0;
        if (info) m[(L.deg + d) * L.plane + i] = ok ? info[d * n + o] : (T)0;
    }
}

// --------------------------------------------------------------------------
// host launchers
// --------------------------------------------------------------------------
static inline int tiles_of(const Lattice &L) {
    return L.tiles_x * ((L.ny + 3) / 4);
}

template <typename T>
static hipError_t launch_iter_t(const Lattice &L, const void *min, void *mout, const void *adiag,
                                const void *bw, double eta, uint32_t *flag, uint32_t t,
                                hipStream_t s) {
    dim3 grid(tiles_of(L)), block(256);
    if (L.alpha == 1)
        hipLaunchKernelGGL((k_iter_direct<T, 1>), grid, block, 0, s, L, (const T *)min, (T *)mout,
                           (const T *)adiag, (const T *)bw, (T)eta, flag, t);
    else
        hipLaunchKernelGGL((k_iter_direct<T, 2>), grid, block, 0, s, L, (const T *)min,
                           (T *)mout, (const T *)adiag, (const T *)bw, (T)eta, flag, t);
    return hipGetLastError();
}

hipError_t launch_iter(int dtype, const Lattice &L, const void *min, void *mout,
                       const void *adiag, const void *bw, double eta, uint32_t *flag,
                       uint32_t t, hipStream_t s) {
    return dtype == 0 ? launch_iter_t<float>(L, min, mout, adiag, bw, eta, flag, t, s)
                      : launch_iter_t<double>(L, min, mout, adiag, bw, eta, flag, t, s);
}

hipError_t launch_post(int dtype, const Lattice &L, const void *m, const double *adiag64,
                       const double *b64, double *mu_plane, double *mean, double *var,
                       hipStream_t s) {
    dim3 grid(tiles_of(L)), block(256);
    if (dtype == 0)
        hipLaunchKernelGGL((k_post<float>), grid, block, 0, s, L, (const float *)m, adiag64, b64,
                           mu_plane, mean, var);
    else
        hipLaunchKernelGGL((k_post<double>), grid, block, 0, s, L, (const double *)m, adiag64,
                           b64, mu_plane, mean, var);
    return hipGetLastError();
}

hipError_t launch_resid(const Lattice &L, const double *mu, const double *adiag64,
                        const double *b64, double *partials, int npart, double *out,
                        hipStream_t s) {
    const int nt = tiles_of(L);
    const int nb = nt < npart ? nt : npart;
    if (L.alpha == 1)
        hipLaunchKernelGGL((k_resid<1>), dim3(nb), dim3(256), 0, s, L, mu, adiag64, b64, partials,
                           nt);
    else
        hipLaunchKernelGGL((k_resid<2>), dim3(nb), dim3(256), 0, s, L, mu, adiag64, b64, partials,
                           nt);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, (const double *)partials, nb, out);
    return hipGetLastError();
}

hipError_t launch_abs_change(int dtype, const void *a, const void *b, int64_t n,
                             double *partials, int npart, double *out, hipStream_t s) {
    int64_t want = (n + 255) / 256;
    const int nb = (int)(want < npart ? (want > 0 ? want : 1) : npart);
    if (dtype == 0)
        hipLaunchKernelGGL((k_abs_change<float>), dim3(nb), dim3(256), 0, s, (const float *)a,
                           (const float *)b, n, partials);
    else
        hipLaunchKernelGGL((k_abs_change<double>), dim3(nb), dim3(256), 0, s, (const double *)a,
                           (const double *)b, n, partials);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, (const double *)partials, nb, out);
    return hipGetLastError();
}

hipError_t launch_setup(int dtype, const Lattice &L, int64_t nobs, const int64_t *cell,
                        const double *y, const double *var, double sigma2, double *adiag64,
                        double *b64, const double *prior_mean, void *adiag_w, void *b_w,
                        uint32_t *err_flag, hipStream_t s) {
    if (nobs > 0)
        hipLaunchKernelGGL(k_obs_scatter, dim3((unsigned)((nobs + 255) / 256)), dim3(256), 0, s, L,
                           nobs, cell, y, var, sigma2, adiag64, b64, err_flag);
    dim3 grid(tiles_of(L)), block(256);
    if (dtype == 0)
        hipLaunchKernelGGL((k_node_init<float>), grid, block, 0, s, L, adiag64, b64, prior_mean,
                           (float *)adiag_w, (float *)b_w, err_flag);
    else
        hipLaunchKernelGGL((k_node_init<double>), grid, block, 0, s, L, adiag64, b64, prior_mean,
                           (double *)nullptr, (double *)nullptr, err_flag);
    return hipGetLastError();
}

hipError_t launch_msgs_get(int dtype, const Lattice &L, const void *m, void *prec, void *info,
                           hipStream_t s) {
    dim3 grid(tiles_of(L)), block(256);
    if (dtype == 0)
        hipLaunchKernelGGL((k_msgs_get<float>), grid, block, 0, s, L, (const float *)m,
                           (float *)prec, (float *)info);
    else
        hipLaunchKernelGGL((k_msgs_get<double>), grid, block, 0, s, L, (const double *)m,
                           (double *)prec, (double *)info);
    return hipGetLastError();
}

hipError_t launch_msgs_set(int dtype, const Lattice &L, void *m, const void *prec,
                           const void *info, hipStream_t s) {
    dim3 grid(tiles_of(L)), block(256);
    if (dtype == 0)
        hipLaunchKernelGGL((k_msgs_set<float>), grid, block, 0, s, L, (float *)m,
                           (const float *)prec, (const float *)info);
    else
        hipLaunchKernelGGL((k_msgs_set<double>), grid, block, 0, s, L, (double *)m,
                           (const double *)prec, (const double *)info);
    return hipGetLastError();
}

}  // namespace gabp

// Learned warm start: the kernels of a small 3x3 convolutional network that
// predicts posterior means and message precisions from the observations,
// trained on solutions the solver itself produced, and the message
// initialisation that turns a prediction into a starting state.
//
// Tensors: activations NHWC in BF16 ([B][H][W][C], C in {16, 32}); weights
// [32][9*Cin] BF16 with k = tap * Cin + ci, tap = 3 * (dy + 1) + (dx + 1)
// (rows beyond the layer's output channels are zero); FP32 biases, FP32
// master weights and FP32 gradients.
//
// The convolutions are implicit GEMMs on the gfx950 matrix cores
// (v_mfma_f32_32x32x16_bf16: BF16 operands, FP32 accumulation).  Operand
// layout of that instruction (A: 32 x 16, B: 16 x 32, D: 32 x 32): lane l
// holds A[l % 32][8 (l / 32) + j] and B[8 (l / 32) + j][l % 32] for j < 8,
// and D[8 i + 4 (l / 32) + j][l % 32] in accumulator 4 i + j.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>

#include "gabp.h"
#include "internal.h"
#include "lattice.h"
#include "numerics.h"

namespace gabp {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

__device__ __forceinline__ bf16x8 zero_bf16x8() {
    bf16x8 z;
#pragma unroll
    for (int j = 0; j < 8; ++j) z[j] = (__bf16)0.0f;
    return z;
}

// --------------------------------------------------------------------------
// Convolution, forward: y[p][co] = act(bias[co] + sum_{tap, ci}
// w[co][tap][ci] x[p + dil * off(tap)][ci]), zero padding.  One wave = 32
// consecutive pixels of one row and all 32 output-channel rows of the
// weight matrix (M = channel, N = pixel, K = 9 * CIN).  The same kernel with
// flipped, transposed weights computes the data gradient.
// --------------------------------------------------------------------------
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv_fwd(const __bf16 *__restrict__ x,
                                                  const __bf16 *__restrict__ w,
                                                  const float *__restrict__ bias, int B, int H,
                                                  int W, int dil, int relu,
                                                  __bf16 *__restrict__ yb,
                                                  float *__restrict__ yf) {
    constexpr int K = 9 * CIN;
    const int tpr = (W + 31) / 32;
    const long wave = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= (long)B * H * tpr) return;
    const int b = (int)(wave / ((long)H * tpr));
    const int rem = (int)(wave % ((long)H * tpr));
    const int y = rem / tpr;
    const int x0 = (rem % tpr) * 32;
    const int lane = (int)(threadIdx.x & 63u);
    const int n = lane & 31, kh = lane >> 5;
    const int px = x0 + n;
    f32x16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
#pragma unroll 3
    for (int s = 0; s < K / 16; ++s) {
        const int k = s * 16 + kh * 8;
        const int tap = k / CIN, ci0 = k % CIN;
        const int yy = y + (tap / 3 - 1) * dil, xx = px + (tap % 3 - 1) * dil;
        const bf16x8 a = *(const bf16x8 *)(w + (size_t)n * K + k);
        bf16x8 bv = zero_bf16x8();
        if (px < W && yy >= 0 && yy < H && xx >= 0 && xx < W)
            bv = *(const bf16x8 *)(x + (((size_t)b * H + yy) * W + xx) * CIN + ci0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bv, acc, 0, 0, 0);
    }
    if (px >= W) return;
    const size_t o = (((size_t)b * H + y) * W + px) * COUT;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int co = 8 * i + 4 * kh + j;
            if (co >= COUT) continue;
            float v = acc[4 * i + j] + (bias ? bias[co] : 0.0f);
            if (relu) v = v > 0.0f ? v : 0.0f;
            if (yb) yb[o + co] = (__bf16)v;
            if (yf) yf[o + co] = v;
        }
}

// Flipped, transposed weights for the data gradient:
// wt[ci][tap'][co] = w[co][8 - tap'][ci] (rows ci >= CIN and columns co >=
// COUT are zero).
__global__ __launch_bounds__(256) void k_flip_weights(const __bf16 *__restrict__ w, int cin,
                                                      int cout, __bf16 *__restrict__ wt) {
    const int idx = (int)(blockIdx.x * 256 + threadIdx.x);
    const int K2 = 9 * cout;               // row length of wt
    if (idx >= 32 * K2) return;
    const int ci = idx / K2, r = idx % K2;
    const int tp = r / cout, co = r % cout;
    __bf16 v = (__bf16)0.0f;
    if (ci < cin) v = w[(size_t)co * (9 * cin) + (8 - tp) * cin + ci];
    wt[idx] = v;
}

// dZ = dY * relu'(y) in BF16 (mask = 1 where the layer has no activation),
// and its transpose dZT[c][p] for the weight gradient (rows c >= C zero).
__global__ __launch_bounds__(256) void k_relu_bwd(const float *__restrict__ dy,
                                                  const __bf16 *__restrict__ y, long P, int C,
                                                  int relu, __bf16 *__restrict__ dz,
                                                  __bf16 *__restrict__ dzt, long Ppad) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= 32 * Ppad) return;
    const int c = (int)(idx / Ppad);
    const long p = idx % Ppad;
    float v = 0.0f;
    if (c < C && p < P) {
        v = dy[p * C + c];
        if (relu && !((float)y[p * C + c] > 0.0f)) v = 0.0f;
        dz[p * C + c] = (__bf16)v;
    }
    dzt[idx] = (__bf16)v;
}

// Transposed im2col of x for the weight gradient:
// xt[tap * CIN + ci][p] = x[p + dil * off(tap)][ci] (0 outside the image),
// rows up to nrows (multiple of 32) zero beyond 9 * CIN.
__global__ __launch_bounds__(256) void k_im2col_t(const __bf16 *__restrict__ x, int B, int H,
                                                  int W, int cin, int dil, int nrows, long Ppad,
                                                  __bf16 *__restrict__ xt) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (long)nrows * Ppad) return;
    const int r = (int)(idx / Ppad);
    const long p = idx % Ppad;
    __bf16 v = (__bf16)0.0f;
    const long P = (long)B * H * W;
    if (r < 9 * cin && p < P) {
        const int tap = r / cin, ci = r % cin;
        const int b = (int)(p / ((long)H * W));
        const int rem = (int)(p % ((long)H * W));
        const int yy = rem / W + (tap / 3 - 1) * dil, xx = rem % W + (tap % 3 - 1) * dil;
        if (yy >= 0 && yy < H && xx >= 0 && xx < W)
            v = x[(((size_t)b * H + yy) * W + xx) * cin + ci];
    }
    xt[idx] = v;
}

// Weight gradient as a split-K GEMM on the matrix cores:
// part[kc][m][n] = sum_{p in chunk kc} dzt[m][p] xt[n][p]  (m < 32, n < N).
// One wave = one 32 x 32 block of (m, n) over one chunk of pixels.
__global__ __launch_bounds__(64) void k_gemm_nt(const __bf16 *__restrict__ dzt,
                                                const __bf16 *__restrict__ xt, long Ppad,
                                                int N, int chunk, float *__restrict__ part) {
    const int nb = (int)blockIdx.x, kc = (int)blockIdx.y;
    const int lane = (int)threadIdx.x;
    const int r = lane & 31, kh = lane >> 5;
    const long k0 = (long)kc * chunk;
    long k1 = k0 + chunk;
    if (k1 > Ppad) k1 = Ppad;
    f32x16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
    const __bf16 *arow = dzt + (size_t)r * Ppad;
    const __bf16 *brow = xt + (size_t)(nb * 32 + r) * Ppad;
    // wave-uniform trip count (Ppad and chunk are multiples of 16)
    for (long kb = k0; kb < k1; kb += 16) {
        const long k = kb + kh * 8;
        const bf16x8 a = *(const bf16x8 *)(arow + k);
        const bf16x8 bv = *(const bf16x8 *)(brow + k);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bv, acc, 0, 0, 0);
    }
    float *out = part + (size_t)kc * 32 * N;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = 8 * i + 4 * kh + j;
            out[(size_t)m * N + nb * 32 + r] = acc[4 * i + j];
        }
}

// dw[m][n] = sum_kc part[kc][m][n] (fixed order), db[m] = sum_p dzt[m][p].
__global__ __launch_bounds__(256) void k_reduce_dw(const float *__restrict__ part, int nchunks,
                                                   int N, int ncols, float *__restrict__ dw) {
    const int idx = (int)(blockIdx.x * 256 + threadIdx.x);
    if (idx >= 32 * ncols) return;
    const int m = idx / ncols, n = idx % ncols;
    float s = 0.0f;
    for (int kc = 0; kc < nchunks; ++kc) s += part[(size_t)kc * 32 * N + (size_t)m * N + n];
    dw[idx] = s;
}

__global__ __launch_bounds__(256) void k_row_sums(const __bf16 *__restrict__ dzt, long Ppad,
                                                  float *__restrict__ db) {
    __shared__ float sh[4];
    const int m = (int)blockIdx.x;
    float s = 0.0f;
    for (long p = threadIdx.x; p < Ppad; p += 256) s += (float)dzt[(size_t)m * Ppad + p];
#pragma unroll
    for (int k = 32; k >= 1; k >>= 1) s += __shfl_xor(s, k, 64);
    if ((threadIdx.x & 63u) == 0u) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) db[m] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Adam step on FP32 master weights (bias-corrected moments); refreshes the
// BF16 copy used by the matrix cores.
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ w, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v,
                                              __bf16 *__restrict__ wb, long n, float lr, float b1,
                                              float b2, float eps, float c1, float c2) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = (__bf16)wi;
}

// Loss and output gradient.  pred[p][16]: channel 0 the mean, channels 1..12
// log(-Lam) of the sender-indexed precision messages.  Mean term:
// (mu^ - mu*)^2 averaged over pixels; precision term: weight times the mean
// of (l^ - l*)^2 over existing edges (valid > 0).  Per-block partial loss
// sums in a fixed order.
__global__ __launch_bounds__(256) void k_warm_loss(const float *__restrict__ pred,
                                                   const float *__restrict__ mu_t,
                                                   const float *__restrict__ lam_t,
                                                   const float *__restrict__ valid, long P,
                                                   int ndir, float inv_np, float lam_w_inv_ne,
                                                   float *__restrict__ grad,
                                                   double *__restrict__ part) {
    __shared__ double sh[4];
    const long p = (long)blockIdx.x * 256 + threadIdx.x;
    double l = 0.0;
    if (p < P) {
        const float e = pred[p * 16] - mu_t[p];
        grad[p * 16] = 2.0f * e * inv_np;
        l += (double)e * e * inv_np;
        for (int d = 0; d < ndir; ++d) {
            const float ok = valid[(size_t)d * P + p];
            const float ed = ok > 0.0f ? pred[p * 16 + 1 + d] - lam_t[(size_t)d * P + p] : 0.0f;
            grad[p * 16 + 1 + d] = 2.0f * ed * lam_w_inv_ne;
            l += (double)ed * ed * lam_w_inv_ne;
        }
        for (int c = 1 + ndir; c < 16; ++c) grad[p * 16 + c] = 0.0f;
    }
#pragma unroll
    for (int k = 32; k >= 1; k >>= 1) l += __shfl_xor(l, k, 64);
    if ((threadIdx.x & 63u) == 0u) sh[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Input features of a lattice problem, NHWC BF16 [ny][nx][16]: channel 0 the
// observation mask, 1 the mean observed value (0 where unobserved), 2 the
// log prior scale kappa (shifted), the rest zero.  cnt/sum are FP32
// scratch planes of nx*ny, zeroed by the caller.
__global__ __launch_bounds__(256) void k_feat_scatter(long n, const int64_t *__restrict__ cell,
                                                      const double *__restrict__ yv, long N,
                                                      float *__restrict__ cnt,
                                                      float *__restrict__ sum) {
    const long k = (long)blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const int64_t c = cell[k];
    if (c < 0 || c >= N) return;
    atomicAdd(&cnt[c], 1.0f);
    atomicAdd(&sum[c], (float)yv[k]);
}

// p[0 .. n) = 0 (a kernel, not a memset, so that callers may capture it in
// a graph)
__global__ __launch_bounds__(256) void k_zero_f32(float *__restrict__ p, long n) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

__global__ __launch_bounds__(256) void k_feat_build(long N, const float *__restrict__ cnt,
                                                    const float *__restrict__ sum, float kfeat,
                                                    __bf16 *__restrict__ x) {
    const long p = (long)blockIdx.x * 256 + threadIdx.x;
    if (p >= N) return;
    const float c = cnt[p];
    __bf16 *o = x + p * 16;
    o[0] = (__bf16)(c > 0.0f ? 1.0f : 0.0f);
    o[1] = (__bf16)(c > 0.0f ? sum[p] / c : 0.0f);
    o[2] = (__bf16)kfeat;
#pragma unroll
    for (int k = 3; k < 16; ++k) o[k] = (__bf16)0.0f;
}

// Warm start of the messages from a prediction (mean mu^ and log(-Lam^) per
// sender-indexed edge): Lam_{i->j} = -exp(l^), and the information message
// that makes every edge consistent with the predicted means,
// th_{i->j} = Lam_{i->j} mu^_j - (Q_ij / c) mu^_i.  With exact means and
// converged precisions this is the fixed point; in general the beliefs
// become mu_i = mu^_i + (b - A mu^)_i / Lam_i.  keep_prec keeps the current
// precision messages instead of the predicted ones.
template <typename T, int ALPHA>
__global__ __launch_bounds__(256) void k_warm_init(Lattice L, const float *__restrict__ pred,
                                                   int keep_prec, T *__restrict__ m) {
    constexpr int DEG = ALPHA == 1 ? 4 : 12;
    const int tile = (int)blockIdx.x;
    const int x = (tile % L.tiles_x) * 64 + (int)(threadIdx.x & 63u);
    const int y = (tile / L.tiles_x) * 4 + (int)(threadIdx.x >> 6);
    if (x >= L.nx || y >= L.ny) return;
    const uint32_t i = (uint32_t)(y * L.pitch + x);
    const size_t pi = (size_t)y * L.nx + x;
    const float mui = pred[pi * 16];
    const T li = ALPHA == 2 ? ell<T>(L, x, y) : (T)0;
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        int xn, yn;
        if (!neighbour(L, x, y, d, xn, yn)) continue;
        const float muj = pred[((size_t)yn * L.nx + xn) * 16];
        T lam;
        if (keep_prec) lam = (m + (size_t)d * L.plane)[i];
        else lam = -(T)expf(pred[pi * 16 + 1 + d]);
        const T q = q_over_c<T, ALPHA>(L, d, li, xn, yn);
        (m + (size_t)d * L.plane)[i] = lam;
        (m + (size_t)(DEG + d) * L.plane)[i] = lam * (T)muj - q * (T)mui;
    }
}

// --------------------------------------------------------------------------
// host launchers
// --------------------------------------------------------------------------
hipError_t launch_warm_init(int dtype, const Lattice &L, const float *pred, int keep_prec,
                            void *m, hipStream_t s) {
    dim3 grid(L.tiles_x * ((L.ny + 3) / 4)), block(256);
    if (dtype == 0) {
        if (L.alpha == 1)
            hipLaunchKernelGGL((k_warm_init<float, 1>), grid, block, 0, s, L, pred, keep_prec, (float *)m);
        else
            hipLaunchKernelGGL((k_warm_init<float, 2>), grid, block, 0, s, L, pred, keep_prec, (float *)m);
    } else {
        if (L.alpha == 1)
            hipLaunchKernelGGL((k_warm_init<double, 1>), grid, block, 0, s, L, pred, keep_prec, (double *)m);
        else
            hipLaunchKernelGGL((k_warm_init<double, 2>), grid, block, 0, s, L, pred, keep_prec, (double *)m);
    }
    return hipGetLastError();
}

}  // namespace gabp

// ==========================================================================
// C ABI of the network primitives
// ==========================================================================
// Scratch of gabp_warm_features_noalloc: the two FP32 planes (observation
// counts and sums) of at most kFeatScratchCells cells, 16 MiB that each GPU
// the library runs on holds until the process ends.  Host code must not pass
// this name to a kernel (it is a host-side stand-in): the device address
// comes from hipGetSymbolAddress, once per device.
constexpr long kFeatScratchCells = 1L << 21;
static __device__ __align__(256) float scratch[2 * kFeatScratchCells];

namespace {
thread_local std::string g_net_error;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_dev[kMaxDevices] = {};   // device address of `scratch`, per device

// The current device's address of `scratch`, looked up on the device's first
// call (with that device current); allocates nothing.
hipError_t scratch_address(float **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = (float *)p;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

// Input features from observations with cnt/sum scratch planes of N cells
// (2 N floats, cleared here by a kernel).
hipError_t features_into(int64_t nobs, const int64_t *cell, const double *y, long N,
                         double kappa, float *scr, void *x_bf16, hipStream_t s) {
    hipLaunchKernelGGL(gabp::k_zero_f32, dim3((unsigned)((2 * N + 255) / 256)), dim3(256), 0, s,
                       scr, 2 * N);
    if (nobs > 0)
        hipLaunchKernelGGL(gabp::k_feat_scatter, dim3((unsigned)((nobs + 255) / 256)), dim3(256), 0, s,
                           (long)nobs, cell, y, N, scr, scr + N);
    const float kf = (float)(std::log(kappa) + 2.5);
    hipLaunchKernelGGL(gabp::k_feat_build, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N,
                       (const float *)scr, (const float *)(scr + N), kf, (__bf16 *)x_bf16);
    return hipGetLastError();
}

gabp_status nfail(gabp_status st, const std::string &m) {
    g_net_error = m;
    return st;
}

bool chan_ok(int c) { return c == 16 || c == 32; }

#define NHIP(call)                                                                      \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return nfail(GABP_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

hipError_t conv_dispatch(const void *x, int B, int H, int W, int cin, const void *w,
                         const float *bias, int cout, int dil, int relu, void *yb, float *yf,
                         hipStream_t s) {
    const long waves = (long)B * H * ((W + 31) / 32);
    dim3 grid((unsigned)((waves + 3) / 4)), block(256);
    const __bf16 *xx = (const __bf16 *)x, *ww = (const __bf16 *)w;
    __bf16 *ybb = (__bf16 *)yb;
    if (cin == 16 && cout == 16)
        hipLaunchKernelGGL((gabp::k_conv_fwd<16, 16>), grid, block, 0, s, xx, ww, bias, B, H, W, dil, relu, ybb, yf);
    else if (cin == 16)
        hipLaunchKernelGGL((gabp::k_conv_fwd<16, 32>), grid, block, 0, s, xx, ww, bias, B, H, W, dil, relu, ybb, yf);
    else if (cout == 16)
        hipLaunchKernelGGL((gabp::k_conv_fwd<32, 16>), grid, block, 0, s, xx, ww, bias, B, H, W, dil, relu, ybb, yf);
    else
        hipLaunchKernelGGL((gabp::k_conv_fwd<32, 32>), grid, block, 0, s, xx, ww, bias, B, H, W, dil, relu, ybb, yf);
    return hipGetLastError();
}

long pad16(long p) { return (p + 15) / 16 * 16; }
}  // namespace

extern "C" {

const char *gabp_net_last_error(void) { return g_net_error.c_str(); }

gabp_status gabp_conv3x3_fwd(const void *x, int32_t B, int32_t H, int32_t W, int32_t cin,
                             const void *w, const float *bias, int32_t cout, int32_t dil,
                             int32_t relu, void *y_bf16, float *y_f32, void *stream) {
    if (!x || !w || B < 1 || H < 1 || W < 1 || !chan_ok(cin) || !chan_ok(cout) || dil < 1 ||
        (!y_bf16 && !y_f32))
        return nfail(GABP_E_INVALID, "conv3x3_fwd: bad arguments (channels must be 16 or 32)");
    NHIP(conv_dispatch(x, B, H, W, cin, w, bias, cout, dil, relu, y_bf16, y_f32, (hipStream_t)stream));
    return GABP_OK;
}

size_t gabp_conv3x3_bwd_workspace(int32_t B, int32_t H, int32_t W, int32_t cin, int32_t cout) {
    const long P = (long)B * H * W, Pp = pad16(P);
    const int nrows = ((9 * cin + 31) / 32) * 32;
    const long chunk = 8192;
    const long nchunks = (Pp + chunk - 1) / chunk;
    size_t bytes = 0;
    bytes += (size_t)32 * 9 * 32 * 2 + 256;                  // flipped weights
    bytes += (size_t)P * cout * 2 + 256;                     // dz (NHWC)
    bytes += (size_t)32 * Pp * 2 + 256;                      // dz transposed
    bytes += (size_t)nrows * Pp * 2 + 256;                   // im2col transposed
    bytes += (size_t)nchunks * 32 * nrows * 4 + 256;         // split-K partials
    return bytes;
}

// Backward of one layer y = act(conv(x, w) + b): from dy (FP32 NHWC, cout
// channels) and the layer's input x and output y (BF16), the weight and bias
// gradients dw [32][9*cin], db [32] (FP32, rows >= cout zero) and, when dx is
// not NULL, the input gradient dx (FP32 NHWC, cin channels).  Deterministic.
gabp_status gabp_conv3x3_bwd(const void *x, const void *y, const float *dy, int32_t B, int32_t H,
                             int32_t W, int32_t cin, const void *w, int32_t cout, int32_t dil,
                             int32_t relu, float *dw, float *db, float *dx, void *workspace,
                             size_t workspace_bytes, void *stream) {
    if (!x || !y || !dy || !w || !dw || !db || B < 1 || H < 1 || W < 1 || !chan_ok(cin) ||
        !chan_ok(cout) || dil < 1 || !workspace)
        return nfail(GABP_E_INVALID, "conv3x3_bwd: bad arguments");
    if (workspace_bytes < gabp_conv3x3_bwd_workspace(B, H, W, cin, cout))
        return nfail(GABP_E_NOMEM, "conv3x3_bwd: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const long P = (long)B * H * W, Pp = pad16(P);
    const int nrows = ((9 * cin + 31) / 32) * 32;
    const long chunk = 8192;
    const int nchunks = (int)((Pp + chunk - 1) / chunk);
    char *ws = (char *)workspace;
    auto take = [&](size_t bytes) {
        char *p = ws;
        ws += (bytes + 255) / 256 * 256;
        return p;
    };
    __bf16 *wt = (__bf16 *)take((size_t)32 * 9 * 32 * 2);
    __bf16 *dz = (__bf16 *)take((size_t)P * cout * 2);
    __bf16 *dzt = (__bf16 *)take((size_t)32 * Pp * 2);
    __bf16 *xt = (__bf16 *)take((size_t)nrows * Pp * 2);
    float *part = (float *)take((size_t)nchunks * 32 * nrows * 4);
    hipLaunchKernelGGL(gabp::k_relu_bwd, dim3((unsigned)((32 * Pp + 255) / 256)), dim3(256), 0, s,
                       dy, (const __bf16 *)y, P, cout, relu, dz, dzt, Pp);
    hipLaunchKernelGGL(gabp::k_im2col_t, dim3((unsigned)((nrows * Pp + 255) / 256)), dim3(256), 0, s,
                       (const __bf16 *)x, B, H, W, cin, dil, nrows, Pp, xt);
    hipLaunchKernelGGL(gabp::k_gemm_nt, dim3(nrows / 32, nchunks), dim3(64), 0, s,
                       (const __bf16 *)dzt, (const __bf16 *)xt, Pp, nrows, (int)chunk, part);
    hipLaunchKernelGGL(gabp::k_reduce_dw, dim3((32 * 9 * cin + 255) / 256), dim3(256), 0, s,
                       (const float *)part, nchunks, nrows, 9 * cin, dw);
    hipLaunchKernelGGL(gabp::k_row_sums, dim3(32), dim3(256), 0, s, (const __bf16 *)dzt, Pp, db);
    if (dx) {
        hipLaunchKernelGGL(gabp::k_flip_weights, dim3((32 * 9 * cout + 255) / 256), dim3(256), 0, s,
                           (const __bf16 *)w, cin, cout, wt);
        NHIP(conv_dispatch(dz, B, H, W, cout, wt, nullptr, cin, dil, 0, nullptr, dx, s));
    }
    NHIP(hipGetLastError());
    return GABP_OK;
}

gabp_status gabp_adam_step(float *w, const float *g, float *m, float *v, void *w_bf16, int64_t n,
                           double lr, double beta1, double beta2, double eps, int32_t step,
                           void *stream) {
    if (!w || !g || !m || !v || n < 0 || step < 1)
        return nfail(GABP_E_INVALID, "adam_step: bad arguments");
    const float c1 = (float)(1.0 - std::pow(beta1, step)), c2 = (float)(1.0 - std::pow(beta2, step));
    hipLaunchKernelGGL(gabp::k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, w, g, m, v, (__bf16 *)w_bf16, (long)n, (float)lr,
                       (float)beta1, (float)beta2, (float)eps, c1, c2);
    NHIP(hipGetLastError());
    return GABP_OK;
}

gabp_status gabp_warm_loss(const float *pred, const float *mu_t, const float *lam_t,
                           const float *valid, int64_t P, int32_t ndir, double lam_weight,
                           float *grad, double *partials, int32_t *nparts, void *stream) {
    if (!pred || !mu_t || !grad || !partials || !nparts || P < 1 || ndir < 0 || ndir > 12 ||
        (ndir > 0 && (!lam_t || !valid)))
        return nfail(GABP_E_INVALID, "warm_loss: bad arguments");
    const int nb = (int)((P + 255) / 256);
    *nparts = nb;
    const float inv_np = (float)(1.0 / (double)P);
    const float lw = (float)(lam_weight / ((double)P * (ndir > 0 ? ndir : 1)));
    hipLaunchKernelGGL(gabp::k_warm_loss, dim3(nb), dim3(256), 0, (hipStream_t)stream, pred, mu_t,
                       lam_t, valid, (long)P, ndir, inv_np, lw, grad, partials);
    NHIP(hipGetLastError());
    return GABP_OK;
}

gabp_status gabp_warm_features(int64_t nobs, const int64_t *cell, const double *y, int64_t nx,
                               int64_t ny, double kappa, float *work, void *x_bf16,
                               void *stream) {
    if (nx < 1 || ny < 1 || !work || !x_bf16 || nobs < 0 || (nobs > 0 && (!cell || !y)) ||
        !(kappa > 0))
        return nfail(GABP_E_INVALID, "warm_features: bad arguments");
    NHIP(features_into(nobs, cell, y, (long)nx * ny, kappa, work, x_bf16, (hipStream_t)stream));
    return GABP_OK;
}

gabp_status gabp_warm_features_noalloc(int64_t nobs, const int64_t *cell, const double *y,
                                       int64_t nx, int64_t ny, double kappa, void *x_bf16,
                                       void *stream) {
    if (nx < 1 || ny < 1 || !x_bf16 || nobs < 0 || (nobs > 0 && (!cell || !y)) ||
        !(kappa > 0))
        return nfail(GABP_E_INVALID, "warm_features_noalloc: bad arguments");
    if (nx > kFeatScratchCells || ny > kFeatScratchCells || nx * ny > kFeatScratchCells)
        return nfail(GABP_E_INVALID,
                     "warm_features_noalloc: nx * ny exceeds the static scratch of 2^21 cells");
    float *scr = nullptr;
    NHIP(scratch_address(&scr));
    NHIP(features_into(nobs, cell, y, (long)nx * ny, kappa, scr, x_bf16, (hipStream_t)stream));
    return GABP_OK;
}

}  // extern "C"

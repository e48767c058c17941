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
// w[co][tap][ci] x[p + dil * off(tap)][ci]), zero padding.  M = output
// channel (32 weight rows), N = pixel, K = 9 * CIN.  The work-group stages
// the weight matrix in LDS once (rows padded by 8 values to spread the LDS
// banks); each wave then computes NP tiles of 32 consecutive pixels of a row
// (tiles numbered over (image, row, column tile)), reusing each K step's
// weight fragment for its NP tiles.  The epilogue adds the bias, applies the
// activation and stores four consecutive channels per lane and row of the
// accumulator.  The same kernel with flipped, transposed weights computes
// the data gradient.
// --------------------------------------------------------------------------
template <int CIN, int COUT, int NP>
__global__ __launch_bounds__(256) void k_conv_fwd(const __bf16 *__restrict__ x,
                                                  const __bf16 *__restrict__ w,
                                                  const float *__restrict__ bias, int B, int H,
                                                  int W, int dil, int relu,
                                                  __bf16 *__restrict__ yb,
                                                  float *__restrict__ yf) {
    constexpr int K = 9 * CIN;
    constexpr int KP = K + 8;
    __shared__ __bf16 wl[32 * KP];
    for (int e = (int)threadIdx.x; e < 32 * (K / 8); e += 256) {
        const int row = e / (K / 8), c8 = e % (K / 8);
        *(bf16x8 *)(wl + row * KP + c8 * 8) = *(const bf16x8 *)(w + (size_t)row * K + c8 * 8);
    }
    __syncthreads();
    const int tpr = (W + 31) / 32;
    const long ntiles = (long)B * H * tpr;
    const long t0 = ((long)blockIdx.x * 4 + (threadIdx.x >> 6)) * NP;
    const int lane = (int)(threadIdx.x & 63u);
    const int n = lane & 31, kh = lane >> 5;
    int tb[NP], ty[NP], tx[NP];
    bool tv[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const long t = t0 + q;
        tv[q] = t < ntiles;
        const long tt = tv[q] ? t : 0;
        tb[q] = (int)(tt / ((long)H * tpr));
        const int rem = (int)(tt % ((long)H * tpr));
        ty[q] = rem / tpr;
        tx[q] = (rem % tpr) * 32 + n;
    }
    f32x16 acc[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[q][v] = 0.0f;
#pragma unroll 3
    for (int s = 0; s < K / 16; ++s) {
        const int k = s * 16 + kh * 8;
        const int tap = k / CIN, ci0 = k % CIN;
        const int oy = (tap / 3 - 1) * dil, ox = (tap % 3 - 1) * dil;
        const bf16x8 a = *(const bf16x8 *)(wl + n * KP + k);
        bf16x8 bv[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int yy = ty[q] + oy, xx = tx[q] + ox;
            bv[q] = zero_bf16x8();
            if (tv[q] && tx[q] < W && yy >= 0 && yy < H && xx >= 0 && xx < W)
                bv[q] = *(const bf16x8 *)(x + (((size_t)tb[q] * H + yy) * W + xx) * CIN + ci0);
        }
#pragma unroll
        for (int q = 0; q < NP; ++q)
            acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bv[q], acc[q], 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        if (!tv[q] || tx[q] >= W) continue;
        const size_t o = (((size_t)tb[q] * H + ty[q]) * W + tx[q]) * COUT;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int c0 = 8 * i + 4 * kh;    // channels c0 .. c0 + 3 of this lane
            if (c0 >= COUT) continue;
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                v[j] = acc[q][4 * i + j] + (bias ? bias[c0 + j] : 0.0f);
                if (relu) v[j] = v[j] > 0.0f ? v[j] : 0.0f;
            }
            if (yb) {
                typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
                bf16x4 pk;
#pragma unroll
                for (int j = 0; j < 4; ++j) pk[j] = (__bf16)v[j];
                *(bf16x4 *)(yb + o + c0) = pk;
            }
            if (yf) *(float4 *)(yf + o + c0) = make_float4(v[0], v[1], v[2], v[3]);
        }
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

// Backward of one layer, y = act(conv(x, w) + bias).  dZ = dY * relu'(y)
// (BF16), then three products:
//   data gradient    dX = conv(dZ, flipped w)          (k_conv_fwd)
//   weight gradient  dW[co][tap][ci] = sum_p dZ[p][co] x[p + dil off(tap)][ci]
//   bias gradient    db[co] = sum_p dZ[p][co]
// The weight gradient is an implicit GEMM on the matrix cores with the pixels
// as the reduction dimension (M = 32 output channels, N = 9 cin taps x
// channels, K = pixels): no im2col is formed; each operand fragment is eight
// consecutive pixels of one channel, read from channel-major copies of dZ
// and x (dZT, xT: [channel][pixel], made by LDS-tiled transposes) at the
// tap's pixel shift.  Work-groups take fixed pixel chunks (split-K) and the
// partial sums are reduced in a fixed order, so the result is deterministic.

constexpr int kTP = 64;   // pixels per transpose tile

// dZ = dY * relu'(y): dz [P][C] BF16 (NHWC) and dzt [32][Ppad] (channel-major;
// rows c >= C and columns p >= P zero), through a 32 x 64 LDS tile.
__global__ __launch_bounds__(256) void k_relu_bwd_t(const float *__restrict__ dy,
                                                    const __bf16 *__restrict__ y, long P, int C,
                                                    int relu, __bf16 *__restrict__ dz,
                                                    __bf16 *__restrict__ dzt, long Ppad) {
    __shared__ __bf16 tile[32][kTP + 2];
    const long p0 = (long)blockIdx.x * kTP;
    for (int e = (int)threadIdx.x; e < kTP * 32; e += 256) {
        const int p = e >> 5, c = e & 31;
        float v = 0.0f;
        if (c < C && p0 + p < P) {
            const long o = (p0 + p) * C + c;
            v = dy[o];
            if (relu && !((float)y[o] > 0.0f)) v = 0.0f;
            dz[o] = (__bf16)v;
        }
        tile[c][p] = (__bf16)v;
    }
    __syncthreads();
    for (int e = (int)threadIdx.x; e < 32 * kTP; e += 256) {
        const int c = e / kTP, p = e % kTP;
        dzt[(size_t)c * Ppad + p0 + p] = tile[c][p];
    }
}

// x [P][C] BF16 -> xt [C][Ppad] (columns p >= P zero), through an LDS tile.
__global__ __launch_bounds__(256) void k_to_cmajor(const __bf16 *__restrict__ x, long P, int C,
                                                   __bf16 *__restrict__ xt, long Ppad) {
    __shared__ __bf16 tile[32][kTP + 2];
    const long p0 = (long)blockIdx.x * kTP;
    for (int e = (int)threadIdx.x; e < kTP * 32; e += 256) {
        const int p = e >> 5, c = e & 31;
        __bf16 v = (__bf16)0.0f;
        if (c < C && p0 + p < P) v = x[(p0 + p) * C + c];
        tile[c][p] = v;
    }
    __syncthreads();
    for (int e = (int)threadIdx.x; e < C * kTP; e += 256) {
        const int c = e / kTP, p = e % kTP;
        xt[(size_t)c * Ppad + p0 + p] = tile[c][p];
    }
}

// Weight and bias gradients of one layer.  One work-group per chunk of
// `chunk` pixels (a multiple of 16); its waves split the N tiles, TPW tiles
// each, and every wave walks all 16-pixel steps of the chunk.  For each step
// a lane loads its A fragment (dZT row co = lane % 32, pixels p .. p + 7 with
// p = step + 8 (lane / 32)) and one B fragment per tile of the wave (xT row
// ci at the tap's shift, eight consecutive pixels: one 16-byte load when
// they stay in one image row, masked element loads at the image edges), then
// runs one MFMA per tile; the next step's loads are issued before this
// step's MFMAs.  Each wave writes its tiles of the chunk's partial dW
// [32][9 CIN], wave 0 also the partial db [32]; k_sum_rows sums the chunks
// in order.
template <int CIN, int TPW>
__global__ __launch_bounds__(64 * (((9 * CIN + 31) / 32 + TPW - 1) / TPW)) void k_wgrad(
    const __bf16 *__restrict__ dzt, const __bf16 *__restrict__ xt, int H, int W, int dil, long P,
    long Ppad, int chunk, float *__restrict__ part, float *__restrict__ dbpart) {
    constexpr int NN = 9 * CIN;
    constexpr int NT = (NN + 31) / 32;     // N tiles of 32 (tap, channel) columns
    const int lane = (int)(threadIdx.x & 63u), w = (int)(threadIdx.x >> 6);
    const int r = lane & 31, h = lane >> 5;
    const long HW = (long)H * W;
    f32x16 acc[TPW];
#pragma unroll
    for (int k = 0; k < TPW; ++k)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[k][v] = 0.0f;
    float bsum = 0.0f;
    // this lane's (tap, channel) in each of the wave's tiles
    int tdy[TPW], tdx[TPW], tci[TPW];
#pragma unroll
    for (int k = 0; k < TPW; ++k) {
        const int n = 32 * (w * TPW + k) + r;
        const int tap = n / CIN;
        tci[k] = n % CIN;
        const bool real = tap < 9 && w * TPW + k < NT;
        tdy[k] = real ? (tap / 3 - 1) * dil : 1 << 28;   // huge: never inside
        tdx[k] = real ? (tap % 3 - 1) * dil : 0;
        if (!real) tci[k] = 0;
    }
    const int c0 = (int)((long)blockIdx.x * chunk);
    const int c1 = (int)(c0 + chunk < Ppad ? c0 + chunk : Ppad);
    const int Pi = (int)P, HWi = (int)HW;
    // eight aligned pixels stay in one image row (and a 16-pixel step moves
    // at most one row on)
    const bool rows8 = (W & 7) == 0 && W >= 16;
    // image, row and column of this lane's first pixel of the next step to
    // load, advanced by 16 pixels per step (no division in the loop)
    int pb = (c0 + 8 * h) / HWi, prem = (c0 + 8 * h) - pb * HWi;
    int py = prem / W, px = prem - py * W;
    // operands of the 16-pixel step at s (zero past the chunk)
    auto load_step = [&](int s, bf16x8 &a, bf16x8 *bv) {
        a = zero_bf16x8();
#pragma unroll
        for (int k = 0; k < TPW; ++k) bv[k] = zero_bf16x8();
        const int p = s + 8 * h;
        const int b = pb, y = py, x = px;
        px += 16;
        if (px >= W) {
            px -= W;
            if (++py == H) {
                py = 0;
                ++pb;
            }
        }
        if (s >= c1) return;
        a = *(const bf16x8 *)(dzt + (size_t)r * Ppad + p);
#pragma unroll
        for (int k = 0; k < TPW; ++k) {
            const __bf16 *src = xt + (size_t)tci[k] * Ppad;
            if (rows8 && p + 8 <= Pi) {
                const int yy = y + tdy[k];
                if (yy >= 0 && yy < H) {
                    const int xs = x + tdx[k];
                    const int q = (b * H + yy) * W + xs;
                    if (xs >= 0 && xs + 8 <= W) {
                        __builtin_memcpy(&bv[k], src + q, 16);
                    } else {
#pragma unroll
                        for (int j = 0; j < 8; ++j)
                            if (xs + j >= 0 && xs + j < W) bv[k][j] = src[q + j];
                    }
                }
            } else {
                // general position: each pixel on its own (rows of any width,
                // the last pixels of the batch)
#pragma unroll 1
                for (int j = 0; j < 8; ++j) {
                    const int pj = p + j;
                    if (pj >= Pi) break;
                    const int bj = pj / HWi, rj = pj - bj * HWi;
                    const int yj = rj / W + tdy[k], xj = rj % W + tdx[k];
                    if (yj >= 0 && yj < H && xj >= 0 && xj < W)
                        bv[k][j] = src[(bj * H + yj) * W + xj];
                }
            }
        }
    };
    auto mma_step = [&](const bf16x8 &a, const bf16x8 *bv) {
#pragma unroll
        for (int j = 0; j < 8; ++j) bsum += (float)a[j];
#pragma unroll
        for (int k = 0; k < TPW; ++k)
            acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bv[k], acc[k], 0, 0, 0);
    };
    bf16x8 a0, a1, b0[TPW], b1[TPW];
    int s = c0;
    load_step(s, a0, b0);
#pragma unroll 1
    for (; s < c1; s += 32) {
        load_step(s + 16, a1, b1);
        mma_step(a0, b0);
        if (s + 16 >= c1) break;
        load_step(s + 32, a0, b0);
        mma_step(a1, b1);
    }
    // this wave's tiles of the partial: D[co][n] with co = 8 i + 4 h + j in
    // accumulator 4 i + j, n = 32 tile + lane % 32
    float *out = part + (size_t)blockIdx.x * 32 * NN;
#pragma unroll
    for (int k = 0; k < TPW; ++k) {
        const int n = 32 * (w * TPW + k) + r;
        if (n >= NN) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) out[(size_t)(8 * i + 4 * h + j) * NN + n] = acc[k][4 * i + j];
    }
    bsum += __shfl_xor(bsum, 32, 64);   // lanes r and r + 32 hold the same channel
    if (w == 0 && h == 0) dbpart[(size_t)blockIdx.x * 32 + r] = bsum;
}

// out[g][i] = sum of in[r][i] over rows r in [g rpg, (g + 1) rpg) of nrows,
// in order: the split-K partials of the weight and bias gradients are summed
// in two such passes (groups, then the groups), a fixed order.
__global__ __launch_bounds__(256) void k_sum_rows(const float *__restrict__ in, int nrows,
                                                  int rpg, int ncols, float *__restrict__ out) {
    const int i = (int)(blockIdx.x * 256 + threadIdx.x);
    const int g = (int)blockIdx.y;
    if (i >= ncols) return;
    const int r0 = g * rpg, r1 = min(nrows, r0 + rpg);
    float acc = 0.0f;
    for (int r = r0; r < r1; ++r) acc += in[(size_t)r * ncols + i];
    out[(size_t)g * ncols + i] = acc;
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
        // the pixel's 16 prediction channels as four 16-byte rows
        const float4 *pr = (const float4 *)(pred + p * 16);
        float v[16], g[16];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 t = pr[q];
            v[4 * q] = t.x; v[4 * q + 1] = t.y; v[4 * q + 2] = t.z; v[4 * q + 3] = t.w;
        }
        const float e = v[0] - mu_t[p];
        g[0] = 2.0f * e * inv_np;
        l += (double)e * e * inv_np;
#pragma unroll
        for (int d = 0; d < 15; ++d) {
            float ed = 0.0f;
            if (d < ndir) {
                const float ok = valid[(size_t)d * P + p];
                ed = ok > 0.0f ? v[1 + d] - lam_t[(size_t)d * P + p] : 0.0f;
            }
            g[1 + d] = 2.0f * ed * lam_w_inv_ne;
            l += (double)ed * ed * lam_w_inv_ne;
        }
        float4 *gr = (float4 *)(grad + p * 16);
#pragma unroll
        for (int q = 0; q < 4; ++q) gr[q] = make_float4(g[4 * q], g[4 * q + 1], g[4 * q + 2], g[4 * q + 3]);
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

// Training targets of the precision outputs from a solver state:
// lam[d][y][x] = log(-Lam) of the message from (x, y) to its neighbour in
// direction d (the sender-indexed plane d of the message buffer m) and
// valid[d][y][x] = 1 where that neighbour exists; 0 in both elsewhere and
// for d >= deg (12 planes are always written).  -Lam is floored at 1e-30.
template <typename T, int ALPHA>
__global__ __launch_bounds__(256) void k_log_prec(Lattice L, const T *__restrict__ m,
                                                  float *__restrict__ lam,
                                                  float *__restrict__ valid) {
    constexpr int DEG = ALPHA == 1 ? 4 : 12;
    const int tile = (int)blockIdx.x;
    const int x = (tile % L.tiles_x) * 64 + (int)(threadIdx.x & 63u);
    const int y = (tile / L.tiles_x) * 4 + (int)(threadIdx.x >> 6);
    if (x >= L.nx || y >= L.ny) return;
    const uint32_t i = (uint32_t)(y * L.pitch + x);
    const size_t np = (size_t)L.nx * L.ny, pi = (size_t)y * L.nx + x;
#pragma unroll
    for (int d = 0; d < 12; ++d) {
        float l = 0.0f, v = 0.0f;
        int xn, yn;
        if (d < DEG && neighbour(L, x, y, d, xn, yn)) {
            const float neg = -(float)(m + (size_t)d * L.plane)[i];
            l = logf(neg > 1e-30f ? neg : 1e-30f);
            v = 1.0f;
        }
        lam[(size_t)d * np + pi] = l;
        if (valid) valid[(size_t)d * np + pi] = v;
    }
}

// --------------------------------------------------------------------------
// host launchers
// --------------------------------------------------------------------------
hipError_t launch_log_prec(int dtype, const Lattice &L, const void *m, float *lam, float *valid,
                           hipStream_t s) {
    dim3 grid(L.tiles_x * ((L.ny + 3) / 4)), block(256);
    if (dtype == 0) {
        if (L.alpha == 1)
            hipLaunchKernelGGL((k_log_prec<float, 1>), grid, block, 0, s, L, (const float *)m, lam, valid);
        else
            hipLaunchKernelGGL((k_log_prec<float, 2>), grid, block, 0, s, L, (const float *)m, lam, valid);
    } else {
        if (L.alpha == 1)
            hipLaunchKernelGGL((k_log_prec<double, 1>), grid, block, 0, s, L, (const double *)m, lam, valid);
        else
            hipLaunchKernelGGL((k_log_prec<double, 2>), grid, block, 0, s, L, (const double *)m, lam, valid);
    }
    return hipGetLastError();
}

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

constexpr int kConvNP = 2;   // 32-pixel tiles per wave of the convolution

hipError_t conv_dispatch(const void *x, int B, int H, int W, int cin, const void *w,
                         const float *bias, int cout, int dil, int relu, void *yb, float *yf,
                         hipStream_t s) {
    const long tiles = (long)B * H * ((W + 31) / 32);
    const long waves = (tiles + kConvNP - 1) / kConvNP;
    dim3 grid((unsigned)((waves + 3) / 4)), block(256);
    const __bf16 *xx = (const __bf16 *)x, *ww = (const __bf16 *)w;
    __bf16 *ybb = (__bf16 *)yb;
    if (cin == 16 && cout == 16)
        hipLaunchKernelGGL((gabp::k_conv_fwd<16, 16, kConvNP>), grid, block, 0, s, xx, ww, bias, B, H, W, dil, relu, ybb, yf);
    else if (cin == 16)
        hipLaunchKernelGGL((gabp::k_conv_fwd<16, 32, kConvNP>), grid, block, 0, s, xx, ww, bias, B, H, W, dil, relu, ybb, yf);
    else if (cout == 16)
        hipLaunchKernelGGL((gabp::k_conv_fwd<32, 16, kConvNP>), grid, block, 0, s, xx, ww, bias, B, H, W, dil, relu, ybb, yf);
    else
        hipLaunchKernelGGL((gabp::k_conv_fwd<32, 32, kConvNP>), grid, block, 0, s, xx, ww, bias, B, H, W, dil, relu, ybb, yf);
    return hipGetLastError();
}

long pad64(long p) { return (p + 63) / 64 * 64; }
// pixels per work-group of the weight gradient (split-K chunk), and the
// groups of chunks its first summation pass forms
constexpr long kWgradChunk = 1024;
constexpr int kWgradTPW = 3;     // N tiles per wave
constexpr int kSumGroups = 16;
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
    const long P = (long)B * H * W, Pp = pad64(P);
    const long nchunks = (Pp + kWgradChunk - 1) / kWgradChunk;
    size_t bytes = 0;
    bytes += (size_t)32 * 9 * 32 * 2 + 256;                  // flipped weights
    bytes += (size_t)P * cout * 2 + 256;                     // dz (NHWC)
    bytes += (size_t)32 * Pp * 2 + 256;                      // dz channel-major
    bytes += (size_t)cin * Pp * 2 + 256;                     // x channel-major
    bytes += (size_t)nchunks * 32 * 9 * cin * 4 + 256;       // split-K partials of dw
    bytes += (size_t)nchunks * 32 * 4 + 256;                 // and of db
    bytes += (size_t)kSumGroups * 32 * (9 * cin + 1) * 4 + 512;   // group sums
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
    if ((long)B * H * W >= (1L << 31) - 64)
        return nfail(GABP_E_INVALID, "conv3x3_bwd: more than 2^31 - 64 pixels");
    if (workspace_bytes < gabp_conv3x3_bwd_workspace(B, H, W, cin, cout))
        return nfail(GABP_E_NOMEM, "conv3x3_bwd: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const long P = (long)B * H * W, Pp = pad64(P);
    const int nchunks = (int)((Pp + kWgradChunk - 1) / kWgradChunk);
    char *ws = (char *)workspace;
    auto take = [&](size_t bytes) {
        char *p = ws;
        ws += (bytes + 255) / 256 * 256;
        return p;
    };
    __bf16 *wt = (__bf16 *)take((size_t)32 * 9 * 32 * 2);
    __bf16 *dz = (__bf16 *)take((size_t)P * cout * 2);
    __bf16 *dzt = (__bf16 *)take((size_t)32 * Pp * 2);
    __bf16 *xt = (__bf16 *)take((size_t)cin * Pp * 2);
    float *part = (float *)take((size_t)nchunks * 32 * 9 * cin * 4);
    float *dbpart = (float *)take((size_t)nchunks * 32 * 4);
    float *gpart = (float *)take((size_t)kSumGroups * 32 * 9 * cin * 4);
    float *gdb = (float *)take((size_t)kSumGroups * 32 * 4);
    const unsigned tiles = (unsigned)(Pp / gabp::kTP);
    hipLaunchKernelGGL(gabp::k_relu_bwd_t, dim3(tiles), dim3(256), 0, s, dy, (const __bf16 *)y, P,
                       cout, relu, dz, dzt, Pp);
    hipLaunchKernelGGL(gabp::k_to_cmajor, dim3(tiles), dim3(256), 0, s, (const __bf16 *)x, P, cin,
                       xt, Pp);
    // waves per work-group: the N tiles (5 for 16 input channels, 9 for 32)
    // in groups of kWgradTPW
    if (cin == 16)
        hipLaunchKernelGGL((gabp::k_wgrad<16, kWgradTPW>), dim3(nchunks),
                           dim3(64 * ((5 + kWgradTPW - 1) / kWgradTPW)), 0, s,
                           (const __bf16 *)dzt, (const __bf16 *)xt, H, W, dil, P, Pp,
                           (int)kWgradChunk, part, dbpart);
    else
        hipLaunchKernelGGL((gabp::k_wgrad<32, kWgradTPW>), dim3(nchunks),
                           dim3(64 * ((9 + kWgradTPW - 1) / kWgradTPW)), 0, s,
                           (const __bf16 *)dzt, (const __bf16 *)xt, H, W, dil, P, Pp,
                           (int)kWgradChunk, part, dbpart);
    const int nn = 32 * 9 * cin;
    const int rpg = (nchunks + kSumGroups - 1) / kSumGroups;
    hipLaunchKernelGGL(gabp::k_sum_rows, dim3((nn + 255) / 256, kSumGroups), dim3(256), 0, s,
                       (const float *)part, nchunks, rpg, nn, gpart);
    hipLaunchKernelGGL(gabp::k_sum_rows, dim3((nn + 255) / 256, 1), dim3(256), 0, s,
                       (const float *)gpart, kSumGroups, kSumGroups, nn, dw);
    hipLaunchKernelGGL(gabp::k_sum_rows, dim3(1, kSumGroups), dim3(256), 0, s,
                       (const float *)dbpart, nchunks, rpg, 32, gdb);
    hipLaunchKernelGGL(gabp::k_sum_rows, dim3(1, 1), dim3(256), 0, s, (const float *)gdb,
                       kSumGroups, kSumGroups, 32, db);
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

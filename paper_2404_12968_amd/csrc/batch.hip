// Batched solving of many independent lattice problems of uneven sizes
// (C ABI: gabp_batch_* in include/gabp.h).
//
// Every instance keeps its own sender-indexed message planes and node planes
// inside one workspace.  A device-resident instance table describes them.
// One iteration of the whole batch is one launch of a persistent-grid kernel
// that walks a work list of (instance, tile) items over the instances still
// running: the launch boundary is the flooding barrier (every message of
// iteration t must exist before any of t + 1 is computed), so no workgroup
// ever waits on another.  Converged or diverged instances leave the work
// list; each instance switches to the information-only iteration on its own
// once its precision messages freeze.  A chunk of k iterations plus the
// per-instance FP64 check is captured once in a hipGraph and replayed while
// the set of running instances does not change.
//
// The per-node bodies are those of the single-lattice kernels (iter_node.h,
// check_node.h): a batched instance computes bitwise what a lone context
// computes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "check_node.h"
#include "gabp.h"
#include "host_common.h"
#include "internal.h"
#include "iter_node.h"
#include "pair_tile.h"
#include "lattice.h"
#include "numerics.h"

#pragma clang fp contract(off)

namespace gabp {

// Device record of one instance.
struct BatchInst {
    Lattice L;
    void *msg[2];
    void *gain;
    const void *adiag_w, *b_w;
    double *adiag64, *b64, *mu64, *bel64;
};

// Largest a in [0, n) with prefix[a] <= w (prefix[0] = 0, increasing).
__device__ __forceinline__ int find_item(const int *__restrict__ prefix, int n, int w) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= w) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// One flooding iteration of every running instance.  Work item w maps to
// instance act[a] and tile w - prefix[a] of that instance (64 x 4*RPT nodes);
// each workgroup of the persistent grid takes one contiguous range of items,
// so neighbouring tiles share a CU and its XCD's L2.
template <typename T, int RPT>
__global__ __launch_bounds__(256) void k_batch_iter(const BatchInst *__restrict__ inst,
                                                    const int *__restrict__ act,
                                                    const int *__restrict__ prefix, int nact,
                                                    int total, const int *__restrict__ frozen,
                                                    const uint32_t *__restrict__ t_dev,
                                                    int t_off, T eta,
                                                    uint32_t *__restrict__ diverged_at) {
    constexpr int TH = 4 * RPT;
    const uint32_t t = *t_dev + (uint32_t)t_off;   // this iteration's number
    const int per = (total + (int)gridDim.x - 1) / (int)gridDim.x;
    const int w1 = min(total, ((int)blockIdx.x + 1) * per);
    for (int w = (int)blockIdx.x * per; w < w1; ++w) {
        const int a = __builtin_amdgcn_readfirstlane(find_item(prefix, nact, w));
        const int I = __builtin_amdgcn_readfirstlane(act[a]);
        if (diverged_at[I] != 0u) continue;
        const BatchInst &B = inst[I];
        const Lattice L = B.L;
        const int tile = w - prefix[a];
        const int tx = tile % L.tiles_x, ty = tile / L.tiles_x;
        const int x = tx * 64 + (int)(threadIdx.x & 63u);
        const int y0 = ty * TH + (int)(threadIdx.x >> 6);
        const bool interior = tx * 64 >= 2 && tx * 64 + 66 <= L.nx && ty * TH >= 2 &&
                              ty * TH + TH + 2 <= L.ny;
        const T *m_in = (const T *)B.msg[(t - 1u) & 1u];
        T *m_out = (T *)B.msg[t & 1u];
        const bool fz = frozen[I] != 0;
        bool bad = false;
        if (x < L.nx) {
#pragma unroll 1
            for (int k = 0; k < RPT; ++k) {
                const int y = y0 + 4 * k;
                if (y >= L.ny) break;
                if (L.alpha == 1) {
                    if (fz) {
                        if (interior) iter_theta_node<T, 1, true>(L, m_in, m_out, (const T *)B.gain, (const T *)B.b_w, eta, bad, x, y);
                        else iter_theta_node<T, 1, false>(L, m_in, m_out, (const T *)B.gain, (const T *)B.b_w, eta, bad, x, y);
                    } else {
                        if (interior) iter_node<T, 1, true>(L, m_in, m_out, (const T *)B.adiag_w, (const T *)B.b_w, eta, bad, x, y);
                        else iter_node<T, 1, false>(L, m_in, m_out, (const T *)B.adiag_w, (const T *)B.b_w, eta, bad, x, y);
                    }
                } else {
                    if (fz) {
                        if (interior) iter_theta_node<T, 2, true>(L, m_in, m_out, (const T *)B.gain, (const T *)B.b_w, eta, bad, x, y);
                        else iter_theta_node<T, 2, false>(L, m_in, m_out, (const T *)B.gain, (const T *)B.b_w, eta, bad, x, y);
                    } else {
                        if (interior) iter_node<T, 2, true>(L, m_in, m_out, (const T *)B.adiag_w, (const T *)B.b_w, eta, bad, x, y);
                        else iter_node<T, 2, false>(L, m_in, m_out, (const T *)B.adiag_w, (const T *)B.b_w, eta, bad, x, y);
                    }
                }
            }
        }
        if (bad) diverged_at[I] = t;
    }
}

// Two information-only iterations of every frozen running instance with the
// prior order ALPHA: one workgroup per work item, item w (XCD-remapped so
// that each XCD takes a contiguous range) maps to instance act[a] and 64 x TH
// tile w - prefix[a].  Launches come in couples: the first (second == 0)
// reads the buffer of the state it starts from, iteration t, and writes the
// other one; the second reads that one and writes back, so after a couple
// each instance is in the buffer its iteration number selects, as after
// single iterations.
template <typename T, int ALPHA, int TH, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_batch_pair(const BatchInst *__restrict__ inst,
                                                           const int *__restrict__ act,
                                                           const int *__restrict__ prefix,
                                                           int nact,
                                                           const uint32_t *__restrict__ t_dev,
                                                           int t_off, int second, T eta,
                                                           uint32_t *__restrict__ diverged_at) {
    __shared__ T lds[(ALPHA == 1 ? 4 : 12) * TH * 64];
    const int w = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int a = __builtin_amdgcn_readfirstlane(find_item(prefix, nact, w));
    const int I = __builtin_amdgcn_readfirstlane(act[a]);
    if (diverged_at[I] != 0u) return;   // waves that return leave the tile's barrier
    const uint32_t t = *t_dev + (uint32_t)t_off;   // iteration the launch starts from
    const BatchInst &B = inst[I];
    const Lattice L = B.L;
    const int tile = w - prefix[a];
    const int tx = tile % L.tiles_x, ty = tile / L.tiles_x;
    const uint32_t own = t & 1u;
    const T *m_in = (const T *)B.msg[second ? own ^ 1u : own];
    T *m_out = (T *)B.msg[second ? own : own ^ 1u];
    bool bad1 = false, bad2 = false;
    // interior tiles on the path compiled without boundary code (uniform
    // across the workgroup)
    if (interior_tiles(L.nx, L.ny, ALPHA == 1 ? 1 : 2, TH).interior(tx, ty))
        pair_tile<T, ALPHA, TH, WAVES, true>(L, m_in, m_out, (const T *)B.gain, (const T *)B.b_w,
                                             eta, tx, ty, lds, bad1, bad2);
    else
        pair_tile<T, ALPHA, TH, WAVES, false>(L, m_in, m_out, (const T *)B.gain,
                                              (const T *)B.b_w, eta, tx, ty, lds, bad1, bad2);
    if (bad1 || bad2) record_divergence(&diverged_at[I], bad1 ? t + 1u : t + 2u);
}

// Marginals of every running instance (64 x 4 tiles), writing each
// instance's FP64 mean plane; probe[I] asks for the belief precisions too.
template <typename T>
__global__ __launch_bounds__(256) void k_batch_post(const BatchInst *__restrict__ inst,
                                                    const int *__restrict__ act,
                                                    const int *__restrict__ prefix, int nact,
                                                    int total, const int *__restrict__ frozen,
                                                    const int *__restrict__ probe,
                                                    const uint32_t *__restrict__ t_dev,
                                                    int t_off) {
    const uint32_t t = *t_dev + (uint32_t)t_off;
    const int per = (total + (int)gridDim.x - 1) / (int)gridDim.x;
    const int w1 = min(total, ((int)blockIdx.x + 1) * per);
    for (int w = (int)blockIdx.x * per; w < w1; ++w) {
        const int a = find_item(prefix, nact, w);
        const int I = act[a];
        const BatchInst &B = inst[I];
        const Lattice L = B.L;
        const int tile = w - prefix[a];
        const int x = (tile % L.tiles_x) * 64 + (int)(threadIdx.x & 63u);
        const int y = (tile / L.tiles_x) * 4 + (int)(threadIdx.x >> 6);
        if (x >= L.nx || y >= L.ny) continue;
        const T *m = (const T *)B.msg[t & 1u];
        double *bel_out = probe[I] ? B.bel64 : nullptr;
        if (L.alpha == 1) {
            if (frozen[I]) post_node<T, 1, true>(L, m, B.adiag64, B.b64, B.bel64, B.mu64, nullptr, nullptr, nullptr, x, y);
            else post_node<T, 1, false>(L, m, B.adiag64, B.b64, nullptr, B.mu64, nullptr, nullptr, bel_out, x, y);
        } else {
            if (frozen[I]) post_node<T, 2, true>(L, m, B.adiag64, B.b64, B.bel64, B.mu64, nullptr, nullptr, nullptr, x, y);
            else post_node<T, 2, false>(L, m, B.adiag64, B.b64, nullptr, B.mu64, nullptr, nullptr, bel_out, x, y);
        }
    }
}

// FP64 residual partial sums, one (r^2, b^2) pair per work item, each summed
// in a fixed order.
__global__ __launch_bounds__(256) void k_batch_resid(const BatchInst *__restrict__ inst,
                                                     const int *__restrict__ act,
                                                     const int *__restrict__ prefix, int nact,
                                                     int total, double *__restrict__ partials) {
    __shared__ double sh[2][4];
    const int per = (total + (int)gridDim.x - 1) / (int)gridDim.x;
    const int w1 = min(total, ((int)blockIdx.x + 1) * per);
    for (int w = (int)blockIdx.x * per; w < w1; ++w) {
        const int a = find_item(prefix, nact, w);
        const BatchInst &B = inst[act[a]];
        const Lattice L = B.L;
        const int tile = w - prefix[a];
        const int tx = tile % L.tiles_x, ty = tile / L.tiles_x;
        const int x = tx * 64 + (int)(threadIdx.x & 63u);
        const int y = ty * 4 + (int)(threadIdx.x >> 6);
        const bool interior = tx * 64 >= 2 && tx * 64 + 66 <= L.nx && ty * 4 >= 2 &&
                              ty * 4 + 6 <= L.ny;
        double rr = 0.0, bb = 0.0;
        if (L.alpha == 1) {
            if (interior) resid_node<1, true>(L, B.mu64, B.adiag64, B.b64, x, y, rr, bb);
            else if (x < L.nx && y < L.ny) resid_node<1, false>(L, B.mu64, B.adiag64, B.b64, x, y, rr, bb);
        } else {
            if (interior) resid_node<2, true>(L, B.mu64, B.adiag64, B.b64, x, y, rr, bb);
            else if (x < L.nx && y < L.ny) resid_node<2, false>(L, B.mu64, B.adiag64, B.b64, x, y, rr, bb);
        }
        rr = wave_sum(rr);
        bb = wave_sum(bb);
        const int wv = (int)(threadIdx.x >> 6);
        __syncthreads();
        if ((threadIdx.x & 63u) == 0u) {
            sh[0][wv] = rr;
            sh[1][wv] = bb;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            partials[2 * (int64_t)w] = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
            partials[2 * (int64_t)w + 1] = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
        }
    }
}

// One workgroup per running instance: fixed-order sum of its partials.
__global__ __launch_bounds__(256) void k_batch_reduce(const int *__restrict__ act,
                                                      const int *__restrict__ prefix,
                                                      const double *__restrict__ partials,
                                                      double *__restrict__ out) {
    __shared__ double sh[2][4];
    const int a = (int)blockIdx.x;
    const int lo = prefix[a], hi = prefix[a + 1];
    double r = 0.0, b = 0.0;
    for (int k = lo + (int)threadIdx.x; k < hi; k += 256) {
        r += partials[2 * (int64_t)k];
        b += partials[2 * (int64_t)k + 1];
    }
    r = wave_sum(r);
    b = wave_sum(b);
    const int wv = (int)(threadIdx.x >> 6);
    if ((threadIdx.x & 63u) == 0u) {
        sh[0][wv] = r;
        sh[1][wv] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int I = act[a];
        out[2 * I] = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
        out[2 * I + 1] = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
    }
}

// Advances the device iteration counter after a chunk (a kernel node, so a
// replayed graph numbers its iterations correctly).
__global__ void k_batch_advance(uint32_t *t_dev, int k) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *t_dev += (uint32_t)k;
}

}  // namespace gabp

// ==========================================================================
// host side
// ==========================================================================
using gabp::BatchInst;
using gabp::Lattice;
using namespace gabp::host;

namespace {

thread_local std::string g_batch_create_error;

struct InstHost {
    Lattice L;
    int dtype;
    Layout lay;
    size_t base = 0;            // byte offset of the instance's region
    int tiles_iter = 0;         // work items of the iteration kernel
    int tiles_pair = 0;         // work items of the two-iteration kernel
    int tiles_check = 0;        // work items of the check kernels (64 x 4)
    bool running = true;
    bool frozen = false;
    int64_t frozen_at = -1;
    int status = GABP_E_NOT_CONVERGED;
    int64_t iters = 0;          // iterations applied to this instance
    double rel = INFINITY;
    double first_rel = -1.0;
    double prev_rel = -1.0;     // residual and iteration count at the check before
    int64_t prev_iters = 0;
    bool prev_valid = false;
    int64_t diverged_at = 0;    // first invalid iteration (0: none)
    int dbuf = -1;              // after a divergence: the buffer holding the kept state
};

// Buffer holding an instance's current messages: its iteration's parity,
// except after a divergence inside a two-iteration launch.
int state_buf(const InstHost &H) { return H.dbuf >= 0 ? H.dbuf : (int)(H.iters & 1); }

// One run of iterations since the last check read-back: its length, the
// couples of two-iteration launches it made, and each instance's iteration
// and frozen flag at its start (-1: not running).
struct BatchRun {
    int k = 0;
    int couples = 0;
    std::vector<int64_t> t0;
    std::vector<char> frozen;
};

struct BatchHostMirror;

}  // namespace

struct gabp_batch {
    int n = 0;
    int dtype = 0;
    size_t esize = 4;
    int device = 0;
    hipStream_t ustream = nullptr;   // the caller's stream (may be the null stream)
    hipStream_t stream = nullptr;    // internal stream (graphs cannot capture the null stream)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    std::vector<InstHost> h;
    // device arrays (inside the workspace)
    BatchInst *d_inst = nullptr;
    int *d_act = nullptr, *d_wprefix = nullptr, *d_pprefix = nullptr;
    int *d_frozen = nullptr, *d_probe = nullptr;
    int *d_actu = nullptr, *d_wprefu = nullptr;   // running, precision not frozen (1 iteration)
    int *d_actf[2] = {nullptr, nullptr}, *d_wpreff[2] = {nullptr, nullptr};
                                                  // running, frozen, by prior order (2 per launch)
    uint32_t *d_div = nullptr, *d_t = nullptr, *d_err = nullptr;
    unsigned long long *d_cnt = nullptr;   // changed precision messages per instance
    uint32_t *d_mrel = nullptr;            // their largest relative change (float bits)
    double *d_partials = nullptr, *d_out = nullptr;
    size_t partial_cap = 0;     // work items of the check kernels
    // pinned host mirror
    double *p_out = nullptr;
    uint32_t *p_div = nullptr, *p_mrel = nullptr, *p_t = nullptr;
    unsigned long long *p_cnt = nullptr;
    int *p_lists = nullptr;     // staging for act / prefixes / frozen / probe
    int rpt = 4;
    int pair = 0;               // tile height of the two-iteration kernel, 0 = unused
    int64_t freeze_slots = 0;   // freeze tolerance (gabp_batch_set_freeze_tolerance)
    double freeze_rel = 0.0;
    int64_t t = 0;              // iterations applied to the running set
    // current work lists
    int nact = 0, wtotal = 0, ptotal = 0;
    int nu = 0, wtotu = 0, nf[2] = {0, 0}, wtotf[2] = {0, 0};
    bool lists_dirty = true;
    // captured chunk
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<BatchRun> runs;   // runs since the last check read-back
    int graph_k = 0, graph_rpt = 0;
    double graph_eta = 0.0;
    std::string err;
};

namespace {

// Order the internal stream after the caller's stream (entry) and the
// caller's stream after the internal one (exit).
struct StreamJoin {
    gabp_batch *b;
    bool ok;
    explicit StreamJoin(gabp_batch *bb) : b(bb), ok(true) {
        ok = hipSetDevice(b->device) == hipSuccess &&
             hipEventRecord(b->ev_in, b->ustream) == hipSuccess &&
             hipStreamWaitEvent(b->stream, b->ev_in, 0) == hipSuccess;
    }
    ~StreamJoin() {
        if (hipEventRecord(b->ev_out, b->stream) == hipSuccess)
            (void)hipStreamWaitEvent(b->ustream, b->ev_out, 0);
    }
};

gabp_status bfail(gabp_batch *b, gabp_status st, const std::string &m) {
    if (b) b->err = m;
    else g_batch_create_error = m;
    return st;
}

#define BHIP(b, call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return bfail((b), GABP_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kBatchGrid = 256 * 32;  // persistent grid: ranges of work items per workgroup

int tiles_iter_of(const Lattice &L, int rpt) {
    return L.tiles_x * ((L.ny + 4 * rpt - 1) / (4 * rpt));
}

int tiles_pair_of(const Lattice &L, int th) {
    return L.tiles_x * ((L.ny + th - 1) / th);
}

// lists staging / device layout: act[n] wprefix[n+1] pprefix[n+1] frozen[n]
// probe[n] actu[n] wprefu[n+1], then actf[n] wpreff[n+1] for alpha = 1 and 2
constexpr int lists_ints(int n) { return 11 * n + 5; }
// flag region: div[n], t, err, mrel[n] (uint32), then cnt[n] (uint64, 8-aligned)
constexpr size_t flag_bytes(int n) { return 4 * (2 * (size_t)n + 2) + 4 + 8 * (size_t)n; }

void drop_graph(gabp_batch *b) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
}

// Rebuild the work lists of the running instances (host staging, then one
// copy into the device arrays).
gabp_status upload_lists(gabp_batch *b) {
    const int n = b->n;
    int *act = b->p_lists, *wp = act + n, *pp = wp + n + 1, *fz = pp + n + 1, *pr = fz + n;
    int *actu = pr + n, *wpu = actu + n;
    int *actf[2], *wpf[2];
    actf[0] = wpu + n + 1;
    wpf[0] = actf[0] + n;
    actf[1] = wpf[0] + n + 1;
    wpf[1] = actf[1] + n;
    int na = 0, w = 0, p = 0, nu = 0, wu = 0, nf[2] = {0, 0}, wf[2] = {0, 0};
    for (int i = 0; i < n; ++i) {
        InstHost &H = b->h[i];
        fz[i] = H.frozen ? 1 : 0;
        pr[i] = (H.running && !H.frozen && H.prev_valid && H.iters >= 2) ? 1 : 0;
        if (!H.running) continue;
        H.tiles_iter = tiles_iter_of(H.L, b->rpt);
        act[na] = i;
        wp[na] = w;
        pp[na] = p;
        w += H.tiles_iter;
        p += H.tiles_check;
        ++na;
        if (H.frozen && b->pair > 0) {
            const int q = H.L.alpha == 1 ? 0 : 1;
            H.tiles_pair = tiles_pair_of(H.L, b->pair);
            actf[q][nf[q]] = i;
            wpf[q][nf[q]] = wf[q];
            wf[q] += H.tiles_pair;
            ++nf[q];
        } else {
            actu[nu] = i;
            wpu[nu] = wu;
            wu += H.tiles_iter;
            ++nu;
        }
    }
    wp[na] = w;
    pp[na] = p;
    wpu[nu] = wu;
    wpf[0][nf[0]] = wf[0];
    wpf[1][nf[1]] = wf[1];
    b->nact = na;
    b->wtotal = w;
    b->ptotal = p;
    b->nu = nu;
    b->wtotu = wu;
    for (int q = 0; q < 2; ++q) {
        b->nf[q] = nf[q];
        b->wtotf[q] = wf[q];
    }
    // all lists are contiguous from d_act on
    BHIP(b, hipMemcpyAsync(b->d_act, b->p_lists, sizeof(int) * (size_t)lists_ints(n),
                           hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));   // staging buffer is reused
    b->lists_dirty = false;
    drop_graph(b);
    return GABP_OK;
}

// One iteration of the instances in one work list (single-iteration kernel).
gabp_status launch_single(gabp_batch *b, const int *act, const int *prefix, int na, int total,
                          int s, double eta) {
    if (na == 0) return GABP_OK;
    const int grid = std::min(kBatchGrid, std::max(1, total));
    if (b->dtype == GABP_F32) {
        switch (b->rpt) {
#define RPT_CASE(R) case R: hipLaunchKernelGGL((gabp::k_batch_iter<float, R>), dim3(grid), dim3(256), 0, b->stream, b->d_inst, act, prefix, na, total, b->d_frozen, b->d_t, s, (float)eta, b->d_div); break;
            RPT_CASE(1) RPT_CASE(2) RPT_CASE(4) default: RPT_CASE(8)
#undef RPT_CASE
        }
    } else {
        switch (b->rpt) {
#define RPT_CASE(R) case R: hipLaunchKernelGGL((gabp::k_batch_iter<double, R>), dim3(grid), dim3(256), 0, b->stream, b->d_inst, act, prefix, na, total, b->d_frozen, b->d_t, s, eta, b->d_div); break;
            RPT_CASE(1) RPT_CASE(2) RPT_CASE(4) default: RPT_CASE(8)
#undef RPT_CASE
        }
    }
    BHIP(b, hipGetLastError());
    return GABP_OK;
}

// Two iterations (starting from iteration offset s0) of the frozen lists.
gabp_status launch_pair(gabp_batch *b, int s0, int second, double eta) {
    for (int q = 0; q < 2; ++q) {
        if (b->nf[q] == 0) continue;
        const dim3 grid((unsigned)b->wtotf[q]);
        const int *act = b->d_actf[q], *pre = b->d_wpreff[q];
        if (b->dtype == GABP_F32) {
            if (q == 0)
                hipLaunchKernelGGL((gabp::k_batch_pair<float, 1, 12, 12>), grid, dim3(768), 0,
                                   b->stream, b->d_inst, act, pre, b->nf[q], b->d_t, s0, second,
                                   (float)eta, b->d_div);
            else
                hipLaunchKernelGGL((gabp::k_batch_pair<float, 2, 12, 12>), grid, dim3(768), 0,
                                   b->stream, b->d_inst, act, pre, b->nf[q], b->d_t, s0, second,
                                   (float)eta, b->d_div);
        } else {
            if (q == 0)
                hipLaunchKernelGGL((gabp::k_batch_pair<double, 1, 4, 4>), grid, dim3(256), 0,
                                   b->stream, b->d_inst, act, pre, b->nf[q], b->d_t, s0, second,
                                   eta, b->d_div);
            else
                hipLaunchKernelGGL((gabp::k_batch_pair<double, 2, 4, 4>), grid, dim3(256), 0,
                                   b->stream, b->d_inst, act, pre, b->nf[q], b->d_t, s0, second,
                                   eta, b->d_div);
        }
        BHIP(b, hipGetLastError());
    }
    return GABP_OK;
}

// k iterations of the running set.  Frozen instances run couples of
// two-iteration launches (4 iterations each) while at least 5 iterations
// remain, the others single iterations alongside; the last 1 to 4
// iterations run singly for everyone, so that every instance ends on its
// two newest iterations in its two buffers.
int couples_of(const gabp_batch *b, int k) {
    return (b->pair > 0 && b->nf[0] + b->nf[1] > 0 && k >= 5) ? (k - 1) / 4 : 0;
}

// Record a run of k iterations about to be applied to the running set.
void record_run(gabp_batch *b, int k) {
    BatchRun r;
    r.k = k;
    r.couples = couples_of(b, k);
    r.t0.resize(b->n);
    r.frozen.resize(b->n);
    for (int i = 0; i < b->n; ++i) {
        r.t0[i] = b->h[i].running ? b->h[i].iters : -1;
        r.frozen[i] = b->h[i].frozen ? 1 : 0;
    }
    b->runs.push_back(std::move(r));
}

gabp_status launch_iters(gabp_batch *b, int k, double eta) {
    if (b->nact == 0) return GABP_OK;
    const int couples = couples_of(b, k);
    gabp_status st = GABP_OK;
    int s = 1;
    for (int c = 0; c < couples && st == GABP_OK; ++c, s += 4) {
        st = launch_pair(b, s - 1, 0, eta);
        for (int q = 0; q < 2 && st == GABP_OK; ++q)
            st = launch_single(b, b->d_actu, b->d_wprefu, b->nu, b->wtotu, s + q, eta);
        if (st == GABP_OK) st = launch_pair(b, s + 1, 1, eta);
        for (int q = 2; q < 4 && st == GABP_OK; ++q)
            st = launch_single(b, b->d_actu, b->d_wprefu, b->nu, b->wtotu, s + q, eta);
    }
    for (; s <= k && st == GABP_OK; ++s)
        st = launch_single(b, b->d_act, b->d_wprefix, b->nact, b->wtotal, s, eta);
    if (st != GABP_OK) return st;
    hipLaunchKernelGGL(gabp::k_batch_advance, dim3(1), dim3(64), 0, b->stream, b->d_t, k);
    BHIP(b, hipGetLastError());
    return GABP_OK;
}

// Check of the running set: marginals, residual partials, per-instance
// reduction, read-back of results and divergence flags.
gabp_status launch_check(gabp_batch *b) {
    if (b->nact == 0) return GABP_OK;
    const int grid = std::min(kBatchGrid, std::max(1, b->ptotal));
    if (b->dtype == GABP_F32)
        hipLaunchKernelGGL((gabp::k_batch_post<float>), dim3(grid), dim3(256), 0, b->stream,
                           b->d_inst, b->d_act, b->d_pprefix, b->nact, b->ptotal, b->d_frozen,
                           b->d_probe, b->d_t, 0);
    else
        hipLaunchKernelGGL((gabp::k_batch_post<double>), dim3(grid), dim3(256), 0, b->stream,
                           b->d_inst, b->d_act, b->d_pprefix, b->nact, b->ptotal, b->d_frozen,
                           b->d_probe, b->d_t, 0);
    hipLaunchKernelGGL(gabp::k_batch_resid, dim3(grid), dim3(256), 0, b->stream, b->d_inst,
                       b->d_act, b->d_pprefix, b->nact, b->ptotal, b->d_partials);
    hipLaunchKernelGGL(gabp::k_batch_reduce, dim3(b->nact), dim3(256), 0, b->stream, b->d_act,
                       b->d_pprefix, b->d_partials, b->d_out);
    BHIP(b, hipGetLastError());
    BHIP(b, hipMemcpyAsync(b->p_out, b->d_out, sizeof(double) * 2 * (size_t)b->n,
                           hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipMemcpyAsync(b->p_div, b->d_div, sizeof(uint32_t) * (size_t)b->n,
                           hipMemcpyDeviceToHost, b->stream));
    return GABP_OK;
}

// Precision-message change (count and largest relative change) of every
// running, not yet frozen instance whose previous buffer is valid (outside
// the captured graph).
gabp_status launch_probes(gabp_batch *b) {
    bool any = false;
    for (int i = 0; i < b->n; ++i) {
        InstHost &H = b->h[i];
        if (!(H.running && !H.frozen && H.prev_valid && H.iters >= 2)) continue;
        any = true;
        const int dt = b->dtype == GABP_F32 ? 0 : 1;
        char *base = b->ws + H.base;
        BHIP(b, gabp::launch_prec_change(dt, base + H.lay.msg[H.iters & 1],
                                         base + H.lay.msg[(H.iters - 1) & 1],
                                         (int64_t)H.L.deg * H.L.plane, b->d_cnt + i,
                                         b->d_mrel + i, b->stream));
    }
    if (any) {
        BHIP(b, hipMemcpyAsync(b->p_cnt, b->d_cnt, sizeof(unsigned long long) * (size_t)b->n,
                               hipMemcpyDeviceToHost, b->stream));
        BHIP(b, hipMemcpyAsync(b->p_mrel, b->d_mrel, sizeof(uint32_t) * (size_t)b->n,
                               hipMemcpyDeviceToHost, b->stream));
    }
    return GABP_OK;
}

gabp_status ensure_graph(gabp_batch *b, int k, double eta) {
    if (b->gexec && b->graph_k == k && b->graph_eta == eta && b->graph_rpt == b->rpt)
        return GABP_OK;
    drop_graph(b);
    BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    gabp_status st = launch_iters(b, k, eta);
    if (st == GABP_OK) st = launch_check(b);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (st != GABP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return bfail(b, GABP_E_DEVICE, "hipStreamEndCapture failed");
    b->graph = g;
    BHIP(b, hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
    b->graph_k = k;
    b->graph_eta = eta;
    b->graph_rpt = b->rpt;
    return GABP_OK;
}

}  // namespace

extern "C" {

const char *gabp_batch_last_error(const gabp_batch *b) {
    return b ? b->err.c_str() : g_batch_create_error.c_str();
}

void gabp_batch_destroy(gabp_batch *b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    if (b->own_ws && b->ws) (void)hipFree(b->ws);
    if (b->p_out) (void)hipHostFree(b->p_out);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

static gabp_status batch_layout(int32_t n, const gabp_instance *inst, int32_t dtype,
                                std::vector<InstHost> *hs, size_t *tables_off, size_t *total,
                                size_t *partial_cap, std::string &why) {
    if (n < 1 || !inst) return why = "need n >= 1 instances", GABP_E_INVALID;
    const size_t es = dtype == GABP_F32 ? 4 : 8;
    size_t off = 0, pc = 0;
    if (hs) hs->assign((size_t)n, InstHost());
    for (int i = 0; i < n; ++i) {
        std::string w;
        gabp_status st = check_grid_stencil(&inst[i].grid, &inst[i].stencil, dtype, w);
        if (st != GABP_OK) return why = "instance " + std::to_string(i) + ": " + w, st;
        const int deg = inst[i].stencil.alpha == 1 ? 4 : 12;
        Layout lay = make_layout(inst[i].grid.nx, inst[i].grid.ny, deg, es, dtype == GABP_F32);
        Lattice L = make_lattice(&inst[i].grid, &inst[i].stencil, lay);
        const int tc = L.tiles_x * ((L.ny + 3) / 4);
        pc += (size_t)tc;
        if (hs) {
            InstHost &H = (*hs)[(size_t)i];
            H.L = L;
            H.dtype = dtype;
            H.lay = lay;
            H.base = off;
            H.tiles_check = tc;
        }
        off = round_up(off + lay.total, kAlign);
    }
    *tables_off = off;
    // instance table, int lists, flag arrays (divergence, counter, error and
    // largest precision changes as uint32, then 64-bit change counts),
    // partials, results
    off = round_up(off + sizeof(BatchInst) * (size_t)n, kAlign);
    off = round_up(off + sizeof(int) * (size_t)lists_ints(n), kAlign);
    off = round_up(off + flag_bytes(n), kAlign);
    off = round_up(off + sizeof(double) * 2 * pc, kAlign);
    off = round_up(off + sizeof(double) * 2 * (size_t)n, kAlign);
    *total = off;
    *partial_cap = pc;
    return GABP_OK;
}

gabp_status gabp_batch_workspace_size(int32_t n, const gabp_instance *inst, int32_t dtype,
                                      size_t *bytes) {
    std::string why;
    size_t toff = 0, total = 0, pc = 0;
    gabp_status st = batch_layout(n, inst, dtype, nullptr, &toff, &total, &pc, why);
    if (st != GABP_OK) return bfail(nullptr, st, why);
    if (!bytes) return bfail(nullptr, GABP_E_INVALID, "bytes is NULL");
    *bytes = total;
    return GABP_OK;
}

gabp_status gabp_batch_create(int32_t n, const gabp_instance *inst, const gabp_opts *opts,
                              gabp_batch **out) {
    if (!out) return bfail(nullptr, GABP_E_INVALID, "out is NULL");
    *out = nullptr;
    const int32_t dtype = opts ? opts->dtype : GABP_F32;
    if (opts && opts->prior_mean)
        return bfail(nullptr, GABP_E_INVALID, "batched instances take no prior mean");
    std::vector<InstHost> hs;
    std::string why;
    size_t toff = 0, total = 0, pc = 0;
    gabp_status st = batch_layout(n, inst, dtype, &hs, &toff, &total, &pc, why);
    if (st != GABP_OK) return bfail(nullptr, st, why);
    for (int i = 0; i < n; ++i) {
        const gabp_obs &o = inst[i].obs;
        const gabp_noise &nz = inst[i].noise;
        const int64_t N = inst[i].grid.nx * inst[i].grid.ny;
        if (!nz.var && (!(nz.sigma > 0) || !std::isfinite(nz.sigma)))
            return bfail(nullptr, GABP_E_INVALID, "instance " + std::to_string(i) + ": sigma must be positive");
        if (o.n < 0 || (o.n > 0 && (!o.cell || !o.y)))
            return bfail(nullptr, GABP_E_INVALID, "instance " + std::to_string(i) + ": bad observations");
        if (o.n > 0 && !o.on_device)
            for (int64_t k = 0; k < o.n; ++k)
                if (o.cell[k] < 0 || o.cell[k] >= N || !std::isfinite(o.y[k]) ||
                    (nz.var && !(nz.var[k] > 0)))
                    return bfail(nullptr, GABP_E_INVALID, "instance " + std::to_string(i) +
                                                              ": invalid observation " + std::to_string(k));
    }
    gabp_batch *b = new (std::nothrow) gabp_batch();
    if (!b) return bfail(nullptr, GABP_E_NOMEM, "host allocation failed");
    auto bail = [&](gabp_status s2) {
        g_batch_create_error = b->err;
        gabp_batch_destroy(b);
        return s2;
    };
    b->n = n;
    b->dtype = dtype;
    b->pair = dtype == GABP_F32 ? 12 : 4;   // matches the k_batch_pair instances launched
    b->esize = dtype == GABP_F32 ? 4 : 8;
    b->h = hs;
    b->partial_cap = pc;
    if (hipGetDevice(&b->device) != hipSuccess) {
        b->err = "no HIP device";
        return bail(GABP_E_DEVICE);
    }
    b->ustream = opts ? (hipStream_t)opts->stream : nullptr;
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess) {
        b->err = "creating the batch stream or events failed";
        return bail(GABP_E_DEVICE);
    }
    // the internal stream starts after everything already queued on the
    // caller's stream (e.g. the observation arrays' uploads)
    if (hipEventRecord(b->ev_in, b->ustream) != hipSuccess ||
        hipStreamWaitEvent(b->stream, b->ev_in, 0) != hipSuccess) {
        b->err = "ordering the batch stream failed";
        return bail(GABP_E_DEVICE);
    }
    if (opts && opts->workspace) {
        if (opts->workspace_bytes < total) {
            b->err = "workspace too small: " + std::to_string(total) + " bytes needed";
            return bail(GABP_E_NOMEM);
        }
        if (((uintptr_t)opts->workspace) % kAlign != 0) {
            b->err = "workspace must be 256-byte aligned";
            return bail(GABP_E_INVALID);
        }
        b->ws = (char *)opts->workspace;
        b->ws_bytes = opts->workspace_bytes;
    } else {
        if (hipMalloc((void **)&b->ws, total) != hipSuccess) {
            b->ws = nullptr;
            b->err = "hipMalloc of the batch workspace failed";
            return bail(GABP_E_NOMEM);
        }
        b->own_ws = true;
        b->ws_bytes = total;
    }
    // device tables
    size_t off = toff;
    b->d_inst = (BatchInst *)(b->ws + off);
    off = round_up(off + sizeof(BatchInst) * (size_t)n, kAlign);
    b->d_act = (int *)(b->ws + off);
    b->d_wprefix = b->d_act + n;
    b->d_pprefix = b->d_wprefix + n + 1;
    b->d_frozen = b->d_pprefix + n + 1;
    b->d_probe = b->d_frozen + n;
    b->d_actu = b->d_probe + n;
    b->d_wprefu = b->d_actu + n;
    b->d_actf[0] = b->d_wprefu + n + 1;
    b->d_wpreff[0] = b->d_actf[0] + n;
    b->d_actf[1] = b->d_wpreff[0] + n + 1;
    b->d_wpreff[1] = b->d_actf[1] + n;
    off = round_up(off + sizeof(int) * (size_t)lists_ints(n), kAlign);
    b->d_div = (uint32_t *)(b->ws + off);
    b->d_t = b->d_div + n;
    b->d_err = b->d_t + 1;
    b->d_mrel = b->d_err + 1;
    b->d_cnt = (unsigned long long *)(b->ws + round_up(off + sizeof(uint32_t) * (size_t)(2 * n + 2), 8));
    off = round_up(off + flag_bytes(n), kAlign);
    b->d_partials = (double *)(b->ws + off);
    off = round_up(off + sizeof(double) * 2 * pc, kAlign);
    b->d_out = (double *)(b->ws + off);
    // pinned mirror: out[2n], cnt[n], div[n], mrel[n], t, lists
    const size_t pin_bytes = sizeof(double) * 2 * (size_t)n + sizeof(unsigned long long) * (size_t)n +
                             sizeof(uint32_t) * (2 * (size_t)n + 2) +
                             sizeof(int) * (size_t)lists_ints(n) + 64;
    if (hipHostMalloc((void **)&b->p_out, pin_bytes, hipHostMallocDefault) != hipSuccess) {
        b->p_out = nullptr;
        b->err = "pinned host allocation failed";
        return bail(GABP_E_NOMEM);
    }
    b->p_cnt = (unsigned long long *)(b->p_out + 2 * n);
    b->p_div = (uint32_t *)(b->p_cnt + n);
    b->p_mrel = b->p_div + n;
    b->p_t = b->p_mrel + n;
    b->p_lists = (int *)(b->p_t + 2);
    if (hipMemsetAsync(b->ws, 0, total, b->stream) != hipSuccess) {
        b->err = "hipMemsetAsync failed";
        return bail(GABP_E_DEVICE);
    }
    // instance records and per-instance set-up
    std::vector<BatchInst> rec((size_t)n);
    for (int i = 0; i < n; ++i) {
        InstHost &H = b->h[i];
        char *base = b->ws + H.base;
        BatchInst &R = rec[(size_t)i];
        R.L = H.L;
        R.msg[0] = base + H.lay.msg[0];
        R.msg[1] = base + H.lay.msg[1];
        R.gain = base + H.lay.gain;
        R.adiag64 = (double *)(base + H.lay.adiag64);
        R.b64 = (double *)(base + H.lay.b64);
        R.mu64 = (double *)(base + H.lay.mu64);
        R.bel64 = (double *)(base + H.lay.bel64);
        R.adiag_w = dtype == GABP_F32 ? (const void *)(base + H.lay.adiag_w) : (const void *)R.adiag64;
        R.b_w = dtype == GABP_F32 ? (const void *)(base + H.lay.b_w) : (const void *)R.b64;
        const gabp_obs &o = inst[i].obs;
        const gabp_noise &nz = inst[i].noise;
        int64_t *tc = nullptr;
        double *ty = nullptr, *tv = nullptr;
        const int64_t *dc = o.cell;
        const double *dy = o.y, *dv = nz.var;
        if (o.n > 0 && !o.on_device) {
            bool ok = hipMalloc((void **)&tc, o.n * sizeof(int64_t)) == hipSuccess &&
                      hipMalloc((void **)&ty, o.n * sizeof(double)) == hipSuccess &&
                      (!nz.var || hipMalloc((void **)&tv, o.n * sizeof(double)) == hipSuccess) &&
                      hipMemcpyAsync(tc, o.cell, o.n * sizeof(int64_t), hipMemcpyHostToDevice, b->stream) == hipSuccess &&
                      hipMemcpyAsync(ty, o.y, o.n * sizeof(double), hipMemcpyHostToDevice, b->stream) == hipSuccess &&
                      (!nz.var || hipMemcpyAsync(tv, nz.var, o.n * sizeof(double), hipMemcpyHostToDevice, b->stream) == hipSuccess);
            if (!ok) {
                (void)hipStreamSynchronize(b->stream);
                (void)hipFree(tc);
                (void)hipFree(ty);
                (void)hipFree(tv);
                b->err = "staging observations failed";
                return bail(GABP_E_NOMEM);
            }
            dc = tc;
            dy = ty;
            dv = tv;
        }
        hipError_t e = gabp::launch_setup(dtype == GABP_F32 ? 0 : 1, H.L, o.n, dc, dy, dv,
                                          nz.var ? 0.0 : nz.sigma * nz.sigma, R.adiag64, R.b64,
                                          nullptr, dtype == GABP_F32 ? base + H.lay.adiag_w : nullptr,
                                          dtype == GABP_F32 ? base + H.lay.b_w : nullptr, b->d_err,
                                          b->stream);
        if (tc || ty || tv) {
            (void)hipStreamSynchronize(b->stream);
            (void)hipFree(tc);
            (void)hipFree(ty);
            (void)hipFree(tv);
        }
        if (e != hipSuccess) {
            b->err = std::string("setup failed: ") + hipGetErrorString(e);
            return bail(GABP_E_DEVICE);
        }
    }
    if (hipMemcpyAsync(b->d_inst, rec.data(), sizeof(BatchInst) * (size_t)n, hipMemcpyHostToDevice,
                       b->stream) != hipSuccess ||
        hipMemcpyAsync(b->p_t, b->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess) {
        b->err = "uploading the instance table failed";
        return bail(GABP_E_DEVICE);
    }
    if (b->p_t[0] != 0u) {
        b->err = "invalid observation (cell out of range, non-finite value or non-positive variance)";
        return bail(GABP_E_INVALID);
    }
    if (upload_lists(b) != GABP_OK) return bail(GABP_E_DEVICE);
    *out = b;
    return GABP_OK;   // create synchronised the internal stream
}

gabp_status gabp_batch_iterate(gabp_batch *b, int32_t n_iters, double damping) {
    if (!b) return GABP_E_INVALID;
    StreamJoin join(b);
    if (!join.ok) return bfail(b, GABP_E_DEVICE, "stream ordering failed");
    if (n_iters < 0 || !(damping > 0.0) || !(damping <= 1.0))
        return bfail(b, GABP_E_INVALID, "need n_iters >= 0 and damping in (0, 1]");
    if (b->lists_dirty) {
        gabp_status st = upload_lists(b);
        if (st != GABP_OK) return st;
    }
    if (b->nact > 0 && n_iters > 0) record_run(b, n_iters);
    gabp_status st = launch_iters(b, n_iters, damping);
    if (st != GABP_OK) return st;
    b->t += n_iters;
    for (auto &H : b->h)
        if (H.running) {
            H.iters += n_iters;
            if (n_iters > 0) H.prev_valid = true;
        }
    return GABP_OK;
}

// Fold one check's read-back into the per-instance state.  Returns true when
// the running set (or a frozen flag) changed.
static bool fold_check(gabp_batch *b, double rel_tol, bool probed) {
    bool changed = false;
    for (int i = 0; i < b->n; ++i) {
        InstHost &H = b->h[i];
        if (!H.running) continue;
        if (b->p_div[i] != 0u) {
            const int64_t t = (int64_t)b->p_div[i];
            H.running = false;
            H.status = GABP_E_DIVERGED;
            H.diverged_at = t;
            H.iters = t;
            H.dbuf = (int)(t & 1);
            // the kept messages are those of the launch that diverged
            for (const BatchRun &r : b->runs) {
                if (r.t0[i] < 0 || t <= r.t0[i] || t > r.t0[i] + r.k) continue;
                const HeldState hs = held_after_batch_run(r.t0[i], r.frozen[i] != 0, r.couples, t);
                H.iters = hs.iter;
                H.dbuf = hs.buf;
                break;
            }
            changed = true;
            continue;
        }
        const double a = std::sqrt(b->p_out[2 * i]), bb = std::sqrt(b->p_out[2 * i + 1]);
        const double rel = bb > 0 ? a / bb : a;
        H.rel = rel;
        if (!std::isfinite(rel) || (H.first_rel > 0 && rel > 1e3 * H.first_rel)) {
            H.running = false;
            H.status = GABP_E_DIVERGED;
            changed = true;
            continue;
        }
        if (H.first_rel < 0) H.first_rel = rel;
        if (rel <= rel_tol) {
            H.running = false;
            H.status = GABP_OK;
            changed = true;
            continue;
        }
        if (probed && !H.frozen && H.prev_valid && H.iters >= 2 &&
            freeze_now(b->p_cnt[i], b->p_mrel[i], b->freeze_slots, b->freeze_rel)) {
            H.frozen = true;
            H.frozen_at = H.iters;
            changed = true;
        }
    }
    return changed;
}

gabp_status gabp_batch_solve(gabp_batch *b, int64_t max_iters, double damping, double rel_tol,
                             int32_t check_every, int64_t *iters_done, double *rel_residual,
                             int32_t *status) {
    if (!b) return GABP_E_INVALID;
    StreamJoin join(b);
    if (!join.ok) return bfail(b, GABP_E_DEVICE, "stream ordering failed");
    if (max_iters < 0 || check_every == 0 || !(rel_tol >= 0) || !(damping > 0.0) ||
        !(damping <= 1.0))
        return bfail(b, GABP_E_INVALID, "need max_iters >= 0, check_every != 0, rel_tol >= 0, damping in (0, 1]");
    // check_every < 0: adaptive chunks, as gabp_solve's, on the slowest
    // running instance; powers of two times |check_every|, at most kMaxChunk,
    // so that few chunk graphs are captured
    constexpr int kMaxChunk = 1280;
    const bool adaptive = check_every < 0;
    const int kmin = adaptive ? -check_every : check_every;
    int next = kmin;
    int64_t run = 0;
    while (run < max_iters) {
        if (b->lists_dirty) {
            gabp_status st = upload_lists(b);
            if (st != GABP_OK) return st;
        }
        if (b->nact == 0) break;
        const int k = (int)std::min<int64_t>(next, max_iters - run);
        // precision-change probes of instances not yet frozen: compare the
        // two newest buffers right after this chunk, outside the graph
        bool need_probe = false;
        for (auto &H : b->h)
            if (H.running && !H.frozen) need_probe = true;
        // the probe's marginal pass must also record belief precisions
        if (need_probe) {
            for (int i = 0; i < b->n; ++i) {
                const InstHost &H = b->h[i];
                b->p_lists[4 * b->n + 2 + i] = (H.running && !H.frozen) ? 1 : 0;
            }
            BHIP(b, hipMemcpyAsync(b->d_probe, b->p_lists + 4 * b->n + 2, sizeof(int) * (size_t)b->n,
                                   hipMemcpyHostToDevice, b->stream));
            BHIP(b, hipStreamSynchronize(b->stream));
        }
        gabp_status st = ensure_graph(b, k, damping);
        if (st != GABP_OK) return st;
        record_run(b, k);
        BHIP(b, hipGraphLaunch(b->gexec, b->stream));
        b->t += k;
        for (auto &H : b->h)
            if (H.running) {
                H.iters += k;
                H.prev_valid = true;
            }
        run += k;
        if (need_probe) {
            st = launch_probes(b);
            if (st != GABP_OK) return st;
            // zero the change flags for the next probe after reading them
        }
        BHIP(b, hipStreamSynchronize(b->stream));
        const bool changed = fold_check(b, rel_tol, need_probe);
        b->runs.clear();
        if (need_probe) {
            BHIP(b, hipMemsetAsync(b->d_cnt, 0, sizeof(unsigned long long) * (size_t)b->n, b->stream));
            BHIP(b, hipMemsetAsync(b->d_mrel, 0, sizeof(uint32_t) * (size_t)b->n, b->stream));
            for (int i = 0; i < b->n; ++i) {
                InstHost &H = b->h[i];
                if (H.frozen && H.frozen_at == H.iters) {
                    char *base = b->ws + H.base;
                    BHIP(b, gabp::launch_gain(b->dtype == GABP_F32 ? 0 : 1, H.L,
                                              base + H.lay.msg[H.iters & 1],
                                              b->dtype == GABP_F32 ? (void *)(base + H.lay.adiag_w)
                                                                   : (void *)(base + H.lay.adiag64),
                                              base + H.lay.gain, b->stream));
                    // frozen within the tolerance: both buffers get the
                    // precision messages the gains come from
                    if (b->p_cnt[i] != 0u)
                        BHIP(b, hipMemcpyAsync(base + H.lay.msg[(H.iters - 1) & 1],
                                               base + H.lay.msg[H.iters & 1],
                                               (size_t)H.L.deg * (size_t)H.L.plane *
                                                   (b->dtype == GABP_F32 ? sizeof(float)
                                                                         : sizeof(double)),
                                               hipMemcpyDeviceToDevice, b->stream));
                }
            }
        }
        if (changed) b->lists_dirty = true;
        next = kmin;
        if (adaptive) {
            double want = (double)kMaxChunk;
            for (auto &H : b->h) {
                if (!H.running) continue;
                double ki = kmin;
                if (H.frozen && H.prev_rel > 0 && H.rel < H.prev_rel && H.rel > 0 &&
                    H.iters > H.prev_iters) {
                    const double rate = std::log(H.rel / H.prev_rel) / (double)(H.iters - H.prev_iters);
                    ki = 0.5 * std::log(rel_tol / H.rel) / rate;
                }
                want = std::min(want, ki);
            }
            while (next * 2 <= kMaxChunk && next * 2 <= want) next *= 2;
        }
        for (auto &H : b->h)
            if (H.running) {
                H.prev_rel = H.rel;
                H.prev_iters = H.iters;
            }
    }
    for (int i = 0; i < b->n; ++i) {
        const InstHost &H = b->h[i];
        if (iters_done) iters_done[i] = H.iters;
        if (rel_residual) rel_residual[i] = H.rel;
        if (status) status[i] = H.running ? GABP_E_NOT_CONVERGED : H.status;
    }
    bool all_ok = true;
    for (const auto &H : b->h) all_ok = all_ok && !H.running && H.status == GABP_OK;
    return all_ok ? GABP_OK : GABP_E_NOT_CONVERGED;
}

gabp_status gabp_batch_posterior(gabp_batch *b, int32_t i, double *mean, double *var) {
    if (!b || i < 0 || i >= b->n) return GABP_E_INVALID;
    StreamJoin join(b);
    if (!join.ok) return bfail(b, GABP_E_DEVICE, "stream ordering failed");
    const InstHost &H = b->h[i];
    char *base = b->ws + H.base;
    BHIP(b, gabp::launch_post(b->dtype == GABP_F32 ? 0 : 1, H.L, base + H.lay.msg[state_buf(H)],
                              (const double *)(base + H.lay.adiag64), (const double *)(base + H.lay.b64),
                              H.frozen ? (const double *)(base + H.lay.bel64) : nullptr, nullptr, mean,
                              var, nullptr, b->stream));
    return GABP_OK;
}

gabp_status gabp_batch_get_messages(gabp_batch *b, int32_t i, void *prec, void *info) {
    if (!b || i < 0 || i >= b->n) return GABP_E_INVALID;
    StreamJoin join(b);
    if (!join.ok) return bfail(b, GABP_E_DEVICE, "stream ordering failed");
    const InstHost &H = b->h[i];
    char *base = b->ws + H.base;
    BHIP(b, gabp::launch_msgs_get(b->dtype == GABP_F32 ? 0 : 1, H.L, base + H.lay.msg[state_buf(H)],
                                  prec, info, b->stream));
    return GABP_OK;
}

gabp_status gabp_batch_log_precisions(gabp_batch *b, int32_t i, float *lam, float *valid) {
    if (!b) return GABP_E_INVALID;
    if (i < 0 || i >= b->n || !lam) return bfail(b, GABP_E_INVALID, "need 0 <= i < n and lam");
    StreamJoin join(b);
    if (!join.ok) return bfail(b, GABP_E_DEVICE, "stream ordering failed");
    const InstHost &H = b->h[i];
    char *base = b->ws + H.base;
    BHIP(b, gabp::launch_log_prec(b->dtype == GABP_F32 ? 0 : 1, H.L, base + H.lay.msg[state_buf(H)],
                                  lam, valid, b->stream));
    return GABP_OK;
}

gabp_status gabp_batch_warm_init(gabp_batch *b, int32_t i, const float *pred,
                                 int32_t keep_precisions) {
    if (!b) return GABP_E_INVALID;
    if (i < 0 || i >= b->n || !pred) return bfail(b, GABP_E_INVALID, "need 0 <= i < n and a pred");
    StreamJoin join(b);
    if (!join.ok) return bfail(b, GABP_E_DEVICE, "stream ordering failed");
    InstHost &H = b->h[i];
    if (H.status == GABP_E_DIVERGED) return bfail(b, GABP_E_DIVERGED, "instance has diverged");
    char *base = b->ws + H.base;
    BHIP(b, gabp::launch_warm_init(b->dtype == GABP_F32 ? 0 : 1, H.L, pred, keep_precisions ? 1 : 0,
                                   base + H.lay.msg[state_buf(H)], b->stream));
    H.prev_valid = false;
    if (H.frozen) b->lists_dirty = true;
    H.frozen = false;
    H.frozen_at = -1;
    return GABP_OK;
}

gabp_status gabp_batch_upscale_precisions(gabp_batch *b, int32_t i, float *pred, int64_t nxf,
                                          int64_t nyf, double scale) {
    if (!b) return GABP_E_INVALID;
    if (i < 0 || i >= b->n || !pred) return bfail(b, GABP_E_INVALID, "need 0 <= i < n and a pred");
    const InstHost &H = b->h[i];
    if (nxf < 1 || nyf < 1 || (nxf + 1) / 2 != H.L.nx || (nyf + 1) / 2 != H.L.ny)
        return bfail(b, GABP_E_INVALID,
                     "upscale_precisions: need ceil(nxf / 2) = nx and ceil(nyf / 2) = ny of the instance");
    if (!(scale > 0.0) || !std::isfinite(scale))
        return bfail(b, GABP_E_INVALID, "upscale_precisions: scale must be finite and > 0");
    StreamJoin join(b);
    if (!join.ok) return bfail(b, GABP_E_DEVICE, "stream ordering failed");
    char *base = b->ws + H.base;
    BHIP(b, gabp::launch_upscale_prec(b->dtype == GABP_F32 ? 0 : 1, H.L,
                                      base + H.lay.msg[state_buf(H)], (float)scale, pred, (int)nxf,
                                      (int)nyf, b->stream));
    return GABP_OK;
}

gabp_status gabp_batch_set_freeze_tolerance(gabp_batch *b, int64_t max_slots, double max_rel) {
    if (!b) return GABP_E_INVALID;
    if (max_slots < 0 || !(max_rel >= 0.0) || !std::isfinite(max_rel))
        return bfail(b, GABP_E_INVALID, "need max_slots >= 0 and a finite max_rel >= 0");
    b->freeze_slots = max_slots;
    b->freeze_rel = max_rel;
    return GABP_OK;
}

gabp_status gabp_batch_autotune(gabp_batch *b, int32_t trials, double damping, int32_t *chosen) {
    if (!b || trials < 1) return GABP_E_INVALID;
    StreamJoin join(b);
    if (!join.ok) return bfail(b, GABP_E_DEVICE, "stream ordering failed");
    hipEvent_t e0, e1;
    BHIP(b, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return bfail(b, GABP_E_DEVICE, "hipEventCreate failed");
    }
    float best = INFINITY;
    int best_r = b->rpt;
    gabp_status st = gabp_batch_iterate(b, 1, damping);
    for (int pass = 0; pass < 2 && st == GABP_OK; ++pass)
        for (int r : gabp::kRptChoices) {
            b->rpt = r;
            b->lists_dirty = true;   // work-item counts depend on the tile shape
            if (hipEventRecord(e0, b->stream) != hipSuccess) { st = GABP_E_DEVICE; break; }
            st = gabp_batch_iterate(b, trials, damping);
            if (st != GABP_OK) break;
            float ms = 0.f;
            if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { st = GABP_E_DEVICE; break; }
            if (ms < best) {
                best = ms;
                best_r = r;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->rpt = best_r;
    b->lists_dirty = true;
    if (st != GABP_OK) return st == GABP_E_DEVICE ? bfail(b, st, "autotune timing failed") : st;
    if (chosen) *chosen = best_r;
    return GABP_OK;
}

gabp_status gabp_batch_info(const gabp_batch *b, int32_t i, int64_t *iters, int64_t *frozen_at,
                            int32_t *running) {
    if (!b || i < 0 || i >= b->n) return GABP_E_INVALID;
    const InstHost &H = b->h[i];
    if (iters) *iters = H.iters;
    if (frozen_at) *frozen_at = H.frozen ? H.frozen_at : -1;
    if (running) *running = H.running ? 1 : 0;
    return GABP_OK;
}

}  // extern "C"

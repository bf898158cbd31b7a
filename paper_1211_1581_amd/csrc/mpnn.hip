// mpnn.hip -- learned factor G of the preconditioner M^-1 = G G^T.
//
// A message-passing network reads the Jacobi-scaled matrix
// A~ = D^-1/2 A D^-1/2 and predicts, on A's own lower-triangular pattern,
// L~ with L~_ii = exp(o_ii) and L~_ij = o_ij (j < i); G = D^-1/2 L~.  Then
// G^T A G = L~^T A~ L~, M^-1 = G G^T is SPD for any output, and a zero head
// gives G = D^-1/2 (Jacobi).  Width 32, SiLU, 4 layers:
//   h_i = W f_i + b,  f_i = [1, log a_ii - mean log a]
//   e_ij = W g_ij + b,  g_ij = [a~_ij, log max(|a~_ij|, 1e-30)]   (i != j)
//   layer: m_ij = W2e silu(W1e [h_i; h_j; e_ij] + c1e) + c2e
//          agg_i = sum over the off-diagonal entries of row i of m_ij
//          h_i += W2n silu(W1n [h_i; agg_i] + c1n) + c2n;  e_ij = m_ij
//   head:  o_ij = w_e . e_ij + c_e (j < i),  o_ii = w_n . h_i + c_n
// Training minimises sum over probes v of ||G^T A G v - v||^2 / (n m).
//
// Layout: activations are BF16 row-major [item][32]; every per-edge and
// per-node MLP runs on 32-row tiles with v_mfma_f32_32x32x16_bf16 (FP32
// accumulation), one tile per wavefront.  Segment sums over a row's edges and
// the backward scatter to column nodes are gathers in fixed order (the
// column-node sum reads the reverse edges of the node's own row), so results
// are deterministic.  Weight gradients are per-workgroup partials reduced in
// fixed order.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "internal.h"
#include "scan.h"
#include "mfma.h"

namespace spcg {
namespace mp {

constexpr int H = 32;
constexpr int NL = 4;
constexpr int L0 = 192;        // first layer's offset in the flat weights
constexpr int LSZ = 7296;      // floats per layer
constexpr int HEAD = L0 + NL * LSZ;
enum : int { E1W = 0, E1B = 3072, E2W = 3104, E2B = 4128, N1W = 4160, N1B = 6208, N2W = 6240, N2B = 7264 };
enum : int { ENW = 0, ENB = 64, EEW = 96, EEB = 160 };
enum : int { HEW = 0, HEB = 32, HNW = 33, HNB = 65 };

// BF16 copies of one layer's weights, row-major [out][in], and transposes [in][out]
struct LayerBf {
    __bf16 w1e[32 * 96], w2e[32 * 32], w1n[32 * 64], w2n[32 * 32];
    __bf16 w1eT[96 * 32], w2eT[32 * 32], w1nT[64 * 32], w2nT[32 * 32];
};

constexpr int kWavesPerWg = 4;  // 256-thread workgroups, one tile per wave at a time

}  // namespace mp
}  // namespace spcg

using namespace spcg;
using namespace spcg::mp;

// Per-matrix state: edge lists, factor patterns, features, factor values.
struct spcg_mpnn {
    spcg_csr *A = nullptr;
    int n = 0, E = 0, nG = 0;
    bool train = false;
    int32_t *erow = nullptr, *ecol = nullptr, *eptr = nullptr, *rev = nullptr, *dpos = nullptr;
    int32_t *cntL = nullptr, *cntU = nullptr;
    int32_t *g_rp = nullptr, *g_col = nullptr, *g_row = nullptr, *gdiag = nullptr;
    int32_t *gt_rp = nullptr, *gt_col = nullptr, *gt_src = nullptr;
    double *s64 = nullptr;
    float *s32 = nullptr, *logd = nullptr, *fe = nullptr, *ge = nullptr;
    float *gvals = nullptr, *gtvals = nullptr, *a32 = nullptr, *lpart = nullptr;
    spcg_csr *G = nullptr, *GT = nullptr, *A32 = nullptr;
    int32_t *flags = nullptr;
    float *scal = nullptr;  // [0] mean log a_ii
    void *h_pinned = nullptr;
};

// Activations and training scratch: a view of slices of the caller's
// workspace (carve_ws), shareable by the graphs of many matrices used one at a
// time on one stream.
struct spcg_mpnn_ws {
    int64_t max_n = 0, max_E = 0, max_nG = 0;
    bool train = false;
    __bf16 *h[NL + 1] = {}, *e[NL + 1] = {};
    LayerBf *wbf = nullptr;
    float *dh[2] = {}, *de[2] = {}, *dxi = nullptr, *dxj = nullptr, *dagg = nullptr;
    float *pw = nullptr, *pu = nullptr, *ps = nullptr, *py = nullptr, *pq = nullptr;
    float *gG = nullptr, *wpart = nullptr, *lpart = nullptr, *scal = nullptr;
};

namespace spcg {
namespace mp {

// ---------------------------------------------------------- graph prep --

// flags[0] error bits: 1 missing/duplicate diagonal, 2 unsorted row,
// 4 structurally unsymmetric, 8 non-positive diagonal
__global__ void k_rowprep(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                          int32_t *dpos, int32_t *cntL, int32_t *cntU, int32_t *eptr,
                          int32_t *erow, int32_t *ecol, int32_t *flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int a = rp[i], b = rp[i + 1];
    int nd = 0, lower = 0, prev = -1, dp = a, err = 0;
    for (int k = a; k < b; ++k) {
        const int c = col[k];
        if (c <= prev) err |= 2;
        prev = c;
        if (c == i) {
            ++nd;
            dp = k;
        } else if (c < i) {
            ++lower;
        }
    }
    if (nd != 1) err |= 1;
    if (err) {
        atomicOr(&flags[0], err);
        return;
    }
    dpos[i] = dp;
    cntL[i] = lower + 1;
    cntU[i] = (b - a - 1 - lower) + 1;
    const int e0 = a - i;
    eptr[i] = e0;
    if (i == n - 1) eptr[n] = b - n;
    for (int k = a; k < b; ++k) {
        if (k == dp) continue;
        const int e = e0 + (k - a) - (k > dp ? 1 : 0);
        erow[e] = i;
        ecol[e] = col[k];
    }
}

// rev[e]: index of the edge (j, i) for e = (i, j)
__global__ void k_rev(int E, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                      const int32_t *__restrict__ erow, const int32_t *__restrict__ ecol,
                      const int32_t *__restrict__ dpos, int32_t *rev, int32_t *flags) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int i = erow[e], j = ecol[e];
    int lo = rp[j], hi = rp[j + 1];
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (col[mid] < i) lo = mid + 1;
        else hi = mid;
    }
    if (lo >= rp[j + 1] || col[lo] != i) {
        atomicOr(&flags[0], 4);
        rev[e] = e;
        return;
    }
    rev[e] = (rp[j] - j) + (lo - rp[j]) - (lo > dpos[j] ? 1 : 0);
}

// G (tril) and G^T (triu) patterns, and the G^T <- G value map
__global__ void k_gmap(int n, const int32_t *__restrict__ eptr, const int32_t *__restrict__ ecol,
                       const int32_t *__restrict__ rev, const int32_t *__restrict__ cntL,
                       const int32_t *__restrict__ g_rp, const int32_t *__restrict__ gt_rp,
                       int32_t *g_col, int32_t *g_row, int32_t *gdiag, int32_t *gt_col,
                       int32_t *gt_src) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int L = cntL[i] - 1;
    const int g0 = g_rp[i], e0 = eptr[i], e1 = eptr[i + 1];
    for (int t = 0; t < L; ++t) {
        g_col[g0 + t] = ecol[e0 + t];
        g_row[g0 + t] = i;
    }
    g_col[g0 + L] = i;
    g_row[g0 + L] = i;
    gdiag[i] = g0 + L;
    const int t0 = gt_rp[i];
    gt_col[t0] = i;
    gt_src[t0] = g0 + L;
    for (int t = L; t < e1 - e0; ++t) {
        const int e = e0 + t;
        const int j = ecol[e];                 // j > i: (j, i) is a lower entry of row j
        const int tr = rev[e] - eptr[j];       // its index among row j's edges
        gt_col[t0 + 1 + (t - L)] = j;
        gt_src[t0 + 1 + (t - L)] = g_rp[j] + tr;
    }
}

// s_i = a_ii^-1/2 and log a_ii; partial sums of log a_ii per workgroup
__global__ void __launch_bounds__(256) k_nodefeat(int n, const double *__restrict__ vals,
                                                  const int32_t *__restrict__ dpos, double *s64,
                                                  float *s32, float *logd, float *lpart,
                                                  int32_t *flags) {
    __shared__ float red[4];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.0f;
    if (i < n) {
        const double d = vals[dpos[i]];
        if (!(d > 0.0)) atomicOr(&flags[0], 8);
        const double s = 1.0 / sqrt(d);
        s64[i] = s;
        s32[i] = (float)s;
        l = (float)log(d);
        logd[i] = l;
    }
    const float t = block_sum(l, red);
    if (threadIdx.x == 0) lpart[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kFinThreads) k_mean(int nparts, const float *part, int n, float *out) {
    float t[1];
    finalize_sum<float, 1>(part, nparts, t);
    if (threadIdx.x == 0) out[0] = t[0] / (float)max(n, 1);
}

// node features [1, log d - mean] and edge features [a~, log |a~|]
__global__ void k_feat(int n, int E, const float *__restrict__ logd, const float *__restrict__ scal,
                       const double *__restrict__ vals, const int32_t *__restrict__ rp,
                       const int32_t *__restrict__ erow, const int32_t *__restrict__ ecol,
                       const int32_t *__restrict__ dpos, const double *__restrict__ s64,
                       float *fe, float *ge) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        fe[2 * t] = 1.0f;
        fe[2 * t + 1] = logd[t] - scal[0];
    }
    if (t < E) {
        const int i = erow[t], j = ecol[t];
        // position of edge t in A: row i, skipping the diagonal
        const int k = rp[i] + (t - (rp[i] - i)) + ((rp[i] + (t - (rp[i] - i))) >= dpos[i] ? 1 : 0);
        const double at = vals[k] * s64[i] * s64[j];
        ge[2 * t] = (float)at;
        ge[2 * t + 1] = (float)log(fmax(fabs(at), 1e-30));
    }
}

__global__ void k_to_f32v(int64_t n, const double *__restrict__ a, float *__restrict__ b) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

__global__ void k_zero_i32(int32_t *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// ----------------------------------------------------------- weights --

__global__ void k_prep_weights(const float *__restrict__ w, LayerBf *wb) {
    const int l = blockIdx.x;
    const float *L = w + L0 + l * LSZ;
    LayerBf &B = wb[l];
    for (int t = threadIdx.x; t < 32 * 96; t += blockDim.x) {
        const int o = t / 96, k = t % 96;
        B.w1e[t] = (__bf16)L[E1W + t];
        B.w1eT[k * 32 + o] = (__bf16)L[E1W + t];
    }
    for (int t = threadIdx.x; t < 32 * 64; t += blockDim.x) {
        const int o = t / 64, k = t % 64;
        B.w1n[t] = (__bf16)L[N1W + t];
        B.w1nT[k * 32 + o] = (__bf16)L[N1W + t];
    }
    for (int t = threadIdx.x; t < 32 * 32; t += blockDim.x) {
        const int o = t / 32, k = t % 32;
        B.w2e[t] = (__bf16)L[E2W + t];
        B.w2eT[k * 32 + o] = (__bf16)L[E2W + t];
        B.w2n[t] = (__bf16)L[N2W + t];
        B.w2nT[k * 32 + o] = (__bf16)L[N2W + t];
    }
}

// ---------------------------------------------------------- encoders --

// encoded edge state, one output: the 2 -> 32 linear map of the edge features,
// rounded once to BF16 (the encoder and the fused first edge layer both use it,
// so the two round identically)
__device__ __forceinline__ __bf16 edge_code(float wg0, float wg1, float b, float g0, float g1) {
    return (__bf16)__fmaf_rn(wg1, g1, __fmaf_rn(wg0, g0, b));
}

__global__ void k_encode(int n, int E, const float *__restrict__ w, const float *__restrict__ fe,
                         const float *__restrict__ ge, __bf16 *h0, __bf16 *e0) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        const float f0 = fe[2 * t], f1 = fe[2 * t + 1];
        for (int o = 0; o < H; ++o)
            h0[(size_t)t * H + o] = (__bf16)(w[ENW + 2 * o] * f0 + w[ENW + 2 * o + 1] * f1 + w[ENB + o]);
    }
    if (t < E) {
        const float g0 = ge[2 * t], g1 = ge[2 * t + 1];
        for (int o = 0; o < H; ++o)
            e0[(size_t)t * H + o] = edge_code(w[EEW + 2 * o], w[EEW + 2 * o + 1], w[EEB + o], g0, g1);
    }
}

// ----------------------------------------------------- layer forward --

// Edge MLP of one layer: m = W2e silu(W1e [h_i; h_j; e] + c1e) + c2e.
// ENC: first layer without a stored edge state; e is encoded from the two edge
// features (weights w) as the fragments are formed.
template <bool ENC>
__global__ void __launch_bounds__(256) k_edge_fwd(int E, const int32_t *__restrict__ erow,
                                                  const int32_t *__restrict__ ecol,
                                                  const __bf16 *__restrict__ hin,
                                                  const __bf16 *__restrict__ ein,
                                                  const float *__restrict__ ge,
                                                  const float *__restrict__ w,
                                                  __bf16 *__restrict__ eout,
                                                  const LayerBf *__restrict__ B,
                                                  const float *__restrict__ Lw) {
    __shared__ __bf16 lds[kWavesPerWg][32 * 40];
    __shared__ float4 encw[H];
    if constexpr (ENC) {
        if (threadIdx.x < H) {
            const int o = threadIdx.x;
            encw[o] = make_float4(w[EEW + 2 * o], w[EEW + 2 * o + 1], w[EEB + o], 0.0f);
        }
        __syncthreads();
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __bf16 *T = lds[wv];
    bf16x8 w1[6], w2[2];
#pragma unroll
    for (int c = 0; c < 6; ++c) w1[c] = frag(B->w1e, 96, c);
#pragma unroll
    for (int c = 0; c < 2; ++c) w2[c] = frag(B->w2e, 32, c);
    const float b1 = Lw[E1B + (lane & 31)], b2 = Lw[E2B + (lane & 31)];
    const int ntiles = (E + 31) / 32;
    const int hh = lane >> 5;
    const int stride = gridDim.x * kWavesPerWg;
    // Software pipeline, one tile deep: each pass issues the next tile's
    // input gathers and the endpoints of the tile after it, then runs this
    // tile's products on inputs gathered one pass earlier.
    auto ends = [&](int t, int &i, int &j) {
        const int e = min(t * 32 + (lane & 31), E - 1);
        i = erow[e];
        j = ecol[e];
    };
    constexpr int NF = ENC ? 4 : 6;  // fragments gathered from memory
    auto gather = [&](int t, int i, int j, bf16x8 (&a)[6], float2 &gf) {
        const int e = min(t * 32 + (lane & 31), E - 1);
        const __bf16 *src[3] = {hin + (size_t)i * H, hin + (size_t)j * H, ein + (size_t)e * H};
#pragma unroll
        for (int c = 0; c < NF; ++c)
            a[c] = *reinterpret_cast<const bf16x8 *>(src[c >> 1] + 16 * (c & 1) + 8 * hh);
        if constexpr (ENC) gf = make_float2(ge[2 * e], ge[2 * e + 1]);
    };
    int tile = blockIdx.x * kWavesPerWg + wv;
    bf16x8 a[6];
    float2 gf = make_float2(0.0f, 0.0f);
    int i_nx = 0, j_nx = 0;
    if (tile < ntiles) {
        int i0, j0;
        ends(tile, i0, j0);
        gather(tile, i0, j0, a, gf);
        if (tile + stride < ntiles) ends(tile + stride, i_nx, j_nx);
    }
    for (; tile < ntiles; tile += stride) {
        bf16x8 a_nx[6];
        float2 gf_nx = make_float2(0.0f, 0.0f);
        const int t1 = tile + stride;
        if (t1 < ntiles) {
            gather(t1, i_nx, j_nx, a_nx, gf_nx);
            if (t1 + stride < ntiles) ends(t1 + stride, i_nx, j_nx);
        }
        if constexpr (ENC) {
#pragma unroll
            for (int c = 4; c < 6; ++c)
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const float4 q = encw[16 * (c & 1) + 8 * hh + k];
                    a[c][k] = edge_code(q.x, q.y, q.z, gf.x, gf.y);
                }
        }
        f32x16 z = splat16(b1);
#pragma unroll
        for (int c = 0; c < 6; ++c) z = mfma32(a[c], w1[c], z);
#pragma unroll
        for (int q = 0; q < 16; ++q) z[q] = silu(z[q]);
        acc_to_lds(z, T, 40, false);
        wave_lds_sync();
        f32x16 m = splat16(b2);
#pragma unroll
        for (int c = 0; c < 2; ++c) m = mfma32(frag(T, 40, c), w2[c], m);
        wave_lds_sync();
        // the message tile goes out through LDS: each lane stores 16
        // consecutive BF16 of one row with two 16-byte stores
        acc_to_lds(m, T, 40, false);
        wave_lds_sync();
        {
            const int rr = lane >> 1, half = lane & 1;
            const int r = tile * 32 + rr;
            if (r < E) {
                const bf16x8 *src = reinterpret_cast<const bf16x8 *>(T + rr * 40 + 16 * half);
                bf16x8 *dst = reinterpret_cast<bf16x8 *>(eout + (size_t)r * H + 16 * half);
                dst[0] = src[0];
                dst[1] = src[1];
            }
        }
        wave_lds_sync();
#pragma unroll
        for (int c = 0; c < NF; ++c) a[c] = a_nx[c];
        gf = gf_nx;
    }
}

// Node MLP of one layer: h += W2n silu(W1n [h; agg] + c1n) + c2n, agg_i = sum of m over row i
__global__ void __launch_bounds__(256) k_node_fwd(int n, const int32_t *__restrict__ eptr,
                                                  const __bf16 *__restrict__ hin,
                                                  const __bf16 *__restrict__ m,
                                                  __bf16 *__restrict__ hout,
                                                  const LayerBf *__restrict__ B,
                                                  const float *__restrict__ Lw) {
    __shared__ __bf16 lds[kWavesPerWg][32 * 40];
    __shared__ float Dl[kWavesPerWg][32 * 33];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __bf16 *T = lds[wv];
    bf16x8 w1[4], w2[2];
#pragma unroll
    for (int c = 0; c < 4; ++c) w1[c] = frag(B->w1n, 64, c);
#pragma unroll
    for (int c = 0; c < 2; ++c) w2[c] = frag(B->w2n, 32, c);
    const float b1 = Lw[N1B + (lane & 31)], b2 = Lw[N2B + (lane & 31)];
    const int ntiles = (n + 31) / 32;
    const int hh = lane >> 5;
    for (int tile = blockIdx.x * kWavesPerWg + wv; tile < ntiles; tile += gridDim.x * kWavesPerWg) {
        const int v = min(tile * 32 + (lane & 31), n - 1);
        float a0[8], a1[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) a0[t] = a1[t] = 0.0f;
        for (int e = eptr[v]; e < eptr[v + 1]; ++e) {
            const bf16x8 x0 = *reinterpret_cast<const bf16x8 *>(m + (size_t)e * H + 8 * hh);
            const bf16x8 x1 = *reinterpret_cast<const bf16x8 *>(m + (size_t)e * H + 16 + 8 * hh);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                a0[t] += (float)x0[t];
                a1[t] += (float)x1[t];
            }
        }
        const __bf16 *hv = hin + (size_t)v * H;
        f32x16 u = splat16(b1);
        u = mfma32(*reinterpret_cast<const bf16x8 *>(hv + 8 * hh), w1[0], u);
        u = mfma32(*reinterpret_cast<const bf16x8 *>(hv + 16 + 8 * hh), w1[1], u);
        u = mfma32(to_bf16x8(a0), w1[2], u);
        u = mfma32(to_bf16x8(a1), w1[3], u);
#pragma unroll
        for (int q = 0; q < 16; ++q) u[q] = silu(u[q]);
        acc_to_lds(u, T, 40, false);
        wave_lds_sync();
        f32x16 d = splat16(b2);
#pragma unroll
        for (int c = 0; c < 2; ++c) d = mfma32(frag(T, 40, c), w2[c], d);
        // the update goes out through LDS (FP32, so the residual sum is the
        // same): each lane adds 16 consecutive values of one row to h and
        // writes them with two 16-byte stores
        float *D = Dl[wv];
#pragma unroll
        for (int q = 0; q < 16; ++q) D[acc_row(q, lane) * 33 + (lane & 31)] = d[q];
        wave_lds_sync();
        {
            const int rr = lane >> 1, half = lane & 1;
            const int r = tile * 32 + rr;
            if (r < n) {
                const size_t o = (size_t)r * H + 16 * half;
                const bf16x8 h0 = *reinterpret_cast<const bf16x8 *>(hin + o);
                const bf16x8 h1 = *reinterpret_cast<const bf16x8 *>(hin + o + 8);
                bf16x8 u0, u1;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    u0[k] = (__bf16)((float)h0[k] + D[rr * 33 + 16 * half + k]);
                    u1[k] = (__bf16)((float)h1[k] + D[rr * 33 + 16 * half + 8 + k]);
                }
                *reinterpret_cast<bf16x8 *>(hout + o) = u0;
                *reinterpret_cast<bf16x8 *>(hout + o + 8) = u1;
            }
        }
        wave_lds_sync();
    }
}

// ------------------------------------------------------------------ head --

// o_ii = w_n . h_i + c_n -> G_ii = s_i exp(o_ii); o_ij = w_e . e_ij + c_e -> G_ij = s_i o_ij
__global__ void k_head(int n, const int32_t *__restrict__ eptr, const int32_t *__restrict__ cntL,
                       const int32_t *__restrict__ g_rp, const __bf16 *__restrict__ h,
                       const __bf16 *__restrict__ e, const float *__restrict__ w,
                       const float *__restrict__ s32, float *gvals) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float *hw = w + HEAD;
    float od = hw[HNB];
    for (int o = 0; o < H; ++o) od += hw[HNW + o] * (float)h[(size_t)i * H + o];
    const int L = cntL[i] - 1, g0 = g_rp[i], e0 = eptr[i];
    const float si = s32[i];
    gvals[g0 + L] = si * __expf(od);
    for (int t = 0; t < L; ++t) {
        float oe = hw[HEB];
        for (int o = 0; o < H; ++o) oe += hw[HEW + o] * (float)e[(size_t)(e0 + t) * H + o];
        gvals[g0 + t] = si * oe;
    }
}

__global__ void k_gt_fill(int nG, const int32_t *__restrict__ src, const float *__restrict__ g,
                          float *gt) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nG) gt[p] = g[src[p]];
}

}  // namespace mp
}  // namespace spcg

namespace spcg {
namespace mp {

// ---------------------------------------------- probe loss and its gradient --

struct EpiStore32 {
    float *__restrict__ y;
    __device__ __forceinline__ NoOperand load(int) const { return {}; }
    __device__ __forceinline__ void row(int i, float s, NoOperand) { y[i] = s; }
};

// t = G^T u (row sums), r = t - v, s = 2 r / (n m); partial sum of r^2
struct EpiResidLoss {
    const float *__restrict__ v;
    float *__restrict__ s;
    float scale;
    float acc;
    __device__ __forceinline__ float load(int i) const { return v[i]; }
    __device__ __forceinline__ void row(int i, float t, float vi) {
        const float r = t - vi;
        s[i] = scale * r;
        acc += r * r;
    }
};

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
k_sp32(CsrDev A, const float *__restrict__ vals, const float *__restrict__ x, float *__restrict__ y) {
    __shared__ SpmvSmem<float, kChunkWide> sm;  // A over its handle's wide partition
    int bs, be;
    block_range(A.n_blocks, bs, be);
    EpiStore32 epi{y};
    for (int b = bs; b < be; ++b) spmv_block<float, float, float>(A, vals, x, b, sm, epi);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
k_sp32_resid(CsrDev A, const float *__restrict__ vals, const float *__restrict__ x,
             const float *__restrict__ v, float *__restrict__ s, float scale, float *part) {
    __shared__ SpmvSmem<float, kChunkWide> sm;  // A over its handle's wide partition
    int bs, be;
    const int slot = block_range(A.n_blocks, bs, be);
    EpiResidLoss epi{v, s, scale, 0.0f};
    for (int b = bs; b < be; ++b) spmv_block<float, float, float>(A, vals, x, b, sm, epi);
    const float t = block_sum(epi.acc, sm.red);
    if (threadIdx.x == 0) part[slot] = t;
}

// dL/dG_p += u_i s_j + q_i v_j for the factor entry p = (i, j)
__global__ void k_sddmm(int nG, const int32_t *__restrict__ g_row, const int32_t *__restrict__ g_col,
                        const float *__restrict__ u, const float *__restrict__ s,
                        const float *__restrict__ q, const float *__restrict__ v, float *gG,
                        int first) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nG) return;
    const int i = g_row[p], j = g_col[p];
    const float g = u[i] * s[j] + q[i] * v[j];
    gG[p] = first ? g : gG[p] + g;
}

__global__ void __launch_bounds__(kFinThreads) k_loss_fin(int nparts, const float *part, float *out) {
    float t[1];
    finalize_sum<float, 1>(part, nparts, t);
    if (threadIdx.x == 0) out[1] = t[0];
}

// ------------------------------------------------------------ backward --

// Head: do_ii = dG_ii G_ii, do_ij = dG_ij s_i; dh4 = do_ii w_n; de4 = do_ij w_e
// (upper edges 0); per-workgroup partials of the head weights [66].
__global__ void __launch_bounds__(256) k_head_bwd(int n, const int32_t *__restrict__ eptr,
                                                  const int32_t *__restrict__ cntL,
                                                  const int32_t *__restrict__ g_rp,
                                                  const __bf16 *__restrict__ h,
                                                  const __bf16 *__restrict__ e,
                                                  const float *__restrict__ w,
                                                  const float *__restrict__ s32,
                                                  const float *__restrict__ gvals,
                                                  const float *__restrict__ gG, float *dh,
                                                  float *de, float *part) {
    __shared__ float red[66][8];
    const float *hw = w + HEAD;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    float acc[66];
#pragma unroll
    for (int k = 0; k < 66; ++k) acc[k] = 0.0f;
    if (i < n) {
        const int L = cntL[i] - 1, g0 = g_rp[i], e0 = eptr[i], e1 = eptr[i + 1];
        const float dod = gG[g0 + L] * gvals[g0 + L];
        for (int o = 0; o < H; ++o) {
            dh[(size_t)i * H + o] = dod * hw[HNW + o];
            acc[HNW + o] += dod * (float)h[(size_t)i * H + o];
        }
        acc[HNB] += dod;
        const float si = s32[i];
        for (int t = 0; t < e1 - e0; ++t) {
            const size_t eo = (size_t)(e0 + t) * H;
            if (t < L) {
                const float doe = gG[g0 + t] * si;
                for (int o = 0; o < H; ++o) {
                    de[eo + o] = doe * hw[HEW + o];
                    acc[HEW + o] += doe * (float)e[eo + o];
                }
                acc[HEB] += doe;
            } else {
                for (int o = 0; o < H; ++o) de[eo + o] = 0.0f;
            }
        }
    }
    // fixed-order workgroup reduction: waves in order, then lanes by butterfly
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 66; ++k) {
        const float t = wave_sum(acc[k]);
        if ((threadIdx.x & 63) == 0) red[k][wv] = t;
    }
    __syncthreads();
    if (threadIdx.x < 66) {
        float t = 0.0f;
        for (int q = 0; q < 4; ++q) t += red[threadIdx.x][q];
        part[(size_t)blockIdx.x * 66 + threadIdx.x] = t;
    }
}

// column sums of an accumulator tile: lane l (< 32) receives the sum of column l
__device__ __forceinline__ float acc_colsum(const f32x16 &d) {
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < 16; ++i) s += d[i];
    s += __shfl_xor(s, 32, 64);
    return s;
}

// write an accumulator tile of a weight gradient [32 rows][ld] at column offset c0
__device__ __forceinline__ void acc_store_w(const f32x16 &d, float *dst, int ld, int c0) {
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < 16; ++i) dst[acc_row(i, l) * ld + c0 + (l & 31)] = d[i];
}

// Node MLP backward of one layer (per 32-node tile and wavefront):
//   dV = dh_l;  dW2n += dV^T S;  dS = dV W2n;  dU = dS * silu'(U);
//   dW1n += dU^T [h; agg];  [dh_part; dagg] = dU W1n;  dh_prev = dh_l + dh_part
// Partials per wave: layer floats N1W .. N2B+32 (3136) in flat order.
__global__ void __launch_bounds__(256) k_node_bwd(int n, const int32_t *__restrict__ eptr,
                                                  const __bf16 *__restrict__ hin,
                                                  const __bf16 *__restrict__ m,
                                                  const float *__restrict__ dh_l,
                                                  float *__restrict__ dh_prev,
                                                  float *__restrict__ dagg,
                                                  const LayerBf *__restrict__ B,
                                                  const float *__restrict__ Lw, float *part) {
    __shared__ __attribute__((aligned(16))) __bf16 lds[kWavesPerWg][4 * 32 * 40 + 64 * 40];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, hh = lane >> 5;
    __bf16 *TA = lds[wv], *TB = TA + 32 * 40, *TC = TB + 32 * 40, *TD = TC + 32 * 40;
    __bf16 *TX = TD + 32 * 40;  // [64][40]: X^T
    bf16x8 w1[4], w2[2];
#pragma unroll
    for (int c = 0; c < 4; ++c) w1[c] = frag(B->w1n, 64, c);
#pragma unroll
    for (int c = 0; c < 2; ++c) w2[c] = frag(B->w2n, 32, c);
    const float b1 = Lw[N1B + (lane & 31)];
    f32x16 gW1[2] = {splat16(0.0f), splat16(0.0f)}, gW2 = splat16(0.0f);
    float gb1 = 0.0f, gb2 = 0.0f;
    const int ntiles = (n + 31) / 32;
    for (int tile = blockIdx.x * kWavesPerWg + wv; tile < ntiles; tile += gridDim.x * kWavesPerWg) {
        const int v = min(tile * 32 + (lane & 31), n - 1);
        float a0[8], a1[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) a0[t] = a1[t] = 0.0f;
        for (int e = eptr[v]; e < eptr[v + 1]; ++e) {
            const bf16x8 x0 = *reinterpret_cast<const bf16x8 *>(m + (size_t)e * H + 8 * hh);
            const bf16x8 x1 = *reinterpret_cast<const bf16x8 *>(m + (size_t)e * H + 16 + 8 * hh);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                a0[t] += (float)x0[t];
                a1[t] += (float)x1[t];
            }
        }
        const __bf16 *hv = hin + (size_t)v * H;
        bf16x8 xf[4];
        xf[0] = *reinterpret_cast<const bf16x8 *>(hv + 8 * hh);
        xf[1] = *reinterpret_cast<const bf16x8 *>(hv + 16 + 8 * hh);
        xf[2] = to_bf16x8(a0);
        xf[3] = to_bf16x8(a1);
        f32x16 u = splat16(b1);
#pragma unroll
        for (int c = 0; c < 4; ++c) u = mfma32(xf[c], w1[c], u);
        // dV from dh_l; rows past n are zero
        f32x16 dv, sv;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int r = tile * 32 + acc_row(q, lane);
            dv[q] = r < n ? dh_l[(size_t)r * H + (lane & 31)] : 0.0f;
            sv[q] = silu(u[q]);
        }
        // X^T into LDS: lane holds X[l%32][16c + 8hh + t]
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int t = 0; t < 8; ++t) TX[(16 * c + 8 * hh + t) * 40 + (lane & 31)] = xf[c][t];
        acc_to_lds(dv, TA, 40, true);   // dV^T [o][node]
        acc_to_lds(sv, TB, 40, true);   // S^T  [hd][node]
        acc_to_lds(dv, TC, 40, false);  // dV   [node][o]
        wave_lds_sync();
        // dW2n[o][hd] += sum_node dV[node][o] S[node][hd]
#pragma unroll
        for (int c = 0; c < 2; ++c) gW2 = mfma32(frag(TA, 40, c), frag(TB, 40, c), gW2);
        gb2 += acc_colsum(dv);
        // dS = dV W2n ; dU = dS * silu'(U)
        f32x16 du = splat16(0.0f);
#pragma unroll
        for (int c = 0; c < 2; ++c) du = mfma32(frag(TC, 40, c), frag(B->w2nT, 32, c), du);
#pragma unroll
        for (int q = 0; q < 16; ++q) du[q] *= silu_grad(u[q]);
        gb1 += acc_colsum(du);
        wave_lds_sync();
        acc_to_lds(du, TA, 40, true);   // dU^T [o][node]
        acc_to_lds(du, TC, 40, false);  // dU   [node][o]
        wave_lds_sync();
        // dW1n[o][f] += sum_node dU[node][o] X[node][f], f in two tiles of 32
#pragma unroll
        for (int ft = 0; ft < 2; ++ft)
#pragma unroll
            for (int c = 0; c < 2; ++c)
                gW1[ft] = mfma32(frag(TA, 40, c), frag(TX + ft * 32 * 40, 40, c), gW1[ft]);
        // dX = dU W1n: tile 0 -> dh_part, tile 1 -> dagg
        f32x16 dx0 = splat16(0.0f), dx1 = splat16(0.0f);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const bf16x8 a = frag(TC, 40, c);
            dx0 = mfma32(a, frag(B->w1nT, 32, c), dx0);
            dx1 = mfma32(a, frag(B->w1nT + 32 * 32, 32, c), dx1);
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int r = tile * 32 + acc_row(q, lane);
            if (r < n) {
                const size_t o = (size_t)r * H + (lane & 31);
                dh_prev[o] = dh_l[o] + dx0[q];
                dagg[o] = dx1[q];
            }
        }
        wave_lds_sync();
    }
    float *P = part + (size_t)(blockIdx.x * kWavesPerWg + wv) * 3136;
    acc_store_w(gW1[0], P, 64, 0);
    acc_store_w(gW1[1], P, 64, 32);
    acc_store_w(gW2, P + (N2W - N1W), 32, 0);
    if (lane < 32) {
        P[N1B - N1W + lane] = gb1;
        P[N2B - N1W + lane] = gb2;
    }
}

// Edge MLP backward of one layer (per 32-edge tile and wavefront):
//   dm = de_l + dagg[row];  dW2e += dm^T S;  dS = dm W2e;  dZ = dS * silu'(Z);
//   dW1e += dZ^T X;  dX = dZ W1e -> (dxi, dxj, de_prev)
// Partials per wave: layer floats E1W .. E2B+32 (4160) in flat order.
__global__ void __launch_bounds__(256) k_edge_bwd(int E, const int32_t *__restrict__ erow,
                                                  const int32_t *__restrict__ ecol,
                                                  const __bf16 *__restrict__ hin,
                                                  const __bf16 *__restrict__ ein,
                                                  const float *__restrict__ de_l,
                                                  const float *__restrict__ dagg,
                                                  float *__restrict__ dxi, float *__restrict__ dxj,
                                                  float *__restrict__ de_prev,
                                                  const LayerBf *__restrict__ B,
                                                  const float *__restrict__ Lw, float *part) {
    __shared__ __attribute__((aligned(16))) __bf16 lds[kWavesPerWg][3 * 32 * 40 + 96 * 40];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, hh = lane >> 5;
    __bf16 *TA = lds[wv], *TB = TA + 32 * 40, *TC = TB + 32 * 40, *TX = TC + 32 * 40;
    bf16x8 w1[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) w1[c] = frag(B->w1e, 96, c);
    const float b1 = Lw[E1B + (lane & 31)];
    f32x16 gW1[3] = {splat16(0.0f), splat16(0.0f), splat16(0.0f)}, gW2 = splat16(0.0f);
    float gb1 = 0.0f, gb2 = 0.0f;
    const int ntiles = (E + 31) / 32;
    for (int tile = blockIdx.x * kWavesPerWg + wv; tile < ntiles; tile += gridDim.x * kWavesPerWg) {
        const int e = min(tile * 32 + (lane & 31), E - 1);
        const int i = erow[e], j = ecol[e];
        const __bf16 *src[3] = {hin + (size_t)i * H, hin + (size_t)j * H, ein + (size_t)e * H};
        bf16x8 xf[6];
        f32x16 z = splat16(b1);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            xf[c] = *reinterpret_cast<const bf16x8 *>(src[c >> 1] + 16 * (c & 1) + 8 * hh);
            z = mfma32(xf[c], w1[c], z);
        }
        f32x16 dm, sv;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int r = tile * 32 + acc_row(q, lane);
            float g = 0.0f;
            if (r < E) g = de_l[(size_t)r * H + (lane & 31)] + dagg[(size_t)erow[r] * H + (lane & 31)];
            dm[q] = g;
            sv[q] = silu(z[q]);
        }
#pragma unroll
        for (int c = 0; c < 6; ++c)
#pragma unroll
            for (int t = 0; t < 8; ++t) TX[(16 * c + 8 * hh + t) * 40 + (lane & 31)] = xf[c][t];
        acc_to_lds(dm, TA, 40, true);   // dm^T
        acc_to_lds(sv, TB, 40, true);   // S^T
        acc_to_lds(dm, TC, 40, false);  // dm
        wave_lds_sync();
#pragma unroll
        for (int c = 0; c < 2; ++c) gW2 = mfma32(frag(TA, 40, c), frag(TB, 40, c), gW2);
        gb2 += acc_colsum(dm);
        f32x16 dz = splat16(0.0f);
#pragma unroll
        for (int c = 0; c < 2; ++c) dz = mfma32(frag(TC, 40, c), frag(B->w2eT, 32, c), dz);
#pragma unroll
        for (int q = 0; q < 16; ++q) dz[q] *= silu_grad(z[q]);
        gb1 += acc_colsum(dz);
        wave_lds_sync();
        acc_to_lds(dz, TA, 40, true);
        acc_to_lds(dz, TC, 40, false);
        wave_lds_sync();
#pragma unroll
        for (int ft = 0; ft < 3; ++ft)
#pragma unroll
            for (int c = 0; c < 2; ++c)
                gW1[ft] = mfma32(frag(TA, 40, c), frag(TX + ft * 32 * 40, 40, c), gW1[ft]);
        float *outs[3] = {dxi, dxj, de_prev};
#pragma unroll
        for (int ft = 0; ft < 3; ++ft) {
            f32x16 dx = splat16(0.0f);
#pragma unroll
            for (int c = 0; c < 2; ++c) dx = mfma32(frag(TC, 40, c), frag(B->w1eT + ft * 32 * 32, 32, c), dx);
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int r = tile * 32 + acc_row(q, lane);
                if (r < E) outs[ft][(size_t)r * H + (lane & 31)] = dx[q];
            }
        }
        wave_lds_sync();
    }
    float *P = part + (size_t)(blockIdx.x * kWavesPerWg + wv) * 4160;
    for (int ft = 0; ft < 3; ++ft) acc_store_w(gW1[ft], P, 96, 32 * ft);
    acc_store_w(gW2, P + (E2W - E1W), 32, 0);
    if (lane < 32) {
        P[E1B - E1W + lane] = gb1;
        P[E2B - E1W + lane] = gb2;
    }
}

// dh_prev[i] += sum over row i's edges e of dxi[e] + dxj[rev(e)]  (fixed order)
__global__ void k_node_gather(int n, const int32_t *__restrict__ eptr, const int32_t *__restrict__ rev,
                              const float *__restrict__ dxi, const float *__restrict__ dxj,
                              float *dh_prev) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * H) return;
    const int i = (int)(t / H), o = (int)(t % H);
    float s = dh_prev[t];
    for (int e = eptr[i]; e < eptr[i + 1]; ++e) s += dxi[(size_t)e * H + o] + dxj[(size_t)rev[e] * H + o];
    dh_prev[t] = s;
}

// encoder gradients, per-workgroup partials [192] in flat order
__global__ void __launch_bounds__(256) k_enc_bwd(int n, int E, const float *__restrict__ fe,
                                                 const float *__restrict__ ge,
                                                 const float *__restrict__ dh0,
                                                 const float *__restrict__ de0, float *part) {
    __shared__ float red[8][192];
    const int o = threadIdx.x & 31, sub = threadIdx.x >> 5;
    float a[6] = {0, 0, 0, 0, 0, 0};
    for (int i = blockIdx.x * 8 + sub; i < n; i += gridDim.x * 8) {
        const float g = dh0[(size_t)i * H + o];
        a[0] += g * fe[2 * i];
        a[1] += g * fe[2 * i + 1];
        a[2] += g;
    }
    for (int e = blockIdx.x * 8 + sub; e < E; e += gridDim.x * 8) {
        const float g = de0[(size_t)e * H + o];
        a[3] += g * ge[2 * e];
        a[4] += g * ge[2 * e + 1];
        a[5] += g;
    }
    red[sub][ENW + 2 * o] = a[0];
    red[sub][ENW + 2 * o + 1] = a[1];
    red[sub][ENB + o] = a[2];
    red[sub][EEW + 2 * o] = a[3];
    red[sub][EEW + 2 * o + 1] = a[4];
    red[sub][EEB + o] = a[5];
    __syncthreads();
    if (threadIdx.x < 192) {
        float s = 0.0f;
        for (int q = 0; q < 8; ++q) s += red[q][threadIdx.x];
        part[(size_t)blockIdx.x * 192 + threadIdx.x] = s;
    }
}

// grads[off + j] = sum over slots (in order) of part[slot * len + j]
__global__ void k_wreduce(int slots, int len, const float *__restrict__ part, float *grads, int off) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= len) return;
    float s = 0.0f;
    for (int q = 0; q < slots; ++q) s += part[(size_t)q * len + j];
    grads[off + j] = s;
}

__global__ void k_adam(int64_t n, float *w, const float *g, float *m, float *v, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace mp
}  // namespace spcg

// ================================================================= C ABI ==

namespace {

template <typename T>
void free_dev(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

int release(spcg_mpnn *g) {
    if (!g) return SPCG_OK;
    if (g->G) spcg_csr_destroy(g->G);
    if (g->GT) spcg_csr_destroy(g->GT);
    if (g->A32) spcg_csr_destroy(g->A32);
    free_dev(g->erow); free_dev(g->ecol); free_dev(g->eptr); free_dev(g->rev); free_dev(g->dpos);
    free_dev(g->cntL); free_dev(g->cntU); free_dev(g->g_rp); free_dev(g->g_col); free_dev(g->g_row);
    free_dev(g->gdiag); free_dev(g->gt_rp); free_dev(g->gt_col); free_dev(g->gt_src);
    free_dev(g->s64); free_dev(g->s32); free_dev(g->logd); free_dev(g->fe); free_dev(g->ge);
    free_dev(g->gvals); free_dev(g->gtvals); free_dev(g->a32); free_dev(g->lpart);
    free_dev(g->flags); free_dev(g->scal);
    if (g->h_pinned) (void)hipHostFree(g->h_pinned);
    delete g;
    return SPCG_OK;
}

unsigned g1(int64_t n, int per = 256) { return (unsigned)std::max<int64_t>((n + per - 1) / per, 1); }

// workgroups of the tile kernels: forward, and backward (bounded: per-wave partials).
// The edge forward kernel holds 148 registers per lane (3 wavefronts per SIMD),
// so 768 = 256 CUs x 3 workgroups of 4 wavefronts is the resident grid: one
// generation of workgroups, no tail.
unsigned tile_wgs(int64_t items, int cap) {
    const int64_t tiles = (items + 31) / 32;
    return (unsigned)std::max<int64_t>(std::min<int64_t>((tiles + kWavesPerWg - 1) / kWavesPerWg, cap), 1);
}
constexpr int kFwdCap = 2048, kEdgeCap = 768, kBwdCap = 256, kSmallCap = 512, kMaxProbes = 64;

__bf16 *hbuf(const spcg_mpnn_ws *w, int l) { return w->train ? w->h[l] : w->h[l & 1]; }
__bf16 *ebuf(const spcg_mpnn_ws *w, int l) { return w->train ? w->e[l] : w->e[l & 1]; }

// Workspace slices (256-byte aligned) for graphs of up to n rows and E edges:
// per layer BF16 node and edge activations (all layers when training, two
// alternating ones for inference), the BF16 weight copies, scalars and, for
// training, the gradient and probe-product scratch.  base = nullptr only sizes.
size_t carve_ws(int64_t n, int64_t E, bool train, char *base, spcg_mpnn_ws *w) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        char *q = base ? base + off : nullptr;
        off += align256(std::max<size_t>(bytes, 1));
        return q;
    };
    spcg_mpnn_ws W;
    W.max_n = n;
    W.max_E = E;
    W.max_nG = n + E / 2;
    W.train = train;
    const int nbuf = train ? NL + 1 : 2;
    for (int l = 0; l < nbuf; ++l) {
        W.h[l] = (__bf16 *)take(sizeof(__bf16) * n * H);
        W.e[l] = (__bf16 *)take(sizeof(__bf16) * E * H);
    }
    W.wbf = (LayerBf *)take(sizeof(LayerBf) * NL);
    W.scal = (float *)take(sizeof(float) * 64);
    if (train) {
        for (int q = 0; q < 2; ++q) {
            W.dh[q] = (float *)take(sizeof(float) * n * H);
            W.de[q] = (float *)take(sizeof(float) * E * H);
        }
        W.dxi = (float *)take(sizeof(float) * E * H);
        W.dxj = (float *)take(sizeof(float) * E * H);
        W.dagg = (float *)take(sizeof(float) * n * H);
        float **vecs[] = {&W.pw, &W.pu, &W.ps, &W.py, &W.pq};
        for (float **v : vecs) *v = (float *)take(sizeof(float) * n);
        W.gG = (float *)take(sizeof(float) * W.max_nG);
        W.wpart = (float *)take(sizeof(float) * std::max<int64_t>((int64_t)kBwdCap * kWavesPerWg * 4160,
                                                                    (int64_t)g1(n) * 66));
        W.lpart = (float *)take(sizeof(float) * (size_t)kMaxProbes * kMaxGrid);
    }
    if (w) *w = W;
    return off;
}

// The caller's workspace as slices for graph g, or an error if it is too small
// or misaligned.
int bind_ws(const spcg_mpnn *g, bool train, void *d_work, size_t work_bytes, spcg_mpnn_ws *w) {
    if (!d_work || ((uintptr_t)d_work & 255) != 0) return SPCG_INVALID_ARG;
    if (work_bytes < carve_ws(g->n, g->E, train, nullptr, nullptr)) return SPCG_INVALID_ARG;
    carve_ws(g->n, g->E, train, (char *)d_work, w);
    return SPCG_OK;
}

int forward(spcg_mpnn *g, spcg_mpnn_ws *ws, const float *w, hipStream_t s) {
    hipLaunchKernelGGL(k_prep_weights, dim3(NL), dim3(256), 0, s, w, ws->wbf);
    // Without training the encoded edge state is never stored: the first edge
    // layer forms it from the edge features. Training keeps it for the backward pass.
    const bool fuse = !ws->train;
    const int64_t E_enc = fuse ? 0 : g->E;
    hipLaunchKernelGGL(k_encode, dim3(g1(std::max<int64_t>(g->n, E_enc))), dim3(256), 0, s, g->n, (int)E_enc,
                       w, (const float *)g->fe, (const float *)g->ge, hbuf(ws, 0), ebuf(ws, 0));
    for (int l = 1; l <= NL; ++l) {
        const float *Lw = w + L0 + (l - 1) * LSZ;
        if (g->E > 0) {
            const dim3 grid(tile_wgs(g->E, kEdgeCap));
            if (l == 1 && fuse)
                hipLaunchKernelGGL(k_edge_fwd<true>, grid, dim3(256), 0, s, g->E, g->erow, g->ecol,
                                   hbuf(ws, 0), (const __bf16 *)nullptr, (const float *)g->ge, w,
                                   ebuf(ws, 1), ws->wbf, Lw);
            else
                hipLaunchKernelGGL(k_edge_fwd<false>, grid, dim3(256), 0, s, g->E, g->erow, g->ecol,
                                   hbuf(ws, l - 1), ebuf(ws, l - 1), (const float *)nullptr, w,
                                   ebuf(ws, l), ws->wbf + (l - 1), Lw);
        }
        hipLaunchKernelGGL(k_node_fwd, dim3(tile_wgs(g->n, kFwdCap)), dim3(256), 0, s, g->n,
                           g->eptr, hbuf(ws, l - 1), ebuf(ws, l), hbuf(ws, l), ws->wbf + (l - 1), Lw);
    }
    hipLaunchKernelGGL(k_head, dim3(g1(g->n)), dim3(256), 0, s, g->n, g->eptr, g->cntL, g->g_rp,
                       hbuf(ws, NL), ebuf(ws, NL), w, (const float *)g->s32, g->gvals);
    hipLaunchKernelGGL(k_gt_fill, dim3(g1(g->nG)), dim3(256), 0, s, g->nG, g->gt_src,
                       (const float *)g->gvals, g->gtvals);
    SPCG_LAUNCH_CHECK("mpnn forward");
    return SPCG_OK;
}

}  // namespace

extern "C" {

size_t spcg_mpnn_workspace_bytes(int64_t max_rows, int64_t max_edges, int32_t flags) {
    if (max_rows < 1 || max_edges < 0) return 0;
    return carve_ws(max_rows, max_edges, (flags & SPCG_MPNN_TRAIN) != 0, nullptr, nullptr);
}

int spcg_mpnn_create(spcg_mpnn_t *out, spcg_csr_t A, int32_t flags, hipStream_t s) {
    if (!out || !A) return SPCG_INVALID_ARG;
    *out = nullptr;
    if (A->dtype != SPCG_F64 || A->n_rows != A->n_cols || A->n_rows < 1) return SPCG_INVALID_ARG;
    spcg_mpnn *g = new (std::nothrow) spcg_mpnn;
    if (!g) return SPCG_INVALID_ARG;
    g->A = A;
    g->n = A->n_rows;
    g->E = (int)(A->nnz - A->n_rows);
    g->train = (flags & SPCG_MPNN_TRAIN) != 0;
    const int n = g->n;
    const int64_t E = std::max(g->E, 0);
#define MP_TRY(expr)                                                         \
    do {                                                                     \
        hipError_t e_ = (expr);                                              \
        if (e_ != hipSuccess) { release(g); return hip_status(e_, #expr); } \
    } while (0)
#define MP_ALLOC(ptr, count) MP_TRY(hipMalloc(&(ptr), sizeof(*(ptr)) * (size_t)std::max<int64_t>((count), 1)))
    if (g->E < 0) { release(g); return SPCG_INVALID_CSR; }
    MP_ALLOC(g->flags, 64);
    MP_ALLOC(g->scal, 64);
    MP_TRY(hipHostMalloc(&g->h_pinned, 256, hipHostMallocDefault));
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, g->flags, 64);
    MP_ALLOC(g->erow, E);
    MP_ALLOC(g->ecol, E);
    MP_ALLOC(g->rev, E);
    MP_ALLOC(g->eptr, n + 1);
    MP_ALLOC(g->dpos, n);
    MP_ALLOC(g->cntL, n);
    MP_ALLOC(g->cntU, n);
    MP_ALLOC(g->g_rp, n + 1);
    MP_ALLOC(g->gt_rp, n + 1);
    hipLaunchKernelGGL(k_rowprep, dim3(g1(n)), dim3(256), 0, s, n, A->row_ptr, A->col, g->dpos,
                       g->cntL, g->cntU, g->eptr, g->erow, g->ecol, g->flags);
    if (E > 0)
        hipLaunchKernelGGL(k_rev, dim3(g1(E)), dim3(256), 0, s, (int)E, A->row_ptr, A->col,
                           g->erow, g->ecol, g->dpos, g->rev, g->flags);
    {
        const int nb = (n + kScanChunk - 1) / kScanChunk;
        MP_ALLOC(g->lpart, std::max<int64_t>(nb + 1, g1(n)));
        int32_t *sums = reinterpret_cast<int32_t *>(g->lpart);
        const int32_t *cnts[2] = {g->cntL, g->cntU};
        int32_t *outs[2] = {g->g_rp, g->gt_rp};
        for (int q = 0; q < 2; ++q) {
            hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(256), 0, s, n, cnts[q], sums);
            hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, nb, sums);
            hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(256), 0, s, n, cnts[q],
                               (const int32_t *)sums, outs[q]);
        }
    }
    MP_TRY(hipGetLastError());
    int32_t *hp = (int32_t *)g->h_pinned;
    MP_TRY(hipMemcpyAsync(hp, g->flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MP_TRY(hipMemcpyAsync(hp + 1, g->g_rp + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MP_TRY(hipMemcpyAsync(hp + 2, g->gt_rp + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MP_TRY(hipStreamSynchronize(s));
    if (hp[0] != 0 || hp[1] != hp[2]) {
        release(g);
        return SPCG_INVALID_CSR;
    }
    g->nG = hp[1];
    MP_ALLOC(g->g_col, g->nG);
    MP_ALLOC(g->g_row, g->nG);
    MP_ALLOC(g->gt_col, g->nG);
    MP_ALLOC(g->gt_src, g->nG);
    MP_ALLOC(g->gdiag, n);
    MP_ALLOC(g->gvals, g->nG);
    MP_ALLOC(g->gtvals, g->nG);
    hipLaunchKernelGGL(k_gmap, dim3(g1(n)), dim3(256), 0, s, n, g->eptr, g->ecol, g->rev, g->cntL,
                       g->g_rp, g->gt_rp, g->g_col, g->g_row, g->gdiag, g->gt_col, g->gt_src);
    MP_ALLOC(g->s64, n);
    MP_ALLOC(g->s32, n);
    MP_ALLOC(g->logd, n);
    MP_ALLOC(g->fe, 2 * (int64_t)n);
    MP_ALLOC(g->ge, 2 * E);
    const int nfp = (int)g1(n);
    hipLaunchKernelGGL(k_nodefeat, dim3(nfp), dim3(256), 0, s, n, (const double *)A->vals, g->dpos,
                       g->s64, g->s32, g->logd, g->lpart, g->flags);
    hipLaunchKernelGGL(k_mean, dim3(1), dim3(kFinThreads), 0, s, nfp, (const float *)g->lpart, n,
                       g->scal);
    hipLaunchKernelGGL(k_feat, dim3(g1(std::max<int64_t>(n, E))), dim3(256), 0, s, n, (int)E,
                       (const float *)g->logd, (const float *)g->scal, (const double *)A->vals,
                       A->row_ptr, g->erow, g->ecol, g->dpos, (const double *)g->s64, g->fe, g->ge);
    MP_TRY(hipGetLastError());
    if (g->train) {
        MP_ALLOC(g->a32, A->nnz);
        hipLaunchKernelGGL(k_to_f32v, dim3(g1(A->nnz, 2048)), dim3(256), 0, s, A->nnz,
                           (const double *)A->vals, g->a32);
    }
    MP_TRY(hipStreamSynchronize(s));
    MP_TRY(hipMemcpyAsync(hp, g->flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MP_TRY(hipStreamSynchronize(s));
    if (hp[0] != 0) {
        release(g);
        return (hp[0] & 8) ? SPCG_NOT_SPD : SPCG_INVALID_CSR;
    }
    int rc = spcg_csr_create(&g->G, n, n, g->nG, g->g_rp, g->g_col, g->gvals, SPCG_F32, s);
    if (rc == SPCG_OK)
        rc = spcg_csr_create(&g->GT, n, n, g->nG, g->gt_rp, g->gt_col, g->gtvals, SPCG_F32, s);
    if (rc == SPCG_OK && g->train)
        rc = spcg_csr_create(&g->A32, n, n, A->nnz, A->row_ptr, A->col, g->a32, SPCG_F32, s);
    if (rc != SPCG_OK) {
        release(g);
        return rc;
    }
#undef MP_ALLOC
#undef MP_TRY
    *out = g;
    return SPCG_OK;
}

int spcg_mpnn_destroy(spcg_mpnn_t g) {
    if (!g) return SPCG_INVALID_ARG;
    hipError_t e = hipDeviceSynchronize();
    release(g);
    return e == hipSuccess ? SPCG_OK : hip_status(e, "hipDeviceSynchronize");
}

int spcg_mpnn_info(spcg_mpnn_t g, int64_t *n_edges, int64_t *nnz_factor) {
    if (!g) return SPCG_INVALID_ARG;
    if (n_edges) *n_edges = g->E;
    if (nnz_factor) *nnz_factor = g->nG;
    return SPCG_OK;
}

int spcg_mpnn_factor(spcg_mpnn_t g, spcg_csr_t *G, spcg_csr_t *GT) {
    if (!g || !G || !GT) return SPCG_INVALID_ARG;
    *G = g->G;
    *GT = g->GT;
    return SPCG_OK;
}

int spcg_mpnn_factor_arrays(spcg_mpnn_t g, const int32_t **d_row_ptr, const int32_t **d_col,
                            const float **d_vals, const float **d_t_vals) {
    if (!g) return SPCG_INVALID_ARG;
    if (d_row_ptr) *d_row_ptr = g->g_rp;
    if (d_col) *d_col = g->g_col;
    if (d_vals) *d_vals = g->gvals;
    if (d_t_vals) *d_t_vals = g->gtvals;
    return SPCG_OK;
}

int spcg_mpnn_predict(spcg_mpnn_t g, const float *d_w, void *d_work, size_t work_bytes,
                      hipStream_t s) {
    if (!g || !d_w) return SPCG_INVALID_ARG;
    spcg_mpnn_ws view;
    int rc = bind_ws(g, false, d_work, work_bytes, &view);
    if (rc) return rc;
    return forward(g, &view, d_w, s);
}

int spcg_mpnn_loss_grad(spcg_mpnn_t g, const float *d_w, const float *d_probes, int32_t m,
                        float *d_grad, double *h_loss, void *d_work, size_t work_bytes,
                        hipStream_t s) {
    if (!g || !d_w || !d_probes || m < 1 || m > kMaxProbes || !g->train) return SPCG_INVALID_ARG;
    spcg_mpnn_ws view;
    int rc = bind_ws(g, true, d_work, work_bytes, &view);
    if (rc) return rc;
    spcg_mpnn_ws *ws = &view;
    rc = forward(g, ws, d_w, s);
    if (rc) return rc;
    const int n = g->n, E = g->E;
    // the FP32 products over the handles' wide row-block partitions
    const CsrDev Gd = dev_view_wide(g->G), GTd = dev_view_wide(g->GT), Ad = dev_view_wide(g->A32);
    const unsigned gG = spmv_grid(g->G->n_wblocks), gGT = spmv_grid(g->GT->n_wblocks),
                   gA = spmv_grid(g->A32->n_wblocks);
    const float scale = 2.0f / ((float)n * (float)m);
    for (int k = 0; k < m; ++k) {
        const float *v = d_probes + (size_t)k * n;
        hipLaunchKernelGGL(k_sp32, dim3(gG), dim3(256), 0, s, Gd, (const float *)g->gvals, v, ws->pw);
        hipLaunchKernelGGL(k_sp32, dim3(gA), dim3(256), 0, s, Ad, (const float *)g->a32,
                           (const float *)ws->pw, ws->pu);
        hipLaunchKernelGGL(k_sp32_resid, dim3(gGT), dim3(256), 0, s, GTd, (const float *)g->gtvals,
                           (const float *)ws->pu, v, ws->ps, scale, ws->lpart + (size_t)k * gGT);
        hipLaunchKernelGGL(k_sp32, dim3(gG), dim3(256), 0, s, Gd, (const float *)g->gvals,
                           (const float *)ws->ps, ws->py);
        hipLaunchKernelGGL(k_sp32, dim3(gA), dim3(256), 0, s, Ad, (const float *)g->a32,
                           (const float *)ws->py, ws->pq);
        hipLaunchKernelGGL(k_sddmm, dim3(g1(g->nG)), dim3(256), 0, s, g->nG, g->g_row, g->g_col,
                           (const float *)ws->pu, (const float *)ws->ps, (const float *)ws->pq, v,
                           ws->gG, k == 0 ? 1 : 0);
    }
    hipLaunchKernelGGL(k_loss_fin, dim3(1), dim3(kFinThreads), 0, s, (int)(m * gGT),
                       (const float *)ws->lpart, ws->scal);
    SPCG_LAUNCH_CHECK("mpnn loss");
    if (d_grad) {
        const unsigned hw = g1(n);
        hipLaunchKernelGGL(k_head_bwd, dim3(hw), dim3(256), 0, s, n, g->eptr, g->cntL, g->g_rp,
                           (const __bf16 *)ws->h[NL], (const __bf16 *)ws->e[NL], d_w,
                           (const float *)g->s32, (const float *)g->gvals, (const float *)ws->gG,
                           ws->dh[0], ws->de[0], ws->wpart);
        hipLaunchKernelGGL(k_wreduce, dim3(1), dim3(128), 0, s, (int)hw, 66,
                           (const float *)ws->wpart, d_grad, HEAD);
        int c = 0;
        for (int l = NL; l >= 1; --l) {
            const int li = l - 1;
            const float *Lw = d_w + L0 + li * LSZ;
            const unsigned wn = tile_wgs(n, kBwdCap), we = tile_wgs(E, kBwdCap);
            hipLaunchKernelGGL(k_node_bwd, dim3(wn), dim3(256), 0, s, n, g->eptr,
                               (const __bf16 *)ws->h[l - 1], (const __bf16 *)ws->e[l],
                               (const float *)ws->dh[c], ws->dh[1 - c], ws->dagg, ws->wbf + li, Lw,
                               ws->wpart);
            hipLaunchKernelGGL(k_wreduce, dim3(g1(3136)), dim3(256), 0, s, (int)(wn * kWavesPerWg),
                               3136, (const float *)ws->wpart, d_grad, L0 + li * LSZ + N1W);
            if (E > 0) {
                hipLaunchKernelGGL(k_edge_bwd, dim3(we), dim3(256), 0, s, E, g->erow, g->ecol,
                                   (const __bf16 *)ws->h[l - 1], (const __bf16 *)ws->e[l - 1],
                                   (const float *)ws->de[c], (const float *)ws->dagg, ws->dxi,
                                   ws->dxj, ws->de[1 - c], ws->wbf + li, Lw, ws->wpart);
                hipLaunchKernelGGL(k_wreduce, dim3(g1(4160)), dim3(256), 0, s,
                                   (int)(we * kWavesPerWg), 4160, (const float *)ws->wpart, d_grad,
                                   L0 + li * LSZ + E1W);
                hipLaunchKernelGGL(k_node_gather, dim3(g1((int64_t)n * H)), dim3(256), 0, s, n,
                                   g->eptr, g->rev, (const float *)ws->dxi, (const float *)ws->dxj,
                                   ws->dh[1 - c]);
            } else {
                hipLaunchKernelGGL(k_wreduce, dim3(g1(4160)), dim3(256), 0, s, 0, 4160,
                                   (const float *)ws->wpart, d_grad, L0 + li * LSZ + E1W);
            }
            c = 1 - c;
        }
        const unsigned we = (unsigned)std::min<int64_t>(g1(std::max(n, E), 8), kSmallCap);
        hipLaunchKernelGGL(k_enc_bwd, dim3(we), dim3(256), 0, s, n, E, (const float *)g->fe,
                           (const float *)g->ge, (const float *)ws->dh[c], (const float *)ws->de[c],
                           ws->wpart);
        hipLaunchKernelGGL(k_wreduce, dim3(1), dim3(256), 0, s, (int)we, 192,
                           (const float *)ws->wpart, d_grad, 0);
        SPCG_LAUNCH_CHECK("mpnn backward");
    }
    if (h_loss) {
        float *hp = (float *)g->h_pinned;
        SPCG_TRY(hipMemcpyAsync(hp, ws->scal + 1, sizeof(float), hipMemcpyDeviceToHost, s));
        SPCG_TRY(hipStreamSynchronize(s));
        *h_loss = (double)hp[0] / ((double)n * (double)m);
    }
    return SPCG_OK;
}

int spcg_adam_step(float *d_w, const float *d_g, float *d_m, float *d_v, int64_t n, int32_t t,
                   float lr, float b1, float b2, float eps, hipStream_t s) {
    if (!d_w || !d_g || !d_m || !d_v || n < 0 || t < 1) return SPCG_INVALID_ARG;
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(g1(n)), dim3(256), 0, s, n, d_w, d_g, d_m, d_v, lr, b1, b2, eps,
                       c1, c2);
    SPCG_LAUNCH_CHECK("k_adam");
    return SPCG_OK;
}

}  // extern "C"

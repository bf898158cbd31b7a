// cg.hip -- preconditioned conjugate gradients on the device (arXiv 1211.1581,
// Sec. 3.4: per pass one SpMV, two inner products and three vector updates).
//
// Schedule of one pass (FP64 Jacobi-PCG; the scalars never leave the device):
//   K1  q = A p            SpMV with p.q folded into the row epilogue
//   F1  sigma = sum of K1's partials, alpha = rho / sigma   (one workgroup)
//   K2  x += alpha p, r -= alpha q, z = D^-1 r   (z not stored); partials r.z, r.r
//   K3F every workgroup sums K2's partials (rho', ||r||^2 -> beta, stop
//       decision) and updates p = D^-1 r + beta p; workgroup 0 records the
//       pass (history entry, state)
// Every kernel carries the pass number it belongs to and does nothing unless
// the device state is at that pass and running, so the host can enqueue a
// batch of passes and read one status word per batch.
//
// Mixed precision: the same kernels in FP32 on fl32(A) with FP32 vectors and
// reductions; when ||r32|| falls below delta * ||r at the last replacement||
// (or below tol ||b||, or at maxit) the state halts with "replace": x64 += x32,
// r64 = b - A x64 in FP64, r32 = fl32(r64), rho recomputed, p kept.
//
// Learned: M^-1 = G G^T with G lower-triangular (FP32 values, FP64 vectors):
// t = G^T r and z = G t are two SpMV-shaped launches on the handles of G^T
// and G, with r.z folded into the second one.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include <hip/hip_ext.h>

#include "internal.h"

namespace spcg {

enum Halt : int {
    RUN = 0,
    H_CONV = 1,     // recursive residual below tol ||b||
    H_MAXIT = 2,
    H_BREAK = 3,    // breakdown; status holds NOT_SPD / NON_FINITE
    H_REPLACE = 4,  // mixed: FP64 residual replacement due
    H_BUDGET = 5,   // learned: pass budget used up
    H_ZERO = 6,     // ||b|| = 0
};

struct CgState {
    double rho, alpha, beta, rr, nb, thresh, rlast, delta, true_rr, r2_64;
    float rho32, alpha32, beta32, rr32;
    int k, maxit, halt, status, budget, n_updates, bad_diag, c16_bad;
    // folded pass end (K3F): rho by pass parity, so that the workgroup that
    // records pass e + 1 never writes what the others of pass e still read;
    // kq = the last pass whose F1 ran (K3F's gate)
    double rho_pp[2];
    float rho32_pp[2];
    int kq, pad;
    // learned form: constant-offset (DIA) check of G (0) and G^T (1): the
    // offsets col - row of a probe row, their count, and whether some entry
    // has another offset
    int dia_off[2][8];
    int dia_w[2], dia_bad[2], dia_probe[2];
};

constexpr int kVecPer = 4;
constexpr int kVecBlock = kBlock * kVecPer;
constexpr int kSmallThreads = 1024;

inline int64_t vec_blocks(int64_t n) { return (n + kVecBlock - 1) / kVecBlock; }

template <typename T> __device__ __forceinline__ T st_alpha(const CgState *s);
template <> __device__ __forceinline__ double st_alpha<double>(const CgState *s) { return s->alpha; }
template <> __device__ __forceinline__ float st_alpha<float>(const CgState *s) { return s->alpha32; }

__device__ __forceinline__ bool finite_d(double v) { return isfinite(v); }

__device__ __forceinline__ void set_break(CgState *s, double v) {
    s->status = finite_d(v) ? SPCG_NOT_SPD : SPCG_NON_FINITE;
    s->halt = H_BREAK;
}

// ------------------------------------------------------------- set-up --
// ------------------------------------------------------------- set-up --

// k0: passes already taken (a fallback phase continues the pass count and
// the history of the phase before it, and maxit bounds both together)
__global__ void k_init_state(CgState *st, int maxit, double delta, int budget, int k0) {
    if (threadIdx.x == 0) {
        CgState s;
        memset(&s, 0, sizeof s);
        s.k = k0;
        s.maxit = maxit;
        s.delta = delta;
        s.budget = budget;
        s.kq = -1;
        s.dia_probe[0] = s.dia_probe[1] = INT32_MAX;
        *st = s;
    }
}

// state fields for a restart from the true residual: keep nb, thresh, k
__global__ void k_phase_state(CgState *st) {
    if (threadIdx.x == 0) {
        st->halt = RUN;
        st->status = SPCG_OK;
        st->kq = -1;
    }
}

// dinv_i = 1 / (sum of row i's diagonal entries); dinv32 = fl32(dinv)
__global__ void __launch_bounds__(kBlock)
k_diag_inv(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
           const double *__restrict__ vals, double *__restrict__ dinv, float *__restrict__ dinv32,
           CgState *st) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double d = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k)
        if (col[k] == i) d += vals[k];
    if (!(d > 0.0)) atomicOr(&st->bad_diag, isfinite(d) ? 1 : 2);
    const double v = 1.0 / d;
    dinv[i] = v;
    if (dinv32) dinv32[i] = (float)v;
}

__global__ void __launch_bounds__(kBlock)
k_to_f32(int64_t n, const double *__restrict__ a, float *__restrict__ b) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

template <typename T>
__global__ void k_fill(int64_t n, T *p, T v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_copy(int64_t n, const double *__restrict__ a, double *__restrict__ b) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

// ------------------------------------------- residual r = b - A x (FP64) --

enum ResidMode : int { R_INIT = 0, R_TRUE = 1, R_REPLACE = 2 };

struct EpiResid {
    const double *__restrict__ b;
    double *__restrict__ r;
    float *__restrict__ r32;
    double bb, rr;
    __device__ __forceinline__ double load(int i) const { return b[i]; }
    __device__ __forceinline__ void row(int i, double s, double bi) {
        const double ri = bi - s;
        r[i] = ri;
        if (r32) r32[i] = (float)ri;
        bb += bi * bi;
        rr += ri * ri;
    }
};

// r = b - A x (and r32 = fl32(r)); partials (b.b, r.r).  Every row belongs to
// exactly one row block, so r is fully written.
SPCG_ROWBLOCK_KERNEL
k_resid(CsrDev A, const double *__restrict__ vals, const double *__restrict__ x,
        const double *__restrict__ b, double *__restrict__ r, float *__restrict__ r32,
        const CgState *st, double *part, int mode) {
    __shared__ SpmvSmem<double> sm;
    if (mode == R_REPLACE && st->halt != H_REPLACE) return;
    int bs, be;
    const int slot = block_range(A.n_blocks, bs, be);
    EpiResid epi{b, r, r32, 0.0, 0.0};
    for (int k = bs; k < be; ++k) spmv_block<double, double, double>(A, vals, x, k, sm, epi, k + 1 < be);
    const double v[2] = {epi.bb, epi.rr};
    store_block_partials(part, slot, v, sm.red);
}

__global__ void __launch_bounds__(kFinThreads)
k_fin_resid(CgState *st, const double *part, int nslots, double *hist, int mode, double tol) {
    if (mode == R_REPLACE && st->halt != H_REPLACE) return;
    double t[2];
    finalize_sum(part, nslots, t);
    if (threadIdx.x != 0) return;
    if (mode == R_INIT) {
        st->nb = sqrt(t[0]);
        st->thresh = tol * st->nb;
        st->rr = t[1];
        st->rlast = sqrt(t[1]);
        if (!(t[0] > 0.0)) {
            if (finite_d(t[0])) st->halt = H_ZERO;
            else set_break(st, t[0]);
        } else if (!finite_d(t[1])) {
            set_break(st, t[1]);
        }
    } else if (mode == R_TRUE) {
        st->true_rr = t[1];
    } else {
        st->rlast = sqrt(t[1]);
        st->r2_64 = t[1];
        st->n_updates += 1;
        hist[st->k] = st->rlast / st->nb;
    }
}

// z = M^-1 r, p = z; partials (r.z, r.r)  (start of a phase; r is set)
template <int PRE>
__global__ void __launch_bounds__(kBlock)
k_start(int n, const double *__restrict__ r, const double *__restrict__ dinv,
        const double *__restrict__ zin, double *__restrict__ p, const CgState *st, double *part) {
    __shared__ double red[kWaves * 2];
    if (st->halt != RUN) return;
    double rz = 0.0, rr = 0.0;
    const int base = blockIdx.x * kVecBlock + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kVecPer; ++u) {
        const int i = base + u * kBlock;
        if (i < n) {
            const double ri = r[i];
            const double zi = PRE == SPCG_PRECOND_JACOBI ? dinv[i] * ri
                              : PRE == SPCG_PRECOND_NONE ? ri
                                                         : zin[i];
            p[i] = zi;
            rz += ri * zi;
            rr += ri * ri;
        }
    }
    const double v[2] = {rz, rr};
    store_block_partials(part, blockIdx.x, v, red);
}

__global__ void __launch_bounds__(kFinThreads)
k_fin_start(CgState *st, const double *part, int nslots, double *hist) {
    if (st->halt != RUN) return;
    double t[2];
    finalize_sum(part, nslots, t);
    if (threadIdx.x != 0) return;
    st->rho = t[0];
    st->rho_pp[st->k & 1] = t[0];
    st->rr = t[1];
    hist[st->k] = sqrt(t[1]) / st->nb;
    if (!finite_d(t[0]) || !finite_d(t[1])) set_break(st, NAN);
    else if (sqrt(t[1]) <= st->thresh) st->halt = H_CONV;
    else if (!(t[0] > 0.0)) set_break(st, t[0]);
    else if (st->k >= st->maxit) st->halt = H_MAXIT;
}

// ------------------------------------------------------ one CG pass --

template <typename T>
struct EpiPQ {
    T *__restrict__ q;
    const T *__restrict__ p;
    T acc;
    __device__ __forceinline__ T load(int i) const { return p[i]; }
    __device__ __forceinline__ void row(int i, T s, T pi) {
        q[i] = s;
        acc += pi * s;
    }
};

// K1: q = A p; partial p.q.  KEEP: load policy of A's streams (keep_bytes);
// without it, the blocks k with (k & 15) < kq16 still use cache-allocating
// loads (a matrix above the limit keeps that share of its blocks in the
// memory-side cache, spread over every XCD's range of blocks).  C16: compact
// columns (A.off16); CH: span of A's partition (kChunk, or kChunkWide for the
// mixed form's FP32 inner product).
template <typename TV, typename T, bool KEEP, bool C16 = false, int CH = kChunk>
SPCG_ROWBLOCK_KERNEL
k_cg_q(CsrDev A, const TV *__restrict__ vals, const T *__restrict__ p, T *__restrict__ q,
       const CgState *st, T *part, int expect, int kq16) {
    __shared__ SpmvSmem<T, CH> sm;
    if (st->halt != RUN || st->k != expect) return;
    int bs, be;
    const int slot = block_range(A.n_blocks, bs, be);
    EpiPQ<T> epi{q, p, T(0)};
    for (int k = bs; k < be; ++k) {
        if (KEEP || (k & 15) < kq16)
            spmv_block<TV, T, T, true, C16>(A, vals, p, k, sm, epi, k + 1 < be);
        else
            spmv_block<TV, T, T, false, C16>(A, vals, p, k, sm, epi, k + 1 < be);
    }
    const T v[1] = {epi.acc};
    store_block_partials(part, slot, v, sm.red);
}

// F1: sigma = p.q, alpha = rho / sigma.  PP: rho by pass parity, and kq set
// for the folded pass end (K3F).
template <typename T, bool PP = false>
__global__ void __launch_bounds__(kFinThreads)
k_fin_q(CgState *st, const T *part, int nslots, int expect) {
    if (st->halt != RUN || st->k != expect) return;
    T t[1];
    finalize_sum(part, nslots, t);
    if (threadIdx.x != 0) return;
    const T sigma = t[0];
    if (!(sigma > T(0)) || !finite_d((double)sigma)) {
        set_break(st, (double)sigma);
        return;
    }
    if constexpr (sizeof(T) == 8) {
        st->alpha = (PP ? st->rho_pp[expect & 1] : st->rho) / sigma;
    } else {
        st->alpha32 = (PP ? st->rho32_pp[expect & 1] : st->rho32) / sigma;
    }
    if (PP) st->kq = expect;
}

// K2: r -= alpha q, z = M^-1 r; partials (r.z, r.r).  x += alpha p is done by
// the pass end (K3F, K3L), which reads p anyway, so this kernel reads neither
// x nor p.  PRE = LEARNED: r.r only (z comes from two SpMVs).  T = float: mixed
// inner.
template <typename T, int PRE>
__global__ void __launch_bounds__(kBlock)
k_cg_xr(int n, int expect, T *__restrict__ r, const T *__restrict__ q, const T *__restrict__ dinv,
        const CgState *st, T *part) {
    __shared__ T red[kWaves * 2];
    if (st->halt != RUN || st->k != expect) return;
    const T alpha = st_alpha<T>(st);
    T rz = T(0), rr = T(0);
    for (int tile = blockIdx.x; tile * kVecBlock < n; tile += gridDim.x) {
        const int base = tile * kVecBlock + threadIdx.x;
#pragma unroll
        for (int u = 0; u < kVecPer; ++u) {
            const int i = base + u * kBlock;
            if (i < n) {
                // q is not read again before it is next written: a
                // non-temporal load leaves the MALL to the matrix and to the
                // vectors that are
                const T ri = r[i] - alpha * __builtin_nontemporal_load(q + i);
                r[i] = ri;
                if constexpr (PRE == SPCG_PRECOND_JACOBI) rz += ri * (dinv[i] * ri);
                rr += ri * ri;
            }
        }
    }
    if constexpr (PRE == SPCG_PRECOND_NONE) rz = rr;
    const T v[2] = {rz, rr};
    store_block_partials(part, blockIdx.x, v, red);
}

// Fixed-order totals of a[j * SA + OA] (j < na) and b[j * SB + OB] (j < nb)
// in every thread of a kBlock workgroup (na, nb >= 1).  Loads go in batches of
// 8 per thread at clamped, in-bounds indices, all in flight together; the
// order of the sums depends only on na and nb, so every workgroup that calls
// this on the same partials gets the same totals.
template <int SA, int OA, int SB, int OB, typename T>
__device__ __forceinline__ void wg_totals(const T *__restrict__ a, int na, const T *__restrict__ b,
                                          int nb, T &ta, T &tb, T *sh /* kWaves * 2 */) {
    constexpr int kPer = 8;
    const int tid = threadIdx.x;
    T acc_a = T(0), acc_b = T(0);
    const int nmax = na > nb ? na : nb;
    for (int base = 0; base < nmax; base += kBlock * kPer) {
        T va[kPer], vb[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int j = base + tid + u * kBlock;
            va[u] = a[(size_t)min(j, na - 1) * SA + OA];
            vb[u] = b[(size_t)min(j, nb - 1) * SB + OB];
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int j = base + tid + u * kBlock;
            acc_a += j < na ? va[u] : T(0);
            acc_b += j < nb ? vb[u] : T(0);
        }
    }
    acc_a = wave_sum(acc_a);
    acc_b = wave_sum(acc_b);
    if ((tid & 63) == 0) {
        sh[2 * (tid >> 6)] = acc_a;
        sh[2 * (tid >> 6) + 1] = acc_b;
    }
    __syncthreads();
    ta = T(0);
    tb = T(0);
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        ta += sh[2 * w];
        tb += sh[2 * w + 1];
    }
}

// Update kernels of the folded pass end run with at most kXrGrid workgroups
// (each walks a range of tiles), so K3F sums at most 2 kXrGrid partials.
constexpr int kXrGrid = 1024;
// Workgroups of the learned form's t = G^T r in CSR form (each walks a range
// of row blocks or short-row steps): K3L sums one partial per workgroup.
constexpr int kApplyGrid = 4096;

// K3F: the end-of-pass finalize folded into p = z + beta p.  Every workgroup
// sums K2's partials itself, in the same fixed order, so all of them get the
// same rho' and ||r||^2 and take the same stop decision; unless the pass ends
// the loop (converged, out of passes, breakdown) they update p.  Workgroup 0
// records the pass: count, history, rho' (into the other parity slot), beta,
// decision.  The gate is kq (F1 of this pass ran, and so K2), which those
// writes do not touch.  x += alpha p of the pass is done here for every pass
// K2 ran, also one that ends the loop, so K2 reads neither x nor p.
// T = float: the mixed inner loop (replacement instead of stop).
template <typename T, int PRE, bool MIXED>
__global__ void __launch_bounds__(kBlock)
k_cg_pf(int n, int expect, const T *__restrict__ r, const T *__restrict__ dinv,
        T *__restrict__ p, T *__restrict__ x, CgState *st, const T *__restrict__ part, int nslots,
        double *__restrict__ hist) {
    __shared__ T sh[kWaves * 2];
    if (st->kq != expect) return;
    const T alpha = st_alpha<T>(st);  // set by F1 of this pass; not written below
    // the first tile's operands are requested before the partials are summed
    const int tid = threadIdx.x;
    int tile = blockIdx.x;
    T rv[kVecPer], dv[kVecPer], pv[kVecPer], xv[kVecPer];
#pragma unroll
    for (int u = 0; u < kVecPer; ++u) {
        const int i = min(tile * kVecBlock + tid + u * kBlock, n - 1);
        rv[u] = r[i];
        dv[u] = PRE == SPCG_PRECOND_JACOBI ? dinv[i] : T(1);
        pv[u] = p[i];
        xv[u] = __builtin_nontemporal_load(x + i);
    }
    T t0, t1;
    wg_totals<2, 0, 2, 1>(part, nslots, part, nslots, t0, t1, sh);
    // the decision of the former end-of-pass finalize, in every workgroup
    const int k = expect + 1;
    const double rrd = (double)t1;
    const double est = sqrt(rrd);
    bool brk = false;
    double brk_v = 0.0;
    if (!finite_d((double)t0) || !finite_d(rrd)) {
        brk = true;
        brk_v = NAN;
    } else if (rrd > 0.0 && !(t0 > T(0))) {
        brk = true;
        brk_v = (double)t0;
    }
    int halt = RUN;
    T beta = T(0);
    if (!brk) {
        if constexpr (MIXED) {
            beta = t0 / st->rho32_pp[expect & 1];
            if (est < st->delta * st->rlast || est <= st->thresh || k >= st->maxit) halt = H_REPLACE;
        } else {
            beta = T((double)t0 / st->rho_pp[expect & 1]);
            if (est <= st->thresh) halt = H_CONV;
            else if (k >= st->maxit) halt = H_MAXIT;
        }
    }
    if (blockIdx.x == 0 && tid == 0) {
        st->k = k;
        hist[k] = est / st->nb;
        if (brk) {
            set_break(st, brk_v);
        } else {
            if constexpr (MIXED) {
                st->beta32 = beta;
                st->rho32 = t0;
                st->rho32_pp[k & 1] = t0;
                st->rr32 = t1;
            } else {
                st->beta = (double)beta;
                st->rho = (double)t0;
                st->rho_pp[k & 1] = (double)t0;
                st->rr = rrd;
            }
            if (halt != RUN) st->halt = halt;
        }
    }
    // p is left as it is when the pass ends the loop; x is always updated
    const bool upd_p = !(brk || (halt != RUN && halt != H_REPLACE));
    for (;;) {
#pragma unroll
        for (int u = 0; u < kVecPer; ++u) {
            const int i = tile * kVecBlock + tid + u * kBlock;
            if (i < n) {
                __builtin_nontemporal_store(xv[u] + alpha * pv[u], x + i);
                const T zi = PRE == SPCG_PRECOND_JACOBI ? dv[u] * rv[u] : rv[u];
                if (upd_p) p[i] = zi + beta * pv[u];
            }
        }
        tile += gridDim.x;
        if (tile * kVecBlock >= n) break;
#pragma unroll
        for (int u = 0; u < kVecPer; ++u) {
            const int i = min(tile * kVecBlock + tid + u * kBlock, n - 1);
            rv[u] = r[i];
            dv[u] = PRE == SPCG_PRECOND_JACOBI ? dinv[i] : T(1);
            pv[u] = p[i];
            xv[u] = __builtin_nontemporal_load(x + i);
        }
    }
}

// ------------------------------------------- learned: z = G (G^T r) --

struct EpiStore64 {
    double *__restrict__ y;
    __device__ __forceinline__ NoOperand load(int) const { return {}; }
    __device__ __forceinline__ void row(int i, double s, NoOperand) { y[i] = s; }
};

// G^T and G handles as the apply kernels see them
struct FactorDev {
    CsrDev A;
    const float *__restrict__ vals;
    int n;
};

struct EpiTT {
    double *__restrict__ t;
    double acc;
    __device__ __forceinline__ NoOperand load(int) const { return {}; }
    __device__ __forceinline__ void row(int i, double s, NoOperand) {
        t[i] = s;
        acc += s * s;
    }
};

// t = G^T r; partial t.t per workgroup, which is r.z for z = G t
// (r.z = r^T G G^T r = |G^T r|^2), so the G apply need not read r.  kexp:
// pass number the state must be at, or -1 at a phase start.  SHORT: every row
// of G^T has at most kShortLen entries.  KEEP: load policy of the factor's
// streams (keep_bytes).
template <bool SHORT, bool KEEP>
SPCG_ROWBLOCK_KERNEL
k_gt_apply(FactorDev GT, const double *__restrict__ r, double *__restrict__ t, const CgState *st,
           double *part, int kexp) {
    __shared__ SpmvSmem<double> sm;
    if (st->halt != RUN || (kexp >= 0 && st->k != kexp)) return;
    int bs, be;
    EpiTT epi{t, 0.0};
    int slot;
    if constexpr (SHORT) {
        slot = block_range((int)short_steps(GT.n), bs, be);
        for (int k = bs; k < be; ++k)
            spmv_short<float, double, double, KEEP>(GT.A.row_ptr, GT.A.col, GT.vals, r, GT.n, k, epi);
    } else {
        slot = block_range(GT.A.n_blocks, bs, be);
        for (int k = bs; k < be; ++k) spmv_block<float, double, double, KEEP>(GT.A, GT.vals, r, k, sm, epi, k + 1 < be);
    }
    const double v[1] = {epi.acc};
    store_block_partials(part, slot, v, sm.red);
}

// z = G t
template <bool SHORT, bool KEEP>
SPCG_ROWBLOCK_KERNEL
k_g_apply(FactorDev G, const double *__restrict__ t, double *__restrict__ z, const CgState *st,
          int kexp) {
    __shared__ SpmvSmem<double> sm;
    if (st->halt != RUN || (kexp >= 0 && st->k != kexp)) return;
    int bs, be;
    EpiStore64 epi{z};
    if constexpr (SHORT) {
        block_range((int)short_steps(G.n), bs, be);
        for (int k = bs; k < be; ++k)
            spmv_short<float, double, double, KEEP>(G.A.row_ptr, G.A.col, G.vals, t, G.n, k, epi);
    } else {
        block_range(G.A.n_blocks, bs, be);
        for (int k = bs; k < be; ++k) spmv_block<float, double, double, KEEP>(G.A, G.vals, t, k, sm, epi, k + 1 < be);
    }
}

// ----------------------------------- learned: factors as padded ELL --
//
// A factor whose rows hold at most kEllMax entries (the triangles of a
// 7-point stencil hold 4) is copied at the start of a solve into the
// workspace as W column-major planes, col[w * n + i] and val[w * n + i] for
// the w-th entry of row i (padding: column i, value 0).  One thread per row
// then loads its W columns and values with coalesced loads that depend on
// nothing, gathers, and sums in the row's order: one round trip fewer than
// the CSR kernels, which must read row_ptr first.
constexpr int kEllMax = 8;
constexpr int kEllGrid = 2048;  // workgroups of an ELL apply (each walks a range of rows)

inline int ell_width(const spcg_csr *F) {
    return !F || F->max_len > kEllMax ? 0 : (F->max_len <= 4 ? 4 : kEllMax);
}

template <int W>
__global__ void __launch_bounds__(kBlock)
k_to_ell(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
         const float *__restrict__ vals, int32_t *__restrict__ ec, float *__restrict__ ev) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const int a = rp[i], e = rp[i + 1];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const bool in = a + w < e;
            ec[(size_t)w * n + i] = in ? col[a + w] : i;
            ev[(size_t)w * n + i] = in ? vals[a + w] : 0.0f;
        }
    }
}

struct EllDev {
    const int32_t *__restrict__ col;
    const float *__restrict__ val;
    int n;
};

// Rows per thread of an ELL apply: every thread loads the columns and values
// of R rows at once (clamped, in-bounds indices), then gathers, so a batch
// costs two round trips to memory however many rows it holds.
template <int W> constexpr int ell_rows() { return W <= 4 ? 4 : 2; }

// Rows base + u kBlock + threadIdx.x (u < R) of an ELL factor times x, each
// in its row's order (FP32 values, FP64 sums); rows past n are clamped to
// n - 1 (the caller drops them).
template <int W, int R, bool KEEP>
__device__ __forceinline__ void ell_rows_times(const EllDev &F, const double *__restrict__ x,
                                               int base, double (&s)[R]) {
    int c[R][W];
    float v[R][W];
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const int i = min(base + u * kBlock + (int)threadIdx.x, F.n - 1);
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const size_t o = (size_t)w * F.n + i;
            c[u][w] = KEEP ? F.col[o] : __builtin_nontemporal_load(F.col + o);
            v[u][w] = KEEP ? F.val[o] : __builtin_nontemporal_load(F.val + o);
        }
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
        double a = 0.0;
#pragma unroll
        for (int w = 0; w < W; ++w) a += (double)v[u][w] * x[c[u][w]];
        s[u] = a;
    }
}

// t = G^T r  (ELL); partial t.t per workgroup, which is r.z for z = G t
// (r.z = r^T G G^T r = |G^T r|^2), so the G apply need not read r.
// kexp: pass number, or -1 at a phase start.
template <int W, bool KEEP>
__global__ void __launch_bounds__(kBlock)
k_gt_ell(EllDev GT, const double *__restrict__ r, double *__restrict__ t, const CgState *st,
         double *part, int kexp) {
    constexpr int R = ell_rows<W>();
    __shared__ double red[kWaves];
    if (st->halt != RUN || (kexp >= 0 && st->k != kexp)) return;
    double acc = 0.0;
    for (int base = blockIdx.x * kBlock * R; base < GT.n; base += gridDim.x * kBlock * R) {
        double sv[R];
        ell_rows_times<W, R, KEEP>(GT, r, base, sv);
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int i = base + u * kBlock + threadIdx.x;
            if (i < GT.n) {
                t[i] = sv[u];
                acc += sv[u] * sv[u];
            }
        }
    }
    const double v[1] = {acc};
    store_block_partials(part, blockIdx.x, v, red);
}

// z = G t (ELL)
template <int W, bool KEEP>
__global__ void __launch_bounds__(kBlock)
k_g_ell(EllDev G, const double *__restrict__ t, double *__restrict__ z, const CgState *st,
        int kexp) {
    constexpr int R = ell_rows<W>();
    if (st->halt != RUN || (kexp >= 0 && st->k != kexp)) return;
    for (int base = blockIdx.x * kBlock * R; base < G.n; base += gridDim.x * kBlock * R) {
        double sv[R];
        ell_rows_times<W, R, KEEP>(G, t, base, sv);
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int i = base + u * kBlock + threadIdx.x;
            if (i < G.n) z[i] = sv[u];
        }
    }
}

// ------------------------------------- learned: factors as DIA planes --
//
// When every entry of a factor lies on one of at most kEllMax diagonals
// (col - row in a fixed set: the triangles of a stencil matrix), the solve's
// copy keeps only values, one plane per diagonal in ascending offset order
// (val[w * n + i] for column i + off[w]; 0 where row i has no such entry).
// An apply then needs no column loads: each thread requests its rows' values
// and the gathered x at known addresses together, one round trip per batch.
struct DiaOff {
    int o[kEllMax];
};

// The first row of the longest length becomes the probe row (its offsets are
// the candidates).  f: 0 for G, 1 for G^T.
__global__ void __launch_bounds__(kBlock)
k_dia_probe(int n, const int32_t *__restrict__ rp, int max_len, CgState *st, int f) {
    __shared__ int wmin[kWaves];
    int first = INT32_MAX;  // this thread's first row of the longest length
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        if (rp[i + 1] - rp[i] == max_len) {
            first = i;
            break;
        }
    // workgroup minimum: DPP inside rows of 16, then the row minima
    first = min(first, dpp_mov<kDppXor1>(first));
    first = min(first, dpp_mov<kDppXor2>(first));
    first = min(first, dpp_mov<kDppHalfMirror>(first));
    first = min(first, dpp_mov<kDppMirror>(first));
    first = min(min(lane_value(first, 0), lane_value(first, 16)),
                min(lane_value(first, 32), lane_value(first, 48)));
    if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = first;
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = wmin[0];
        for (int w = 1; w < kWaves; ++w) m = min(m, wmin[w]);
        // most workgroups hold no smaller row than one already recorded: a
        // plain read first keeps the atomics (which serialise) few
        const int cur = __hip_atomic_load(&st->dia_probe[f], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (m < cur) atomicMin(&st->dia_probe[f], m);
    }
}

// Read the probe row's offsets, then check every entry against them
__global__ void __launch_bounds__(kBlock)
k_dia_check(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col, CgState *st,
            int f) {
    const int m = min(max(st->dia_probe[f], 0), n - 1);
    const int a = rp[m], len = rp[m + 1] - a;
    if (len < 1 || len > kEllMax) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->dia_bad[f] = 1;
        return;
    }
    int off[kEllMax];
#pragma unroll
    for (int w = 0; w < kEllMax; ++w) off[w] = w < len ? col[a + w] - m : 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int w = 0; w < len; ++w) st->dia_off[f][w] = off[w];
        st->dia_w[f] = len;
    }
    int bad = 0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            const int d = col[k] - i;
            bool found = false;
#pragma unroll
            for (int w = 0; w < kEllMax; ++w) found |= w < len && d == off[w];
            bad |= !found;
        }
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(&st->dia_bad[f], 1);
}

// DIA planes of a factor whose entries all lie on the diagonals off[0..cnt);
// planes cnt..W are padding (offset 0, value 0)
template <int W>
__global__ void __launch_bounds__(kBlock)
k_to_dia(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
         const float *__restrict__ vals, DiaOff off, int cnt, float *__restrict__ ev) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        float v[W];
#pragma unroll
        for (int w = 0; w < W; ++w) v[w] = 0.0f;
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            const int d = col[k] - i;
            bool done = false;  // the first plane with this offset takes the entry
#pragma unroll
            for (int w = 0; w < W; ++w) {
                if (!done && w < cnt && d == off.o[w]) {
                    v[w] += vals[k];
                    done = true;
                }
            }
        }
#pragma unroll
        for (int w = 0; w < W; ++w) ev[(size_t)w * n + i] = v[w];
    }
}

struct DiaDev {
    const float *__restrict__ val;
    DiaOff off;
    int n;
};

// Rows base + u kBlock + threadIdx.x (u < R) of a DIA factor times x, each in
// ascending offset order (FP32 values, FP64 sums); rows past n are clamped
template <int W, int R, bool KEEP>
__device__ __forceinline__ void dia_rows_times(const DiaDev &F, const double *__restrict__ x,
                                               int base, double (&s)[R]) {
    float v[R][W];
    double xv[R][W];
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const int i = min(base + u * kBlock + (int)threadIdx.x, F.n - 1);
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const size_t o = (size_t)w * F.n + i;
            v[u][w] = KEEP ? F.val[o] : __builtin_nontemporal_load(F.val + o);
            xv[u][w] = x[min(max(i + F.off.o[w], 0), F.n - 1)];
        }
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
        double a = 0.0;
#pragma unroll
        for (int w = 0; w < W; ++w) a += (double)v[u][w] * xv[u][w];
        s[u] = a;
    }
}

// t = G^T r  (DIA); partial t.t per workgroup, which is r.z for z = G t
// (r.z = r^T G G^T r = |G^T r|^2), so the G apply need not read r.
// kexp: pass number, or -1 at a phase start.
template <int W, bool KEEP>
__global__ void __launch_bounds__(kBlock)
k_gt_dia(DiaDev GT, const double *__restrict__ r, double *__restrict__ t, const CgState *st,
         double *part, int kexp) {
    constexpr int R = ell_rows<W>();
    __shared__ double red[kWaves];
    if (st->halt != RUN || (kexp >= 0 && st->k != kexp)) return;
    double acc = 0.0;
    for (int base = blockIdx.x * kBlock * R; base < GT.n; base += gridDim.x * kBlock * R) {
        double sv[R];
        dia_rows_times<W, R, KEEP>(GT, r, base, sv);
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int i = base + u * kBlock + threadIdx.x;
            if (i < GT.n) {
                t[i] = sv[u];
                acc += sv[u] * sv[u];
            }
        }
    }
    const double v[1] = {acc};
    store_block_partials(part, blockIdx.x, v, red);
}

// z = G t (DIA)
template <int W, bool KEEP>
__global__ void __launch_bounds__(kBlock)
k_g_dia(DiaDev G, const double *__restrict__ t, double *__restrict__ z, const CgState *st,
        int kexp) {
    constexpr int R = ell_rows<W>();
    if (st->halt != RUN || (kexp >= 0 && st->k != kexp)) return;
    for (int base = blockIdx.x * kBlock * R; base < G.n; base += gridDim.x * kBlock * R) {
        double sv[R];
        dia_rows_times<W, R, KEEP>(G, t, base, sv);
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int i = base + u * kBlock + threadIdx.x;
            if (i < G.n) z[i] = sv[u];
        }
    }
}

// The decision of a learned pass from ||r||^2 and r.z (converged, out of
// passes, budget used up, breakdown), taken alike by every workgroup of a
// kernel that folds the pass end in; workgroup 0 records the pass: count,
// history, rho (into the other parity slot), beta, decision.  Returns whether
// the loop goes on (then p = z + beta p).
__device__ __forceinline__ bool learned_pass_end(CgState *st, int expect, double rr, double rho,
                                                 double *__restrict__ hist, double &beta) {
    const int k = expect + 1;
    const double est = sqrt(rr);
    bool brk = false;
    double brk_v = NAN;
    int halt = RUN;
    beta = 0.0;
    if (!finite_d(rr) || !finite_d(rho)) {
        brk = true;
    } else if (est <= st->thresh) {
        halt = H_CONV;
    } else if (k >= st->maxit) {
        halt = H_MAXIT;
    } else if (k >= st->budget) {
        halt = H_BUDGET;
    } else if (rr > 0.0 && !(rho > 0.0)) {
        brk = true;
        brk_v = rho;
    } else {
        beta = rho / st->rho_pp[expect & 1];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->k = k;
        hist[k] = est / st->nb;
        if (brk) {
            set_break(st, brk_v);
        } else {
            st->rr = rr;
            if (halt != RUN) {
                st->halt = halt;
            } else {
                st->beta = beta;
                st->rho = rho;
                st->rho_pp[k & 1] = rho;
            }
        }
    }
    return !(brk || halt != RUN);
}

// K3L: the learned pass's end folded into p = z + beta p, as K3F: every
// workgroup sums ||r||^2 from K2's partials (second value of each slot) and
// r.z from the G apply's partials in one fixed order, takes the decision of a
// learned pass (converged, out of passes, budget used up, breakdown) and
// updates p unless the pass ends the loop; workgroup 0 records the pass.  As
// in K3F, x += alpha p of the pass is done here, also in a pass that ends the
// loop.
__global__ void __launch_bounds__(kBlock)
k_cg_pl(int n, int expect, const double *__restrict__ z, double *__restrict__ p,
        double *__restrict__ x, CgState *st, const double *__restrict__ part_xr, int n_xr,
        const double *__restrict__ part_g, int n_g, double *__restrict__ hist) {
    __shared__ double sh[kWaves * 2];
    if (st->kq != expect) return;
    const double alpha = st->alpha;  // set by F1 of this pass; not written below
    const int tid = threadIdx.x;
    int tile = blockIdx.x;
    double zv[kVecPer], pv[kVecPer], xv[kVecPer];
#pragma unroll
    for (int u = 0; u < kVecPer; ++u) {
        const int i = min(tile * kVecBlock + tid + u * kBlock, n - 1);
        zv[u] = z[i];
        pv[u] = p[i];
        xv[u] = __builtin_nontemporal_load(x + i);
    }
    double rr, rho;
    wg_totals<2, 1, 1, 0>(part_xr, n_xr, part_g, n_g, rr, rho, sh);
    double beta;
    // p is left as it is when the pass ends the loop; x is always updated
    const bool upd_p = learned_pass_end(st, expect, rr, rho, hist, beta);
    for (;;) {
#pragma unroll
        for (int u = 0; u < kVecPer; ++u) {
            const int i = tile * kVecBlock + tid + u * kBlock;
            if (i < n) {
                __builtin_nontemporal_store(xv[u] + alpha * pv[u], x + i);
                if (upd_p) p[i] = zv[u] + beta * pv[u];
            }
        }
        tile += gridDim.x;
        if (tile * kVecBlock >= n) break;
#pragma unroll
        for (int u = 0; u < kVecPer; ++u) {
            const int i = min(tile * kVecBlock + tid + u * kBlock, n - 1);
            zv[u] = z[i];
            pv[u] = p[i];
            xv[u] = __builtin_nontemporal_load(x + i);
        }
    }
}

// K3G: z = G t from the ELL or DIA copy with the learned pass's end folded in.
// The G^T apply of the pass has already written the r.z = t.t partials, so
// every workgroup sums ||r||^2 and r.z as K3L does, takes the same decision,
// and uses each z_i at once: x += alpha p, and p = z + beta p unless the pass
// ends the loop.  z is neither stored nor read back, and K3L is not launched.
// Gate: kq, as K3L (workgroup 0 rewrites k and halt while the others run).
template <int W, bool KEEP, bool DIA, class Dev>
__global__ void __launch_bounds__(kBlock)
k_g_pass(Dev G, const double *__restrict__ t, double *__restrict__ p, double *__restrict__ x,
         CgState *st, const double *__restrict__ part_xr, int n_xr,
         const double *__restrict__ part_g, int n_g, double *__restrict__ hist, int expect) {
    constexpr int R = ell_rows<W>();
    __shared__ double sh[kWaves * 2];
    if (st->kq != expect) return;
    const double alpha = st->alpha;  // set by F1 of this pass; not written below
    const int n = G.n, tid = threadIdx.x;
    const int stride = gridDim.x * kBlock * R;
    double sv[R], pv[R], xv[R];
    auto fetch = [&](int b) {
        if constexpr (DIA) dia_rows_times<W, R, KEEP>(G, t, b, sv);
        else ell_rows_times<W, R, KEEP>(G, t, b, sv);
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int i = min(b + u * kBlock + tid, n - 1);
            pv[u] = p[i];
            xv[u] = __builtin_nontemporal_load(x + i);
        }
    };
    // the first rows' products and operands are requested before the partials are summed
    int base = blockIdx.x * kBlock * R;
    if (base < n) fetch(base);
    double rr, rho;
    wg_totals<2, 1, 1, 0>(part_xr, n_xr, part_g, n_g, rr, rho, sh);
    double beta;
    const bool upd_p = learned_pass_end(st, expect, rr, rho, hist, beta);
    for (; base < n; base += stride) {
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int i = base + u * kBlock + tid;
            if (i < n) {
                __builtin_nontemporal_store(xv[u] + alpha * pv[u], x + i);
                if (upd_p) p[i] = sv[u] + beta * pv[u];
            }
        }
        if (base + stride < n) fetch(base + stride);
    }
}

// ------------------------------- single reduction (Chronopoulos-Gear) --
//
// u = M^-1 r, w = A u and s = A p (kept by recurrence) let one joint
// reduction (r.u, w.u, r.r) serve a whole pass:
//   K1  p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s, u = M^-1 r
//   K2  w = A u with the three partial sums folded into the row epilogue
//   F   gamma' = r.u, delta = w.u -> beta = gamma'/gamma,
//       alpha = gamma' / (delta - beta gamma' / alpha), stop decision

// start of a phase (r is set): u = M^-1 r, p = s = 0
template <int PRE>
__global__ void __launch_bounds__(kBlock)
k_sr_start(int n, const double *__restrict__ r, const double *__restrict__ dinv,
           double *__restrict__ u, double *__restrict__ p, double *__restrict__ s, const CgState *st) {
    if (st->halt != RUN) return;
    const int base = blockIdx.x * kVecBlock + threadIdx.x;
#pragma unroll
    for (int v = 0; v < kVecPer; ++v) {
        const int i = base + v * kBlock;
        if (i < n) {
            u[i] = PRE == SPCG_PRECOND_JACOBI ? dinv[i] * r[i] : r[i];
            p[i] = 0.0;
            s[i] = 0.0;
        }
    }
}

// K1 of pass `expect`
template <int PRE>
__global__ void __launch_bounds__(kBlock)
k_sr_vec(int n, int expect, double *__restrict__ x, double *__restrict__ r, double *__restrict__ p,
         double *__restrict__ s, double *__restrict__ u, const double *__restrict__ w,
         const double *__restrict__ dinv, const CgState *st) {
    if (st->halt != RUN || st->k != expect) return;
    const double alpha = st->alpha, beta = st->beta;
    const int base = blockIdx.x * kVecBlock + threadIdx.x;
    // p, s and x are next read by this kernel in the following pass: their
    // accesses are non-temporal so they do not displace A, u, r and w from
    // the memory-side cache
#pragma unroll
    for (int v = 0; v < kVecPer; ++v) {
        const int i = base + v * kBlock;
        if (i < n) {
            const double pi = u[i] + beta * __builtin_nontemporal_load(p + i);
            const double si = w[i] + beta * __builtin_nontemporal_load(s + i);
            __builtin_nontemporal_store(__builtin_nontemporal_load(x + i) + alpha * pi, x + i);
            const double ri = r[i] - alpha * si;
            __builtin_nontemporal_store(pi, p + i);
            __builtin_nontemporal_store(si, s + i);
            r[i] = ri;
            u[i] = PRE == SPCG_PRECOND_JACOBI ? dinv[i] * ri : ri;
        }
    }
}

struct RU {
    double r, u;
};

struct EpiSR {
    double *__restrict__ w;
    const double *__restrict__ r;
    const double *__restrict__ u;
    double g, d, rr;
    __device__ __forceinline__ RU load(int i) const { return RU{r[i], u[i]}; }
    __device__ __forceinline__ void row(int i, double s, RU v) {
        w[i] = s;
        g += v.r * v.u;
        d += s * v.u;
        rr += v.r * v.r;
    }
};

// K2: w = A u; partials (r.u, w.u, r.r).  kexp: pass number, or -1 at a phase start.
template <bool KEEP>
SPCG_ROWBLOCK_KERNEL
k_sr_w(CsrDev A, const double *__restrict__ vals, const double *__restrict__ u,
       const double *__restrict__ r, double *__restrict__ w, const CgState *st, double *part,
       int kexp) {
    __shared__ SpmvSmem<double> sm;
    if (st->halt != RUN || (kexp >= 0 && st->k != kexp)) return;
    int bs, be;
    const int slot = block_range(A.n_blocks, bs, be);
    EpiSR epi{w, r, u, 0.0, 0.0, 0.0};
    for (int k = bs; k < be; ++k) spmv_block<double, double, double, KEEP>(A, vals, u, k, sm, epi, k + 1 < be);
    const double v[3] = {epi.g, epi.d, epi.rr};
    store_block_partials(part, slot, v, sm.red);
}

// F at a phase start: gamma, delta -> alpha, beta = 0, history entry
__global__ void __launch_bounds__(kFinThreads)
k_fin_sr_start(CgState *st, const double *part, int nslots, double *hist) {
    if (st->halt != RUN) return;
    double t[3];
    finalize_sum(part, nslots, t);
    if (threadIdx.x != 0) return;
    const double gamma = t[0], delta = t[1], rr = t[2];
    hist[st->k] = sqrt(rr) / st->nb;
    st->rr = rr;
    if (!finite_d(gamma) || !finite_d(delta) || !finite_d(rr)) set_break(st, NAN);
    else if (sqrt(rr) <= st->thresh) st->halt = H_CONV;
    else if (!(gamma > 0.0)) set_break(st, gamma);
    else if (!(delta > 0.0)) set_break(st, delta);
    else {
        st->rho = gamma;
        st->alpha = gamma / delta;
        st->beta = 0.0;
        if (st->k >= st->maxit) st->halt = H_MAXIT;
    }
}

// F of pass `expect`
__global__ void __launch_bounds__(kFinThreads)
k_fin_sr(CgState *st, const double *part, int nslots, double *hist, int expect) {
    if (st->halt != RUN || st->k != expect) return;
    double t[3];
    finalize_sum(part, nslots, t);
    if (threadIdx.x != 0) return;
    const int k = expect + 1;
    st->k = k;
    const double gamma = t[0], delta = t[1], rr = t[2];
    const double est = sqrt(rr);
    hist[k] = est / st->nb;
    st->rr = rr;
    if (!finite_d(gamma) || !finite_d(delta) || !finite_d(rr)) {
        set_break(st, NAN);
        return;
    }
    if (est <= st->thresh) {
        st->halt = H_CONV;
        return;
    }
    if (!(gamma > 0.0)) {
        set_break(st, gamma);
        return;
    }
    const double beta = gamma / st->rho;
    const double denom = delta - beta * gamma / st->alpha;
    if (!finite_d(denom)) set_break(st, NAN);
    else if (!(denom > 0.0)) set_break(st, denom);
    else {
        st->beta = beta;
        st->alpha = gamma / denom;
        st->rho = gamma;
        if (k >= st->maxit) st->halt = H_MAXIT;
    }
}

// ------------------------------------------------------------ mixed --

// Compact columns of the FP32 inner matrix: off16[k] = col[k] - block_row[b]
// for the entries k of row block b (2 instead of 4 bytes per entry); c16_bad
// is set when an offset does not fit int16, and the inner loop then reads col.
__global__ void __launch_bounds__(kBlock)
k_make_off16(CsrDev A, int16_t *__restrict__ off16, CgState *st) {
    int bad = 0;
    for (int b = blockIdx.x; b < A.n_blocks; b += gridDim.x) {
        const int r0 = A.block_row[b], k1 = A.block_k[b + 1];
        for (int k = A.block_k[b] + threadIdx.x; k < k1; k += kBlock) {
            const int d = A.col[k] - r0;
            bad |= d < -32768 || d > 32767;
            off16[k] = (int16_t)d;
        }
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(&st->c16_bad, 1);
}

// x64 += x32, x32 = 0  (replacement or final fold)
__global__ void __launch_bounds__(kBlock)
k_mp_fold(int n, double *__restrict__ x, float *__restrict__ x32, const CgState *st, int always) {
    if (!always && st->halt != H_REPLACE) return;
    const int base = blockIdx.x * kVecBlock + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kVecPer; ++u) {
        const int i = base + u * kBlock;
        if (i < n) {
            x[i] += (double)x32[i];
            x32[i] = 0.0f;
        }
    }
}

// z32 = dinv32 r32; partial r32.z32 (FP32); init: p32 = z32 as well
__global__ void __launch_bounds__(kBlock)
k_mp_rz(int n, const float *__restrict__ r32, const float *__restrict__ dinv32,
        float *__restrict__ p32, const CgState *st, float *part, int init) {
    __shared__ float red[kWaves];
    if (init ? st->halt != RUN : st->halt != H_REPLACE) return;
    float rz = 0.0f;
    const int base = blockIdx.x * kVecBlock + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kVecPer; ++u) {
        const int i = base + u * kBlock;
        if (i < n) {
            const float ri = r32[i];
            const float zi = dinv32[i] * ri;
            if (init) p32[i] = zi;
            rz += ri * zi;
        }
    }
    const float v[1] = {rz};
    store_block_partials(part, blockIdx.x, v, red);
}

// Ends a replacement (or the start): converged, out of passes, or running.
__global__ void __launch_bounds__(kFinThreads)
k_fin_mprz(CgState *st, const float *part, int nslots, double *hist, int init) {
    if (init ? st->halt != RUN : st->halt != H_REPLACE) return;
    float t[1];
    finalize_sum(part, nslots, t);
    if (threadIdx.x != 0) return;
    st->rho32 = t[0];
    st->rho32_pp[st->k & 1] = t[0];
    if (init) hist[st->k] = st->rlast / st->nb;
    if (!finite_d((double)t[0]) || !finite_d(st->rlast)) set_break(st, NAN);
    else if (st->rlast <= st->thresh) st->halt = H_CONV;
    else if (!(t[0] > 0.0f)) set_break(st, (double)t[0]);
    else if (st->k >= st->maxit) st->halt = H_MAXIT;
    else st->halt = RUN;
}

// ------------------------------------- single-workgroup solver (small n) --

template <typename T>
__device__ __forceinline__ T wg_sum(T v, T *sh16) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh16[w] = v;
    __syncthreads();
    T s = T(0);
#pragma unroll
    for (int i = 0; i < kSmallThreads / 64; ++i) s += sh16[i];
    __syncthreads();
    return s;
}

// The whole loop in one 1024-thread workgroup (vectors stay in L2); the
// state was prepared by k_resid / k_start.  Exits at convergence, maxit or
// breakdown: every thread evaluates the same stop test on the same sums.  The
// product gives each row a group of L lanes (L a power of two <= 16 near the
// mean row length) that stride over its entries and add up by group_sum.
template <int PRE>
__global__ void __launch_bounds__(kSmallThreads)
k_cg_small(int n, int L, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
           const double *__restrict__ vals, double *__restrict__ x, double *__restrict__ r,
           double *__restrict__ p, double *__restrict__ q, const double *__restrict__ dinv,
           CgState *st, double *hist) {
    __shared__ double sh[kSmallThreads / 64];
    if (st->halt != RUN) return;
    double rho = st->rho;
    const double thresh = st->thresh, nb = st->nb;
    const int maxit = st->maxit;
    int k = st->k;
    int halt = RUN, status = SPCG_OK;
    double rr = st->rr, alpha = 0.0, beta = 0.0;
    const int lane = threadIdx.x & (L - 1);
    while (true) {
        double pq = 0.0;
        // the row loop's bound is uniform over each group of L lanes
        for (int i = threadIdx.x / L; i < n; i += kSmallThreads / L) {
            double s = 0.0;
            for (int e = rp[i] + lane; e < rp[i + 1]; e += L) s += vals[e] * p[col[e]];
            s = group_sum(s, L);
            if (lane == 0) {
                q[i] = s;
                pq += p[i] * s;
            }
        }
        // wg_sum's barrier also completes q before the update loop reads it
        // through another thread-to-row mapping
        const double sigma = wg_sum(pq, sh);
        if (!(sigma > 0.0) || !isfinite(sigma)) {
            halt = H_BREAK;
            status = isfinite(sigma) ? SPCG_NOT_SPD : SPCG_NON_FINITE;
            break;
        }
        alpha = rho / sigma;
        double rz = 0.0, rl = 0.0;
        for (int i = threadIdx.x; i < n; i += kSmallThreads) {
            x[i] += alpha * p[i];
            const double ri = r[i] - alpha * q[i];
            r[i] = ri;
            const double zi = PRE == SPCG_PRECOND_JACOBI ? dinv[i] * ri : ri;
            rz += ri * zi;
            rl += ri * ri;
        }
        const double rzs = wg_sum(rz, sh);
        rr = wg_sum(rl, sh);
        ++k;
        const double est = sqrt(rr);
        if (threadIdx.x == 0) hist[k] = est / nb;
        if (!isfinite(rzs) || !isfinite(rr)) {
            halt = H_BREAK;
            status = SPCG_NON_FINITE;
            break;
        }
        if (rr > 0.0 && !(rzs > 0.0)) {
            halt = H_BREAK;
            status = SPCG_NOT_SPD;
            break;
        }
        beta = rzs / rho;
        rho = rzs;
        if (est <= thresh) { halt = H_CONV; break; }
        if (k >= maxit) { halt = H_MAXIT; break; }
        for (int i = threadIdx.x; i < n; i += kSmallThreads) {
            const double zi = PRE == SPCG_PRECOND_JACOBI ? dinv[i] * r[i] : r[i];
            p[i] = zi + beta * p[i];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->k = k;
        st->rho = rho;
        st->rr = rr;
        st->halt = halt;
        st->status = status;
    }
}

// Register-resident variant for n <= R * 1024 rows of at most ML entries: each
// thread keeps its R rows (columns, values, x) in registers for the whole
// solve, and p, r and D^-1 live in LDS, so a pass reads no global memory: the
// SpMV gathers p from LDS, and the only synchronisation is the two workgroup
// reductions and the barrier after the direction update.
template <int PRE, int R, int ML>
__global__ void __launch_bounds__(kSmallThreads)
k_cg_regs(int n, int64_t nnz, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
          const double *__restrict__ vals, double *__restrict__ x, double *__restrict__ r,
          const double *__restrict__ p_in, const double *__restrict__ dinv, CgState *st,
          double *hist) {
    constexpr int MP = (ML + 1) / 2;  // column indices (< 2^16) packed two per register
    __shared__ double pl[R * kSmallThreads];
    // this thread's own entries of r and D^-1 (only it reads them): LDS keeps
    // the registers for the matrix
    __shared__ double rl_[R * kSmallThreads], dl[R * kSmallThreads];
    // wavefront partials: sh[0] p.q, sh[1] r.z, sh[2] r.r.  sigma is read from
    // sh[0] after the first barrier of a pass and sh[0] is next written after
    // the barrier that ends the pass, so no slot is rewritten while a slower
    // wavefront may still read it
    __shared__ double sh[3][kSmallThreads / 64];
    if (st->halt != RUN) return;
    const int tid = threadIdx.x;
    uint32_t c[R][MP];
    double v[R][ML], xr[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = tid + j * kSmallThreads;
        const bool real = i < n;
        const int lo = real ? rp[i] : 0;
        const int len = real ? rp[i + 1] - lo : 0;
#pragma unroll
        for (int t = 0; t < MP; ++t) c[j][t] = 0u;
#pragma unroll
        for (int t = 0; t < ML; ++t) {
            const int64_t e = min((int64_t)lo + t, nnz - 1);
            const bool use = t < len;
            const uint32_t cj = use ? (uint32_t)col[e] : 0u;
            c[j][t / 2] |= (t & 1) ? (cj << 16) : cj;
            v[j][t] = use ? vals[e] : 0.0;
        }
        xr[j] = real ? x[i] : 0.0;
        rl_[i] = real ? r[i] : 0.0;
        dl[i] = real && PRE == SPCG_PRECOND_JACOBI ? dinv[i] : 0.0;
        pl[i] = real ? p_in[i] : 0.0;
    }
    __syncthreads();
    double rho = st->rho;
    const double thresh = st->thresh, nb = st->nb;
    const int maxit = st->maxit;
    int k = st->k;
    int halt = RUN, status = SPCG_OK;
    double rr = st->rr;
    while (true) {
        double q[R], pq = 0.0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            double sj = 0.0;
#pragma unroll
            for (int t = 0; t < ML; ++t) {
                const uint32_t cj = (t & 1) ? (c[j][t / 2] >> 16) : (c[j][t / 2] & 0xffffu);
                sj += v[j][t] * pl[cj];
            }
            q[j] = sj;
            pq += pl[tid + j * kSmallThreads] * sj;
            // keep one row's LDS gathers in flight at a time (register pressure)
            __builtin_amdgcn_sched_barrier(0);
        }
        pq = wave_sum(pq);
        if ((tid & 63) == 0) sh[0][tid >> 6] = pq;
        __syncthreads();
        double sigma = 0.0;
#pragma unroll
        for (int w = 0; w < kSmallThreads / 64; ++w) sigma += sh[0][w];
        if (!(sigma > 0.0) || !isfinite(sigma)) {
            halt = H_BREAK;
            status = isfinite(sigma) ? SPCG_NOT_SPD : SPCG_NON_FINITE;
            break;
        }
        const double alpha = rho / sigma;
        double rz = 0.0, rl = 0.0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int i = tid + j * kSmallThreads;
            xr[j] += alpha * pl[i];
            const double ri = rl_[i] - alpha * q[j];
            rl_[i] = ri;
            const double zj = PRE == SPCG_PRECOND_JACOBI ? dl[i] * ri : ri;
            rz += ri * zj;
            rl += ri * ri;
        }
        rz = wave_sum(rz);
        rl = wave_sum(rl);
        if ((tid & 63) == 0) {
            sh[1][tid >> 6] = rz;
            sh[2][tid >> 6] = rl;
        }
        __syncthreads();
        double rzs = 0.0;
        rr = 0.0;
#pragma unroll
        for (int w = 0; w < kSmallThreads / 64; ++w) {
            rzs += sh[1][w];
            rr += sh[2][w];
        }
        ++k;
        const double est = sqrt(rr);
        if (tid == 0) hist[k] = est / nb;
        if (!isfinite(rzs) || !isfinite(rr)) {
            halt = H_BREAK;
            status = SPCG_NON_FINITE;
            break;
        }
        if (rr > 0.0 && !(rzs > 0.0)) {
            halt = H_BREAK;
            status = SPCG_NOT_SPD;
            break;
        }
        const double beta = rzs / rho;
        rho = rzs;
        if (est <= thresh) { halt = H_CONV; break; }
        if (k >= maxit) { halt = H_MAXIT; break; }
        // each thread updates only its own entries of p, which no other thread
        // reads before the barrier
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int i = tid + j * kSmallThreads;
            const double zj = PRE == SPCG_PRECOND_JACOBI ? dl[i] * rl_[i] : rl_[i];
            pl[i] = zj + beta * pl[i];
        }
        __syncthreads();  // the new direction is complete before the next product reads it
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = tid + j * kSmallThreads;
        if (i < n) {
            x[i] = xr[j];
            r[i] = rl_[i];
        }
    }
    if (tid == 0) {
        st->k = k;
        st->rho = rho;
        st->rr = rr;
        st->halt = halt;
        st->status = status;
    }
}

// ----------------------------------------------------------- workspace --

struct Work {
    CgState *st;
    double *hist;
    double *r, *p, *q, *dinv, *z, *t, *x0;
    float *r32, *p32, *q32, *x32, *dinv32, *vals32;
    int16_t *off16;  // mixed: compact columns of the FP32 inner matrix
    int32_t *g_col, *gt_col;  // learned: ELL copies of G and G^T (w_g, w_gt planes)
    float *g_val, *gt_val;
    int w_g, w_gt;
    double *partd;  // [nslots * 2]
    double *partg;  // [nslots]  (learned: r.z partials of the G apply)
    float *partf;   // [nslots * 2]
    int64_t nslots;
};

// Workgroups of a factor apply (row-block or short-row kernel)
static unsigned factor_grid(const spcg_csr *F) {
    return uses_short_rows(F) ? short_grid(F->n_rows) : spmv_grid(F->n_blocks);
}

static FactorDev factor_view(const spcg_csr *F) {
    return FactorDev{dev_view(F), (const float *)F->vals, F->n_rows};
}

// Partial-sum slots of the largest producing kernel (one per workgroup)
static int64_t n_slots(const spcg_csr *A, const spcg_cg_opts *o) {
    int64_t s = std::max<int64_t>(spmv_grid(A->n_blocks), vec_blocks(A->n_rows));
    if (o->precond == SPCG_PRECOND_LEARNED) {
        for (const spcg_csr *F : {o->G, o->GT})
            if (F) s = std::max<int64_t>(s, factor_grid(F));
        s = std::max<int64_t>(s, std::min<int64_t>((A->n_rows + kBlock - 1) / kBlock, kEllGrid));  // ELL apply
    }
    return std::max<int64_t>(s, 1);
}

static size_t carve(const spcg_csr *A, const spcg_cg_opts *o, char *base, Work *w) {
    const int64_t n = A->n_rows;
    const bool mixed = o->precision == SPCG_PREC_MIXED;
    const bool learned = o->precond == SPCG_PRECOND_LEARNED;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *q = base ? base + off : nullptr;
        off += align256(bytes);
        return q;
    };
    Work W;
    memset(&W, 0, sizeof W);
    W.nslots = n_slots(A, o);
    W.st = (CgState *)take(sizeof(CgState));
    W.hist = (double *)take(sizeof(double) * ((size_t)std::max(o->maxit, 0) + 1));
    W.r = (double *)take(sizeof(double) * n);
    W.dinv = (double *)take(sizeof(double) * n);
    if (!mixed) {
        W.p = (double *)take(sizeof(double) * n);
        W.q = (double *)take(sizeof(double) * n);
    }
    if (learned || o->variant == SPCG_CG_SINGLE_REDUCTION) {
        W.z = (double *)take(sizeof(double) * n);  // learned: z;  single reduction: u
        W.t = (double *)take(sizeof(double) * n);  // learned: t;  single reduction: w = A u
    }
    if (learned) W.x0 = (double *)take(sizeof(double) * n);
    if (learned && ell_width(o->G) && ell_width(o->GT)) {
        W.w_g = ell_width(o->G);
        W.w_gt = ell_width(o->GT);
        W.g_col = (int32_t *)take(sizeof(int32_t) * (size_t)W.w_g * n);
        W.g_val = (float *)take(sizeof(float) * (size_t)W.w_g * n);
        W.gt_col = (int32_t *)take(sizeof(int32_t) * (size_t)W.w_gt * n);
        W.gt_val = (float *)take(sizeof(float) * (size_t)W.w_gt * n);
    }
    if (mixed) {
        W.r32 = (float *)take(sizeof(float) * n);
        W.p32 = (float *)take(sizeof(float) * n);
        W.q32 = (float *)take(sizeof(float) * n);
        W.x32 = (float *)take(sizeof(float) * n);
        W.dinv32 = (float *)take(sizeof(float) * n);
        W.vals32 = (float *)take(sizeof(float) * (size_t)A->nnz);
        W.off16 = (int16_t *)take(sizeof(int16_t) * (size_t)A->nnz);
    }
    W.partd = (double *)take(sizeof(double) * 2 * W.nslots);
    if (learned) W.partg = (double *)take(sizeof(double) * W.nslots);
    W.partf = (float *)take(sizeof(float) * 2 * W.nslots);
    if (w) *w = W;
    return off;
}

static unsigned grid_of(int64_t n, int per) { return (unsigned)std::max<int64_t>((n + per - 1) / per, 1); }

struct Solver {
    spcg_csr *A;
    const spcg_cg_opts *o;
    Work w;
    hipStream_t s;
    CgState *h;  // pinned host copy
    double *x;
    const double *b;
    // timing mode: event pair around the SpMV launch of every timing_every-th
    // pass of the loop, with its pass number
    bool timing = false;
    int timing_every = 1;
    bool timed(int e) const { return timing && e % timing_every == 0; }
    // Ordinary (cache-allocating) loads for the matrices streamed every pass
    // when they fit keep_bytes(): A (or its FP32 copy in the mixed inner loop,
    // with 2-byte columns when c16); in the learned form A, G and G^T
    // together, else the two factors alone (measured at 128^3: keeping the
    // factors, 150 MB, beats keeping A).
    bool keep = false, keep_g = false, c16 = false;
    // a matrix above the limit: sixteenths of its row blocks read with
    // cache-allocating loads all the same (k_cg_q)
    int kq16 = 0;
    // learned form: factors as DIA planes (dia) with their offsets and widths
    bool dia = false;
    DiaOff dia_g{}, dia_gt{};
    int wd_g = 0, wd_gt = 0;
    void set_keep() {
        const bool mixed = o->precision == SPCG_PREC_MIXED;
        const int64_t a = mixed ? A->nnz * (c16 ? 6 : 8) + 4 * (int64_t)(A->n_rows + 1)
                                : matrix_bytes(A->n_rows, A->nnz, 8);
        int64_t f = 0;
        if (o->precond == SPCG_PRECOND_LEARNED) {
            if (dia)  // the DIA planes (4 bytes per slot)
                f = (int64_t)(wd_g + wd_gt) * A->n_rows * 4;
            else if (ell_width(o->G) && ell_width(o->GT))  // the ELL copies (8 bytes per slot)
                f = (int64_t)(ell_width(o->G) + ell_width(o->GT)) * A->n_rows * 8;
            else
                for (const spcg_csr *F : {o->G, o->GT})
                    if (F) f += matrix_bytes(F->n_rows, F->nnz, F->dtype == SPCG_F32 ? 4 : 8);
        }
        const int64_t lim = keep_bytes();
        keep = a + f <= lim;
        keep_g = f > 0 && f <= lim;
        if (dia && !keep && a <= lim) {
            // DIA applies stream their planes well: keep A instead of them
            keep = true;
            keep_g = false;
        }
        // Above the limit, the product of the standard and mixed loops keeps
        // the share of A that fits beside the vectors the pass reads with
        // cache-allocating loads (p, r and D^-1: 24 bytes per row in FP64,
        // 12 in FP32), in sixteenths rounded to nearest: at 160^3 (358 MB of
        // FP64 A, 4.6 sixteenths) 5/16 of the blocks,
        // Jacobi-PCG 107.5 -> 100.2 ms, where keeping all of A thrashes the
        // cache (114.4 -> 118.8 ms when that was measured)
        kq16 = 0;
        if (!keep && o->precond != SPCG_PRECOND_LEARNED && !single_reduction() && a > 0) {
            const int64_t vec = (int64_t)A->n_rows * (mixed ? 12 : 24);
            if (lim > vec) kq16 = (int)std::min<int64_t>(15, (32 * (lim - vec) / a + 1) / 2);  // nearest
        }
    }
    int n_timed = 0;
    int *timed_k = nullptr;

    int ensure_events(int pairs) {
        if (A->n_events >= 2 * pairs) return SPCG_OK;
        const int want = 2 * pairs;
        hipEvent_t *ev = new hipEvent_t[want];
        for (int i = 0; i < A->n_events; ++i) ev[i] = A->events[i];
        for (int i = A->n_events; i < want; ++i) {
            hipError_t e = hipEventCreate(&ev[i]);
            if (e != hipSuccess) {
                for (int j = A->n_events; j < i; ++j) (void)hipEventDestroy(ev[j]);
                delete[] ev;
                return hip_status(e, "hipEventCreate");
            }
        }
        delete[] A->events;
        A->events = ev;
        A->n_events = want;
        return SPCG_OK;
    }
    int cap_timed = 0;
    int grow_timed(int need) {
        if (need <= cap_timed) return SPCG_OK;
        const int cap = std::max(need, 2 * cap_timed);
        int *t = new int[cap];
        for (int i = 0; i < n_timed; ++i) t[i] = timed_k[i];
        delete[] timed_k;
        timed_k = t;
        cap_timed = cap;
        return SPCG_OK;
    }
    ~Solver() { delete[] timed_k; }
    // summed duration of the timed launches whose pass actually ran (k < k_end)
    void collect(int k_end, spcg_cg_result *res) {
        float tot = 0.0f;
        int calls = 0;
        for (int i = 0; i < n_timed; ++i) {
            if (timed_k[i] >= k_end) continue;
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, A->events[2 * i], A->events[2 * i + 1]) == hipSuccess) {
                tot += ms;
                ++calls;
            }
        }
        res->spmv_ms += tot;
        res->spmv_calls += calls;
        n_timed = 0;
    }

    int read_state() {
        SPCG_TRY(hipMemcpyAsync(h, w.st, sizeof(CgState), hipMemcpyDeviceToHost, s));
        SPCG_TRY(hipStreamSynchronize(s));
        return SPCG_OK;
    }
    unsigned gv() const { return grid_of(A->n_rows, kVecBlock); }
    unsigned gxr() const { return std::min<unsigned>(gv(), kXrGrid); }
    unsigned gA() const { return spmv_grid(A->n_blocks); }
    unsigned gA32() const { return spmv_grid(A->n_wblocks); }  // wide partition (mixed inner product)
    // the G^T apply's workgroups (and r.z partials, which every workgroup of K3L sums)
    unsigned gG() const {
        return w.w_g ? ell_grid() : std::min<unsigned>(factor_grid(o->GT), kApplyGrid);
    }

    // z = G (G^T r); r.z partials (t.t from the G^T apply) in w.partg
    unsigned ell_grid() const { return std::min<unsigned>(grid_of(A->n_rows, kBlock), kEllGrid); }

    // the G apply with the pass end folded in (K3G) in place of z = G t and K3L;
    // on the update kernels' grid (at most 1024 workgroups, each walking a range
    // of rows), since every workgroup sums all the partials first
    template <int WG, bool KEEP, bool DIA, class Dev>
    void g_pass(const Dev &g, int e) {
        hipLaunchKernelGGL((k_g_pass<WG, KEEP, DIA, Dev>), dim3(std::min(ell_grid(), gxr())), dim3(kBlock), 0, s, g,
                           (const double *)w.t, w.p, x, w.st, (const double *)w.partd, (int)gxr(),
                           (const double *)w.partg, (int)gG(), w.hist, e);
    }

    template <int WG, int WT, bool KEEP>
    void apply_ell(int kexp, bool fused) {
        const EllDev gt{w.gt_col, w.gt_val, A->n_rows}, g{w.g_col, w.g_val, A->n_rows};
        hipLaunchKernelGGL((k_gt_ell<WT, KEEP>), dim3(ell_grid()), dim3(kBlock), 0, s, gt,
                           (const double *)w.r, w.t, w.st, w.partg, kexp);
        if (fused)
            g_pass<WG, KEEP, false>(g, kexp);
        else
            hipLaunchKernelGGL((k_g_ell<WG, KEEP>), dim3(ell_grid()), dim3(kBlock), 0, s, g,
                               (const double *)w.t, w.z, w.st, kexp);
    }

    template <int WG, int WT, bool KEEP>
    void apply_dia(int kexp, bool fused) {
        const DiaDev gt{w.gt_val, dia_gt, A->n_rows}, g{w.g_val, dia_g, A->n_rows};
        hipLaunchKernelGGL((k_gt_dia<WT, KEEP>), dim3(ell_grid()), dim3(kBlock), 0, s, gt,
                           (const double *)w.r, w.t, w.st, w.partg, kexp);
        if (fused)
            g_pass<WG, KEEP, true>(g, kexp);
        else
            hipLaunchKernelGGL((k_g_dia<WG, KEEP>), dim3(ell_grid()), dim3(kBlock), 0, s, g,
                               (const double *)w.t, w.z, w.st, kexp);
    }

    // z = G (G^T r).  fused (a pass, kexp >= 0): with the ELL or DIA copies the
    // G apply also ends the pass (K3G) and z is not stored; returns whether it
    // did, else the caller launches K3L.
    bool apply_factor(int kexp, bool fused = false) {
        if (dia) {
#define SPCG_DIA(WG, WT)                                        \
    if (wd_g == WG && wd_gt == WT) {                            \
        if (keep_g) apply_dia<WG, WT, true>(kexp, fused);       \
        else apply_dia<WG, WT, false>(kexp, fused);             \
        return fused;                                           \
    }
            SPCG_DIA(4, 4) SPCG_DIA(4, 8) SPCG_DIA(8, 4) SPCG_DIA(8, 8)
#undef SPCG_DIA
        }
        if (w.w_g) {
#define SPCG_ELL(WG, WT)                                        \
    if (w.w_g == WG && w.w_gt == WT) {                          \
        if (keep_g) apply_ell<WG, WT, true>(kexp, fused);       \
        else apply_ell<WG, WT, false>(kexp, fused);             \
        return fused;                                           \
    }
            SPCG_ELL(4, 4) SPCG_ELL(4, 8) SPCG_ELL(8, 4) SPCG_ELL(8, 8)
#undef SPCG_ELL
        }
        const bool sgt = uses_short_rows(o->GT), sg = uses_short_rows(o->G);
        auto gt = sgt ? (keep_g ? k_gt_apply<true, true> : k_gt_apply<true, false>)
                      : (keep_g ? k_gt_apply<false, true> : k_gt_apply<false, false>);
        auto g = sg ? (keep_g ? k_g_apply<true, true> : k_g_apply<true, false>)
                    : (keep_g ? k_g_apply<false, true> : k_g_apply<false, false>);
        hipLaunchKernelGGL(gt, dim3(gG()), dim3(kBlock), 0, s, factor_view(o->GT),
                           (const double *)w.r, w.t, w.st, w.partg, kexp);
        hipLaunchKernelGGL(g, dim3(factor_grid(o->G)), dim3(kBlock), 0, s, factor_view(o->G),
                           (const double *)w.t, w.z, w.st, kexp);
        return false;
    }

    int resid(int mode, float *r32) {
        hipLaunchKernelGGL(k_resid, dim3(gA()), dim3(kBlock), 0, s, dev_view(A),
                           (const double *)A->vals, x, b, w.r, r32, w.st, w.partd, mode);
        hipLaunchKernelGGL(k_fin_resid, dim3(1), dim3(kFinThreads), 0, s, w.st,
                           (const double *)w.partd, (int)gA(), w.hist, mode, o->tol);
        SPCG_LAUNCH_CHECK("k_resid");
        return SPCG_OK;
    }

    bool single_reduction() const { return o->variant == SPCG_CG_SINGLE_REDUCTION; }

    // single reduction: u = M^-1 r, p = s = 0, w = A u, (gamma, delta) -> alpha
    int start_sr(int pre) {
        const int n = A->n_rows;
        if (pre == SPCG_PRECOND_JACOBI)
            hipLaunchKernelGGL(k_sr_start<SPCG_PRECOND_JACOBI>, dim3(gv()), dim3(kBlock), 0, s, n,
                               (const double *)w.r, (const double *)w.dinv, w.z, w.p, w.q, w.st);
        else
            hipLaunchKernelGGL(k_sr_start<SPCG_PRECOND_NONE>, dim3(gv()), dim3(kBlock), 0, s, n,
                               (const double *)w.r, (const double *)w.dinv, w.z, w.p, w.q, w.st);
        if (keep)
            hipLaunchKernelGGL(k_sr_w<true>, dim3(gA()), dim3(kBlock), 0, s, dev_view(A),
                               (const double *)A->vals, (const double *)w.z, (const double *)w.r,
                               w.t, w.st, w.partd, -1);
        else
            hipLaunchKernelGGL(k_sr_w<false>, dim3(gA()), dim3(kBlock), 0, s, dev_view(A),
                               (const double *)A->vals, (const double *)w.z, (const double *)w.r,
                               w.t, w.st, w.partd, -1);
        hipLaunchKernelGGL(k_fin_sr_start, dim3(1), dim3(kFinThreads), 0, s, w.st,
                           (const double *)w.partd, (int)gA(), w.hist);
        SPCG_LAUNCH_CHECK("single-reduction start");
        return SPCG_OK;
    }

    int pass_sr(int pre, int e) {
        const int n = A->n_rows;
        if (pre == SPCG_PRECOND_JACOBI)
            hipLaunchKernelGGL(k_sr_vec<SPCG_PRECOND_JACOBI>, dim3(gv()), dim3(kBlock), 0, s, n, e,
                               x, w.r, w.p, w.q, w.z, (const double *)w.t, (const double *)w.dinv,
                               w.st);
        else
            hipLaunchKernelGGL(k_sr_vec<SPCG_PRECOND_NONE>, dim3(gv()), dim3(kBlock), 0, s, n, e, x,
                               w.r, w.p, w.q, w.z, (const double *)w.t, (const double *)w.dinv,
                               w.st);
        {
            auto kern = keep ? k_sr_w<true> : k_sr_w<false>;
            if (timed(e)) {
                hipExtLaunchKernelGGL(kern, dim3(gA()), dim3(kBlock), 0, s, A->events[2 * n_timed],
                                      A->events[2 * n_timed + 1], 0, dev_view(A),
                                  (const double *)A->vals, (const double *)w.z,
                                  (const double *)w.r, w.t, w.st, w.partd, e);
                timed_k[n_timed++] = e;
            } else {
                hipLaunchKernelGGL(kern, dim3(gA()), dim3(kBlock), 0, s, dev_view(A),
                                  (const double *)A->vals, (const double *)w.z,
                                  (const double *)w.r, w.t, w.st, w.partd, e);
            }
        }
        hipLaunchKernelGGL(k_fin_sr, dim3(1), dim3(kFinThreads), 0, s, w.st,
                           (const double *)w.partd, (int)gA(), w.hist, e);
        SPCG_LAUNCH_CHECK("single-reduction pass");
        return SPCG_OK;
    }

    // z = M^-1 r, p = z, rho; the phase's first history entry
    int start(int pre) {
        if (single_reduction()) return start_sr(pre);
        const int n = A->n_rows;
        if (pre == SPCG_PRECOND_LEARNED) {
            apply_factor(-1);
            hipLaunchKernelGGL(k_start<SPCG_PRECOND_LEARNED>, dim3(gv()), dim3(kBlock), 0, s, n,
                               w.r, w.dinv, w.z, w.p, w.st, w.partd);
        } else if (pre == SPCG_PRECOND_JACOBI) {
            hipLaunchKernelGGL(k_start<SPCG_PRECOND_JACOBI>, dim3(gv()), dim3(kBlock), 0, s, n,
                               w.r, w.dinv, w.z, w.p, w.st, w.partd);
        } else {
            hipLaunchKernelGGL(k_start<SPCG_PRECOND_NONE>, dim3(gv()), dim3(kBlock), 0, s, n,
                               w.r, w.dinv, w.z, w.p, w.st, w.partd);
        }
        hipLaunchKernelGGL(k_fin_start, dim3(1), dim3(kFinThreads), 0, s, w.st,
                           (const double *)w.partd, (int)gv(), w.hist);
        SPCG_LAUNCH_CHECK("k_start");
        return SPCG_OK;
    }

    int pass64(int pre, int e) {
        const int n = A->n_rows;
        const double *pd = w.partd;
        {
            auto kern = keep ? k_cg_q<double, double, true> : k_cg_q<double, double, false>;
            if (timed(e)) {
                hipExtLaunchKernelGGL(kern, dim3(gA()), dim3(kBlock), 0, s, A->events[2 * n_timed],
                                      A->events[2 * n_timed + 1], 0, dev_view(A),
                                  (const double *)A->vals, (const double *)w.p, w.q, w.st,
                                  w.partd, e, kq16);
                timed_k[n_timed++] = e;
            } else {
                hipLaunchKernelGGL(kern, dim3(gA()), dim3(kBlock), 0, s, dev_view(A),
                                  (const double *)A->vals, (const double *)w.p, w.q, w.st,
                                  w.partd, e, kq16);
            }
        }
        if (pre != SPCG_PRECOND_LEARNED) {
            // F1, K2 on at most kXrGrid workgroups, K3F (pass end folded in)
            const unsigned gx = gxr();
            hipLaunchKernelGGL((k_fin_q<double, true>), dim3(1), dim3(kFinThreads), 0, s, w.st, pd,
                               (int)gA(), e);
            if (pre == SPCG_PRECOND_JACOBI) {
                hipLaunchKernelGGL((k_cg_xr<double, SPCG_PRECOND_JACOBI>), dim3(gx), dim3(kBlock), 0,
                                   s, n, e, w.r, (const double *)w.q, (const double *)w.dinv, w.st, w.partd);
                hipLaunchKernelGGL((k_cg_pf<double, SPCG_PRECOND_JACOBI, false>), dim3(gx),
                                   dim3(kBlock), 0, s, n, e, (const double *)w.r,
                                   (const double *)w.dinv, w.p, x, w.st, pd, (int)gx, w.hist);
            } else {
                hipLaunchKernelGGL((k_cg_xr<double, SPCG_PRECOND_NONE>), dim3(gx), dim3(kBlock), 0,
                                   s, n, e, w.r, (const double *)w.q, (const double *)w.dinv, w.st, w.partd);
                hipLaunchKernelGGL((k_cg_pf<double, SPCG_PRECOND_NONE, false>), dim3(gx),
                                   dim3(kBlock), 0, s, n, e, (const double *)w.r,
                                   (const double *)w.dinv, w.p, x, w.st, pd, (int)gx, w.hist);
            }
        } else {
            // F1, K2 (r.r), z = G (G^T r) with r.z, K3L (pass end folded in)
            const unsigned gx = gxr();
            hipLaunchKernelGGL((k_fin_q<double, true>), dim3(1), dim3(kFinThreads), 0, s, w.st, pd,
                               (int)gA(), e);
            hipLaunchKernelGGL((k_cg_xr<double, SPCG_PRECOND_LEARNED>), dim3(gx), dim3(kBlock),
                               0, s, n, e, w.r, (const double *)w.q, (const double *)w.dinv, w.st, w.partd);
            if (!apply_factor(e, true))
                hipLaunchKernelGGL(k_cg_pl, dim3(gx), dim3(kBlock), 0, s, n, e, (const double *)w.z, w.p,
                                   x, w.st, pd, (int)gx, (const double *)w.partg, (int)gG(), w.hist);
        }
        SPCG_LAUNCH_CHECK("cg pass");
        return SPCG_OK;
    }

    int pass32(int e) {
        const int n = A->n_rows;
        const float *pf = w.partf;
        {
            // over the wide partition (the compact columns are relative to its blocks)
            constexpr int W = kChunkWide;
            auto kern = keep ? (c16 ? k_cg_q<float, float, true, true, W> : k_cg_q<float, float, true, false, W>)
                             : (c16 ? k_cg_q<float, float, false, true, W> : k_cg_q<float, float, false, false, W>);
            CsrDev d = dev_view_wide(A);
            if (c16) d.off16 = w.off16;
            if (timed(e)) {
                hipExtLaunchKernelGGL(kern, dim3(gA32()), dim3(kBlock), 0, s, A->events[2 * n_timed],
                                      A->events[2 * n_timed + 1], 0, d, (const float *)w.vals32,
                                      (const float *)w.p32, w.q32, w.st, w.partf, e, kq16);
                timed_k[n_timed++] = e;
            } else {
                hipLaunchKernelGGL(kern, dim3(gA32()), dim3(kBlock), 0, s, d, (const float *)w.vals32,
                                   (const float *)w.p32, w.q32, w.st, w.partf, e, kq16);
            }
        }
        const unsigned gx = gxr();
        hipLaunchKernelGGL((k_fin_q<float, true>), dim3(1), dim3(kFinThreads), 0, s, w.st, pf,
                           (int)gA32(), e);
        hipLaunchKernelGGL((k_cg_xr<float, SPCG_PRECOND_JACOBI>), dim3(gx), dim3(kBlock), 0, s,
                           n, e, w.r32, (const float *)w.q32, (const float *)w.dinv32, w.st, w.partf);
        hipLaunchKernelGGL((k_cg_pf<float, SPCG_PRECOND_JACOBI, true>), dim3(gx), dim3(kBlock), 0,
                           s, n, e, (const float *)w.r32, (const float *)w.dinv32, w.p32, w.x32, w.st,
                           pf, (int)gx, w.hist);
        SPCG_LAUNCH_CHECK("mixed pass");
        return SPCG_OK;
    }

    int mp_rz(int init) {
        hipLaunchKernelGGL(k_mp_rz, dim3(gv()), dim3(kBlock), 0, s, A->n_rows, (const float *)w.r32,
                           (const float *)w.dinv32, w.p32, w.st, w.partf, init);
        hipLaunchKernelGGL(k_fin_mprz, dim3(1), dim3(kFinThreads), 0, s, w.st,
                           (const float *)w.partf, (int)gv(), w.hist, init);
        SPCG_LAUNCH_CHECK("k_mp_rz");
        return SPCG_OK;
    }

    // FP64 residual replacement: x64 += x32, r64 = b - A x64, r32 = fl32(r64), rho
    int replace() {
        hipLaunchKernelGGL(k_mp_fold, dim3(gv()), dim3(kBlock), 0, s, A->n_rows, x, w.x32, w.st, 0);
        SPCG_LAUNCH_CHECK("k_mp_fold");
        int rc = resid(R_REPLACE, w.r32);
        if (rc) return rc;
        return mp_rz(0);
    }

    // Run passes until the device state halts.  Batches are sized from the
    // observed residual decay so that few empty passes are enqueued.
    int loop(bool mixed, int pre) {
        int rc;
        double prev_rr = mixed ? h->rlast * h->rlast : h->rr;
        int prev_k = h->k;
        int batch = o->check_every > 0 ? o->check_every : 8;
        while (h->halt == RUN) {
            const int k0 = h->k;
            const int nb = std::min(batch, std::max(h->maxit - k0, 1));
            if (timing && (rc = ensure_events(n_timed + nb))) return rc;
            if (timing && (rc = grow_timed(n_timed + nb))) return rc;
            for (int j = 0; j < nb; ++j) {
                rc = mixed                ? pass32(k0 + j)
                     : single_reduction() ? pass_sr(pre, k0 + j)
                                          : pass64(pre, k0 + j);
                if (rc) return rc;
            }
            if ((rc = read_state())) return rc;
            if (mixed && h->halt == H_REPLACE) {
                if ((rc = replace())) return rc;
                if ((rc = read_state())) return rc;
            }
            if (o->check_every > 0) continue;
            // adaptive batch: passes predicted to reach the next stop test
            const double cur_rr = mixed ? (double)h->rr32 : h->rr;
            const int dk = h->k - prev_k;
            int next = 16;
            if (dk > 0 && cur_rr > 0.0 && prev_rr > cur_rr) {
                const double rate = std::log(prev_rr / cur_rr) / dk;  // per pass, in log(rr)
                double target = h->thresh * h->thresh;
                if (mixed) target = std::max(target, h->delta * h->delta * h->rlast * h->rlast);
                const double need = std::log(cur_rr / target) / rate;
                next = (int)std::ceil(std::max(need, 1.0));
            }
            batch = std::min(std::max(next, 2), 64);
            prev_rr = cur_rr;
            prev_k = h->k;
        }
        return SPCG_OK;
    }
};

// The single-workgroup solver runs on one CU: a pass costs about 6 us plus
// ~0.85 ns per nonzero there, against ~30 us for the five-launch pass of the
// grid-wide kernels on a tiny matrix, so it only pays up to ~32K nonzeros.
static int small_ok(const spcg_csr *A, const spcg_cg_opts *o) {
    return o->small_path && o->precision == SPCG_PREC_F64 && o->precond != SPCG_PRECOND_LEARNED &&
           o->variant == SPCG_CG_STANDARD && A->n_rows <= 16384 && A->nnz <= (int64_t)1 << 15;
}

// Shapes of the register-resident solver: rows per thread R and row length
// bound ML with about R * (2.5 ML + 4) registers within the 128 a 1024-thread
// workgroup allows, and 3 R * 8 KB of LDS (column indices need n < 2^16).
static int regs_shape(const spcg_csr *A) {
    const int64_t n = A->n_rows, ml = A->max_len;
    if (n <= kSmallThreads && ml <= 16) return 1;
    if (n <= 2 * kSmallThreads && ml <= 8) return 2;
    if (n <= 4 * kSmallThreads && ml <= 5) return 4;
    return 0;
}

static bool regs_ok(const spcg_csr *A) { return A->nnz > 0 && regs_shape(A) != 0; }

static int launch_regs(Solver &S, int pre, double *d_x) {
    const spcg_csr *A = S.A;
    Work &w = S.w;
    const int n = A->n_rows;
#define SPCG_REGS(P, RR, MM)                                                                    \
    hipLaunchKernelGGL((k_cg_regs<P, RR, MM>), dim3(1), dim3(kSmallThreads), 0, S.s, n, A->nnz, \
                       A->row_ptr, A->col, (const double *)A->vals, d_x, w.r,                  \
                       (const double *)w.p, (const double *)w.dinv, w.st, w.hist)
    const int R = regs_shape(A);
    if (pre == SPCG_PRECOND_JACOBI) {
        if (R == 1) SPCG_REGS(SPCG_PRECOND_JACOBI, 1, 16);
        else if (R == 2) SPCG_REGS(SPCG_PRECOND_JACOBI, 2, 8);
        else SPCG_REGS(SPCG_PRECOND_JACOBI, 4, 5);
    } else {
        if (R == 1) SPCG_REGS(SPCG_PRECOND_NONE, 1, 16);
        else if (R == 2) SPCG_REGS(SPCG_PRECOND_NONE, 2, 8);
        else SPCG_REGS(SPCG_PRECOND_NONE, 4, 5);
    }
#undef SPCG_REGS
    SPCG_LAUNCH_CHECK("k_cg_regs");
    return SPCG_OK;
}

// ------------------------------------------------ static scratch area --
// The workspace of cg_solve_static.  In host code `scratch` names a host-side
// stand-in, not device memory: the device address comes from
// hipGetSymbolAddress, once per device with that device current, and only
// that address is passed to kernels.
static __device__ __align__(256) char scratch[SPCG_STATIC_WORK_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[kMaxDevices] = {};

static int scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return SPCG_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_status(e, "hipGetSymbolAddress(scratch)");
        if (!p || ((uintptr_t)p & 255) != 0) return SPCG_HIP_ERROR;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return SPCG_OK;
}

}  // namespace spcg

using namespace spcg;

extern "C" {

void spcg_cg_default_opts(spcg_cg_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->tol = 1e-10;
    o->maxit = 20000;
    o->precond = SPCG_PRECOND_JACOBI;
    o->precision = SPCG_PREC_F64;
    o->check_every = 0;
    o->delta = 0.1;
    o->budget = 1 << 30;
    o->small_path = 1;
}

size_t spcg_cg_workspace_bytes(spcg_csr_t A, const spcg_cg_opts *o) {
    if (!A || !o) return 0;
    return carve(A, o, nullptr, nullptr);
}

int cg_solve(spcg_csr_t A, const double *d_b, double *d_x, const spcg_cg_opts *o, void *d_work,
             size_t work_bytes, spcg_cg_result *res, double *h_hist, hipStream_t s) {
    if (!A || !o || !res) return SPCG_INVALID_ARG;
    memset(res, 0, sizeof *res);
    if (A->dtype != SPCG_F64 || A->n_rows != A->n_cols) return SPCG_INVALID_ARG;
    if (o->maxit < 0 || !(o->tol >= 0.0)) return SPCG_INVALID_ARG;
    if (o->precond < SPCG_PRECOND_NONE || o->precond > SPCG_PRECOND_LEARNED) return SPCG_INVALID_ARG;
    if (o->precision != SPCG_PREC_F64 && o->precision != SPCG_PREC_MIXED) return SPCG_INVALID_ARG;
    if (o->variant != SPCG_CG_STANDARD && o->variant != SPCG_CG_SINGLE_REDUCTION) return SPCG_INVALID_ARG;
    if (o->variant == SPCG_CG_SINGLE_REDUCTION &&
        (o->precision != SPCG_PREC_F64 || o->precond == SPCG_PRECOND_LEARNED))
        return SPCG_INVALID_ARG;
    const bool mixed = o->precision == SPCG_PREC_MIXED;
    const bool learned = o->precond == SPCG_PRECOND_LEARNED;
    if (mixed && (o->precond != SPCG_PRECOND_JACOBI || !(o->delta > 0.0 && o->delta < 1.0)))
        return SPCG_INVALID_ARG;
    if (learned) {
        if (!o->G || !o->GT || o->G->dtype != SPCG_F32 || o->GT->dtype != SPCG_F32 ||
            o->G->n_rows != A->n_rows || o->GT->n_rows != A->n_rows ||
            o->G->n_cols != A->n_rows || o->GT->n_cols != A->n_rows || o->budget < 0)
            return SPCG_INVALID_ARG;
    }
    const int n = A->n_rows;
    if (n > 0 && (!d_b || !d_x)) return SPCG_INVALID_ARG;
    if (!d_work || ((uintptr_t)d_work & 255) != 0 || work_bytes < spcg_cg_workspace_bytes(A, o))
        return SPCG_INVALID_ARG;
    if (n == 0) {
        if (h_hist) h_hist[0] = 0.0;
        return SPCG_OK;
    }

    Solver S;
    S.A = A;
    S.o = o;
    S.s = s;
    S.x = d_x;
    S.b = d_b;
    S.set_keep();
    S.h = (CgState *)A->h_pinned;
    S.timing = o->timing > 0;
    S.timing_every = o->timing > 0 ? o->timing : 1;
    static_assert(sizeof(CgState) <= 256, "pinned status buffer");
    carve(A, o, (char *)d_work, &S.w);
    Work &w = S.w;
    int rc;
    const int budget = learned ? std::min(o->budget, o->maxit) : o->maxit;
    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(64), 0, s, w.st, learned ? budget : o->maxit,
                       o->delta, budget, 0);
    SPCG_LAUNCH_CHECK("k_init_state");
    if (o->precond == SPCG_PRECOND_JACOBI || learned) {
        hipLaunchKernelGGL(k_diag_inv, dim3(grid_of(n, kBlock)), dim3(kBlock), 0, s, n,
                           A->row_ptr, A->col, (const double *)A->vals, w.dinv, w.dinv32, w.st);
        SPCG_LAUNCH_CHECK("k_diag_inv");
    }
    if (mixed) {
        hipLaunchKernelGGL(k_to_f32, dim3(grid_of(A->nnz, kBlock * 8)), dim3(kBlock), 0, s,
                           A->nnz, (const double *)A->vals, w.vals32);
        hipLaunchKernelGGL(k_fill<float>, dim3(grid_of(n, kBlock * 8)), dim3(kBlock), 0, s,
                           (int64_t)n, w.x32, 0.0f);
        if (A->n_wblocks > 0)
            hipLaunchKernelGGL(k_make_off16, dim3((unsigned)std::min<int64_t>(A->n_wblocks, 4096)),
                               dim3(kBlock), 0, s, dev_view_wide(A), w.off16, w.st);
        SPCG_LAUNCH_CHECK("mixed set-up");
    }
    if (learned) {
        hipLaunchKernelGGL(k_copy, dim3(grid_of(n, kBlock * 8)), dim3(kBlock), 0, s, (int64_t)n,
                           (const double *)d_x, w.x0);
        SPCG_LAUNCH_CHECK("k_copy");
        for (int f = 0; f < 2 && w.w_g; ++f) {
            const spcg_csr *F = f ? o->GT : o->G;
            const unsigned grid = std::min<unsigned>(grid_of(n, kBlock), 4096);
            hipLaunchKernelGGL(k_dia_probe, dim3(grid), dim3(kBlock), 0, s, n, F->row_ptr,
                               (int)F->max_len, w.st, f);
            hipLaunchKernelGGL(k_dia_check, dim3(grid), dim3(kBlock), 0, s, n, F->row_ptr, F->col,
                               w.st, f);
            SPCG_LAUNCH_CHECK("k_dia_check");
        }
    }
    if ((rc = S.resid(R_INIT, mixed ? w.r32 : nullptr))) return rc;
    if ((rc = S.read_state())) return rc;
    CgState *h = S.h;
    if (mixed && A->n_wblocks > 0 && !h->c16_bad) {
        S.c16 = true;
        S.set_keep();
    }
    if (learned && w.w_g) {
        // the solve's copies of G and G^T: DIA planes when both lie on a few
        // diagonals, else padded ELL planes
        S.dia = !h->dia_bad[0] && !h->dia_bad[1];
        for (int f = 0; f < 2; ++f) {
            const spcg_csr *F = f ? o->GT : o->G;
            float *ev = f ? w.gt_val : w.g_val;
            const unsigned grid = std::min<unsigned>(grid_of(n, kBlock), 4096);
            if (S.dia) {
                DiaOff off{};
                const int cnt = h->dia_w[f];
                for (int j = 0; j < cnt; ++j) off.o[j] = h->dia_off[f][j];
                const int wd = cnt <= 4 ? 4 : kEllMax;
                (f ? S.dia_gt : S.dia_g) = off;
                (f ? S.wd_gt : S.wd_g) = wd;
                auto kern = wd == 4 ? k_to_dia<4> : k_to_dia<kEllMax>;
                hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, n, F->row_ptr, F->col,
                                   (const float *)F->vals, off, cnt, ev);
                SPCG_LAUNCH_CHECK("k_to_dia");
            } else {
                const int wd = f ? w.w_gt : w.w_g;
                int32_t *ec = f ? w.gt_col : w.g_col;
                auto kern = wd == 4 ? k_to_ell<4> : k_to_ell<kEllMax>;
                hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, n, F->row_ptr, F->col,
                                   (const float *)F->vals, ec, ev);
                SPCG_LAUNCH_CHECK("k_to_ell");
            }
        }
        S.set_keep();
    }
    if (h->bad_diag) return (h->bad_diag & 2) ? SPCG_NON_FINITE : SPCG_NOT_SPD;
    if (h->halt == H_ZERO) {
        hipLaunchKernelGGL(k_fill<double>, dim3(grid_of(n, kBlock * 8)), dim3(kBlock), 0, s,
                           (int64_t)n, d_x, 0.0);
        SPCG_LAUNCH_CHECK("k_fill");
        SPCG_TRY(hipStreamSynchronize(s));
        if (h_hist) h_hist[0] = 0.0;
        return SPCG_OK;
    }
    if (h->halt == H_BREAK) return h->status;

    int status = SPCG_OK;
    int restarts = 0;
    bool fell_back = false;
    int learned_iters = 0;
    int pre = o->precond;
    if ((rc = mixed ? S.mp_rz(1) : S.start(pre))) return rc;
    if ((rc = S.read_state())) return rc;

    for (;;) {
        if (h->halt == RUN) {
            if (!mixed && !learned && small_ok(A, o) && regs_ok(A)) {
                if ((rc = launch_regs(S, pre, d_x))) return rc;
                if ((rc = S.read_state())) return rc;
            } else if (!mixed && !learned && small_ok(A, o)) {
                // lanes per row: power-of-two floor of the mean row length, 1..16
                int L = 1;
                while (2 * L <= 16 && (int64_t)2 * L * n <= A->nnz) L *= 2;
                if (pre == SPCG_PRECOND_JACOBI)
                    hipLaunchKernelGGL(k_cg_small<SPCG_PRECOND_JACOBI>, dim3(1),
                                       dim3(kSmallThreads), 0, s, n, L, A->row_ptr, A->col,
                                       (const double *)A->vals, d_x, w.r, w.p, w.q, w.dinv, w.st,
                                       w.hist);
                else
                    hipLaunchKernelGGL(k_cg_small<SPCG_PRECOND_NONE>, dim3(1), dim3(kSmallThreads),
                                       0, s, n, L, A->row_ptr, A->col, (const double *)A->vals, d_x,
                                       w.r, w.p, w.q, w.dinv, w.st, w.hist);
                SPCG_LAUNCH_CHECK("k_cg_small");
                if ((rc = S.read_state())) return rc;
            } else {
                if ((rc = S.loop(mixed, pre))) return rc;
                if (S.timing) S.collect(h->k, res);
            }
        }
        const int halt = h->halt;
        if (pre == SPCG_PRECOND_LEARNED &&
            (halt == H_BUDGET || halt == H_BREAK || halt == H_MAXIT)) {
            // fall back to Jacobi-PCG: from x0 after a breakdown, else from x.
            // Its passes follow the learned ones in the pass count and the
            // history (its first entry replaces the learned phase's last), and
            // maxit bounds the two phases together
            learned_iters = h->k;
            fell_back = true;
            pre = SPCG_PRECOND_JACOBI;
            if (halt == H_BREAK) {
                hipLaunchKernelGGL(k_copy, dim3(grid_of(n, kBlock * 8)), dim3(kBlock), 0, s,
                                   (int64_t)n, (const double *)w.x0, d_x);
                SPCG_LAUNCH_CHECK("k_copy");
            }
            hipLaunchKernelGGL(k_init_state, dim3(1), dim3(64), 0, s, w.st, o->maxit, o->delta,
                               o->maxit, learned_iters);
            SPCG_LAUNCH_CHECK("k_init_state");
            if ((rc = S.resid(R_INIT, nullptr))) return rc;
            if ((rc = S.start(pre))) return rc;
            if ((rc = S.read_state())) return rc;
            if (h->halt == H_BREAK) return h->status;
            continue;
        }
        if (halt == H_BREAK) {
            status = h->status;
            break;
        }
        // exit check: fold the FP32 correction, recompute b - A x in FP64
        if (mixed) {
            hipLaunchKernelGGL(k_mp_fold, dim3(S.gv()), dim3(kBlock), 0, s, n, d_x, w.x32, w.st, 1);
            SPCG_LAUNCH_CHECK("k_mp_fold");
        }
        if ((rc = S.resid(R_TRUE, nullptr))) return rc;
        if ((rc = S.read_state())) return rc;
        const double tr = std::sqrt(h->true_rr) / h->nb;
        res->true_relres = tr;
        if (tr <= o->tol) {
            status = SPCG_OK;
            break;
        }
        if (h->k >= h->maxit || restarts >= 4 || mixed) {
            status = SPCG_NOT_CONVERGED;
            break;
        }
        // residual gap: restart from the true residual (r holds b - A x)
        ++restarts;
        hipLaunchKernelGGL(k_phase_state, dim3(1), dim3(64), 0, s, w.st);
        SPCG_LAUNCH_CHECK("k_phase_state");
        if ((rc = S.start(pre))) return rc;
        if ((rc = S.read_state())) return rc;
    }
    if (fell_back) {
        res->iters = learned_iters;
        res->iters_fallback = h->k - learned_iters;
        if (status == SPCG_OK) status = SPCG_FELL_BACK;
    } else {
        res->iters = h->k;
    }
    res->n_updates = h->n_updates;
    res->n_restarts = restarts;
    if (h_hist) {
        const int kk = h->k;
        SPCG_TRY(hipMemcpyAsync(h_hist, w.hist, sizeof(double) * (kk + 1), hipMemcpyDeviceToHost, s));
        SPCG_TRY(hipStreamSynchronize(s));
    }
    return status;
}

int cg_solve_static(spcg_csr_t A, const double *d_b, double *d_x, const spcg_cg_opts *o,
                    spcg_cg_result *res, double *h_hist, hipStream_t s) {
    if (!A || !o || !res) return SPCG_INVALID_ARG;
    memset(res, 0, sizeof *res);
    if (o->timing > 0) return SPCG_INVALID_ARG;  // timing mode creates events
    int dev = -1;
    SPCG_TRY(hipGetDevice(&dev));
    if (dev != A->device) return SPCG_INVALID_ARG;
    const size_t need = spcg_cg_workspace_bytes(A, o);
    if (need > SPCG_STATIC_WORK_BYTES) {
        char msg[160];
        snprintf(msg, sizeof msg, "cg_solve_static: the solve needs %zu bytes of workspace, the static "
                 "scratch area holds %zu", need, (size_t)SPCG_STATIC_WORK_BYTES);
        set_error_text(msg);
        return SPCG_TOO_LARGE;
    }
    void *work = nullptr;
    const int rc = scratch_address(dev, &work);
    if (rc) return rc;
    return cg_solve(A, d_b, d_x, o, work, SPCG_STATIC_WORK_BYTES, res, h_hist, s);
}

}  // extern "C"

// internal.h -- device building blocks of the gfx950 CSR SpMV / CG library.
//
// Layout of the work (CDNA4, 64-wide wavefronts, 256 CUs in 8 XCDs):
//  * Rows are partitioned once per matrix into row blocks of bounded work:
//    with the merge coordinate f(i) = row_ptr[i] + i (entries plus rows
//    before row i), block b owns the rows with f(i) in [b*kChunk, (b+1)*kChunk).
//    Every row but the last of a block has fewer than kChunk entries; a
//    block's entries fit the LDS slab (kSlab) unless its last row is long,
//    and then that row is reduced separately by the whole workgroup.
//  * One 256-thread workgroup per row block.  Phase 1 streams the block's
//    contiguous values and column indices with coalesced non-temporal loads,
//    gathers x and writes the products into LDS.  Phase 2 reduces each row
//    from LDS with a group of L lanes (L ~ the block's mean row length) and a
//    wavefront butterfly.  The summation order depends only on the matrix,
//    so results are bitwise reproducible.
//  * Block indices are remapped so that each XCD walks one contiguous range
//    of row blocks: x reuse of stencil matrices then stays in that XCD's L2.
//  * Scalar reductions (inner products) are deterministic: per-block partials
//    in fixed slots, reduced by the last block of each group of 256 to a group
//    partial, then by the last group to the final value, each in fixed order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spcg.h"

struct spcg_csr {
    int32_t n_rows = 0, n_cols = 0;
    int64_t nnz = 0;
    const int32_t *row_ptr = nullptr;
    const int32_t *col = nullptr;
    const void *vals = nullptr;
    int32_t dtype = SPCG_F64;
    int device = 0;
    int32_t *block_row = nullptr;  // [n_blocks + 1], owned
    int64_t n_blocks = 0;
    int64_t n_long = 0;            // blocks whose last row is reduced separately
    int64_t max_len = 0;
    int32_t *flags = nullptr;      // small device scratch for the analysis, owned
    void *h_pinned = nullptr;      // pinned host words for status reads, owned
};

namespace spcg {

constexpr int kBlock = 256;              // threads per workgroup of the streaming kernels
constexpr int kChunk = 1024;             // merge-coordinate span of one row block
constexpr int kSlab = 1792;               // LDS products per row block (>= kChunk; longer last rows go strided)
constexpr int kGroup = 256;              // partial slots reduced per group in the two-level reduction

void set_error(hipError_t e, const char *what);
int hip_status(hipError_t e, const char *what);

#define SPCG_TRY(expr)                                   \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return spcg::hip_status(e_, #expr); \
    } while (0)

#define SPCG_LAUNCH_CHECK(name) SPCG_TRY(hipGetLastError())

inline int64_t n_row_blocks(int64_t n_rows, int64_t nnz) {
    if (n_rows == 0) return 0;
    return (nnz + n_rows + kChunk - 1) / kChunk;
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// ------------------------------------------------------------ reductions --

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    // butterfly: every lane ends with the same, order-fixed sum
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over a 256-thread workgroup; every thread receives the result.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *sh4) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh4[threadIdx.x >> 6] = v;
    __syncthreads();
    T r = (sh4[0] + sh4[1]) + (sh4[2] + sh4[3]);
    __syncthreads();
    return r;
}

// Logical index of this workgroup: each of the 8 XCDs (which receive
// workgroups round-robin) gets one contiguous range of logical blocks.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int nb8 = nb & ~7;
    if (b >= nb8) return b;
    const int per = nb8 >> 3;
    return (b & 7) * per + (b >> 3);
}

// Control block of the two-level reduction (lives in the workspace).
template <typename T>
struct Reduce {
    T *partials;          // [nslots * NV]
    T *gpartials;         // [ngroups * NV]
    unsigned *counters;   // [ngroups + 1], zero between uses
};

// Called by every thread of a workgroup after the workgroup has reduced its
// NV values (valid in all threads).  The last workgroup overall calls
// fin(total) from thread 0 with the fixed-order totals.  Counters are left at
// zero for the next kernel.
template <int NV, typename T, class Fin>
__device__ __forceinline__ void reduce_arrive(const T (&v)[NV], int slot, int nslots,
                                              const Reduce<T> &R, Fin &fin) {
    __shared__ int s_last;
    __shared__ T s_red[4];
    const int ngroups = (nslots + kGroup - 1) / kGroup;
    const int g = slot / kGroup;
    const int gsize = min(kGroup, nslots - g * kGroup);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) R.partials[(size_t)slot * NV + j] = v[j];
        __threadfence();
        unsigned prev = atomicAdd(&R.counters[g], 1u);
        s_last = (prev == (unsigned)(gsize - 1));
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    T gs[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        T t = (threadIdx.x < gsize) ? R.partials[(size_t)(g * kGroup + threadIdx.x) * NV + j]
                                    : T(0);
        gs[j] = block_sum(t, s_red);
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) R.gpartials[(size_t)g * NV + j] = gs[j];
        R.counters[g] = 0u;
        __threadfence();
        unsigned prev = atomicAdd(&R.counters[ngroups], 1u);
        s_last = (prev == (unsigned)(ngroups - 1));
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    T tot[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        T t = T(0);
        for (int i = threadIdx.x; i < ngroups; i += kBlock)
            t += R.gpartials[(size_t)i * NV + j];
        tot[j] = block_sum(t, s_red);
    }
    if (threadIdx.x == 0) {
        R.counters[ngroups] = 0u;
        fin(tot);
    }
}

template <typename T>
inline size_t reduce_bytes(int64_t nslots, int nv) {
    const int64_t ng = (nslots + kGroup - 1) / kGroup;
    return align256(sizeof(T) * nslots * nv) + align256(sizeof(T) * ng * nv) +
           align256(sizeof(unsigned) * (ng + 1));
}

template <typename T>
inline Reduce<T> reduce_carve(char *&p, int64_t nslots, int nv) {
    const int64_t ng = (nslots + kGroup - 1) / kGroup;
    Reduce<T> R;
    R.partials = reinterpret_cast<T *>(p);
    p += align256(sizeof(T) * nslots * nv);
    R.gpartials = reinterpret_cast<T *>(p);
    p += align256(sizeof(T) * ng * nv);
    R.counters = reinterpret_cast<unsigned *>(p);
    p += align256(sizeof(unsigned) * (ng + 1));
    return R;
}

// ------------------------------------------------------------- SpMV core --

struct CsrDev {
    const int32_t *__restrict__ row_ptr;
    const int32_t *__restrict__ col;
    const int32_t *__restrict__ block_row;
    int n_blocks;
};

template <typename TA>
struct SpmvSmem {
    TA slab[kSlab];
    int32_t rp[kChunk + 1];
    TA red[4];
};

// Row products of one row block.  TV: value type, TX: vector type, TA:
// accumulation type.  epi.row(i, s) is called exactly once for every row i
// of the block, by one thread.  Must be called by all 256 threads.
template <typename TV, typename TX, typename TA, class Epi>
__device__ __forceinline__ void spmv_block(const CsrDev &A, const TV *__restrict__ vals,
                                           const TX *__restrict__ x, int blk,
                                           SpmvSmem<TA> &sm, Epi &epi) {
    const int tid = threadIdx.x;
    const int r0 = A.block_row[blk];
    const int r1 = A.block_row[blk + 1];
    if (r0 >= r1) return;  // uniform over the workgroup
    const int k0 = A.row_ptr[r0];
    const int klast = A.row_ptr[r1 - 1];
    const int kend = A.row_ptr[r1];
    const bool long_last = (kend - k0) > kSlab;
    const int rs_end = long_last ? r1 - 1 : r1;  // rows reduced from LDS: [r0, rs_end)
    const int cnt = (long_last ? klast : kend) - k0;
    const int nr = rs_end - r0;

    // phase 1: coalesced streams of col/vals, gather of x, products to LDS
    constexpr int U = kSlab / kBlock;
    int c[U];
    TV v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int t = tid + u * kBlock;
        if (t < cnt) {
            c[u] = __builtin_nontemporal_load(A.col + k0 + t);
            v[u] = __builtin_nontemporal_load(vals + k0 + t);
        }
    }
    for (int t = tid; t <= nr; t += kBlock) sm.rp[t] = A.row_ptr[r0 + t] - k0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int t = tid + u * kBlock;
        if (t < cnt) sm.slab[t] = TA(v[u]) * TA(x[c[u]]);
    }
    __syncthreads();

    // phase 2: L lanes per row, L = pow2 floor of the mean row length (<= 64)
    if (nr > 0) {
        const int avg = cnt / nr;
        const int L = avg >= 64 ? 64 : (avg <= 1 ? 1 : (1 << (31 - __clz(avg))));
        const int lane = tid & (L - 1);
        const int grp = tid / L;
        const int ngrp = kBlock / L;
        for (int r = grp; r < nr; r += ngrp) {
            const int a = sm.rp[r], e = sm.rp[r + 1];
            TA s = TA(0);
            for (int t = a + lane; t < e; t += L) s += sm.slab[t];
            for (int o = L >> 1; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
            if (lane == 0) epi.row(r0 + r, s);
        }
    }
    if (long_last) {
        // the block's last row is longer than the slab: whole workgroup, strided
        TA s0 = TA(0), s1 = TA(0), s2 = TA(0), s3 = TA(0);
        int k = klast + tid;
        for (; k + 3 * kBlock < kend; k += 4 * kBlock) {
            s0 += TA(vals[k]) * TA(x[A.col[k]]);
            s1 += TA(vals[k + kBlock]) * TA(x[A.col[k + kBlock]]);
            s2 += TA(vals[k + 2 * kBlock]) * TA(x[A.col[k + 2 * kBlock]]);
            s3 += TA(vals[k + 3 * kBlock]) * TA(x[A.col[k + 3 * kBlock]]);
        }
        for (; k < kend; k += kBlock) s0 += TA(vals[k]) * TA(x[A.col[k]]);
        TA s = block_sum((s0 + s1) + (s2 + s3), sm.red);
        if (tid == 0) epi.row(r1 - 1, s);
    }
}

inline CsrDev dev_view(const spcg_csr *A) {
    return CsrDev{A->row_ptr, A->col, A->block_row, (int)A->n_blocks};
}

}  // namespace spcg

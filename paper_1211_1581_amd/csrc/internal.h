// internal.h -- device building blocks of the gfx950 CSR SpMV / CG library.
//
// Layout of the work (CDNA4, 64-wide wavefronts, 256 CUs in 8 XCDs):
//  * Rows are partitioned once per matrix into row blocks of bounded work:
//    with the merge coordinate f(i) = row_ptr[i] + i (entries plus rows
//    before row i), block b owns the rows with f(i) in [b*kChunk, (b+1)*kChunk).
//    The rows before a block's last one hold fewer than kChunk entries in
//    all; the block's entries fit the LDS slab (kSlab) unless its last row is
//    long, and then that row is reduced separately by the whole workgroup.
//  * A 256-thread workgroup handles a contiguous range of row blocks (one
//    block per workgroup up to kMaxGrid blocks; 8 resident per CU).  Phase 1
//    streams the block's contiguous values and column indices with coalesced
//    loads (cache-allocating or non-temporal, see keep_bytes; 16-byte value
//    vectors of consecutive entries per lane where that pays), gathers x and
//    writes the products into LDS.  Phase 2 reduces each row
//    from LDS with a group of L lanes (L ~ the block's mean row length) and a
//    wavefront butterfly.  The summation order depends only on the matrix,
//    so results are bitwise reproducible.
//  * Workgroup indices are remapped so that each XCD walks one contiguous
//    range of row blocks: x reuse of stencil matrices stays in that XCD's L2.
//  * Scalar reductions (inner products) are deterministic: per-workgroup
//    partials in fixed slots, summed in fixed order by a one-workgroup
//    finalize kernel or, at the end of a CG pass, by every workgroup of the
//    next kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

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
    int32_t *block_k = nullptr;    // [n_blocks + 1], owned
    int64_t n_blocks = 0;
    // the wide partition (span kChunkWide) of the FP32 products; n_rows > 0 only
    int32_t *wblock_row = nullptr;  // [n_wblocks + 1], owned
    int32_t *wblock_k = nullptr;    // [n_wblocks + 1], owned
    int64_t n_wblocks = 0;
    int64_t n_long = 0;            // blocks whose last row is reduced separately
    int64_t max_len = 0;
    int32_t *flags = nullptr;      // small device scratch for the analysis, owned
    void *h_pinned = nullptr;      // pinned host words for status reads, owned
    hipEvent_t *events = nullptr;  // timing mode: event pool, owned
    int n_events = 0;
    // row-length bins (bins.hip): each bin's rows in ascending order with
    // their first entry and length, owned; built when the binning policy at
    // creation asks for them
    int32_t *bin_row = nullptr, *bin_k = nullptr, *bin_len = nullptr;
    int32_t bin_count[SPCG_NUM_BINS] = {}, bin_start[SPCG_NUM_BINS] = {};
    bool has_bins = false;
    // run-compressed columns (runs.hip), owned; built when the run policy at
    // creation asks for them
    unsigned long long *run_mask = nullptr;
    int32_t *run_base = nullptr, *run_col = nullptr, *run_chunk = nullptr;
    int64_t n_chunks = 0, n_heads = 0;
    bool has_runs = false;
    // column panels (panels.hip), owned; built when the panel policy at
    // creation asks for them
    int32_t *pan_range = nullptr, *pan_phase = nullptr, *pan_vstart = nullptr, *pan_base = nullptr;
    uint32_t *pan_key = nullptr;
    void *pan_val = nullptr;
    void *pan_part = nullptr;  // [column groups][n_rows] partial products of spmv_csr
    // the last panel product's stream and completion: a product on another
    // stream waits for it, so products sharing pan_part never overlap
    hipEvent_t pan_done = nullptr;
    hipStream_t pan_last = nullptr;
    bool pan_any = false;
    std::mutex pan_mu;
    int pan_P = 0, pan_R = 0, pan_W = 0;
    int64_t pan_entries = 0;  // entries of the panel copy, padding included
    bool has_panels = false;
};

namespace spcg {

constexpr int kBlock = 256;              // threads per workgroup of the streaming kernels
constexpr int kChunk = 1536;             // merge-coordinate span of one row block
constexpr int kSlabExtra = 240;          // slab slots beyond the span (a moderately long last row stays in LDS)
constexpr int kSlab = kChunk + kSlabExtra;  // LDS products per row block (longer last rows go strided)
// Span of the second ("wide") partition that every handle keeps for the
// products with FP32 values and sums (the standalone product of an FP32
// handle, the mixed-precision solve's inner product, the network's loss
// products): their LDS (slab of floats and row pointers, 17.4 KB) still
// leaves room for 8 workgroups per CU, and a block carries a third more
// entries through the same chain of dependent loads (128^3 FP32 product
// 29.9 -> 28.9 us, a 2^20-row band of width 63 120.5 -> 106 us).  Every
// other kernel, including those that read FP32 values with FP64 sums, uses
// kChunk.
constexpr int kChunkWide = 2048;
constexpr int kMaxGrid = 32768;          // workgroups of a row-block kernel (each walks a range)

// Load policy of the matrix streams (col, vals).  The MI355X keeps a 256 MB
// memory-side cache (MALL) in front of HBM; ordinary loads allocate in it,
// non-temporal loads do not.  A matrix whose streamed bytes per product are at
// most keep_bytes() (default kKeepBytes, set by spcg_keep_bytes) is read with
// ordinary loads, so repeated products (a CG pass loop) find it there: 128^3
// 7-point Poisson in FP64 (183.5 MB) runs its CG product in ~41 instead of
// ~50 us.  Larger matrices stream non-temporally: with ordinary loads the
// 160^3 systems (358 MB FP64, 244 MB FP32) thrash the cache and run 3-5 %
// slower.  Both policies give bitwise-identical results.
constexpr int64_t kKeepBytes = int64_t(192) << 20;
int64_t keep_bytes();

// Bytes one product streams from the matrix: col, vals and row_ptr.
inline int64_t matrix_bytes(int64_t n_rows, int64_t nnz, int val_bytes) {
    return nnz * (4 + val_bytes) + 4 * (n_rows + 1);
}

// Row-block kernels run 8 workgroups of 256 per CU (8 waves per SIMD, the
// most a SIMD holds): the FP64 slab, row pointers and block sums take 20464
// bytes of LDS, just within a 160 KB / 8 share, and the kernels stay within
// 64 VGPRs.  A slab of 1792 (20592 bytes) left room for only 7 and cost the
// FP64 product 4-5 %.
#define SPCG_ROWBLOCK_KERNEL __global__ void __launch_bounds__(256)

void set_error(hipError_t e, const char *what);
void set_error_text(const char *text);
int hip_status(hipError_t e, const char *what);

#define SPCG_TRY(expr)                                   \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) return spcg::hip_status(e_, #expr); \
    } while (0)

#define SPCG_LAUNCH_CHECK(name) SPCG_TRY(hipGetLastError())

inline int64_t n_row_blocks(int64_t n_rows, int64_t nnz, int chunk = kChunk) {
    if (n_rows == 0) return 0;
    return (nnz + n_rows + chunk - 1) / chunk;
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Workgroups launched for a row-block kernel over nb row blocks.
inline unsigned spmv_grid(int64_t nb) {
    return (unsigned)(nb < kMaxGrid ? (nb > 0 ? nb : 1) : kMaxGrid);
}

// ------------------------------------------------------------ reductions --

// Cross-lane moves inside rows of 16 lanes by DPP (v_mov_b32_dpp: a VALU
// operand modifier, no LDS round trip; a 64-lane shuffle goes through the LDS
// crossbar as ds_bpermute).  The source lanes are those of the caller's group,
// which must be active.
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]: lane l <- l ^ 1
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]: lane l <- l ^ 2
constexpr int kDppHalfMirror = 0x141;  // lane l <- 7 - l within each group of 8
constexpr int kDppMirror = 0x140;      // lane l <- 15 - l within each row of 16

template <int CTRL>
__device__ __forceinline__ int dpp_mov(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ int lane_value(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

__device__ __forceinline__ float lane_value(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

__device__ __forceinline__ double lane_value(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over groups of L aligned lanes (L a power of two <= 64, uniform over
// the wavefront): every lane of a group ends with its group's sum.  Within a
// row of 16 the pairs are formed by mirrors and quad permutations, which
// cover each group exactly like an xor butterfly.
template <typename T>
__device__ __forceinline__ T group_sum(T s, int L) {
    if (L >= 64) s += __shfl_xor(s, 32, 64);
    if (L >= 32) s += __shfl_xor(s, 16, 64);
    if (L >= 16) s += dpp_mov<kDppMirror>(s);
    if (L >= 8) s += dpp_mov<kDppHalfMirror>(s);
    if (L >= 4) s += dpp_mov<kDppXor2>(s);
    if (L >= 2) s += dpp_mov<kDppXor1>(s);
    return s;
}

// Sum over a whole wavefront (all lanes active): rows of 16 by DPP, then the
// four row sums read from lanes 0, 16, 32, 48 and added in a fixed order, so
// every lane gets the same value.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    v += dpp_mov<kDppXor1>(v);
    v += dpp_mov<kDppXor2>(v);
    v += dpp_mov<kDppHalfMirror>(v);
    v += dpp_mov<kDppMirror>(v);
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
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

// Deterministic scalar reductions: every workgroup of a producing kernel
// writes its NV partial sums to a fixed slot; a one-workgroup finalize kernel
// (kFinThreads threads) then sums the slots in a fixed order and acts on the
// totals.  (A "last workgroup finishes" scheme inside the producer needs a
// device-scope release/acquire per workgroup, which on CDNA writes back and
// invalidates the XCD's L2 and costs far more than the extra launch.)
constexpr int kFinThreads = 512;

template <typename T, int NV>
__device__ __forceinline__ void store_partials(T *part, int slot, const T (&v)[NV]) {
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) part[(size_t)slot * NV + j] = v[j];
    }
}

// Partial sums of one workgroup at its end: each wavefront reduces its
// values with a butterfly and parks them in LDS, one barrier, then thread 0
// adds the kWaves wavefront sums in order and writes slot `slot`.  Row-block
// kernels skip the barrier that would otherwise follow their last block, so
// the workgroup ends with a single barrier (a workgroup that stays resident
// longer costs the streaming kernels several percent, and per-wavefront
// partials would quadruple what the one-workgroup finalize has to read).
constexpr int kWaves = kBlock / 64;

template <typename T, int NV>
__device__ __forceinline__ void store_block_partials(T *part, int slot, const T (&v)[NV],
                                                     T *red /* LDS, kWaves * NV */) {
    T s[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) s[j] = wave_sum(v[j]);
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) red[(threadIdx.x >> 6) * NV + j] = s[j];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            T t = red[j];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) t += red[w * NV + j];
            part[(size_t)slot * NV + j] = t;
        }
    }
}

// Fixed-order totals of two partial arrays at once: a (na >= 1 slots x NA
// values) and b (nb >= 1 slots x NB values).  Call from all kFinThreads
// threads of a one-workgroup kernel; every thread receives the totals.  The
// slots are loaded kFinPer per thread and round together (clamped indices,
// no branch around the loads), then added in slot order.
template <typename T, int NA, int NB>
__device__ __forceinline__ void finalize_sum2(const T *__restrict__ a, int na, T (&ta)[NA],
                                              const T *__restrict__ b, int nb, T *tb) {
    constexpr int NV = NA + NB;
    // slots per thread and round: two wavefronts per SIMD leave room for many
    // loads in flight (16K single-value or 8K three-value slots per round)
    constexpr int kFinPer = NV >= 3 ? 16 : 32 / NV;
    __shared__ T sh[kFinThreads / 64][NV];
    T acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = T(0);
    const int tid = threadIdx.x;
    const int nmax = na > nb ? na : nb;
    for (int base = 0; base < nmax; base += kFinThreads * kFinPer) {
        T v[kFinPer][NV];
#pragma unroll
        for (int u = 0; u < kFinPer; ++u) {
            const int i = base + tid + u * kFinThreads;
            const int ia = min(i, na - 1);
#pragma unroll
            for (int j = 0; j < NA; ++j) v[u][j] = a[(size_t)ia * NA + j];
            if constexpr (NB > 0) {
                const int ib = min(i, nb - 1);
#pragma unroll
                for (int j = 0; j < NB; ++j) v[u][NA + j] = b[(size_t)ib * NB + j];
            }
        }
#pragma unroll
        for (int u = 0; u < kFinPer; ++u) {
            const int i = base + tid + u * kFinThreads;
#pragma unroll
            for (int j = 0; j < NA; ++j) acc[j] += i < na ? v[u][j] : T(0);
#pragma unroll
            for (int j = NA; j < NV; ++j) acc[j] += i < nb ? v[u][j] : T(0);
        }
    }
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        acc[j] = wave_sum(acc[j]);
        if ((tid & 63) == 0) sh[tid >> 6][j] = acc[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        T t = T(0);
#pragma unroll
        for (int w = 0; w < kFinThreads / 64; ++w) t += sh[w][j];
        if (j < NA) ta[j] = t;
        else if constexpr (NB > 0) tb[j - NA] = t;
    }
    __syncthreads();
}

// Fixed-order total of nslots >= 1 x NV partials (see finalize_sum2).
template <typename T, int NV>
__device__ __forceinline__ void finalize_sum(const T *__restrict__ part, int nslots, T (&tot)[NV]) {
    finalize_sum2<T, NV, 0>(part, nslots, tot, part, 1, nullptr);
}

// ------------------------------------------------------------- SpMV core --

struct CsrDev {
    const int32_t *__restrict__ row_ptr;
    const int32_t *__restrict__ col;
    const int32_t *__restrict__ block_row;  // first row of each row block  [n_blocks + 1]
    const int32_t *__restrict__ block_k;    // row_ptr[block_row[b]]        [n_blocks + 1]
    int n_blocks;
    // optional compact columns: col[k] - block_row[b] as int16 for every
    // entry k of row block b (the kernels instantiated with C16 read these
    // instead of col)
    const int16_t *__restrict__ off16;
    // optional run-compressed columns (runs.hip; the kernels instantiated with
    // RUNS read these instead of col for the entries a block stages in LDS):
    // the staged entries of block b form 64-entry chunks from run_chunk[b] on;
    // bit l of run_mask[c] marks entry l of chunk c as the first of a run of
    // consecutive columns (bit 0 always), run_base[c] is the chunk's first
    // head in run_col, which holds the columns of the heads
    const unsigned long long *__restrict__ run_mask;
    const int32_t *__restrict__ run_base;
    const int32_t *__restrict__ run_col;
    const int32_t *__restrict__ run_chunk;
};

// Column of staged entry t of a block whose chunks start at cb (RUNS layout):
// the nearest run head at or before t in its chunk, plus the distance to it.
__device__ __forceinline__ int run_column(const CsrDev &A, int cb, int t) {
    const int j = t >> 6, l = t & 63;
    const unsigned long long m = A.run_mask[cb + j];
    const unsigned long long upto = l == 63 ? m : (m & ((2ull << l) - 1ull));
    const int nh = __popcll(upto);
    const int hl = 63 - __clzll(upto);
    return A.run_col[A.run_base[cb + j] + nh - 1] + (l - hl);
}

// LDS of a row-block kernel for partitions of span at most CH
template <typename TA, int CH = kChunk>
struct SpmvSmem {
    static constexpr int kSl = CH + kSlabExtra;
    TA slab[kSl + 1];  // + a spare slot for the stores of clamped lanes
    int32_t rp[CH + 1];
    TA red[kBlock / 64 * 3];  // block sums: up to 3 values per wavefront
    TA last;
};

// Products of NU rounds of kBlock entries starting at k0 (cnt >= 1 entries
// are real; the clamped tail re-reads the last one and is not stored).  KEEP:
// ordinary loads of col/vals (see keep_bytes), else non-temporal ones.  C16:
// columns from A.off16 relative to the block's first row r0.  RUNS: columns
// from the run-compressed layout, the block's chunks starting at cb.
template <int NU, bool KEEP, bool C16, bool RUNS, int SPARE, typename TV, typename TX, typename TA>
__device__ __forceinline__ void block_products(const CsrDev &A, const TV *__restrict__ vals,
                                               const TX *__restrict__ x, int k0, int cnt, int r0,
                                               int cb, TA *__restrict__ slab, int first = 0) {
    const int tid = threadIdx.x + first;
    // the block's streams from bases that are uniform over the workgroup
    // (scalar registers) plus 32-bit byte offsets per lane: one register per
    // address instead of a 64-bit pair, so every round's loads stay in
    // registers at eight wavefronts per SIMD (with 64-bit addresses the
    // compiler deferred a round until the others had arrived)
    const char *colb = (const char *)(A.col + k0);
    const char *offb = (const char *)(A.off16 + (C16 ? k0 : 0));
    const char *valb = (const char *)(vals + k0);
    int c[NU];
    TV v[NU];
    TX xv[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const uint32_t t = (uint32_t)min(tid + u * kBlock, cnt - 1);
        if constexpr (RUNS) {
            c[u] = run_column(A, cb, (int)t);
        } else if constexpr (C16) {
            const int16_t *p = (const int16_t *)(offb + t * 2u);
            c[u] = r0 + (KEEP ? *p : __builtin_nontemporal_load(p));
        } else {
            const int32_t *p = (const int32_t *)(colb + t * 4u);
            c[u] = KEEP ? *p : __builtin_nontemporal_load(p);
        }
        const TV *q = (const TV *)(valb + t * (uint32_t)sizeof(TV));
        v[u] = KEEP ? *q : __builtin_nontemporal_load(q);
    }
#pragma unroll
    for (int u = 0; u < NU; ++u) xv[u] = x[c[u]];
    // every lane stores, clamped lanes into the slab's spare slot: a store
    // under a branch let the compiler sink a round's loads into the branch,
    // where they waited for all the others
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int t = tid + u * kBlock;
        slab[t < cnt ? t : SPARE] = TA(v[u]) * TA(xv[u]);
    }
}

// Products of NR rounds of kBlock lanes times V consecutive entries (V kBlock
// entries a round) starting at k0, with cnt >= V: each lane loads its V values
// as one 16-byte vector and its V columns as one vector, so a round takes two
// stream instructions per V entries instead of two per entry.  A lane whose
// group reaches past the block reads the block's last V entries instead and
// stores only those from its own first entry on (the others into the spare
// slot).  The loads need not be aligned to their size (the unaligned access
// mode serves them).
template <int V, int NR, bool KEEP, bool C16, int SPARE, typename TV, typename TX, typename TA>
__device__ __forceinline__ void block_products_vec(const CsrDev &A, const TV *__restrict__ vals,
                                                   const TX *__restrict__ x, int k0, int cnt, int r0,
                                                   TA *__restrict__ slab, int first = 0) {
    typedef TV vals_t __attribute__((ext_vector_type(V)));
    typedef int32_t cols_t __attribute__((ext_vector_type(V)));
    typedef int16_t offs_t __attribute__((ext_vector_type(V)));
    const int tid = threadIdx.x + first;
    const char *colb = (const char *)(A.col + k0);
    const char *offb = (const char *)(A.off16 + (C16 ? k0 : 0));
    const char *valb = (const char *)(vals + k0);
    int c[NR][V];
    vals_t v[NR];
    TX xv[NR][V];
#pragma unroll
    for (int u = 0; u < NR; ++u) {
        const uint32_t t0 = (uint32_t)min(V * (tid + u * kBlock), cnt - V);
        if constexpr (C16) {
            const offs_t *p = (const offs_t *)(offb + t0 * 2u);
            const offs_t o = KEEP ? *p : __builtin_nontemporal_load(p);
#pragma unroll
            for (int q = 0; q < V; ++q) c[u][q] = r0 + o[q];
        } else {
            const cols_t *p = (const cols_t *)(colb + t0 * 4u);
            const cols_t o = KEEP ? *p : __builtin_nontemporal_load(p);
#pragma unroll
            for (int q = 0; q < V; ++q) c[u][q] = o[q];
        }
        const vals_t *q = (const vals_t *)(valb + t0 * (uint32_t)sizeof(TV));
        v[u] = KEEP ? *q : __builtin_nontemporal_load(q);
    }
#pragma unroll
    for (int u = 0; u < NR; ++u)
#pragma unroll
        for (int q = 0; q < V; ++q) xv[u][q] = x[c[u][q]];
#pragma unroll
    for (int u = 0; u < NR; ++u) {
        const int s0 = V * (tid + u * kBlock), t0 = min(s0, cnt - V);
#pragma unroll
        for (int q = 0; q < V; ++q)
            slab[(t0 + q >= s0 && t0 + q < cnt) ? t0 + q : SPARE] = TA(v[u][q]) * TA(xv[u][q]);
    }
}

// Per-row operand of an epilogue that needs none.
struct NoOperand {};

// Read of an array that no kernel running at the same time writes, at an
// index that is uniform over the workgroup (row-block descriptors): through
// the constant address space the compiler issues a scalar load, which does not
// wait for the workgroup's outstanding vector stores the way a vector load
// followed by a full vmcnt wait would.
__device__ __forceinline__ int32_t load_uniform(const int32_t *p, int i) {
    return ((const __attribute__((address_space(4))) int32_t *)p)[i];
}

// Row products of one row block.  TV: value type, TX: vector type, TA:
// accumulation type.  epi.row(i, s, epi.load(i)) is called exactly once for
// every row i of the block, by one thread, with consecutive threads on
// consecutive rows; epi.load(i) (the epilogue's per-row operand, e.g. p_i for
// p.q) is issued at the start of the block so its latency hides behind the
// block's loads.  Must be called by all 256 threads.  more = false (the
// workgroup's last block) leaves out the closing barrier: the caller's
// store_block_partials, or the end of the kernel, follows.  KEEP selects the
// load policy of the matrix streams (keep_bytes); C16 reads the compact
// columns A.off16.  CH (taken from sm) is the largest partition span the LDS
// holds: A's blocks must come from a partition of span at most CH.
template <typename TV, typename TX, typename TA, bool KEEP = false, bool C16 = false,
          bool RUNS = false, int CH = kChunk, class Epi>
__device__ __forceinline__ void spmv_block(const CsrDev &A, const TV *__restrict__ vals,
                                           const TX *__restrict__ x, int blk,
                                           SpmvSmem<TA, CH> &sm, Epi &epi, bool more = true) {
    constexpr int kSl = SpmvSmem<TA, CH>::kSl;
    const int tid = threadIdx.x;
    // all four descriptors requested before any is used: one round trip
    const int r0 = load_uniform(A.block_row, blk);
    const int r1 = load_uniform(A.block_row, blk + 1);
    const int k0 = load_uniform(A.block_k, blk);
    const int kend = load_uniform(A.block_k, blk + 1);
    const int cb = RUNS ? load_uniform(A.run_chunk, blk) : 0;
    // (kend < k0 never holds; testing it keeps the compiler from sinking the
    // entry descriptors' load below this exit into a second round trip)
    if (r0 >= r1 || kend < k0) return;  // uniform over the workgroup
    // a block whose entries overflow the slab ends in a long row (the rows
    // before a block's last one hold fewer than CH entries in all); that row
    // is reduced below
    const bool long_last = (kend - k0) > kSl;
    const int cnt = min(kend - k0, kSl);
    const int nr = r1 - r0;

    // phase 1: coalesced streams of col/vals, then the gather of x, products
    // to LDS.  The loads are straight-line code (indices clamped into the
    // block, nothing guarded by a branch), so each gather waits only for its
    // own column index and all of them are in flight together.
    const int rv = A.row_ptr[r0 + min(tid, nr)];
    const auto pre = epi.load(r0 + min(tid, nr - 1));  // the epilogue's operand of row r0 + tid
    // 16-byte value loads, V = 16 / sizeof(TV) consecutive entries per lane:
    // FP32 blocks always; FP64 blocks of short rows (blocks of long scattered
    // rows gathered slower from pairs, so they keep one entry per lane)
    constexpr int V = 16 / (int)sizeof(TV);
    bool vec = false;
    if constexpr (!RUNS && (V == 2 || V == 4)) {
        vec = cnt >= V && (V == 4 || cnt < 8 * nr);
        if (vec) {
            static_assert(kSl <= 4 * V * kBlock, "four rounds of pairs or quads cover the slab");
            switch ((cnt + V * kBlock - 1) / (V * kBlock)) {
                case 1: block_products_vec<V, 1, KEEP, C16, kSl>(A, vals, x, k0, cnt, r0, sm.slab); break;
                case 2: block_products_vec<V, 2, KEEP, C16, kSl>(A, vals, x, k0, cnt, r0, sm.slab); break;
                case 3:
                    if constexpr (V == 2) {
                        block_products_vec<V, 3, KEEP, C16, kSl>(A, vals, x, k0, cnt, r0, sm.slab);
                    } else {  // quads (wide partition): 2 + 1, within 64 VGPRs
                        block_products_vec<V, 2, KEEP, C16, kSl>(A, vals, x, k0, cnt, r0, sm.slab);
                        __builtin_amdgcn_sched_barrier(0);
                        block_products_vec<V, 1, KEEP, C16, kSl>(A, vals, x, k0, cnt, r0, sm.slab, 2 * kBlock);
                    }
                    break;
                default:  // four rounds: two batches, so the registers of two rounds suffice
                    block_products_vec<V, 2, KEEP, C16, kSl>(A, vals, x, k0, cnt, r0, sm.slab);
                    __builtin_amdgcn_sched_barrier(0);
                    block_products_vec<V, 2, KEEP, C16, kSl>(A, vals, x, k0, cnt, r0, sm.slab, 2 * kBlock);
                    break;
            }
        }
    }
    if (!vec) switch ((cnt + kBlock - 1) / kBlock) {
        case 1: block_products<1, KEEP, C16, RUNS, kSl>(A, vals, x, k0, cnt, r0, cb, sm.slab); break;
        case 2: block_products<2, KEEP, C16, RUNS, kSl>(A, vals, x, k0, cnt, r0, cb, sm.slab); break;
        case 3: block_products<3, KEEP, C16, RUNS, kSl>(A, vals, x, k0, cnt, r0, cb, sm.slab); break;
        case 4: block_products<4, KEEP, C16, RUNS, kSl>(A, vals, x, k0, cnt, r0, cb, sm.slab); break;
        case 5: block_products<5, KEEP, C16, RUNS, kSl>(A, vals, x, k0, cnt, r0, cb, sm.slab); break;
        case 6: block_products<6, KEEP, C16, RUNS, kSl>(A, vals, x, k0, cnt, r0, cb, sm.slab); break;
        case 7:  // a long last row: two batches, so the registers of six rounds suffice
            block_products<4, KEEP, C16, RUNS, kSl>(A, vals, x, k0, cnt, r0, cb, sm.slab);
            __builtin_amdgcn_sched_barrier(0);  // keep the batches apart
            block_products<3, KEEP, C16, RUNS, kSl>(A, vals, x, k0, cnt, r0, cb, sm.slab, 4 * kBlock);
            break;
        case 0: break;  // only empty rows
        default:  // wide partition only: batches of four rounds
            for (int b = 0; b < cnt; b += 4 * kBlock) {
                block_products<4, KEEP, C16, RUNS, kSl>(A, vals, x, k0, cnt, r0, cb, sm.slab, b);
                __builtin_amdgcn_sched_barrier(0);
            }
            break;
    }
    if (tid <= nr) sm.rp[tid] = rv - k0;
    for (int t = tid + kBlock; t <= nr; t += kBlock) sm.rp[t] = A.row_ptr[r0 + t] - k0;
    __syncthreads();

    const int nrs = long_last ? nr - 1 : nr;        // rows reduced from LDS
    const int cnts = long_last ? sm.rp[nr - 1] : cnt;  // their entries
    auto col_at = [&](int k) { return C16 ? r0 + A.off16[k] : A.col[k]; };
    // the long last row: whole workgroup, strided over global memory; every
    // thread receives the sum
    auto long_row = [&]() {
        const int klast = k0 + sm.rp[nr - 1];
        TA s0 = TA(0), s1 = TA(0), s2 = TA(0), s3 = TA(0);
        int k = klast + tid;
        for (; k + 3 * kBlock < kend; k += 4 * kBlock) {
            s0 += TA(vals[k]) * TA(x[col_at(k)]);
            s1 += TA(vals[k + kBlock]) * TA(x[col_at(k + kBlock)]);
            s2 += TA(vals[k + 2 * kBlock]) * TA(x[col_at(k + 2 * kBlock)]);
            s3 += TA(vals[k + 3 * kBlock]) * TA(x[col_at(k + 3 * kBlock)]);
        }
        for (; k < kend; k += kBlock) s0 += TA(vals[k]) * TA(x[col_at(k)]);
        return block_sum((s0 + s1) + (s2 + s3), sm.red);
    };
    if (nrs == 0 || cnts < 8 * nrs) {
        // rows of fewer than 8 entries on average: each epilogue thread adds
        // its row's products straight from the slab (8 independent LDS reads
        // at clamped indices, then a tail for longer rows), with no separate
        // row pass and no second barrier
        const TA slast = long_last ? long_row() : TA(0);
        for (int t = tid; t < nr; t += kBlock) {
            TA s = TA(0);
            if (long_last && t == nr - 1) {
                s = slast;
            } else {
                const int a = sm.rp[t], b = sm.rp[t + 1];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const TA v = sm.slab[max(min(a + j, b - 1), 0)];
                    s += a + j < b ? v : TA(0);
                }
                for (int e = a + 8; e < b; ++e) s += sm.slab[e];
            }
            epi.row(r0 + t, s, t == tid ? pre : epi.load(r0 + t));
        }
        if (more) __syncthreads();  // the LDS slab is reused by the next row block
        return;
    }

    // phase 2: L lanes per row, L = pow2 floor of the mean row length (<= 64);
    // each row's sum is parked in LDS on its first product slot
    {
        const int avg = cnts / nrs;
        const int L = avg >= 64 ? 64 : (avg <= 1 ? 1 : (1 << (31 - __clz(avg))));
        const int lane = tid & (L - 1);
        const int grp = tid / L;
        const int ngrp = kBlock / L;
        for (int r = grp; r < nrs; r += ngrp) {
            const int a = sm.rp[r], e = sm.rp[r + 1];
            TA s = TA(0);
            for (int t = a + lane; t < e; t += L) s += sm.slab[t];
            s = group_sum(s, L);
            if (lane == 0 && e > a) sm.slab[a] = s;
        }
    }
    if (long_last) {
        const TA s = long_row();
        if (tid == 0) sm.last = s;
    }
    __syncthreads();
    // epilogue: consecutive threads take consecutive rows (coalesced y and
    // per-row vector accesses in epi.row)
    for (int t = tid; t < nr; t += kBlock) {
        TA s;
        if (long_last && t == nr - 1) s = sm.last;
        else s = sm.rp[t + 1] > sm.rp[t] ? sm.slab[sm.rp[t]] : TA(0);
        epi.row(r0 + t, s, t == tid ? pre : epi.load(r0 + t));
    }
    if (more) __syncthreads();  // the LDS slab is reused by the next row block
}

// ------------------------------------------------------- short rows --
//
// Matrices whose rows all have at most kShortLen entries (the triangular
// factors of a 7-point stencil have at most 4) skip the LDS staging: a group
// of kShortLen lanes owns one row and reduces it with two butterfly steps.  A
// workgroup handles kShortRounds rounds of 64 consecutive rows at once with
// straight-line loads (indices clamped into the row, the product masked), so
// all column, value and gather loads of those rows are in flight together.
constexpr int kShortLen = 4;
constexpr int kShortRounds = 4;
constexpr int kShortRows = (kBlock / kShortLen) * kShortRounds;  // rows per workgroup step

__host__ __device__ inline int64_t short_steps(int64_t n_rows) { return (n_rows + kShortRows - 1) / kShortRows; }

// Workgroups of a short-row kernel (each walks a contiguous range of steps)
inline unsigned short_grid(int64_t n_rows) { return spmv_grid(short_steps(n_rows)); }

// Rows [b * kShortRows, (b + 1) * kShortRows) of an n-row matrix with nnz >= 1
// and every row at most kShortLen long.  epi.row(i, s, epi.load(i)) is called
// once per row, by the group's first lane (the loads are issued up front).
// KEEP selects the load policy of col/vals (keep_bytes).
template <typename TV, typename TX, typename TA, bool KEEP = false, class Epi>
__device__ __forceinline__ void spmv_short(const int32_t *__restrict__ rp,
                                           const int32_t *__restrict__ col,
                                           const TV *__restrict__ vals, const TX *__restrict__ x,
                                           int n, int b, Epi &epi) {
    constexpr int G = kBlock / kShortLen;
    const int lane = threadIdx.x & (kShortLen - 1);
    const int g = threadIdx.x / kShortLen;
    const int base = b * kShortRows;
    int a[kShortRounds], e[kShortRounds], c[kShortRounds];
    TV v[kShortRounds];
    TA s[kShortRounds];
    decltype(epi.load(0)) pre[kShortRounds];
#pragma unroll
    for (int u = 0; u < kShortRounds; ++u) {
        const int r = min(base + u * G + g, n - 1);
        a[u] = rp[r];
        e[u] = rp[r + 1];
        pre[u] = epi.load(r);
    }
#pragma unroll
    for (int u = 0; u < kShortRounds; ++u) {
        const int k = a[u] + lane;
        const int kc = k < e[u] ? k : max(e[u] - 1, 0);
        if constexpr (KEEP) {
            c[u] = col[kc];
            v[u] = vals[kc];
        } else {
            c[u] = __builtin_nontemporal_load(col + kc);
            v[u] = __builtin_nontemporal_load(vals + kc);
        }
    }
#pragma unroll
    for (int u = 0; u < kShortRounds; ++u) {
        const TX xv = x[c[u]];
        s[u] = a[u] + lane < e[u] ? TA(v[u]) * TA(xv) : TA(0);
    }
#pragma unroll
    for (int u = 0; u < kShortRounds; ++u) {
        s[u] += dpp_mov<kDppXor1>(s[u]);
        s[u] += dpp_mov<kDppXor2>(s[u]);
    }
#pragma unroll
    for (int u = 0; u < kShortRounds; ++u) {
        const int r = base + u * G + g;
        if (lane == 0 && r < n) epi.row(r, s[u], pre[u]);
    }
}

// Contiguous range of row blocks owned by this workgroup; the workgroup's
// logical index (XCD-remapped) is also its partial-sum slot.
__device__ __forceinline__ int block_range(int nb, int &bs, int &be) {
    const int P = gridDim.x;
    const int w = xcd_remap(blockIdx.x, P);
    bs = (int)((int64_t)nb * w / P);
    be = (int)((int64_t)nb * (w + 1) / P);
    return w;
}

// ------------------------------------------------------ row-length bins --

constexpr int kNumBins = SPCG_NUM_BINS;
constexpr int kLongBin = kNumBins - 1;  // rows of more than 4 * 2^(kLongBin - 1) entries

struct BinStarts {
    int s[kNumBins];
};

struct BinView {
    const int32_t *__restrict__ row;  // bin lists (all bins back to back)
    const int32_t *__restrict__ k;
    const int32_t *__restrict__ len;
    const int32_t *__restrict__ col;
    int nnz;
    int off;  // first list entry of the bin at hand
};

struct BinPlan {
    BinView v;
    int start[kNumBins], count[kNumBins];
    int wg[kNumBins];  // first workgroup of each bin
};

int binning_mode();
bool binning_at_create(const spcg_csr *A);
int build_bins(spcg_csr *h, hipStream_t s);
bool use_bins(const spcg_csr *A);
template <typename T>
int launch_spmv_bins(const spcg_csr *A, const T *x, T *y, hipStream_t s);

int runs_mode();
int build_runs(spcg_csr *h, hipStream_t s);
bool use_runs(const spcg_csr *A);

int panels_mode();
int build_panels(spcg_csr *h, hipStream_t s);
bool use_panels(const spcg_csr *A);
int panels_pay(const spcg_csr *h, hipStream_t s, bool *pay);
template <typename T>
int launch_spmv_panels(const spcg_csr *A, const T *x, T *y, hipStream_t s);

// Short-row kernels apply when every row has at most kShortLen entries.
inline bool uses_short_rows(const spcg_csr *A) {
    return A->n_rows > 0 && A->nnz > 0 && A->max_len <= kShortLen;
}

inline CsrDev dev_view(const spcg_csr *A) {
    return CsrDev{A->row_ptr, A->col, A->block_row, A->block_k, (int)A->n_blocks, nullptr,
                  A->run_mask, A->run_base, A->run_col, A->run_chunk};
}

// The same matrix over the wide partition (no runs: those follow kChunk's
// blocks); only kernels instantiated with SpmvSmem<float, kChunkWide> may read it
inline CsrDev dev_view_wide(const spcg_csr *A) {
    return CsrDev{A->row_ptr, A->col, A->wblock_row, A->wblock_k, (int)A->n_wblocks, nullptr,
                  nullptr, nullptr, nullptr, nullptr};
}

}  // namespace spcg

// csr.hip -- matrix handle (validation + row analysis), y = A x, and the
// deterministic inner product.  CSR in three arrays and the row-wise product
// follow Sec. 3.2 of arXiv 1211.1581.
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <new>

#include "internal.h"

namespace spcg {

static thread_local char g_err[512] = "";

static std::atomic<int64_t> g_keep_bytes{kKeepBytes};

int64_t keep_bytes() { return g_keep_bytes.load(std::memory_order_relaxed); }

void set_error(hipError_t e, const char *what) {
    snprintf(g_err, sizeof g_err, "%s: %s", what, hipGetErrorString(e));
}

void set_error_text(const char *text) { snprintf(g_err, sizeof g_err, "%s", text); }

int hip_status(hipError_t e, const char *what) {
    set_error(e, what);
    return SPCG_HIP_ERROR;
}

// ------------------------------------------------------------- analysis --

// flags[0]: error bits (1 row_ptr[0] != 0, 2 decreasing row_ptr, 4 row_ptr[n] != nnz,
// 8 column out of range); flags[1]: longest row; flags[2]: blocks whose
// last row does not fit the LDS slab.
__global__ void k_fill_i32(int32_t *p, int n, int32_t v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

__global__ void __launch_bounds__(kBlock)
k_validate(int n, int ncols, int64_t nnz, const int32_t *__restrict__ rp,
           const int32_t *__restrict__ col, int32_t *flags) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int err = 0, mx = 0;
    for (int64_t i = t0; i <= n; i += stride) {
        const int a = rp[i];
        if (i == 0 && a != 0) err |= 1;
        if (i < n) {
            const int len = rp[i + 1] - a;
            if (len < 0) err |= 2;
            mx = max(mx, len);
        } else if ((int64_t)a != nnz) {
            err |= 4;
        }
    }
    for (int64_t k = t0; k < nnz; k += stride) {
        const int c = col[k];
        if (c < 0 || c >= ncols) err |= 8;
    }
    // one atomic per workgroup (atomics on one address serialise: one per
    // wavefront of a full-size grid cost ~0.3 ms)
    __shared__ int sh[2][kBlock / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        err |= __shfl_xor(err, o, 64);
        mx = max(mx, __shfl_xor(mx, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = err;
        sh[1][threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) {
            err |= sh[0][w];
            mx = max(mx, sh[1][w]);
        }
        if (err) atomicOr(&flags[0], err);
        if (mx) atomicMax(&flags[1], mx);
    }
}

// block_row[b] = first row i with row_ptr[i] + i >= b * chunk (b < nb),
// block_row[nb] = n; block_k[b] = row_ptr[block_row[b]]
__global__ void __launch_bounds__(kBlock)
k_partition(int n, const int32_t *__restrict__ rp, int64_t nb, int chunk, int32_t *block_row,
            int32_t *block_k) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nb) return;
    int lo = n;
    if (b < nb) {
        const int64_t target = b * chunk;
        lo = 0;
        int hi = n;  // answer in [lo, hi]
        while (lo < hi) {
            const int mid = lo + ((hi - lo) >> 1);
            if ((int64_t)rp[mid] + mid >= target) hi = mid;
            else lo = mid + 1;
        }
    }
    block_row[b] = lo;
    block_k[b] = rp[lo];
}

__global__ void __launch_bounds__(kBlock)
k_count_long(const int32_t *__restrict__ rp, const int32_t *__restrict__ block_row, int64_t nb,
             int32_t *flags) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int r0 = block_row[b], r1 = block_row[b + 1];
    if (r0 < r1 && rp[r1] - rp[r0] > kSlab) atomicAdd(&flags[2], 1);
}

// ------------------------------------------------------------------ SpMV --

template <typename T>
struct EpiStore {
    T *__restrict__ y;
    __device__ __forceinline__ NoOperand load(int) const { return {}; }
    __device__ __forceinline__ void row(int i, T s, NoOperand) { y[i] = s; }
};

// RUNS: columns of the LDS-staged entries from the run-compressed layout.
// CH: span of A's partition (kChunk, or kChunkWide for FP32 handles).
template <typename T, bool KEEP, bool RUNS = false, int CH = kChunk>
SPCG_ROWBLOCK_KERNEL
k_spmv(CsrDev A, const T *__restrict__ vals, const T *__restrict__ x, T *__restrict__ y) {
    __shared__ SpmvSmem<T, CH> sm;
    int bs, be;
    block_range(A.n_blocks, bs, be);
    EpiStore<T> epi{y};
    for (int b = bs; b < be; ++b)
        spmv_block<T, T, T, KEEP, false, RUNS>(A, vals, x, b, sm, epi, b + 1 < be);
}

// y = A x for matrices whose rows have at most kShortLen entries
template <typename T>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8)))
k_spmv_short(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
             const T *__restrict__ vals, const T *__restrict__ x, T *__restrict__ y) {
    int bs, be;
    block_range((int)short_steps(n), bs, be);
    EpiStore<T> epi{y};
    for (int b = bs; b < be; ++b) spmv_short<T, T, T>(rp, col, vals, x, n, b, epi);
}

template <typename T>
int launch_spmv(const spcg_csr *A, const T *x, T *y, hipStream_t s) {
    if (A->n_rows == 0) return SPCG_OK;
    if (uses_short_rows(A)) {
        hipLaunchKernelGGL(k_spmv_short<T>, dim3(short_grid(A->n_rows)), dim3(kBlock),
                           0, s, A->n_rows, A->row_ptr, A->col, (const T *)A->vals, x, y);
        SPCG_LAUNCH_CHECK("k_spmv_short");
        return SPCG_OK;
    }
    if (use_panels(A) && ((uintptr_t)x & 15) == 0) return launch_spmv_panels<T>(A, x, y, s);
    if (use_bins(A)) return launch_spmv_bins<T>(A, x, y, s);
    const bool keep = matrix_bytes(A->n_rows, A->nnz, sizeof(T)) <= keep_bytes();
    const bool runs = use_runs(A);
    if constexpr (sizeof(T) == 4) {
        if (!runs && A->wblock_row) {
            auto kern = keep ? k_spmv<T, true, false, kChunkWide> : k_spmv<T, false, false, kChunkWide>;
            hipLaunchKernelGGL(kern, dim3(spmv_grid(A->n_wblocks)), dim3(kBlock), 0, s,
                               dev_view_wide(A), (const T *)A->vals, x, y);
            SPCG_LAUNCH_CHECK("k_spmv");
            return SPCG_OK;
        }
    }
    auto kern = runs ? (keep ? k_spmv<T, true, true> : k_spmv<T, false, true>)
                     : (keep ? k_spmv<T, true> : k_spmv<T, false>);
    hipLaunchKernelGGL(kern, dim3(spmv_grid(A->n_blocks)), dim3(kBlock), 0, s, dev_view(A),
                       (const T *)A->vals, x, y);
    SPCG_LAUNCH_CHECK("k_spmv");
    return SPCG_OK;
}

// ------------------------------------------------------------------- dot --

constexpr int kDotPerBlock = kBlock * 16;

__global__ void __launch_bounds__(kBlock)
k_dot_partials(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
               double *__restrict__ part) {
    __shared__ double red[4];
    const int64_t base = (int64_t)blockIdx.x * kDotPerBlock;
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kDotPerBlock / kBlock; ++u) {
        const int64_t i = base + threadIdx.x + (int64_t)u * kBlock;
        if (i < n) s += a[i] * b[i];
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock)
k_dot_final(int64_t nparts, const double *__restrict__ part, double *out) {
    __shared__ double red[4];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < nparts; i += kBlock) s += part[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) *out = s;
}

}  // namespace spcg

using namespace spcg;

extern "C" {

const char *spcg_status_str(int status) {
    switch (status) {
        case SPCG_OK: return "OK";
        case SPCG_NOT_CONVERGED: return "NOT_CONVERGED";
        case SPCG_FELL_BACK: return "FELL_BACK";
        case SPCG_INVALID_ARG: return "INVALID_ARG";
        case SPCG_INVALID_CSR: return "INVALID_CSR";
        case SPCG_HIP_ERROR: return "HIP_ERROR";
        case SPCG_NOT_SPD: return "NOT_SPD";
        case SPCG_NON_FINITE: return "NON_FINITE";
        case SPCG_TOO_LARGE: return "TOO_LARGE";
        default: return "UNKNOWN";
    }
}

const char *spcg_last_error(void) { return g_err; }

int64_t spcg_keep_bytes(int64_t bytes) {
    return bytes >= 0 ? g_keep_bytes.exchange(bytes) : g_keep_bytes.load();
}

static void release(spcg_csr *h) {
    if (!h) return;
    if (h->block_row) (void)hipFree(h->block_row);
    if (h->block_k) (void)hipFree(h->block_k);
    if (h->wblock_row) (void)hipFree(h->wblock_row);
    if (h->wblock_k) (void)hipFree(h->wblock_k);
    if (h->flags) (void)hipFree(h->flags);
    if (h->h_pinned) (void)hipHostFree(h->h_pinned);
    for (int32_t *p : {h->bin_row, h->bin_k, h->bin_len, h->run_base, h->run_col, h->run_chunk,
                       h->pan_range, h->pan_phase, h->pan_vstart, h->pan_base})
        if (p) (void)hipFree(p);
    for (void *p : {(void *)h->run_mask, (void *)h->pan_key, h->pan_val, h->pan_part})
        if (p) (void)hipFree(p);
    if (h->pan_done) (void)hipEventDestroy(h->pan_done);
    for (int i = 0; i < h->n_events; ++i) (void)hipEventDestroy(h->events[i]);
    delete[] h->events;
    delete h;
}

int spcg_csr_create(spcg_csr_t *out, int32_t n_rows, int32_t n_cols, int64_t nnz,
                    const int32_t *d_row_ptr, const int32_t *d_col, const void *d_vals,
                    int32_t dtype, hipStream_t stream) {
    if (!out) return SPCG_INVALID_ARG;
    *out = nullptr;
    if (n_rows < 0 || n_cols < 0 || nnz < 0 || n_rows > SPCG_MAX_INDEX || n_cols > SPCG_MAX_INDEX ||
        nnz > SPCG_MAX_INDEX)
        return SPCG_INVALID_ARG;
    if (dtype != SPCG_F64 && dtype != SPCG_F32) return SPCG_INVALID_ARG;
    if (!d_row_ptr || (nnz > 0 && (!d_col || !d_vals))) return SPCG_INVALID_ARG;
    spcg_csr *h = new (std::nothrow) spcg_csr;
    if (!h) return SPCG_INVALID_ARG;
    h->n_rows = n_rows;
    h->n_cols = n_cols;
    h->nnz = nnz;
    h->row_ptr = d_row_ptr;
    h->col = d_col;
    h->vals = d_vals;
    h->dtype = dtype;
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) { release(h); return hip_status(e, "hipGetDevice"); }
#define CREATE_TRY(expr)                                            \
    do {                                                            \
        hipError_t e_ = (expr);                                     \
        if (e_ != hipSuccess) { release(h); return hip_status(e_, #expr); } \
    } while (0)
    CREATE_TRY(hipMalloc(&h->flags, 256));
    CREATE_TRY(hipHostMalloc(&h->h_pinned, 256, hipHostMallocDefault));
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, stream, h->flags, 64, 0);
    CREATE_TRY(hipGetLastError());
    {
        const int64_t work = (int64_t)n_rows + 1 > nnz ? (int64_t)n_rows + 1 : nnz;
        const unsigned grid = (unsigned)std::min<int64_t>((work + kBlock - 1) / kBlock, 1024);
        hipLaunchKernelGGL(k_validate, dim3(grid > 0 ? grid : 1), dim3(kBlock), 0, stream, n_rows,
                           n_cols, nnz, d_row_ptr, d_col, h->flags);
        CREATE_TRY(hipGetLastError());
    }
    int32_t *hf = (int32_t *)h->h_pinned;
    CREATE_TRY(hipMemcpyAsync(hf, h->flags, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    CREATE_TRY(hipStreamSynchronize(stream));
    if (hf[0] != 0) {
        release(h);
        return SPCG_INVALID_CSR;
    }
    h->max_len = hf[1];
    h->n_blocks = n_row_blocks(n_rows, nnz);
    if (h->n_blocks > INT32_MAX / 2) { release(h); return SPCG_INVALID_ARG; }
    CREATE_TRY(hipMalloc(&h->block_row, sizeof(int32_t) * (h->n_blocks + 1)));
    CREATE_TRY(hipMalloc(&h->block_k, sizeof(int32_t) * (h->n_blocks + 1)));
    {
        const unsigned grid = (unsigned)((h->n_blocks + 1 + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_partition, dim3(grid), dim3(kBlock), 0, stream, n_rows, d_row_ptr,
                           h->n_blocks, kChunk, h->block_row, h->block_k);
        CREATE_TRY(hipGetLastError());
        if (h->n_blocks > 0) {
            const unsigned g2 = (unsigned)((h->n_blocks + kBlock - 1) / kBlock);
            hipLaunchKernelGGL(k_count_long, dim3(g2), dim3(kBlock), 0, stream, d_row_ptr,
                               h->block_row, h->n_blocks, h->flags);
            CREATE_TRY(hipGetLastError());
        }
    }
    if (n_rows > 0) {
        h->n_wblocks = n_row_blocks(n_rows, nnz, kChunkWide);
        CREATE_TRY(hipMalloc(&h->wblock_row, sizeof(int32_t) * (h->n_wblocks + 1)));
        CREATE_TRY(hipMalloc(&h->wblock_k, sizeof(int32_t) * (h->n_wblocks + 1)));
        const unsigned grid = (unsigned)((h->n_wblocks + 1 + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_partition, dim3(grid), dim3(kBlock), 0, stream, n_rows, d_row_ptr,
                           h->n_wblocks, kChunkWide, h->wblock_row, h->wblock_k);
        CREATE_TRY(hipGetLastError());
    }
    CREATE_TRY(hipMemcpyAsync(hf, h->flags, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    CREATE_TRY(hipStreamSynchronize(stream));
    h->n_long = hf[2];
    if (binning_at_create(h)) {
        const int rc = build_bins(h, stream);
        if (rc != SPCG_OK) {
            release(h);
            return rc;
        }
    }
    if (runs_mode() == SPCG_RUNS_ON) {
        const int rc = build_runs(h, stream);
        if (rc != SPCG_OK) {
            release(h);
            return rc;
        }
    }
    bool panels = panels_mode() == SPCG_PANELS_ON;
    if (panels_mode() == SPCG_PANELS_AUTO && binning_mode() == SPCG_BINNING_OFF && runs_mode() == SPCG_RUNS_OFF) {
        const int rc = panels_pay(h, stream, &panels);
        if (rc != SPCG_OK) {
            release(h);
            return rc;
        }
    }
    if (panels) {
        const int rc = build_panels(h, stream);
        if (rc != SPCG_OK) {
            release(h);
            return rc;
        }
    }
#undef CREATE_TRY
    *out = h;
    return SPCG_OK;
}

int spcg_csr_destroy(spcg_csr_t A) {
    if (!A) return SPCG_INVALID_ARG;
    hipError_t e = hipDeviceSynchronize();
    release(A);
    return e == hipSuccess ? SPCG_OK : hip_status(e, "hipDeviceSynchronize");
}

int spcg_csr_info(spcg_csr_t A, int64_t *n_blocks, int64_t *n_long_rows, int64_t *max_row_len) {
    if (!A) return SPCG_INVALID_ARG;
    if (n_blocks) *n_blocks = A->n_blocks;
    if (n_long_rows) *n_long_rows = A->n_long;
    if (max_row_len) *max_row_len = A->max_len;
    return SPCG_OK;
}

int spcg_csr_wide_blocks(spcg_csr_t A, int64_t *n_wide_blocks) {
    if (!A || !n_wide_blocks) return SPCG_INVALID_ARG;
    *n_wide_blocks = A->wblock_row ? A->n_wblocks : 0;
    return SPCG_OK;
}

int spmv_csr(spcg_csr_t A, const void *d_x, void *d_y, hipStream_t stream) {
    if (!A) return SPCG_INVALID_ARG;
    if (A->n_rows > 0 && !d_y) return SPCG_INVALID_ARG;
    if (A->nnz > 0 && !d_x) return SPCG_INVALID_ARG;
    if (A->dtype == SPCG_F64)
        return launch_spmv<double>(A, (const double *)d_x, (double *)d_y, stream);
    return launch_spmv<float>(A, (const float *)d_x, (float *)d_y, stream);
}

size_t spcg_dot_workspace_bytes(int64_t n) {
    const int64_t parts = n > 0 ? (n + kDotPerBlock - 1) / kDotPerBlock : 1;
    return align256(sizeof(double) * parts);
}

int spcg_dot(int64_t n, const double *d_a, const double *d_b, double *d_out, void *d_work,
             hipStream_t stream) {
    if (n < 0 || !d_out || !d_work || (n > 0 && (!d_a || !d_b))) return SPCG_INVALID_ARG;
    const int64_t parts = n > 0 ? (n + kDotPerBlock - 1) / kDotPerBlock : 0;
    double *part = (double *)d_work;
    if (parts > 0) {
        hipLaunchKernelGGL(k_dot_partials, dim3((unsigned)parts), dim3(kBlock), 0, stream, n, d_a,
                           d_b, part);
        SPCG_LAUNCH_CHECK("k_dot_partials");
    }
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kBlock), 0, stream, parts, part, d_out);
    SPCG_LAUNCH_CHECK("k_dot_final");
    return SPCG_OK;
}

}  // extern "C"

// runs.hip -- run-compressed column indices for y = A x, the index side of
// the paper's contiguous-section SpMV (Sec. 3.2: the second mapped kernel
// finds sections of consecutive column indices and reads x there as one
// contiguous piece).
//
// At analysis, the entries each row block stages in LDS are cut into chunks of
// 64 (the entries one wavefront loads at once); in each chunk an entry starts
// a run unless its column is its predecessor's plus one.  Per chunk the
// library keeps a 64-bit mask of run starts and the position of the chunk's
// first start in a list of start columns; a lane then finds its column as the
// nearest start at or before it plus the distance, so inside a run no column
// index is read and the lanes gather consecutive x.  A 7-point stencil row
// has 5 runs in 7 entries; a banded row of bandwidth 2h + 1 is one run.  The
// products are the same, in the same order, as with the plain column array,
// so the results are bitwise equal.  It reads fewer bytes but adds a
// dependent load (mask and start, then the start column) before the gather,
// and measured slower than plain columns (128^3 stencil 54.5 against 43.5 us,
// a 2^20-row band of width 63 185 against 161 us), so it is off by default.
#include <algorithm>
#include <atomic>

#include "internal.h"
#include "scan.h"

namespace spcg {

static std::atomic<int> g_runs{SPCG_RUNS_OFF};

int runs_mode() { return g_runs.load(std::memory_order_relaxed); }

// Staged chunks of every row block: ceil(min(entries, slab) / 64), 0 for a
// block without rows
__global__ void __launch_bounds__(kBlock)
k_run_nchunks(int nb, const int32_t *__restrict__ block_row, const int32_t *__restrict__ block_k,
              int32_t *__restrict__ cnt) {
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= nb) return;
    int c = 0;
    if (block_row[b] < block_row[b + 1]) {
        const int m = min(block_k[b + 1] - block_k[b], kSlab);
        c = (m + 63) / 64;
    }
    cnt[b] = c;
}

// FILL = false: run-start masks and start counts of every chunk;
// FILL = true: the start columns, at the chunk's base plus their rank.
template <bool FILL>
__global__ void __launch_bounds__(kBlock)
k_run_chunks(int nb, const int32_t *__restrict__ block_row, const int32_t *__restrict__ block_k,
             const int32_t *__restrict__ col, const int32_t *__restrict__ chunk0,
             unsigned long long *__restrict__ mask, int32_t *__restrict__ heads,
             const int32_t *__restrict__ base, int32_t *__restrict__ run_col) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        if (block_row[b] >= block_row[b + 1]) continue;  // uniform
        const int k0 = block_k[b];
        const int m = min(block_k[b + 1] - k0, kSlab);
        const int nch = (m + 63) / 64, cb = chunk0[b];
        for (int j = w; j < nch; j += kBlock / 64) {
            const int t = 64 * j + lane;
            const bool valid = t < m;
            const int c = valid ? col[k0 + t] : 0;
            const int cp = valid && lane > 0 ? col[k0 + t - 1] : 0;
            const bool head = valid && (lane == 0 || c != cp + 1);
            const unsigned long long hm = __ballot(head);
            if constexpr (FILL) {
                if (head) run_col[base[cb + j] + __popcll(hm & below)] = c;
            } else if (lane == 0) {
                mask[cb + j] = hm;
                heads[cb + j] = __popcll(hm);
            }
        }
    }
}

int build_runs(spcg_csr *h, hipStream_t s) {
    const int nb = (int)h->n_blocks;
    if (nb == 0 || h->nnz == 0) return SPCG_OK;
    int32_t *cnt = nullptr, *sums = nullptr, *heads = nullptr;
    auto fail = [&](hipError_t e, const char *what) {
        for (int32_t *p : {cnt, sums, heads})
            if (p) (void)hipFree(p);
        return hip_status(e, what);
    };
    hipError_t e;
    int32_t *hp = (int32_t *)h->h_pinned;
    // chunks per block -> each block's first chunk (run_chunk[nb] = all chunks)
    if ((e = hipMalloc(&cnt, sizeof(int32_t) * nb)) != hipSuccess ||
        (e = hipMalloc(&h->run_chunk, sizeof(int32_t) * ((size_t)nb + 1))) != hipSuccess ||
        (e = hipMalloc(&sums, sizeof(int32_t) * (size_t)scan_sums_slots(nb))) != hipSuccess)
        return fail(e, "hipMalloc(run chunks)");
    hipLaunchKernelGGL(k_run_nchunks, dim3((nb + kBlock - 1) / kBlock), dim3(kBlock), 0, s, nb,
                       h->block_row, h->block_k, cnt);
    exclusive_scan(nb, cnt, sums, h->run_chunk, s);
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = hipMemcpyAsync(hp, h->run_chunk + nb, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return fail(e, "run chunk scan");
    const int nch = hp[0];
    (void)hipFree(sums);
    sums = nullptr;
    if (nch == 0) {
        (void)hipFree(cnt);
        return SPCG_OK;
    }
    // masks and start counts -> each chunk's first start (run_base[nch] = all starts)
    if ((e = hipMalloc(&h->run_mask, sizeof(unsigned long long) * nch)) != hipSuccess ||
        (e = hipMalloc(&heads, sizeof(int32_t) * nch)) != hipSuccess ||
        (e = hipMalloc(&h->run_base, sizeof(int32_t) * ((size_t)nch + 1))) != hipSuccess ||
        (e = hipMalloc(&sums, sizeof(int32_t) * (size_t)scan_sums_slots(nch))) != hipSuccess)
        return fail(e, "hipMalloc(run masks)");
    const unsigned grid = (unsigned)std::min(nb, 8192);
    hipLaunchKernelGGL(k_run_chunks<false>, dim3(grid), dim3(kBlock), 0, s, nb, h->block_row,
                       h->block_k, h->col, (const int32_t *)h->run_chunk, h->run_mask, heads,
                       (const int32_t *)nullptr, (int32_t *)nullptr);
    exclusive_scan(nch, heads, sums, h->run_base, s);
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = hipMemcpyAsync(hp, h->run_base + nch, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return fail(e, "run start scan");
    const int nh = hp[0];
    if ((e = hipMalloc(&h->run_col, sizeof(int32_t) * (size_t)std::max(nh, 1))) != hipSuccess)
        return fail(e, "hipMalloc(run columns)");
    hipLaunchKernelGGL(k_run_chunks<true>, dim3(grid), dim3(kBlock), 0, s, nb, h->block_row,
                       h->block_k, h->col, (const int32_t *)h->run_chunk,
                       (unsigned long long *)nullptr, (int32_t *)nullptr,
                       (const int32_t *)h->run_base, h->run_col);
    if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess)
        return fail(e, "k_run_chunks");
    for (int32_t *p : {cnt, sums, heads}) (void)hipFree(p);
    h->n_chunks = nch;
    h->n_heads = nh;
    h->has_runs = true;
    return SPCG_OK;
}

bool use_runs(const spcg_csr *A) { return A->has_runs && runs_mode() == SPCG_RUNS_ON; }

}  // namespace spcg

extern "C" {

int spcg_run_columns(int mode) {
    if (mode < 0) return spcg::g_runs.load();
    if (mode > SPCG_RUNS_ON) return SPCG_INVALID_ARG;
    return spcg::g_runs.exchange(mode);
}

int spcg_csr_run_info(spcg_csr_t A, int64_t *n_chunks, int64_t *n_starts) {
    if (!A || !A->has_runs) return SPCG_INVALID_ARG;
    if (n_chunks) *n_chunks = A->n_chunks;
    if (n_starts) *n_starts = A->n_heads;
    return SPCG_OK;
}

}  // extern "C"

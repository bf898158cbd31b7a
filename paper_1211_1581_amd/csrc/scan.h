// scan.h -- exclusive prefix sums of int32 counts on the device (the
// per-matrix analyses: factor patterns, run-compressed columns).  Static
// kernels: every source file that includes this gets its own copies.
#pragma once

#include "internal.h"

namespace spcg {

// Exclusive scan of cnt[0..n) into out[0..n] in three steps: chunk sums
// (k_scan_sums), a one-workgroup scan of the chunk sums (k_scan_top), and a
// rescan of every chunk from its offset (k_scan_apply).
constexpr int kScanChunk = 4096;

static __global__ void __launch_bounds__(256) k_scan_sums(int n, const int32_t *__restrict__ cnt,
                                                   int32_t *sums) {
    __shared__ int red[4];
    const int base = blockIdx.x * kScanChunk;
    int s = 0;
    for (int i = base + threadIdx.x; i < min(n, base + kScanChunk); i += 256) s += cnt[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

static __global__ void __launch_bounds__(1024) k_scan_top(int nb, int32_t *sums) {
    __shared__ int32_t sh[1024];
    const int T = 1024, t = threadIdx.x;
    const int per = (nb + T - 1) / T;
    const int a = min(nb, t * per), b = min(nb, a + per);
    int32_t s = 0;
    for (int i = a; i < b; ++i) s += sums[i];
    sh[t] = s;
    __syncthreads();
    for (int o = 1; o < T; o <<= 1) {
        const int32_t v = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    int32_t run = sh[t] - s;
    for (int i = a; i < b; ++i) {
        const int32_t c = sums[i];
        sums[i] = run;
        run += c;
    }
    if (t == T - 1) sums[nb] = sh[T - 1];
}

static __global__ void __launch_bounds__(256) k_scan_apply(int n, const int32_t *__restrict__ cnt,
                                                    const int32_t *__restrict__ offs, int32_t *out) {
    __shared__ int32_t sh[256];
    const int base = blockIdx.x * kScanChunk;
    const int per = kScanChunk / 256;
    const int a = min(n, base + threadIdx.x * per), b = min(n, a + per);
    int32_t s = 0;
    for (int i = a; i < b; ++i) s += cnt[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int32_t v = (int)threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    int32_t run = offs[blockIdx.x] + sh[threadIdx.x] - s;
    for (int i = a; i < b; ++i) {
        out[i] = run;
        run += cnt[i];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 255) out[n] = offs[gridDim.x];
}

// out[0..n] = exclusive scan of cnt[0..n), out[n] = the total; sums: scratch
// of scan_sums_slots(n) int32 (n >= 1).
inline int scan_sums_slots(int n) { return (n + kScanChunk - 1) / kScanChunk + 1; }

inline void exclusive_scan(int n, const int32_t *cnt, int32_t *sums, int32_t *out, hipStream_t s) {
    const int nb = (n + kScanChunk - 1) / kScanChunk;
    hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(256), 0, s, n, cnt, sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, nb, sums);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(256), 0, s, n, cnt, (const int32_t *)sums, out);
}

}  // namespace spcg

// mfma.h -- wave-level 32-row tiles on CDNA4 matrix cores (v_mfma_f32_32x32x16_bf16).
//
// Operand layouts of one 32x32x16 step (checked on gfx950):
//   A (32 x 16, rows = tile rows):  lane l holds A[l % 32][8 * (l / 32) + t], t = 0..7
//   B (16 x 32):                    lane l holds B[8 * (l / 32) + t][l % 32]
//   D (32 x 32, FP32):              lane l, element i holds D[acc_row(i, l)][l % 32]
// Both operands are read as 8 consecutive BF16 (16 bytes) from arrays whose
// reduction index K is contiguous: A row-major [32][K], and B given as its
// transpose Bt row-major [32][K].
#pragma once

#include <hip/hip_runtime.h>

namespace spcg {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

__device__ __forceinline__ int acc_row(int i, int lane) {
    return (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
}

__device__ __forceinline__ f32x16 mfma32(bf16x8 a, bf16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Fragment (A or Bt) of K-chunk c from a row-major [32][ld] BF16 array.
__device__ __forceinline__ bf16x8 frag(const __bf16 *base, int ld, int c) {
    const int l = threadIdx.x & 63;
    return *reinterpret_cast<const bf16x8 *>(base + (l & 31) * ld + 16 * c + 8 * (l >> 5));
}

__device__ __forceinline__ bf16x8 to_bf16x8(const float *v) {
    bf16x8 r;
#pragma unroll
    for (int t = 0; t < 8; ++t) r[t] = (__bf16)v[t];
    return r;
}

__device__ __forceinline__ f32x16 splat16(float v) {
    f32x16 r;
#pragma unroll
    for (int i = 0; i < 16; ++i) r[i] = v;
    return r;
}

// Accumulator tile -> LDS as BF16, row-major [32][ld] (transposed: [col][row]).
__device__ __forceinline__ void acc_to_lds(const f32x16 &d, __bf16 *lds, int ld, bool transposed) {
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int r = acc_row(i, l), c = l & 31;
        lds[transposed ? c * ld + r : r * ld + c] = (__bf16)d[i];
    }
}

// LDS writes of this wave are visible to its later LDS reads.
__device__ __forceinline__ void wave_lds_sync() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0), other counters unchanged
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }

// d silu / dz = sigma(z) (1 + z (1 - sigma(z)))
__device__ __forceinline__ float silu_grad(float z) {
    const float sg = 1.0f / (1.0f + __expf(-z));
    return sg * (1.0f + z * (1.0f - sg));
}

}  // namespace spcg

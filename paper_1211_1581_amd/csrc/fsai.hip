// fsai.hip -- factorized sparse approximate inverse (Kolotilina & Yeremin) on a
// given lower pattern: the non-learned factor G of M^-1 = G G^T.
//
// G lower-triangular with G^T A G having a unit diagonal, each column chosen
// independently: for column i with row set J = {j >= i : G_ji in the pattern}
// (J[0] = i), minimise over that column the Frobenius distance to the inverse
// upper Cholesky factor of A, which gives the small SPD system
//   A[J, J] y = e_1,   G[J, i] = y / sqrt(y_1).
// One thread per column: the system (at most SPCG_FSAI_MAX_SET unknowns) is
// assembled from the rows of A in J, factorised by Cholesky in registers
// (padded with identity rows to a compile-time size) and solved; the column is
// written to G^T's row i and, through a search of each row of G, to G.
#include <math.h>

#include <algorithm>

#include "internal.h"

namespace spcg {

enum FsaiFlag : int { F_BAD_PATTERN = 1, F_NOT_SPD = 2, F_NON_FINITE = 4 };

__global__ void k_fsai_clear(int32_t *flags) {
    if (threadIdx.x == 0) flags[0] = 0;
}

template <int MS>
__global__ void __launch_bounds__(64)
k_fsai(int n, const int32_t *__restrict__ arp, const int32_t *__restrict__ acol,
       const double *__restrict__ avals, const int32_t *__restrict__ grp,
       const int32_t *__restrict__ gcol, float *__restrict__ gvals,
       const int32_t *__restrict__ trp, const int32_t *__restrict__ tcol,
       float *__restrict__ tvals, int32_t *flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t0 = trp[i];
    const int m = trp[i + 1] - t0;
    if (m < 1 || m > MS || tcol[t0] != i) {
        atomicOr(flags, F_BAD_PATTERN);
        return;
    }
    int J[MS];
#pragma unroll
    for (int a = 0; a < MS; ++a) J[a] = a < m ? tcol[t0 + a] : -1;
    // M = A[J, J], identity on the padding
    double M[MS][MS];
#pragma unroll
    for (int a = 0; a < MS; ++a)
#pragma unroll
        for (int b = 0; b < MS; ++b) M[a][b] = (a == b && a >= m) ? 1.0 : 0.0;
#pragma unroll
    for (int a = 0; a < MS; ++a) {
        if (a < m) {
            const int j = J[a];
            for (int k = arp[j]; k < arp[j + 1]; ++k) {
                const int c = acol[k];
                const double v = avals[k];
#pragma unroll
                for (int b = 0; b < MS; ++b)
                    if (c == J[b]) M[a][b] += v;
            }
        }
    }
    // Cholesky M = L L^T in place (lower triangle)
    bool spd = true;
#pragma unroll
    for (int a = 0; a < MS; ++a) {
        double d = M[a][a];
#pragma unroll
        for (int t = 0; t < a; ++t) d -= M[a][t] * M[a][t];
        spd = spd && d > 0.0;
        const double l = sqrt(d > 0.0 ? d : 1.0);
        M[a][a] = l;
#pragma unroll
        for (int b = a + 1; b < MS; ++b) {
            double s = M[b][a];
#pragma unroll
            for (int t = 0; t < a; ++t) s -= M[b][t] * M[a][t];
            M[b][a] = s / l;
        }
    }
    if (!spd) {
        atomicOr(flags, F_NOT_SPD);
        return;
    }
    // L w = e_1, then L^T y = w
    double w[MS], y[MS];
#pragma unroll
    for (int a = 0; a < MS; ++a) {
        double s = a == 0 ? 1.0 : 0.0;
#pragma unroll
        for (int t = 0; t < a; ++t) s -= M[a][t] * w[t];
        w[a] = s / M[a][a];
    }
#pragma unroll
    for (int a = MS - 1; a >= 0; --a) {
        double s = w[a];
#pragma unroll
        for (int t = a + 1; t < MS; ++t) s -= M[t][a] * y[t];
        y[a] = s / M[a][a];
    }
    const double scale = 1.0 / sqrt(y[0]);  // y_1 = (A[J,J]^-1)_11 > 0
    if (!isfinite(scale)) {
        atomicOr(flags, F_NON_FINITE);
        return;
    }
#pragma unroll
    for (int a = 0; a < MS; ++a) {
        if (a < m) {
            const float g = (float)(y[a] * scale);
            tvals[t0 + a] = g;
            // G[J[a], i]: search row J[a] of G for column i
            const int j = J[a];
            int pos = -1;
            for (int k = grp[j]; k < grp[j + 1]; ++k)
                if (gcol[k] == i) pos = k;
            if (pos < 0) atomicOr(flags, F_BAD_PATTERN);
            else gvals[pos] = g;
        }
    }
}

}  // namespace spcg

using namespace spcg;

extern "C" {

int spcg_fsai_values(spcg_csr_t A, spcg_csr_t G, spcg_csr_t GT, hipStream_t stream) {
    if (!A || !G || !GT) return SPCG_INVALID_ARG;
    const int n = A->n_rows;
    if (A->dtype != SPCG_F64 || G->dtype != SPCG_F32 || GT->dtype != SPCG_F32) return SPCG_INVALID_ARG;
    if (A->n_cols != n || G->n_rows != n || G->n_cols != n || GT->n_rows != n || GT->n_cols != n ||
        G->nnz != GT->nnz)
        return SPCG_INVALID_ARG;
    if (GT->max_len > SPCG_FSAI_MAX_SET) return SPCG_INVALID_ARG;
    if (n == 0) return SPCG_OK;
    int32_t *flags = GT->flags;  // the handle's own analysis scratch
    hipLaunchKernelGGL(k_fsai_clear, dim3(1), dim3(64), 0, stream, flags);
    const dim3 grid((n + 63) / 64);
    if (GT->max_len <= 4)
        hipLaunchKernelGGL(k_fsai<4>, grid, dim3(64), 0, stream, n, A->row_ptr, A->col,
                           (const double *)A->vals, G->row_ptr, G->col, (float *)G->vals,
                           GT->row_ptr, GT->col, (float *)GT->vals, flags);
    else
        hipLaunchKernelGGL(k_fsai<SPCG_FSAI_MAX_SET>, grid, dim3(64), 0, stream, n, A->row_ptr,
                           A->col, (const double *)A->vals, G->row_ptr, G->col, (float *)G->vals,
                           GT->row_ptr, GT->col, (float *)GT->vals, flags);
    SPCG_TRY(hipGetLastError());
    int32_t *hf = (int32_t *)GT->h_pinned;
    SPCG_TRY(hipMemcpyAsync(hf, flags, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    SPCG_TRY(hipStreamSynchronize(stream));
    if (hf[0] & F_BAD_PATTERN) return SPCG_INVALID_ARG;
    if (hf[0] & F_NOT_SPD) return SPCG_NOT_SPD;
    if (hf[0] & F_NON_FINITE) return SPCG_NON_FINITE;
    return SPCG_OK;
}

}  // extern "C"

// fb_lu.hip -- the LU function block (the paper's other offloaded block,
// section 5.1(b)): right-looking blocked LU factorization with partial
// pivoting of a row-major n x n binary64 matrix, in place.
//
// For each panel of LU_NB columns starting at column k:
//   lu_panel  factors rows k..n-1 of the panel column by column (pivot =
//             first row of largest magnitude, row swap inside the panel,
//             scaling, rank-1 update of the panel's remaining columns); one
//             workgroup holds the whole panel in registers, two rows per
//             thread, so n <= 2 * 1024;
//   lu_swap   applies the panel's row swaps, in order, to every column
//             outside the panel (one thread per column);
//   lu_trsm   U12 = L11^-1 A12 for the columns right of the panel (one
//             thread per column, L11 in LDS);
//   lu_gemm   A22 -= L21 U12 on 64 x 64 tiles (L21 and U12 tiles in LDS).
// Every element receives its updates in increasing column order j, as in
// unblocked elimination.  On gfx950 the dense binary64 matrix-core rate
// equals the vector rate, and the rank-16 update is bound by memory traffic,
// so the update uses vector FMAs.
#include <hip/hip_runtime.h>

#include "fb_lu.hpp"

namespace fb {

constexpr int LU_PANEL_THREADS = 1024;
constexpr int LU_ROWS = 2;   // rows of the panel per thread

__global__ void lu_init(int32_t *info)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) info[0] = 0;
}

__global__ void __launch_bounds__(LU_PANEL_THREADS)
    lu_panel(double *__restrict__ a, int64_t n, int64_t lda, int64_t k, int nb, int32_t *__restrict__ ipiv,
             int32_t *__restrict__ info)
{
    __shared__ double rowj[LU_NB], rowp[LU_NB];
    __shared__ double wbest[LU_PANEL_THREADS / 64];
    __shared__ int widx[LU_PANEL_THREADS / 64];
    __shared__ int s_p;
    const int tid = threadIdx.x;
    const int m = (int)(n - k);   // rows of the panel (<= LU_ROWS * LU_PANEL_THREADS, checked on the host)
    double v[LU_ROWS][LU_NB];
#pragma unroll
    for (int r = 0; r < LU_ROWS; r++) {
        const int i = tid + LU_PANEL_THREADS * r;
#pragma unroll
        for (int c = 0; c < LU_NB; c++)
            v[r][c] = (i < m && c < nb) ? a[(k + i) * lda + k + c] : 0.0;
    }

#pragma unroll
    for (int j = 0; j < LU_NB; j++) {
        if (j < nb) {   // uniform
            // ---- pivot: the first row i >= j of largest |a[i][j]|
            double best = -1.0;
            int bi = 0x7fffffff;
#pragma unroll
            for (int r = 0; r < LU_ROWS; r++) {
                const int i = tid + LU_PANEL_THREADS * r;
                if (i >= j && i < m) {
                    const double x = fabs(v[r][j]);
                    if (x > best) {
                        best = x;
                        bi = i;
                    }
                }
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double ob = __shfl_xor(best, off);
                const int oi = __shfl_xor(bi, off);
                if (ob > best || (ob == best && oi < bi)) {
                    best = ob;
                    bi = oi;
                }
            }
            if ((tid & 63) == 0) {
                wbest[tid >> 6] = best;
                widx[tid >> 6] = bi;
            }
            __syncthreads();
            if (tid == 0) {
                double b = wbest[0];
                int p = widx[0];
                for (int w = 1; w < LU_PANEL_THREADS / 64; w++)
                    if (wbest[w] > b || (wbest[w] == b && widx[w] < p)) {
                        b = wbest[w];
                        p = widx[w];
                    }
                s_p = p;
                ipiv[k + j] = (int32_t)(k + p);
                if (b == 0.0 && info[0] == 0) info[0] = (int32_t)(k + j + 1);
            }
            __syncthreads();
            const int p = s_p;
            // ---- swap rows j and p of the panel; rowp becomes the pivot row
#pragma unroll
            for (int r = 0; r < LU_ROWS; r++) {
                const int i = tid + LU_PANEL_THREADS * r;
                if (i == p) {
#pragma unroll
                    for (int c = 0; c < LU_NB; c++) rowp[c] = v[r][c];
                }
                if (i == j) {
#pragma unroll
                    for (int c = 0; c < LU_NB; c++) rowj[c] = v[r][c];
                }
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < LU_ROWS; r++) {
                const int i = tid + LU_PANEL_THREADS * r;
                if (i == j) {
#pragma unroll
                    for (int c = 0; c < LU_NB; c++) v[r][c] = rowp[c];
                } else if (i == p) {
#pragma unroll
                    for (int c = 0; c < LU_NB; c++) v[r][c] = rowj[c];
                }
            }
            // ---- scale the column below the pivot, update the panel's right part
            const double piv = rowp[j];
            if (piv != 0.0) {
#pragma unroll
                for (int r = 0; r < LU_ROWS; r++) {
                    const int i = tid + LU_PANEL_THREADS * r;
                    if (i > j && i < m) {
                        const double l = v[r][j] / piv;
                        v[r][j] = l;
#pragma unroll
                        for (int c = j + 1; c < LU_NB; c++) v[r][c] -= l * rowp[c];
                    }
                }
            }
            __syncthreads();   // rowp / rowj are rewritten by the next column
        }
    }

#pragma unroll
    for (int r = 0; r < LU_ROWS; r++) {
        const int i = tid + LU_PANEL_THREADS * r;
        if (i < m) {
#pragma unroll
            for (int c = 0; c < LU_NB; c++)
                if (c < nb) a[(k + i) * lda + k + c] = v[r][c];
        }
    }
}

// The panel's swaps (rows k+j <-> ipiv[k+j], j = 0..nb-1 in order) on every
// column outside the panel.
__global__ void __launch_bounds__(256)
    lu_swap(double *__restrict__ a, int64_t n, int64_t lda, int64_t k, int nb, const int32_t *__restrict__ ipiv)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= n || (c >= k && c < k + nb)) return;
    for (int j = 0; j < nb; j++) {
        const int64_t p = ipiv[k + j];
        if (p != k + j) {
            const double t = a[(k + j) * lda + c];
            a[(k + j) * lda + c] = a[p * lda + c];
            a[p * lda + c] = t;
        }
    }
}

// U12 = L11^-1 A12: columns c >= k + nb of rows k .. k+nb-1.
__global__ void __launch_bounds__(256)
    lu_trsm(double *__restrict__ a, int64_t n, int64_t lda, int64_t k, int nb)
{
    __shared__ double L[LU_NB][LU_NB + 1];
    for (int idx = threadIdx.x; idx < LU_NB * LU_NB; idx += 256) {
        const int i = idx / LU_NB, j = idx % LU_NB;
        L[i][j] = (i < nb && j < nb) ? a[(k + i) * lda + k + j] : 0.0;
    }
    __syncthreads();
    const int64_t c = k + nb + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= n) return;
    double x[LU_NB];
#pragma unroll
    for (int i = 0; i < LU_NB; i++) x[i] = i < nb ? a[(k + i) * lda + c] : 0.0;
#pragma unroll
    for (int i = 1; i < LU_NB; i++) {
#pragma unroll
        for (int j = 0; j < i; j++) x[i] -= L[i][j] * x[j];
    }
#pragma unroll
    for (int i = 1; i < LU_NB; i++)
        if (i < nb) a[(k + i) * lda + c] = x[i];
}

// A22 -= L21 U12 on 64 x 64 tiles: rows and columns >= k + nb.
constexpr int LU_TILE = 64;
__global__ void __launch_bounds__(256)
    lu_gemm(double *__restrict__ a, int64_t n, int64_t lda, int64_t k, int nb)
{
    __shared__ double Ls[LU_TILE][LU_NB + 1];
    __shared__ double Us[LU_NB][LU_TILE + 4];
    const int64_t s = k + nb;   // first row and column of A22
    const int64_t r0 = s + (int64_t)blockIdx.y * LU_TILE, c0 = s + (int64_t)blockIdx.x * LU_TILE;
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    for (int idx = tid; idx < LU_TILE * LU_NB; idx += 256) {
        const int i = idx / LU_NB, j = idx % LU_NB;
        Ls[i][j] = (r0 + i < n && j < nb) ? a[(r0 + i) * lda + k + j] : 0.0;
    }
    for (int idx = tid; idx < LU_NB * LU_TILE; idx += 256) {
        const int j = idx / LU_TILE, c = idx % LU_TILE;
        Us[j][c] = (c0 + c < n && j < nb) ? a[(k + j) * lda + c0 + c] : 0.0;
    }
    __syncthreads();
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int64_t r = r0 + ty * 4 + i;
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const int64_t cc = c0 + tx * 4 + c;
            acc[i][c] = (r < n && cc < n) ? a[r * lda + cc] : 0.0;
        }
    }
#pragma unroll
    for (int j = 0; j < LU_NB; j++) {
        if (j < nb) {
            double l[4], u[4];
#pragma unroll
            for (int i = 0; i < 4; i++) l[i] = Ls[ty * 4 + i][j];
#pragma unroll
            for (int c = 0; c < 4; c++) u[c] = Us[j][tx * 4 + c];
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int c = 0; c < 4; c++) acc[i][c] -= l[i] * u[c];
        }
    }
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int64_t r = r0 + ty * 4 + i;
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const int64_t cc = c0 + tx * 4 + c;
            if (r < n && cc < n) a[r * lda + cc] = acc[i][c];
        }
    }
}

hipError_t launch_lu(double *a, int64_t n, int64_t lda, int32_t *ipiv, int32_t *info, hipStream_t st)
{
    hipLaunchKernelGGL(lu_init, dim3(1), dim3(64), 0, st, info);
    hipError_t e = hipGetLastError();
    for (int64_t k = 0; e == hipSuccess && k < n; k += LU_NB) {
        const int nb = (int)(n - k < LU_NB ? n - k : LU_NB);
        hipLaunchKernelGGL(lu_panel, dim3(1), dim3(LU_PANEL_THREADS), 0, st, a, n, lda, k, nb, ipiv, info);
        hipLaunchKernelGGL(lu_swap, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, n, lda, k, nb, ipiv);
        const int64_t rest = n - k - nb;
        if (rest > 0) {
            hipLaunchKernelGGL(lu_trsm, dim3((unsigned)((rest + 255) / 256)), dim3(256), 0, st, a, n, lda, k, nb);
            const unsigned t = (unsigned)((rest + LU_TILE - 1) / LU_TILE);
            hipLaunchKernelGGL(lu_gemm, dim3(t, t), dim3(256), 0, st, a, n, lda, k, nb);
        }
        e = hipGetLastError();
    }
    return e;
}

}  // namespace fb

// fb_lu.hip -- the LU function block (the paper's other offloaded block,
// section 5.1(b)): right-looking blocked LU factorization with partial
// pivoting of a row-major n x n binary64 matrix, in place.
//
// For each panel of LU_NB columns starting at column k:
//   lu_panel  factors rows k..n-1 of the panel column by column (pivot =
//             first row of largest magnitude, row exchange inside the panel,
//             scaling, rank-1 update of the panel's remaining columns); one
//             workgroup holds the whole panel in registers, four rows per
//             thread of 512, so n <= 2048, and exchanges rows by relabelling
//             them;
//   lu_swap_trsm  applies the panel's row swaps, in order, to every column
//             outside the panel, then U12 = L11^-1 A12 for the columns right
//             of it (one thread per column, L11 in LDS);
//   lu_gemm_mfma  A22 -= L21 U12 on 64 x 64 tiles (L21 and U12 tiles in
//             LDS) on the binary64 matrix cores (lu_gemm: the same on the
//             vector units, FB_LU_MFMA = 0).
// Every element receives its updates in increasing column order j, as in
// unblocked elimination (both update kernels give the same bits).
#include <hip/hip_runtime.h>

#include "fb_device.hpp"
#include "fb_lu.hpp"

namespace fb {

#ifndef FB_LU_PANEL_THREADS
#define FB_LU_PANEL_THREADS 512
#endif
constexpr int LU_PANEL_THREADS = FB_LU_PANEL_THREADS;
constexpr int LU_ROWS = (int)(LU_MAX_N / LU_PANEL_THREADS);   // rows of the panel per thread
static_assert(LU_ROWS * LU_PANEL_THREADS >= LU_MAX_N, "the panel kernel holds every row of a panel");

__global__ void lu_init(int32_t *info)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) info[0] = 0;
}

// ---- pivot search within a wavefront
//
// The pivot is the first row (smallest position) among those of largest
// magnitude.  It is found in two reductions: the largest magnitude M, then
// the smallest position among the candidates whose magnitude equals M, so
// each step is a single max or min instead of a compare-and-select on
// (magnitude, row) pairs.  Magnitudes are compared as binary64 values, so
// ties are exact.  The all-reduce over 64 lanes exchanges with the lanes
// l ^ 1, l ^ 2 (DPP quad permutations), 7 - l within 8 and 15 - l within 16
// (DPP half-row and row mirrors), then with the same lane of the row r ^ 1
// and r ^ 2 (permlane16 / permlane32 swaps): each step pairs disjoint halves
// of a group, so after six steps every lane holds the wave's result.
template <int CTRL> __device__ __forceinline__ int dpp_i(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
template <int CTRL> __device__ __forceinline__ double dpp_d(double x)
{
    const long long u = __double_as_longlong(x);
    const int lo = dpp_i<CTRL>((int)u), hi = dpp_i<CTRL>((int)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// the same lane of row r ^ 1 (ROWS = 1) or r ^ 2 (ROWS = 2)
template <int ROWS> __device__ __forceinline__ int row_partner_i(int x, int lane)
{
    if constexpr (ROWS == 1) {
        const auto r = __builtin_amdgcn_permlane16_swap((unsigned)x, (unsigned)x, false, false);
        return (int)((lane & 16) ? r[0] : r[1]);
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)x, false, false);
        return (int)((lane & 32) ? r[0] : r[1]);
    }
}
template <int ROWS> __device__ __forceinline__ double row_partner_d(double x, int lane)
{
    const long long u = __double_as_longlong(x);
    const int lo = row_partner_i<ROWS>((int)u, lane), hi = row_partner_i<ROWS>((int)(u >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double dmax(double x, double y) { return x > y ? x : y; }
__device__ __forceinline__ int imin(int x, int y) { return x < y ? x : y; }
__device__ __forceinline__ double wave_max(double x, int lane)
{
    x = dmax(x, dpp_d<0xB1>(x));     // quad_perm [1,0,3,2]: l ^ 1
    x = dmax(x, dpp_d<0x4E>(x));     // quad_perm [2,3,0,1]: l ^ 2
    x = dmax(x, dpp_d<0x141>(x));    // row_half_mirror
    x = dmax(x, dpp_d<0x140>(x));    // row_mirror
    x = dmax(x, row_partner_d<1>(x, lane));
    return dmax(x, row_partner_d<2>(x, lane));
}
__device__ __forceinline__ int wave_min(int i, int lane)
{
    i = imin(i, dpp_i<0xB1>(i));
    i = imin(i, dpp_i<0x4E>(i));
    i = imin(i, dpp_i<0x141>(i));
    i = imin(i, dpp_i<0x140>(i));
    i = imin(i, row_partner_i<1>(i, lane));
    return imin(i, row_partner_i<2>(i, lane));
}

struct PanelCand {
    double best;
    int row;
    int pad;
};

// FULL: nb == LU_NB (every panel but possibly the last), with no test per
// column.  The column steps contain no branch apart from the candidate row's
// publication and the barrier, so that the tail of one column's update
// (columns j + 2 ..) can be scheduled into the latency of the next column's
// reductions: rows that are not updated keep their values through selects,
// and the pivots are kept in registers and stored at the end.
template <bool FULL>
__global__ void __launch_bounds__(LU_PANEL_THREADS)
    lu_panel(double *__restrict__ a, int64_t n, int64_t lda, int64_t k, int nb, int32_t *__restrict__ ipiv,
             int32_t *__restrict__ info)
{
    constexpr int W = LU_PANEL_THREADS / 64;   // waves
    // Rows never move between registers: each row held by a thread carries
    // its current position in the panel (its label), and exchanging rows j
    // and p exchanges two labels.  At the end every row is stored at the
    // position its label names.  Ties between pivot candidates go to the
    // smallest label: the first row of largest magnitude in the exchanged
    // order.
    //
    // One barrier per column.  Before it, each wave publishes its candidate
    // (largest magnitude, smallest position of that magnitude) and that
    // candidate's whole row; after it, every wave reduces the W candidates
    // the same way and reads the pivot row.  The buffers alternate with the
    // column's parity: a thread that reaches column j + 1's barrier has
    // finished every read of column j - 1's buffers.
    __shared__ PanelCand cand[2][W];
    __shared__ double crow[2][W][LU_NB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = (int)(n - k);   // rows of the panel (<= LU_ROWS * LU_PANEL_THREADS, checked on the host)
    if (FULL) nb = LU_NB;
    // the first zero pivot, kept in registers (a global read per column
    // would stall every column's barrier on memory latency)
    int32_t zero_at = info[0];
    int piv_at[LU_NB];   // the pivot position of each column
    double v[LU_ROWS][LU_NB];
    int lab[LU_ROWS];   // the row's position; rows past the panel keep positions >= m
#pragma unroll
    for (int r = 0; r < LU_ROWS; r++) {
        const int i = tid + LU_PANEL_THREADS * r;
        lab[r] = i;
#pragma unroll
        for (int c = 0; c < LU_NB; c++)
            v[r][c] = (i < m && c < nb) ? a[(k + i) * lda + k + c] : 0.0;
    }

    // columns as a compile-time sequence, so that every index into v is a
    // constant and v stays in registers
    static_for<0, LU_NB>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (FULL || j < nb) {   // uniform
            constexpr int h = j & 1;
            // ---- pivot candidates: per thread the largest |a[.][j]| among
            // its rows at positions >= j and the smallest such position, then
            // the same per wave
            double x[LU_ROWS];
#pragma unroll
            for (int r = 0; r < LU_ROWS; r++) x[r] = (lab[r] >= j && lab[r] < m) ? fabs(v[r][j]) : -1.0;
            double mt = x[0];
#pragma unroll
            for (int r = 1; r < LU_ROWS; r++) mt = dmax(mt, x[r]);
            int lt = 0x7fffffff, br = 0;
#pragma unroll
            for (int r = LU_ROWS - 1; r >= 0; r--) {
                const bool t = x[r] == mt && lab[r] < lt;
                lt = t ? lab[r] : lt;
                br = t ? r : br;
            }
            const double mw = wave_max(mt, lane);
            const int pwv = wave_min(mt == mw ? lt : 0x7fffffff, lane);
            if (lane == 0) cand[h][wave] = PanelCand{mw, pwv, 0};
            if (lt == pwv) {   // the one lane of the wave that holds the candidate (positions are unique)
#pragma unroll
                for (int r = 0; r < LU_ROWS; r++) {
                    if (br == r) {
#pragma unroll
                        for (int c = 0; c < LU_NB; c++) crow[h][wave][c] = v[r][c];
                        asm volatile("" ::: "memory");   // keeps the four stores apart (merged, they index v at run time)
                    }
                }
            }
            __syncthreads();
            // ---- the pivot: the same two reductions over the W wave
            // candidates, lane l reading candidate l mod W
            static_assert(W == 8, "the candidates are reduced within groups of 8 lanes");
            const PanelCand cl = cand[h][lane & (W - 1)];
            double b = cl.best;
            b = dmax(b, dpp_d<0xB1>(b));
            b = dmax(b, dpp_d<0x4E>(b));
            b = dmax(b, dpp_d<0x141>(b));
            int p = b == cl.best ? cl.row : 0x7fffffff;
            p = imin(p, dpp_i<0xB1>(p));
            p = imin(p, dpp_i<0x4E>(p));
            p = imin(p, dpp_i<0x141>(p));
            // every group of 8 lanes holds the result; the wave that published it
            const int pw = __ffsll((long long)(__ballot(lane < W && cl.row == p) & 0xffull)) - 1;
            piv_at[j] = p;
            zero_at = (b == 0.0 && zero_at == 0) ? (int32_t)(k + j + 1) : zero_at;
            const double *rowp = crow[h][pw];
            double pr[LU_NB];   // the pivot row's columns j .. LU_NB - 1, read once
#pragma unroll
            for (int c = j; c < LU_NB; c++) pr[c] = rowp[c];
            // ---- exchange positions j and p
#pragma unroll
            for (int r = 0; r < LU_ROWS; r++) lab[r] = lab[r] == j ? p : (lab[r] == p ? j : lab[r]);
            // ---- scale the column below the pivot (a zero pivot scales
            // nothing), update the panel's right part; the four quotients are
            // independent, and column j + 1 comes first: the next pivot
            // search waits for it alone
            const double piv = pr[j];
            bool up[LU_ROWS];
            double l[LU_ROWS];
#pragma unroll
            for (int r = 0; r < LU_ROWS; r++) {
                up[r] = lab[r] > j && lab[r] < m && piv != 0.0;
                const double q = v[r][j] / piv;
                l[r] = q;
                v[r][j] = up[r] ? q : v[r][j];
            }
#pragma unroll
            for (int c = j + 1; c < LU_NB; c++) {
#pragma unroll
                for (int r = 0; r < LU_ROWS; r++) v[r][c] = up[r] ? v[r][c] - l[r] * pr[c] : v[r][c];
            }
        }
    });

#pragma unroll
    for (int r = 0; r < LU_ROWS; r++) {
        if (lab[r] < m) {
#pragma unroll
            for (int c = 0; c < LU_NB; c++)
                if (c < nb) a[(k + lab[r]) * lda + k + c] = v[r][c];
        }
    }
    if (tid == 0) {
#pragma unroll
        for (int j = 0; j < LU_NB; j++)
            if (j < nb) ipiv[k + j] = (int32_t)(k + piv_at[j]);
        info[0] = zero_at;
    }
}

// The panel's swaps (rows k+j <-> ipiv[k+j], j = 0..nb-1 in order) on every
// column outside the panel, then U12 = L11^-1 A12 on the columns right of
// it.  The swaps are first composed into one permutation of the at most
// 2 nb rows they touch (each workgroup does it in LDS from ipiv), so that a
// column loads every touched row at once and stores each once, instead of
// nb dependent swaps.  One thread per column: row accesses are coalesced.
constexpr int LU_SWAP_THREADS = 64;
// the value of x in lane l (l uniform over the wave)
__device__ __forceinline__ int64_t lane_i64(int64_t x, int l)
{
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)(uint64_t)x, l);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)((uint64_t)x >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__global__ void __launch_bounds__(LU_SWAP_THREADS)
    lu_swap_trsm(double *__restrict__ a, int64_t n, int64_t lda, int64_t k, int nb, const int32_t *__restrict__ ipiv)
{
    // The kernel is a chain of latencies (the pivots, the permutation, the
    // rows, the solve), so every step keeps its loads in flight together:
    // the pivots and L11 are requested at once, and the row addresses are
    // scalars read from the lanes that composed the permutation, with no LDS
    // round trip between them.
    static_assert(LU_SWAP_THREADS == 64 && 2 * LU_NB <= 64, "one wave composes the permutation");
    static_assert((LU_NB * LU_NB) % LU_SWAP_THREADS == 0, "L11 is loaded in whole rounds");
    constexpr int LR = LU_NB * LU_NB / LU_SWAP_THREADS;
    __shared__ double L[LU_NB][LU_NB + 1];
    const int lane = threadIdx.x;
    const int32_t pv32 = ipiv[k + (lane < nb ? lane : 0)];   // unconditional: no wait at a branch join
    double lv[LR];
#pragma unroll
    for (int t = 0; t < LR; t++) {
        const int idx = lane + LU_SWAP_THREADS * t, i = idx / LU_NB, j = idx % LU_NB;
        const int ic = i < nb ? i : 0, jc = j < nb ? j : 0;   // in bounds also for a short last panel
        lv[t] = a[(k + ic) * lda + k + jc];
    }
    // Lane q holds touched row d and the original row sr whose content it
    // holds after the swaps so far: rows k .. k+nb-1 in lanes 0 .. nb-1,
    // pivot rows below the block appended as they first appear.  j and q are
    // uniform, so every exchange is a scalar read of one lane.
    const int64_t pv = lane < nb ? (int64_t)pv32 : 0;
    int64_t d = lane < nb ? k + lane : -1;
    int64_t sr = d;
    int cnt = nb;
    for (int j = 0; j < nb; j++) {
        const int64_t pr = lane_i64(pv, j);
        int q;
        if (pr - k < nb) {
            q = (int)(pr - k);   // inside the block (pivot rows are >= k + j)
        } else {
            const unsigned long long hit = __ballot(lane >= nb && lane < cnt && d == pr);
            if (hit) {
                q = __ffsll((long long)hit) - 1;
            } else {
                q = cnt++;
                if (lane == q) d = sr = pr;
            }
        }
        const int64_t sj = lane_i64(sr, j), sq = lane_i64(sr, q);
        if (lane == j) sr = sq;
        if (lane == q) sr = sj;
    }
#pragma unroll
    for (int t = 0; t < LR; t++) {
        const int idx = lane + LU_SWAP_THREADS * t, i = idx / LU_NB, j = idx % LU_NB;
        L[i][j] = (i < nb && j < nb) ? lv[t] : 0.0;
    }
    __syncthreads();
    const int64_t c = (int64_t)blockIdx.x * LU_SWAP_THREADS + lane;
    const bool live = c < n && !(c >= k && c < k + nb);   // the panel's own columns are done
    const int64_t cc = live ? c : (k + nb < n ? k + nb : 0);   // a column every lane may read
    double val[2 * LU_NB];
#pragma unroll
    for (int q = 0; q < 2 * LU_NB; q++) val[q] = q < cnt ? a[lane_i64(sr, q) * lda + cc] : 0.0;
    const bool right = c >= k + nb;
    if (right) {
        static_for<1, LU_NB>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
#pragma unroll
            for (int j = 0; j < i; j++) val[i] -= L[i][j] * val[j];
        });
    }
    if (live) {
#pragma unroll
        for (int q = 0; q < 2 * LU_NB; q++) {
            if (q < cnt) {
                const int64_t dq = lane_i64(d, q), sq = lane_i64(sr, q);
                if (dq != sq || (right && q < nb)) a[dq * lda + c] = val[q];
            }
        }
    }
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

// The same update on the binary64 matrix cores (FB_LU_MFMA = 1):
// v_mfma_f64_16x16x4f64 computes D = A B + C for a 16 x 4 block A, a 4 x 16
// block B and a 16 x 16 block C; lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and holds D[4 r + l / 16][l % 16] in its register r < 4
// (rows interleaved over the four 16-lane groups; checked on the device with
// known operands).  Each wave of the 64 x 64 tile computes a 32 x 32
// quadrant as 2 x 2 such blocks over the panel's columns in steps of 4, with
// A = -L21 so that the accumulator starts from A22 and ends at A22 - L21 U12.
#ifndef FB_LU_MFMA
#define FB_LU_MFMA 1
#endif
typedef double lu_d4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256)
    lu_gemm_mfma(double *__restrict__ a, int64_t n, int64_t lda, int64_t k, int nb)
{
    __shared__ double Ls[LU_TILE][LU_NB + 1];
    __shared__ double Us[LU_NB][LU_TILE + 4];
    const int64_t s = k + nb;   // first row and column of A22
    const int64_t r0 = s + (int64_t)blockIdx.y * LU_TILE, c0 = s + (int64_t)blockIdx.x * LU_TILE;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < LU_TILE * LU_NB; idx += 256) {
        const int i = idx / LU_NB, j = idx % LU_NB;
        Ls[i][j] = (r0 + i < n && j < nb) ? -a[(r0 + i) * lda + k + j] : 0.0;
    }
    for (int idx = tid; idx < LU_NB * LU_TILE; idx += 256) {
        const int j = idx / LU_TILE, c = idx % LU_TILE;
        Us[j][c] = (c0 + c < n && j < nb) ? a[(k + j) * lda + c0 + c] : 0.0;
    }
    const int wave = tid >> 6, lane = tid & 63;
    const int qr = 32 * (wave >> 1), qc = 32 * (wave & 1);   // the wave's quadrant of the tile
    const int li = lane & 15, lk = lane >> 4;
    lu_d4 acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; bi++) {
#pragma unroll
        for (int bj = 0; bj < 2; bj++) {
            const int64_t cc = c0 + qc + 16 * bj + li;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int64_t rr = r0 + qr + 16 * bi + 4 * r + lk;
                acc[bi][bj][r] = (rr < n && cc < n) ? a[rr * lda + cc] : 0.0;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < LU_NB; k4 += 4) {
        if (k4 < nb) {   // uniform; columns nb .. k4 + 3 of the tiles are zero
            double av[2], bv[2];
#pragma unroll
            for (int bi = 0; bi < 2; bi++) av[bi] = Ls[qr + 16 * bi + li][k4 + lk];
#pragma unroll
            for (int bj = 0; bj < 2; bj++) bv[bj] = Us[k4 + lk][qc + 16 * bj + li];
#pragma unroll
            for (int bi = 0; bi < 2; bi++) {
#pragma unroll
                for (int bj = 0; bj < 2; bj++)
                    acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bi], bv[bj], acc[bi][bj], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int bi = 0; bi < 2; bi++) {
#pragma unroll
        for (int bj = 0; bj < 2; bj++) {
            const int64_t cc = c0 + qc + 16 * bj + li;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int64_t rr = r0 + qr + 16 * bi + 4 * r + lk;
                if (rr < n && cc < n) a[rr * lda + cc] = acc[bi][bj][r];
            }
        }
    }
}

hipError_t launch_lu(double *a, int64_t n, int64_t lda, int32_t *ipiv, int32_t *info, hipStream_t st)
{
    hipLaunchKernelGGL(lu_init, dim3(1), dim3(64), 0, st, info);
    hipError_t e = hipGetLastError();
    for (int64_t k = 0; e == hipSuccess && k < n; k += LU_NB) {
        const int nb = (int)(n - k < LU_NB ? n - k : LU_NB);
        if (nb == LU_NB)
            hipLaunchKernelGGL(lu_panel<true>, dim3(1), dim3(LU_PANEL_THREADS), 0, st, a, n, lda, k, nb, ipiv, info);
        else
            hipLaunchKernelGGL(lu_panel<false>, dim3(1), dim3(LU_PANEL_THREADS), 0, st, a, n, lda, k, nb, ipiv, info);
        if (n > nb)
            hipLaunchKernelGGL(lu_swap_trsm, dim3((unsigned)((n + LU_SWAP_THREADS - 1) / LU_SWAP_THREADS)),
                               dim3(LU_SWAP_THREADS), 0, st, a, n, lda, k, nb, ipiv);
        const int64_t rest = n - k - nb;
        if (rest > 0) {
            const unsigned t = (unsigned)((rest + LU_TILE - 1) / LU_TILE);
            if (FB_LU_MFMA) hipLaunchKernelGGL(lu_gemm_mfma, dim3(t, t), dim3(256), 0, st, a, n, lda, k, nb);
            else hipLaunchKernelGGL(lu_gemm, dim3(t, t), dim3(256), 0, st, a, n, lda, k, nb);
        }
        e = hipGetLastError();
    }
    return e;
}

}  // namespace fb

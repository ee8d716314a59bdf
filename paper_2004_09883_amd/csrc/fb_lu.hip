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
//   the update of the other columns: the panel's row exchanges, in order,
//             on every column outside the panel, U12 = L11^-1 A12 for the
//             columns right of it, A22 -= L21 U12.
// Two schedules of the same operations:
//   FB_LU_LOOKAHEAD = 1 (default): lu_panel for the first panel, then one
//             lu_step per panel k, whose workgroup 0 updates panel k+1's
//             columns and factors panel k+1 while the other workgroups
//             update the columns right of it (16-column strips) and apply
//             the exchanges left of panel k;
//   FB_LU_LOOKAHEAD = 0: three launches per panel, lu_panel, lu_swap_trsm
//             (exchanges and U12, one thread per column) and lu_gemm_mfma
//             (A22 on 64 x 64 tiles on the binary64 matrix cores; lu_gemm:
//             the same on the vector units, FB_LU_MFMA = 0).
// Every element receives its updates in increasing column order j, as in
// unblocked elimination, so both schedules and both update kernels give
// the same bits.
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

// step S (0 .. 5) of wave_max / wave_min, so that other work can be placed
// between the steps
template <int S> __device__ __forceinline__ double wave_max_step(double x, int lane)
{
    if constexpr (S == 0) return dmax(x, dpp_d<0xB1>(x));
    else if constexpr (S == 1) return dmax(x, dpp_d<0x4E>(x));
    else if constexpr (S == 2) return dmax(x, dpp_d<0x141>(x));
    else if constexpr (S == 3) return dmax(x, dpp_d<0x140>(x));
    else if constexpr (S == 4) return dmax(x, row_partner_d<1>(x, lane));
    else return dmax(x, row_partner_d<2>(x, lane));
}
template <int S> __device__ __forceinline__ int wave_min_step(int i, int lane)
{
    if constexpr (S == 0) return imin(i, dpp_i<0xB1>(i));
    else if constexpr (S == 1) return imin(i, dpp_i<0x4E>(i));
    else if constexpr (S == 2) return imin(i, dpp_i<0x141>(i));
    else if constexpr (S == 3) return imin(i, dpp_i<0x140>(i));
    else if constexpr (S == 4) return imin(i, row_partner_i<1>(i, lane));
    else return imin(i, row_partner_i<2>(i, lane));
}

struct PanelCand {
    double best;
    int row;
    int pad;
};

// The factorization of one panel (columns k .. k+nb-1, rows k .. k+m-1)
// from registers: thread t holds rows in v[r][0 .. nb), each with its
// position in the panel in lab[r] (rows that are not in the panel carry a
// position >= m).  Rows never move between registers: exchanging rows j and
// p exchanges two positions, and at the end every row is stored at the
// position it carries.  Ties between pivot candidates go to the smallest
// position: the first row of largest magnitude in the exchanged order.
//
// One barrier per column.  Before it, each wave publishes its candidate
// (largest magnitude, smallest position of that magnitude) and that
// candidate's whole row; after it, every wave reduces the W candidates the
// same way and reads the pivot row.  The buffers alternate with the
// column's parity: a thread that reaches column j + 1's barrier has finished
// every read of column j - 1's buffers.
//
// R: the register slots that can hold rows of the panel (slot r holds
// physical rows t + LU_PANEL_THREADS r, so a panel of m rows needs
// ceil(m / LU_PANEL_THREADS) of them); the others are not compiled in, which
// shortens every column step of the short panels.
//
// FULL: nb == LU_NB (every panel but possibly the last), with no test per
// column.  The column steps contain no branch apart from the candidate row's
// publication and the barrier (rows that are not updated keep their values
// through selects, the pivots are kept in registers and stored at the end),
// and the reductions of column j + 1 are computed at the end of step j:
// once column j + 1 is updated, its candidates are reduced over the wave
// while the rest of step j's update (columns j + 2 ..) is placed between the
// reduction's dependent steps, whose latency it fills (5.49 -> 5.31 ms for
// the 2048 x 2048 factorization).
constexpr int LU_W = LU_PANEL_THREADS / 64;   // waves of the panel's workgroup
struct PanelShared {
    PanelCand cand[2][LU_W];
    double crow[2][LU_W][LU_NB];
};

template <bool FULL, int R>
__device__ __forceinline__ void panel_columns(double (&v)[LU_ROWS][LU_NB], int (&lab)[LU_ROWS],
                                              double *__restrict__ a, int64_t lda, int64_t k, int m, int nb,
                                              int32_t *__restrict__ ipiv, int32_t *__restrict__ info, PanelShared &sh)
{
    constexpr int W = LU_W;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (FULL) nb = LU_NB;
    // the first zero pivot and the pivot positions, kept in registers (a
    // global access per column would stall every column's barrier on memory
    // latency) and stored at the end; the first panel starts the record
    int32_t zero_at = k == 0 ? 0 : info[0];
    int piv_at[LU_NB];
    // pivot candidates of column j: per thread the largest |a[.][j]| among
    // its rows at positions >= j and the smallest such position
    double mt = 0.0;
    int lt = 0, br = 0;
    auto candidates = [&](auto jc) {
        constexpr int j = decltype(jc)::value;
        double x[LU_ROWS];
#pragma unroll
        for (int r = 0; r < R; r++) x[r] = (lab[r] >= j && lab[r] < m) ? fabs(v[r][j]) : -1.0;
        mt = x[0];
#pragma unroll
        for (int r = 1; r < R; r++) mt = dmax(mt, x[r]);
        lt = 0x7fffffff;
        br = 0;
#pragma unroll
        for (int r = R - 1; r >= 0; r--) {
            const bool t = x[r] == mt && lab[r] < lt;
            lt = t ? lab[r] : lt;
            br = t ? r : br;
        }
    };
    candidates(std::integral_constant<int, 0>{});
    double mw = wave_max(mt, lane);
    int pwv = wave_min(mt == mw ? lt : 0x7fffffff, lane);

    static_for<0, LU_NB>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (FULL || j < nb) {   // uniform
            constexpr int h = j & 1;
            // ---- publish the wave's candidate and its row
            if (lane == 0) sh.cand[h][wave] = PanelCand{mw, pwv, 0};
            if (lt == pwv) {   // the one lane of the wave that holds the candidate (positions are unique)
#pragma unroll
                for (int r = 0; r < R; r++) {
                    if (br == r) {
#pragma unroll
                        for (int c = 0; c < LU_NB; c++) sh.crow[h][wave][c] = v[r][c];
                        asm volatile("" ::: "memory");   // keeps the stores apart (merged, they index v at run time)
                    }
                }
            }
            __syncthreads();
            // ---- the pivot: the same two reductions over the W wave
            // candidates, lane l reading candidate l mod W
            static_assert(W == 8, "the candidates are reduced within groups of 8 lanes");
            const PanelCand cl = sh.cand[h][lane & (W - 1)];
            double b = cl.best;
            b = dmax(b, dpp_d<0xB1>(b));
            b = dmax(b, dpp_d<0x4E>(b));
            b = dmax(b, dpp_d<0x141>(b));
            int p = b == cl.best ? cl.row : 0x7fffffff;
            p = imin(p, dpp_i<0xB1>(p));
            p = imin(p, dpp_i<0x4E>(p));
            p = imin(p, dpp_i<0x141>(p));
            const int pw = __ffsll((long long)(__ballot(lane < W && cl.row == p) & 0xffull)) - 1;
            piv_at[j] = p;
            zero_at = (b == 0.0 && zero_at == 0) ? (int32_t)(k + j + 1) : zero_at;
            const double *rowp = sh.crow[h][pw];
            double pr[LU_NB];
#pragma unroll
            for (int c = j; c < LU_NB; c++) pr[c] = rowp[c];
#pragma unroll
            for (int r = 0; r < R; r++) lab[r] = lab[r] == j ? p : (lab[r] == p ? j : lab[r]);
            // ---- scale the column below the pivot (a zero pivot scales
            // nothing); rows that are not updated keep their values
            const double piv = pr[j];
            bool up[LU_ROWS];
            double l[LU_ROWS];
#pragma unroll
            for (int r = 0; r < R; r++) {
                up[r] = lab[r] > j && lab[r] < m && piv != 0.0;
                const double q = v[r][j] / piv;
                l[r] = q;
                v[r][j] = up[r] ? q : v[r][j];
            }
            auto update = [&](auto cc) {
                constexpr int c = decltype(cc)::value;
                if constexpr (c < LU_NB) {
#pragma unroll
                    for (int r = 0; r < R; r++) {
                        v[r][c] = up[r] ? v[r][c] - l[r] * pr[c] : v[r][c];
                        // computed here, not sunk to its first use (the
                        // next column's publication)
                        asm volatile("" : "+v"(v[r][c]));
                    }
                }
            };
            if constexpr (j + 1 < LU_NB) {
                // ---- column j + 1 first, then its candidates and their
                // reductions, with columns j + 2 .. between the steps
                update(std::integral_constant<int, j + 1>{});
                candidates(std::integral_constant<int, j + 1>{});
                double mwn = mt;
                static_for<0, 6>([&](auto sc) {
                    constexpr int st = decltype(sc)::value;
                    mwn = wave_max_step<st>(mwn, lane);
                    update(std::integral_constant<int, j + 2 + st>{});
                    __builtin_amdgcn_sched_barrier(0);   // keep the pairs apart: the scheduler would bunch them
                });
                int pwn = mt == mwn ? lt : 0x7fffffff;
                static_for<0, 6>([&](auto sc) {
                    constexpr int st = decltype(sc)::value;
                    pwn = wave_min_step<st>(pwn, lane);
                    update(std::integral_constant<int, j + 8 + st>{});
                    __builtin_amdgcn_sched_barrier(0);
                });
                update(std::integral_constant<int, j + 14>{});
                update(std::integral_constant<int, j + 15>{});
                mw = mwn;
                pwv = pwn;
            }
        }
    });

#pragma unroll
    for (int r = 0; r < R; r++) {
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
// The first panel (and, with the lookahead off, every panel): rows k ..
// n-1 of columns k .. k+nb-1 loaded into registers, then factored.
template <bool FULL, int R>
__global__ void __launch_bounds__(LU_PANEL_THREADS)
    lu_panel(double *__restrict__ a, int64_t n, int64_t lda, int64_t k, int nb, int32_t *__restrict__ ipiv,
             int32_t *__restrict__ info)
{
    __shared__ PanelShared sh;
    const int tid = threadIdx.x;
    const int m = (int)(n - k);   // rows of the panel (<= LU_ROWS * LU_PANEL_THREADS, checked on the host)
    if (FULL) nb = LU_NB;
    double v[LU_ROWS][LU_NB];
    int lab[LU_ROWS];   // the row's position; rows past the panel keep positions >= m
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int i = tid + LU_PANEL_THREADS * r;
        lab[r] = i;
#pragma unroll
        for (int c = 0; c < LU_NB; c++)
            v[r][c] = (i < m && c < nb) ? a[(k + i) * lda + k + c] : 0.0;
    }
    panel_columns<FULL, R>(v, lab, a, lda, k, m, nb, ipiv, info, sh);
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
// The panel's swaps composed by one wave into one permutation of the rows
// they touch: lane q < the returned count holds touched row d and the
// original row sr whose content moves there.  pv is ipiv[k + lane] for lanes
// < nb.  Lanes 0 .. nb-1 start with rows k .. k+nb-1; pivot rows below the
// block are appended as they first appear.  j and q are uniform, so every
// exchange is a scalar read of one lane.
__device__ __forceinline__ int compose_perm(int64_t pv, int64_t k, int nb, int lane, int64_t &d, int64_t &sr)
{
    d = lane < nb ? k + lane : -1;
    sr = d;
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
    return cnt;
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
    const int64_t pv = lane < nb ? (int64_t)pv32 : 0;
    int64_t d, sr;
    const int cnt = compose_perm(pv, k, nb, lane, d, sr);
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

// ---- one launch per panel: the previous panel's update and the next panel
//
// lu_step(k) runs after panel k (columns k .. k+nb-1) has been factored.  Its
// workgroups split the work by columns, each owning its columns in every
// row, so that the row exchanges can be applied in place with no other
// workgroup reading or writing those rows' elements:
//   workgroup 0     the next panel's columns s .. s+nb2-1 (s = k + nb): the
//                   exchanges, U12 = L11^-1 A12, A22 -= L21 U12, then the
//                   factorization of panel s from its registers (the
//                   lookahead: the next panel starts as soon as its own
//                   columns are up to date);
//   the next ones   the same update on 16-column strips right of it;
//   the last ones   the exchanges alone on the columns left of the panel,
//                   one column per thread.
// Every element receives the same operations in the same order as in
// lu_swap_trsm and lu_gemm, so the factors are bitwise those of the
// three-launch schedule.
constexpr int LU_STAGE_LD = LU_NB + 2;   // staged row stride in doubles: 16-byte aligned rows, spread banks
struct StripShared {
    double L[LU_NB][LU_NB + 1];          // L11
    double U[LU_NB][LU_NB + 1];          // the strip's U12 block
    double slot[2 * LU_NB][LU_NB];       // the touched rows' contents, by composed index
    int64_t dst[2 * LU_NB], src[2 * LU_NB];
    int np;
    int16_t send[LU_MAX_N], recv[LU_MAX_N];   // per row from k: the slot it sends / receives, or -1
    double stage[LU_PANEL_THREADS * LU_STAGE_LD];   // one register slot's strip rows on their way in
};

// Columns [c0, c0 + w) of rows k .. n-1 after panel k: thread t holds rows
// k + t + LU_PANEL_THREADS r in v[r][0 .. w).  keep: store only the U12 rows
// and leave the rows below them, updated, in v.
template <int R>
__device__ __forceinline__ void strip_update(double *__restrict__ a, int64_t n, int64_t lda, int64_t k, int nb,
                                             const int32_t *__restrict__ ipiv, int64_t c0, int w, bool keep,
                                             double (&v)[LU_ROWS][LU_NB], StripShared &sh)
{
    static_assert(2 * LU_NB <= 64, "one wave composes the permutation");
    static_assert(LU_NB * LU_NB <= LU_PANEL_THREADS, "one L11 element per thread");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = (int)(n - k);
    // ---- every load that does not depend on the permutation goes first:
    // the strip's first rows, the first half of L21, L11 and the pivots.
    // Every load is unconditional (rows past the end read the last row
    // again: they are never stored, published or used as candidates), so
    // that no load waits at a branch.  A strip is called with nb == LU_NB (a
    // panel is followed by columns only when it is whole) and m > nb.
    //
    // The strip's rows go through LDS one register slot (512 rows) at a time:
    // a wavefront's load covers 8 rows (8 lanes per 128-byte row, two
    // adjacent doubles per lane) instead of 64 rows when every lane reads
    // its own row, which costs the load pipeline 8 times the cache-line
    // lookups (on one 2048 x 16 panel, 26-33 thousand cycles against 12.7).
    double g[2 * 8];
    auto load_slot = [&](auto rc) {
        constexpr int r = decltype(rc)::value;
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int e = tid + LU_PANEL_THREADS * u, row = e >> 3, ch = e & 7;
            const int i = LU_PANEL_THREADS * r + row, ic = i < m ? i : m - 1;
            const int c0c = 2 * ch < w ? 2 * ch : w - 1, c1c = 2 * ch + 1 < w ? 2 * ch + 1 : w - 1;
            g[2 * u] = a[(k + ic) * lda + c0 + c0c];
            g[2 * u + 1] = a[(k + ic) * lda + c0 + c1c];
        }
    };
    load_slot(std::integral_constant<int, 0>{});
    // L21, four panel columns per quarter, two quarters in flight: each lane
    // reads its own rows' 32 bytes (the second pair of quarters is read
    // during the first pair's products)
    double lq[2][LU_ROWS][4];
    auto load_quarter = [&](auto qc, double (&dq)[LU_ROWS][4]) {
        constexpr int q = decltype(qc)::value;
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int i = tid + LU_PANEL_THREADS * r, ic = i < nb ? nb : (i < m ? i : m - 1);   // rows of L21
#pragma unroll
            for (int t = 0; t < 4; t++) dq[r][t] = a[(k + ic) * lda + k + 4 * q + t];
        }
    };
    load_quarter(std::integral_constant<int, 0>{}, lq[0]);
    load_quarter(std::integral_constant<int, 1>{}, lq[1]);
    const int li = (tid / LU_NB) % LU_NB, lj = tid % LU_NB;
    const double lv = a[(k + (li < nb ? li : 0)) * lda + k + (lj < nb ? lj : 0)];   // clamped: every thread loads
    const int32_t pv32 = ipiv[k + (lane < nb ? lane : 0)];
    // ---- the permutation, composed by wave 0, as maps over the rows
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int i = tid + LU_PANEL_THREADS * r;
        if (i < m) {
            sh.send[i] = -1;
            sh.recv[i] = -1;
        }
    }
    if (tid < LU_NB * LU_NB) sh.L[li][lj] = (li < nb && lj < nb) ? lv : 0.0;
    int64_t d = -1, sr = -1;
    int cnt = 0;
    if (wave == 0) cnt = compose_perm(lane < nb ? (int64_t)pv32 : 0, k, nb, lane, d, sr);
    static_for<0, R>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        if (r > 0) __syncthreads();   // the previous slot has been read
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int e = tid + LU_PANEL_THREADS * u, row = e >> 3, ch = e & 7;
            sh.stage[row * LU_STAGE_LD + 2 * ch] = g[2 * u];
            sh.stage[row * LU_STAGE_LD + 2 * ch + 1] = g[2 * u + 1];
        }
        if constexpr (r + 1 < R) load_slot(std::integral_constant<int, r + 1>{});
        __syncthreads();   // (the first also orders the maps' initialisation and L11)
#pragma unroll
        for (int c = 0; c < LU_NB; c++) v[r][c] = sh.stage[tid * LU_STAGE_LD + c];
    });
    if (wave == 0 && lane < cnt) {
        sh.send[sr - k] = (int16_t)lane;
        sh.recv[d - k] = (int16_t)lane;
    }
    __syncthreads();
    // ---- the exchanges: the holders of the source rows publish them, the
    // holders of the destination rows take them
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int i = tid + LU_PANEL_THREADS * r;
        const int q = i < m ? sh.send[i] : -1;
        if (q >= 0) {
#pragma unroll
            for (int c = 0; c < LU_NB; c++) sh.slot[q][c] = v[r][c];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int i = tid + LU_PANEL_THREADS * r;
        const int q = i < m ? sh.recv[i] : -1;
        if (q >= 0) {
#pragma unroll
            for (int c = 0; c < LU_NB; c++) v[r][c] = sh.slot[q][c];
        }
    }
    // ---- U12 = L11^-1 A12: rows k .. k+nb-1 are rows r = 0 of threads
    // 0 .. nb-1; one thread per column solves in registers
    if (tid < LU_NB) {
#pragma unroll
        for (int c = 0; c < LU_NB; c++) sh.U[tid][c] = tid < nb ? v[0][c] : 0.0;
    }
    __syncthreads();
    if (tid < w) {
        double col[LU_NB];
#pragma unroll
        for (int i = 0; i < LU_NB; i++) col[i] = sh.U[i][tid];
        static_for<1, LU_NB>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
#pragma unroll
            for (int j = 0; j < i; j++) col[i] -= sh.L[i][j] * col[j];
        });
#pragma unroll
        for (int i = 0; i < LU_NB; i++) sh.U[i][tid] = col[i];
    }
    __syncthreads();
    // ---- A22 -= L21 U12, the panel's columns in order (on every row held:
    // the U12 rows, which read some row of L21, are restored afterwards;
    // rows past the end are never stored)
    static_for<0, 4>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        static_for<0, 4>([&](auto tc) {
            constexpr int t = decltype(tc)::value, j = 4 * q + t;
            if (j < nb) {   // uniform
                double u[LU_NB];
#pragma unroll
                for (int c = 0; c < LU_NB; c++) u[c] = sh.U[j][c];
#pragma unroll
                for (int r = 0; r < R; r++) {
#pragma unroll
                    for (int c = 0; c < LU_NB; c++) v[r][c] -= lq[q & 1][r][t] * u[c];
                }
            }
        });
        if constexpr (q + 2 < 4) load_quarter(std::integral_constant<int, q + 2>{}, lq[q & 1]);
    });
    if (tid < nb) {
#pragma unroll
        for (int c = 0; c < LU_NB; c++) v[0][c] = sh.U[tid][c];
    }
    // ---- store
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int i = tid + LU_PANEL_THREADS * r;
        if (i < m && (!keep || i < nb)) {
            if (w == LU_NB) {
#pragma unroll
                for (int c = 0; c < LU_NB; c++) a[(k + i) * lda + c0 + c] = v[r][c];
            } else {
#pragma unroll
                for (int c = 0; c < LU_NB; c++)
                    if (c < w) a[(k + i) * lda + c0 + c] = v[r][c];
            }
        }
    }
}

// The exchanges alone on columns [c0, min(c0 + LU_PANEL_THREADS, k)), one
// column per thread.
__device__ __forceinline__ void left_swaps(double *__restrict__ a, int64_t lda, int64_t k, int nb,
                                           const int32_t *__restrict__ ipiv, int64_t c0, StripShared &sh)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (wave == 0) {
        const int32_t pv32 = ipiv[k + (lane < nb ? lane : 0)];
        int64_t d, sr;
        const int cnt = compose_perm(lane < nb ? (int64_t)pv32 : 0, k, nb, lane, d, sr);
        if (lane < cnt) {
            sh.dst[lane] = d;
            sh.src[lane] = sr;
        }
        if (lane == 0) sh.np = cnt;
    }
    __syncthreads();
    const int64_t c = c0 + tid;
    if (c >= k) return;
    const int np = sh.np;
    double val[2 * LU_NB];
#pragma unroll
    for (int q = 0; q < 2 * LU_NB; q++) val[q] = q < np ? a[sh.src[q] * lda + c] : 0.0;
#pragma unroll
    for (int q = 0; q < 2 * LU_NB; q++)
        if (q < np && sh.dst[q] != sh.src[q]) a[sh.dst[q] * lda + c] = val[q];
}

#ifndef FB_LU_STRIP_DELAY
#define FB_LU_STRIP_DELAY 0   // pauses of 127 x 64 cycles per register slot before the strips start
#endif

// grid: nfirst (0 or 1: the next panel's workgroup), nstrips, then the
// left-column workgroups.  FULL_NEXT: the next panel is LU_NB wide.  R: the
// register slots that rows k .. n-1 need.
template <bool FULL_NEXT, int R>
__global__ void __launch_bounds__(LU_PANEL_THREADS)
    lu_step(double *__restrict__ a, int64_t n, int64_t lda, int64_t k, int nb, int32_t *__restrict__ ipiv,
            int32_t *__restrict__ info, int nfirst, int nstrips)
{
    __shared__ StripShared ss;
    __shared__ PanelShared ps;
    const int b = blockIdx.x;
    const int64_t s = k + nb;   // the first column right of panel k
    const int nb2 = (int)(n - s < LU_NB ? n - s : LU_NB);   // the next panel's width (when s < n)
    if (b < nfirst) {
        double v[LU_ROWS][LU_NB];
        strip_update<R>(a, n, lda, k, nb, ipiv, s, nb2, true, v, ss);
        // rows k + nb .. n-1 are the next panel's rows 0 .. n-s-1; the U12
        // rows above them are done
        const int m = (int)(n - k);
        int lab[LU_ROWS];
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int i = threadIdx.x + LU_PANEL_THREADS * r;
            lab[r] = (i >= nb && i < m) ? i - nb : 0x3fffffff;
        }
        panel_columns<FULL_NEXT, R>(v, lab, a, lda, s, m - nb, nb2, ipiv, info, ps);
    } else if (b < nfirst + nstrips) {
        // the strips have the length of the next panel's factorization to
        // finish; they start after a pause, so that workgroup 0's own loads
        // do not queue behind theirs
        for (int t = 0; nfirst && t < FB_LU_STRIP_DELAY * R; t++) __builtin_amdgcn_s_sleep(127);
        const int64_t c0 = s + nb2 + (int64_t)LU_NB * (b - nfirst);
        const int w = (int)(n - c0 < LU_NB ? n - c0 : LU_NB);
        double v[LU_ROWS][LU_NB];
        strip_update<R>(a, n, lda, k, nb, ipiv, c0, w, false, v, ss);
    } else {
        for (int t = 0; nfirst && t < FB_LU_STRIP_DELAY * R; t++) __builtin_amdgcn_s_sleep(127);
        left_swaps(a, lda, k, nb, ipiv, (int64_t)LU_PANEL_THREADS * (b - nfirst - nstrips), ss);
    }
}

#ifndef FB_LU_LOOKAHEAD
#define FB_LU_LOOKAHEAD 1   // 0: three launches per panel (lu_panel, lu_swap_trsm, lu_gemm)
#endif

// R = ceil(m / LU_PANEL_THREADS) register slots for m rows
template <int R> struct LuKernels {
    static void panel(bool full, double *a, int64_t n, int64_t lda, int64_t k, int nb, int32_t *ipiv, int32_t *info,
                      hipStream_t st)
    {
        if (full)
            hipLaunchKernelGGL((lu_panel<true, R>), dim3(1), dim3(LU_PANEL_THREADS), 0, st, a, n, lda, k, nb, ipiv, info);
        else
            hipLaunchKernelGGL((lu_panel<false, R>), dim3(1), dim3(LU_PANEL_THREADS), 0, st, a, n, lda, k, nb, ipiv, info);
    }
    static void step(bool full_next, unsigned grid, double *a, int64_t n, int64_t lda, int64_t k, int nb,
                     int32_t *ipiv, int32_t *info, int nfirst, int nstrips, hipStream_t st)
    {
        if (full_next)
            hipLaunchKernelGGL((lu_step<true, R>), dim3(grid), dim3(LU_PANEL_THREADS), 0, st, a, n, lda, k, nb, ipiv,
                               info, nfirst, nstrips);
        else
            hipLaunchKernelGGL((lu_step<false, R>), dim3(grid), dim3(LU_PANEL_THREADS), 0, st, a, n, lda, k, nb, ipiv,
                               info, nfirst, nstrips);
    }
};
static_assert(LU_ROWS == 4, "the launches below instantiate 1 .. 4 register slots");
static void launch_panel(int64_t m, bool full, double *a, int64_t n, int64_t lda, int64_t k, int nb, int32_t *ipiv,
                         int32_t *info, hipStream_t st)
{
    switch ((m + LU_PANEL_THREADS - 1) / LU_PANEL_THREADS) {
    case 1: LuKernels<1>::panel(full, a, n, lda, k, nb, ipiv, info, st); break;
    case 2: LuKernels<2>::panel(full, a, n, lda, k, nb, ipiv, info, st); break;
    case 3: LuKernels<3>::panel(full, a, n, lda, k, nb, ipiv, info, st); break;
    default: LuKernels<4>::panel(full, a, n, lda, k, nb, ipiv, info, st); break;
    }
}
static void launch_step(int64_t m, bool full_next, unsigned grid, double *a, int64_t n, int64_t lda, int64_t k, int nb,
                        int32_t *ipiv, int32_t *info, int nfirst, int nstrips, hipStream_t st)
{
    switch ((m + LU_PANEL_THREADS - 1) / LU_PANEL_THREADS) {
    case 1: LuKernels<1>::step(full_next, grid, a, n, lda, k, nb, ipiv, info, nfirst, nstrips, st); break;
    case 2: LuKernels<2>::step(full_next, grid, a, n, lda, k, nb, ipiv, info, nfirst, nstrips, st); break;
    case 3: LuKernels<3>::step(full_next, grid, a, n, lda, k, nb, ipiv, info, nfirst, nstrips, st); break;
    default: LuKernels<4>::step(full_next, grid, a, n, lda, k, nb, ipiv, info, nfirst, nstrips, st); break;
    }
}

hipError_t launch_lu(double *a, int64_t n, int64_t lda, int32_t *ipiv, int32_t *info, hipStream_t st)
{
    hipError_t e = hipSuccess;
    if (FB_LU_LOOKAHEAD) {
        const int nb0 = (int)(n < LU_NB ? n : LU_NB);
        if (e == hipSuccess) {
            launch_panel(n, nb0 == LU_NB, a, n, lda, 0, nb0, ipiv, info, st);
            e = hipGetLastError();
        }
        for (int64_t k = 0; e == hipSuccess && k < n; k += LU_NB) {
            const int nb = (int)(n - k < LU_NB ? n - k : LU_NB);
            const int64_t s = k + nb;
            const int nfirst = s < n ? 1 : 0;
            const int64_t nb2 = s < n ? (n - s < LU_NB ? n - s : LU_NB) : 0;
            const int nstrips = s < n ? (int)((n - s - nb2 + LU_NB - 1) / LU_NB) : 0;
            const int nleft = (int)((k + LU_PANEL_THREADS - 1) / LU_PANEL_THREADS);
            const unsigned grid = (unsigned)(nfirst + nstrips + nleft);
            if (grid == 0) continue;
            launch_step(n - k, nb2 == LU_NB || nfirst == 0, grid, a, n, lda, k, nb, ipiv, info, nfirst, nstrips, st);
            e = hipGetLastError();
        }
        return e;
    }
    for (int64_t k = 0; e == hipSuccess && k < n; k += LU_NB) {
        const int nb = (int)(n - k < LU_NB ? n - k : LU_NB);
        launch_panel(n - k, nb == LU_NB, a, n, lda, k, nb, ipiv, info, st);
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

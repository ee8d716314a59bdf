// fb_mfma.hpp -- radix-16 DFT stages on the gfx950 matrix cores with
// split-bf16 operands and fp32 accumulation.
//
// A radix-16 DFT of 16 complex values is the real product
//     [Yr; Yi] = [[Wr, -Wi], [Wi, Wr]] [xr; xi],   W[k][q] = w16^(k q),
// a 32 x 32 matrix times a 32-vector.  Sixteen such butterflies form one
// 16 x 16 x 32 matrix product per output half (Yr rows, Yi rows):
// v_mfma_f32_16x16x32_bf16 with A = 16 rows of the DFT matrix (K = 32 real
// inputs) and B = 16 butterflies (columns).
//
// Precision: every data value x is split x = hi + lo with hi = bf16(x),
// lo = bf16(x - hi) (round to nearest even); every matrix entry
// w = whi + wlo + wlo2 likewise in three terms.  The products kept are
//     wlo2 hi + wlo lo + wlo hi + whi lo + whi hi
// (smallest first), accumulated in fp32; the dropped terms are below
// 2^-24 relative, and the representation error of x (below 2^-16) dominates.
//
// Operand layout of the 16x16x32 instruction (64 lanes, lane = c + 16 g):
//   A: lane holds row (lane % 16), K elements 8 g .. 8 g + 7
//   B: lane holds column (lane % 16), K elements 8 g .. 8 g + 7
//   D: lane holds rows 4 g .. 4 g + 3 of column (lane % 16)
// The K index is assigned here as K = 8 g + 2 i + p <-> (element q = 4 g + i,
// part p: 0 real, 1 imaginary), the same for A and B, so lane (c, g) of a
// butterfly group supplies its complex inputs q = 4g..4g+3 and receives its
// complex outputs k = 4g..4g+3.
#pragma once
#include "fb_device.hpp"

namespace fb {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float cos16(int m)
{
    constexpr double c[16] = {1.0, K::C8, K::R2, K::S8, 0.0, -K::S8, -K::R2, -K::C8,
                              -1.0, -K::C8, -K::R2, -K::S8, 0.0, K::S8, K::R2, K::C8};
    return (float)c[m & 15];
}
// sin(2 pi m / 16) = cos(2 pi (m - 4) / 16)
__device__ __forceinline__ float sin16(int m) { return cos16(m - 4); }

// The DFT matrix rows this lane supplies, split into three bf16 terms.
struct MxConsts {
    bf16x8 ar[3];  // rows of Yr: [Wr, -Wi]
    bf16x8 ai[3];  // rows of Yi: [Wi,  Wr]
};

__device__ __forceinline__ void split3(float v, __bf16 &a, __bf16 &b, __bf16 &c)
{
    a = (__bf16)v;
    const float r1 = v - (float)a;
    b = (__bf16)r1;
    c = (__bf16)(r1 - (float)b);
}

__device__ __forceinline__ MxConsts mx_consts(int lane)
{
    MxConsts cs;
    const int kout = lane & 15, g = lane >> 4;
#pragma unroll
    for (int e = 0; e < 8; e++) {
        const int i = e >> 1, p = e & 1, q = 4 * g + i;
        const int m = (kout * q) & 15;
        const float wr = cos16(m), wi = -sin16(m);   // W = wr + i wi (forward)
        const float vr = p ? -wi : wr;
        const float vi = p ? wr : wi;
        __bf16 h, l, l2;
        split3(vr, h, l, l2);
        cs.ar[0][e] = h; cs.ar[1][e] = l; cs.ar[2][e] = l2;
        split3(vi, h, l, l2);
        cs.ai[0][e] = h; cs.ai[1][e] = l; cs.ai[2][e] = l2;
    }
    return cs;
}

__device__ __forceinline__ f32x4 mx_dot(const bf16x8 *w, bf16x8 xh, bf16x8 xl)
{
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[2], xh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[1], xl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[1], xh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[0], xl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[0], xh, acc, 0, 0, 0);
    return acc;
}

// One radix-16 stage of a pass on the matrix cores.
//
// Wave w takes the G groups G w .. G w + G - 1 of 16 butterflies; lane
// (c, g) of group gamma works on butterfly beta = 16 gamma + c, whose pencil
// and index b come from `map` (beta -> pp, b), and supplies its inputs
// q = 4g .. 4g+3 and receives its outputs k = 4g .. 4g+3.  The tile has
// exactly P N / (4 G) threads (G = 4: one thread per butterfly; G = 8: tiles
// of pencil pairs), so the groups cover every butterfly once; waves beyond
// the tile (`active` false, whole wavefronts) only take part in the
// barriers.
//
// Inputs come from `src` (element b + q N/16 of the pencil, twiddled here by
// w_{16 Ns}^(q (b mod Ns)) when Ns > 1) and outputs go to `dst` at the
// Stockham positions (b div Ns) 16 Ns + (b mod Ns) + k Ns.  src and dst are
// either the LDS rows of the tile or the grid in global memory; when both
// are LDS a barrier separates the reads from the writes, and when dst is LDS
// a barrier ends the stage.
template <int N, int Ns, int TWOFF, bool SRC_LDS, bool DST_LDS, int G = 4, class Map, class Src, class Dst>
__device__ __forceinline__ void mx_stage16(const float2 *__restrict__ tw, const MxConsts &A, int wave, int lane,
                                           bool active, const Map &map, const Src &src, const Dst &dst)
{
    constexpr int NBF = N / 16;
    const int c = lane & 15, g = lane >> 4;
    float2 x[G][4];
    int ppv[G], bb[G];
#pragma unroll
    for (int gi = 0; active && gi < G; gi++) {
        const int beta = 16 * (G * wave + gi) + c;
        map(beta, ppv[gi], bb[gi]);
        const int b = bb[gi];
        const auto h = src.open(ppv[gi]);
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int q = 4 * g + i;
            float2 v = src.load(h, b + q * NBF);
            if constexpr (Ns > 1) {
                if (q > 0) v = cmul(v, tw[TWOFF + (q - 1) * Ns + (b % Ns)]);
            }
            x[gi][i] = v;
        }
    }
    if constexpr (SRC_LDS && DST_LDS) __syncthreads();
#pragma unroll
    for (int gi = 0; active && gi < G; gi++) {
        bf16x8 xh, xl;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const __bf16 hr = (__bf16)x[gi][i].x, hi = (__bf16)x[gi][i].y;
            xh[2 * i] = hr;
            xh[2 * i + 1] = hi;
            xl[2 * i] = (__bf16)(x[gi][i].x - (float)hr);
            xl[2 * i + 1] = (__bf16)(x[gi][i].y - (float)hi);
        }
        const f32x4 yr = mx_dot(A.ar, xh, xl);
        const f32x4 yi = mx_dot(A.ai, xh, xl);
        const int b = bb[gi];
        const int idx = (b / Ns) * Ns * 16 + (b % Ns);
        const auto h = dst.open(ppv[gi]);
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int k = 4 * g + e;
            dst.store(h, idx + k * Ns, make_float2(yr[e], yi[e]));
        }
    }
    if constexpr (DST_LDS) __syncthreads();
}

// ---- register exchange between the vector-unit and the matrix-core layout
//
// In the vector-unit layout each lane holds one butterfly: its 16 inputs (or
// outputs) in natural order, as four blocks of four complex values.  The
// matrix-core operand layout above wants, for the 16 butterflies of row
// gamma (lanes 16 gamma .. 16 gamma + 15), block g of butterfly (gamma, c) in
// lane (c, g).  Both are related by a 4 x 4 transpose of (row, block) among
// the four lanes of a column: block j of lane (c, r) trades places with block
// r of lane (c, j).  It takes two rounds of row swaps: rows 0,1 <-> 2,3
// (v_permlane32_swap) and rows 0 <-> 1, 2 <-> 3 (v_permlane16_swap), with no
// LDS traffic, and it is its own inverse.

// a: rows 2,3 <- rows 0,1 of b; b: rows 0,1 <- rows 2,3 of a
__device__ __forceinline__ void swap_row_halves(float &a, float &b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}
// a: rows 1,3 <- rows 0,2 of b; b: rows 0,2 <- rows 1,3 of a
__device__ __forceinline__ void swap_odd_even_rows(float &a, float &b)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}

__device__ __forceinline__ void row_block_transpose(float2 (&x)[4][4])
{
#pragma unroll
    for (int j = 0; j < 2; j++) {
#pragma unroll
        for (int i = 0; i < 4; i++) {
            swap_row_halves(x[j][i].x, x[j + 2][i].x);
            swap_row_halves(x[j][i].y, x[j + 2][i].y);
        }
    }
#pragma unroll
    for (int j = 0; j < 4; j += 2) {
#pragma unroll
        for (int i = 0; i < 4; i++) {
            swap_odd_even_rows(x[j][i].x, x[j + 1][i].x);
            swap_odd_even_rows(x[j][i].y, x[j + 1][i].y);
        }
    }
}

// One radix-16 stage on the matrix cores with register input (IN_REG: the
// first stage of a pass, r[h][q] = input q of the lane's butterfly) and/or
// register output (OUT_REG: the last stage, r[h][k] = output k).  The other
// side is `src` or `dst` (LDS rows) at the positions of mx_stage16.  A lane
// holding a pencil pair carries SETS = 2 butterflies (h = 0, 1: the pair's
// two pencils, whose elements sit side by side in LDS and move as one 16-byte
// access); who(l, pp, b) gives the pencil (pair) and butterfly index b held
// by lane l of this wave.  Whole active wavefronts only; no barriers here.
template <int N, int Ns, int TWOFF, bool IN_REG, bool OUT_REG, int SETS, class Who, class Src, class Dst>
__device__ __forceinline__ void mx_stage16_reg(const float2 *__restrict__ tw, const MxConsts &A, int lane,
                                               float2 (&r)[SETS][16], const Who &who, const Src &src,
                                               const Dst &dst)
{
    static_assert(SETS == 1 || SETS == 2, "one pencil or a pencil pair per lane");
    constexpr int NBF = N / 16;
    const int c = lane & 15, g = lane >> 4;
    float2 x[SETS][4][4];
    if constexpr (IN_REG) {
#pragma unroll
        for (int h = 0; h < SETS; h++) {
#pragma unroll
            for (int j = 0; j < 4; j++) {
#pragma unroll
                for (int i = 0; i < 4; i++) x[h][j][i] = r[h][4 * j + i];
            }
            row_block_transpose(x[h]);
        }
    }
#pragma unroll
    for (int gm = 0; gm < 4; gm++) {
        int pp, b;
        who(16 * gm + c, pp, b);
        if constexpr (!IN_REG) {
            const auto hd = src.open(pp);
#pragma unroll
            for (int i = 0; i < 4; i++) {
                if constexpr (SETS == 2) src.load2(hd, b + (4 * g + i) * NBF, x[0][gm][i], x[1][gm][i]);
                else x[0][gm][i] = src.load(hd, b + (4 * g + i) * NBF);
            }
        }
        if constexpr (Ns > 1) {
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int q = 4 * g + i;
                if (q > 0) {
                    const float2 w = tw[TWOFF + (q - 1) * Ns + (b % Ns)];
#pragma unroll
                    for (int h = 0; h < SETS; h++) x[h][gm][i] = cmul(x[h][gm][i], w);
                }
            }
        }
        f32x4 yr[SETS], yi[SETS];
#pragma unroll
        for (int h = 0; h < SETS; h++) {
            bf16x8 xh, xl;
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const __bf16 hr = (__bf16)x[h][gm][i].x, hi = (__bf16)x[h][gm][i].y;
                xh[2 * i] = hr;
                xh[2 * i + 1] = hi;
                xl[2 * i] = (__bf16)(x[h][gm][i].x - (float)hr);
                xl[2 * i + 1] = (__bf16)(x[h][gm][i].y - (float)hi);
            }
            yr[h] = mx_dot(A.ar, xh, xl);
            yi[h] = mx_dot(A.ai, xh, xl);
        }
        if constexpr (OUT_REG) {
#pragma unroll
            for (int h = 0; h < SETS; h++) {
#pragma unroll
                for (int e = 0; e < 4; e++) x[h][gm][e] = make_float2(yr[h][e], yi[h][e]);
            }
        } else {
            const int idx = (b / Ns) * Ns * 16 + (b % Ns);
            const auto hd = dst.open(pp);
#pragma unroll
            for (int e = 0; e < 4; e++) {
                if constexpr (SETS == 2)
                    dst.store2(hd, idx + (4 * g + e) * Ns, make_float2(yr[0][e], yi[0][e]),
                               make_float2(yr[1][e], yi[1][e]));
                else dst.store(hd, idx + (4 * g + e) * Ns, make_float2(yr[0][e], yi[0][e]));
            }
        }
    }
    if constexpr (OUT_REG) {
#pragma unroll
        for (int h = 0; h < SETS; h++) {
            row_block_transpose(x[h]);
#pragma unroll
            for (int j = 0; j < 4; j++) {
#pragma unroll
                for (int i = 0; i < 4; i++) r[h][4 * j + i] = x[h][j][i];
            }
        }
    }
}

// Neither a source nor a destination (the register side of mx_stage16_reg).
struct MxNone {
    __device__ __forceinline__ float2 *open(int) const { return nullptr; }
    __device__ __forceinline__ float2 load(float2 *, int) const { return make_float2(0.f, 0.f); }
    __device__ __forceinline__ void store(float2 *, int, float2) const {}
};

// LDS rows of a tile as a source or destination of a matrix-core stage.
struct MxLds {
    float2 *lds;
    int LS;
    __device__ __forceinline__ float2 *open(int pp) const { return lds + pp * LS; }
    __device__ __forceinline__ float2 load(float2 *row, int pos) const { return row[lds_pos(pos)]; }
    __device__ __forceinline__ void store(float2 *row, int pos, float2 v) const { row[lds_pos(pos)] = v; }
};

// LDS rows of a tile of pencil pairs: row j holds pencils 2j and 2j + 1
// interleaved (element pos of pencil 2j + h at float2 index 2 lds_pos(pos) + h
// of the row).
struct MxLdsPair {
    float2 *lds;
    int LS;   // row stride in pairs
    __device__ __forceinline__ float2 *open(int pp) const { return lds + (pp >> 1) * 2 * LS + (pp & 1); }
    __device__ __forceinline__ float2 load(float2 *row, int pos) const { return row[2 * lds_pos(pos)]; }
    __device__ __forceinline__ void store(float2 *row, int pos, float2 v) const { row[2 * lds_pos(pos)] = v; }
    // both pencils of the pair (row opened with an even pp), one 16-byte access
    __device__ __forceinline__ void load2(float2 *row, int pos, float2 &a, float2 &b) const
    {
        const float4 v = *(const float4 *)(row + 2 * lds_pos(pos));
        a = make_float2(v.x, v.y);
        b = make_float2(v.z, v.w);
    }
    __device__ __forceinline__ void store2(float2 *row, int pos, float2 a, float2 b) const
    {
        *(float4 *)(row + 2 * lds_pos(pos)) = make_float4(a.x, a.y, b.x, b.y);
    }
};

}  // namespace fb

// fb_device.hpp -- device-side complex arithmetic and the small DFT
// butterflies (radix 2, 3, 4, 8, 16) that the pencil passes are built from.
//
// Every butterfly computes the FORWARD DFT  X[k] = sum_q a[q] w_R^(q k),
// w_R = exp(-2 pi i / R), in place and in natural order.  Inverse transforms
// use conj(DFT(conj(x))), so one set of butterflies serves both directions.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace fb {

// Two complex64 values of adjacent pencils, moved as one 16-byte access;
// every operation acts on both halves (a pair of independent transforms).
struct __attribute__((aligned(16))) c2x {
    float2 a, b;
};

template <typename V> struct vec_traits;
template <> struct vec_traits<double2> { using real = double; using tw = double2; };
template <> struct vec_traits<float2> { using real = float; using tw = float2; };
template <> struct vec_traits<c2x> { using real = float; using tw = float2; };
template <typename V> using real_t = typename vec_traits<V>::real;
// type of the twiddle factors multiplying a V
template <typename V> using tw_t = typename vec_traits<V>::tw;

template <typename V> __device__ __forceinline__ V mk(real_t<V> x, real_t<V> y) { V r; r.x = x; r.y = y; return r; }
template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return mk<V>(a.x + b.x, a.y + b.y); }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return mk<V>(a.x - b.x, a.y - b.y); }
template <typename V> __device__ __forceinline__ V cmul(V a, V b)
{
    return mk<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename V> __device__ __forceinline__ V cconj(V a) { return mk<V>(a.x, -a.y); }
template <typename V> __device__ __forceinline__ V cscale(V a, real_t<V> s) { return mk<V>(a.x * s, a.y * s); }
// a * (-i)
template <typename V> __device__ __forceinline__ V mul_mi(V a) { return mk<V>(a.y, -a.x); }

__device__ __forceinline__ c2x mk2(float2 a, float2 b) { c2x r; r.a = a; r.b = b; return r; }
__device__ __forceinline__ float2 mkf(float x, float y) { return make_float2(x, y); }
__device__ __forceinline__ c2x cadd(c2x p, c2x q) { return mk2(mkf(p.a.x + q.a.x, p.a.y + q.a.y), mkf(p.b.x + q.b.x, p.b.y + q.b.y)); }
__device__ __forceinline__ c2x csub(c2x p, c2x q) { return mk2(mkf(p.a.x - q.a.x, p.a.y - q.a.y), mkf(p.b.x - q.b.x, p.b.y - q.b.y)); }
__device__ __forceinline__ c2x cmul(c2x p, float2 w)
{
    return mk2(mkf(p.a.x * w.x - p.a.y * w.y, p.a.x * w.y + p.a.y * w.x),
               mkf(p.b.x * w.x - p.b.y * w.y, p.b.x * w.y + p.b.y * w.x));
}
__device__ __forceinline__ c2x cconj(c2x p) { return mk2(mkf(p.a.x, -p.a.y), mkf(p.b.x, -p.b.y)); }
__device__ __forceinline__ c2x cscale(c2x p, float s) { return mk2(mkf(p.a.x * s, p.a.y * s), mkf(p.b.x * s, p.b.y * s)); }
__device__ __forceinline__ c2x mul_mi(c2x p) { return mk2(mkf(p.a.y, -p.a.x), mkf(p.b.y, -p.b.x)); }

// Exact-value constants of the small roots of unity (math constants, written
// to more digits than binary64 holds; the compiler rounds them).
struct K {
    static constexpr double C8 = 0.92387953251128675612818318939678828682;  // cos(pi/8)
    static constexpr double S8 = 0.38268343236508977172845998403039886676;  // sin(pi/8)
    static constexpr double R2 = 0.70710678118654752440084436210484903928;  // sqrt(2)/2
    static constexpr double S3 = 0.86602540378443864676372317075293618347;  // sqrt(3)/2
};

// a * w where w = (c, s) given as constants
template <typename V> __device__ __forceinline__ V cmulc(V a, double c, double s)
{
    using R = real_t<V>;
    const R cr = (R)c, ci = (R)s;
    return mk<V>(a.x * cr - a.y * ci, a.x * ci + a.y * cr);
}
__device__ __forceinline__ c2x cmulc(c2x p, double c, double s) { return cmul(p, make_float2((float)c, (float)s)); }

template <typename V> __device__ __forceinline__ void dft2(V &a0, V &a1)
{
    V t = a0;
    a0 = cadd(t, a1);
    a1 = csub(t, a1);
}

// X0 = a0+a1+a2, X1 = a0 - (a1+a2)/2 - i (sqrt3/2)(a1-a2), X2 = conj-partner
template <typename V> __device__ __forceinline__ void dft3(V &a0, V &a1, V &a2)
{
    using R = real_t<V>;
    const V s = cadd(a1, a2);
    const V d = csub(a1, a2);
    const V m = csub(a0, cscale(s, (R)0.5));
    // -i * S3 * d
    const V r = cscale(mul_mi(d), (R)K::S3);
    a0 = cadd(a0, s);
    a1 = cadd(m, r);
    a2 = csub(m, r);
}

template <typename V> __device__ __forceinline__ void dft4(V &a0, V &a1, V &a2, V &a3)
{
    const V t0 = cadd(a0, a2), t1 = csub(a0, a2);
    const V t2 = cadd(a1, a3), t3 = mul_mi(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

// 8 = 4 x 2: index n = 2 n1 + n2, output k = k1 + 4 k2
template <typename V> __device__ __forceinline__ void dft8(V *a)
{
    V e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
    V o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    o1 = cmulc(o1, K::R2, -K::R2);
    o2 = mul_mi(o2);
    o3 = cmulc(o3, -K::R2, -K::R2);
    a[0] = cadd(e0, o0); a[4] = csub(e0, o0);
    a[1] = cadd(e1, o1); a[5] = csub(e1, o1);
    a[2] = cadd(e2, o2); a[6] = csub(e2, o2);
    a[3] = cadd(e3, o3); a[7] = csub(e3, o3);
}

// 16 = 4 x 4: index n = 4 n1 + n2, output k = k1 + 4 k2;
// inner twiddle w16^(n2 k1)
template <typename V> __device__ __forceinline__ void dft16(V *a)
{
    V y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; n2++) {
        V b0 = a[n2], b1 = a[4 + n2], b2 = a[8 + n2], b3 = a[12 + n2];
        dft4(b0, b1, b2, b3);
        y[n2][0] = b0; y[n2][1] = b1; y[n2][2] = b2; y[n2][3] = b3;
    }
    // w16^m = (cos(2 pi m/16), -sin(2 pi m/16))
    y[1][1] = cmulc(y[1][1], K::C8, -K::S8);   // m = 1
    y[1][2] = cmulc(y[1][2], K::R2, -K::R2);   // m = 2
    y[1][3] = cmulc(y[1][3], K::S8, -K::C8);   // m = 3
    y[2][1] = cmulc(y[2][1], K::R2, -K::R2);   // m = 2
    y[2][2] = mul_mi(y[2][2]);                 // m = 4
    y[2][3] = cmulc(y[2][3], -K::R2, -K::R2);  // m = 6
    y[3][1] = cmulc(y[3][1], K::S8, -K::C8);   // m = 3
    y[3][2] = cmulc(y[3][2], -K::R2, -K::R2);  // m = 6
    y[3][3] = cmulc(y[3][3], -K::C8, K::S8);   // m = 9
#pragma unroll
    for (int k1 = 0; k1 < 4; k1++) {
        V b0 = y[0][k1], b1 = y[1][k1], b2 = y[2][k1], b3 = y[3][k1];
        dft4(b0, b1, b2, b3);
        a[k1] = b0; a[k1 + 4] = b1; a[k1 + 8] = b2; a[k1 + 12] = b3;
    }
}

template <int R, typename V> __device__ __forceinline__ void dft(V *a)
{
    if constexpr (R == 2) dft2(a[0], a[1]);
    else if constexpr (R == 3) dft3(a[0], a[1], a[2]);
    else if constexpr (R == 4) dft4(a[0], a[1], a[2], a[3]);
    else if constexpr (R == 8) dft8(a);
    else if constexpr (R == 16) dft16(a);
    else static_assert(R == 2, "unsupported radix");
}

// Padded LDS position of element i of a pencil row: one pad slot every 16.
__device__ __forceinline__ int lds_pos(int i) { return i + (i >> 4); }

// exp(-c k2): binary64 for complex128 grids, binary32 for complex64 grids.
template <typename R> __device__ __forceinline__ R evol_factor(double c, double k2)
{
    if constexpr (std::is_same<R, double>::value) return exp(-c * k2);
    else return expf(-(float)c * (float)k2);
}

// SplitMix64 (Steele, Lea, Flood 2014) at counter c of stream `seed`:
// the (c+1)-th output of the sequential generator started at state `seed`.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Uniform on [-1, 1) from the top 53 bits (exact in binary64).
__device__ __forceinline__ double u_pm1(uint64_t h) { return (double)(h >> 11) * 0x1.0p-52 - 1.0; }

// Element i of the seeded uniform grid: re = U(seed, 2i), im = U(seed, 2i+1),
// rounded to the element's precision; a pencil pair holds elements i, i + 1.
template <typename V> __device__ __forceinline__ V uniform_elem(uint64_t seed, uint64_t i)
{
    if constexpr (std::is_same<V, c2x>::value) {
        return mk2(uniform_elem<float2>(seed, i), uniform_elem<float2>(seed, i + 1));
    } else {
        using R = real_t<V>;
        V v;
        v.x = (R)u_pm1(splitmix64_at(seed, 2 * i));
        v.y = (R)u_pm1(splitmix64_at(seed, 2 * i + 1));
        return v;
    }
}

template <int B, int E, typename F> __device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

}  // namespace fb

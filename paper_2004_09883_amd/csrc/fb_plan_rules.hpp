// fb_plan_rules.hpp -- compile-time and host-side rules of the plan: the radix
// list of an axis length and the launch geometry of a pencil pass.
//
// Radix list of n = 2^a 3^b, in the order the stages are applied to the data:
// b threes, then floor(a/4) sixteens, then 2^(a mod 4) when a mod 4 > 0
// (e.g. 512 -> 16,16,2; 768 -> 3,16,16; 64 -> 16,4; 2304 -> 3,3,16,16).
// A 3D axis may have any such length up to 4096.
#pragma once
#include <stdint.h>

namespace fb {

struct RadixPlan {
    int count;
    int r[16];
    int ns[16];     // product of the radices before stage s
    int twoff[16];  // offset of stage s in the per-axis twiddle table
    int twlen;      // total twiddle entries
};

constexpr RadixPlan radix_plan(int n)
{
    RadixPlan p{};
    p.count = 0;
    int a = 0, b = 0, m = n;
    while (m > 1 && m % 3 == 0) { m /= 3; b++; }
    while (m > 1 && m % 2 == 0) { m /= 2; a++; }
    if (m != 1 || n < 1) { p.count = -1; return p; }
    for (int i = 0; i < b; i++) p.r[p.count++] = 3;
    for (int i = 0; i < a / 4; i++) p.r[p.count++] = 16;
    if (a % 4) p.r[p.count++] = 1 << (a % 4);
    int ns = 1, off = 0;
    for (int s = 0; s < p.count; s++) {
        p.ns[s] = ns;
        p.twoff[s] = off;
        if (ns > 1) off += (p.r[s] - 1) * ns;  // entries w_{ns r}^(q k), 1<=q<r, k<ns
        ns *= p.r[s];
    }
    p.twlen = off;
    return p;
}

// True when n is an axis length the 3D passes support: 2^a 3^b, 1..4096.
constexpr bool supported_length(int64_t n)
{
    if (n < 1 || n > 4096) return false;
    int64_t m = n;
    while (m % 3 == 0) m /= 3;
    while (m % 2 == 0) m /= 2;
    return m == 1;
}

// True for the lengths 2^a and 3 * 2^a (the batched form's pass lengths).
constexpr bool supported_length_b1(int64_t n)
{
    if (n < 1 || n > 4096) return false;
    int64_t m = n;
    if (m % 3 == 0) m /= 3;
    while (m % 2 == 0) m /= 2;
    return m == 1;
}

// Threads that cooperate on one pencil: each holds about 16 elements (n/16
// threads when 16 divides n; one thread for the short lengths up to 32;
// otherwise ceil(n/16), and the stages whose butterfly count is not a
// multiple of it leave the last round part-filled).
constexpr int threads_per_pencil(int n) { return (n % 16 == 0) ? n / 16 : n <= 32 ? 1 : (n + 15) / 16; }

// Largest number of elements one thread holds over all stages.
constexpr int regs_per_thread(int n)
{
    RadixPlan p = radix_plan(n);
    int T = threads_per_pencil(n), M = 0;
    for (int s = 0; s < p.count; s++) {
        int nbf = n / p.r[s];
        int u = (nbf + T - 1) / T;
        if (u * p.r[s] > M) M = u * p.r[s];
    }
    return M;
}

// LDS row of one pencil: one pad element every 16 (breaks the stride-R
// pattern of the first exchange) and an odd total (consecutive pencils land
// on different banks).
constexpr int lds_pencil_stride(int n)
{
    int s = n + n / 16;
    return (s % 2 == 0) ? s + 1 : s;
}

// Build-time tuning knobs (defaults are the measured best on MI355X).
#ifndef FB_LDS_CONTIG_KB
#define FB_LDS_CONTIG_KB 40   // contiguous complex64 passes
#endif
#ifndef FB_LDS_CONTIG16_KB
#define FB_LDS_CONTIG16_KB 20   // contiguous complex128 passes: one wavefront per tile at n = 128, 256
#endif
#ifndef FB_LDS_CONTIG_MX_KB
#define FB_LDS_CONTIG_MX_KB 20   // contiguous complex64 matrix-core passes
#endif
// Complex128 vector-unit passes exchange real and imaginary parts through
// LDS one after the other (FB_SPLIT_EXCHANGE = 1): half the LDS per tile, so
// more tiles fit a CU; their budgets are then FB_LDS_SPLIT_*_KB.
#ifndef FB_SPLIT_EXCHANGE
#define FB_SPLIT_EXCHANGE 1
#endif
#ifndef FB_SPLIT_MAX_N
#define FB_SPLIT_MAX_N 256   // longer passes keep the one-round exchange
#endif
#ifndef FB_LDS_SPLIT_CONTIG_KB
#define FB_LDS_SPLIT_CONTIG_KB 10
#endif
#ifndef FB_LDS_SPLIT_STRIDED_KB
#define FB_LDS_SPLIT_STRIDED_KB 36
#endif
#ifndef FB_LDS_STRIDED_KB
#define FB_LDS_STRIDED_KB 72
#endif
#ifndef FB_LDS_STRIDED_MX_KB
#define FB_LDS_STRIDED_MX_KB 36   // strided complex64 matrix-core passes: half-size tiles
#endif
#ifndef FB_STRIDED_P16
#define FB_STRIDED_P16 16   // target pencils per workgroup, strided complex128
#endif
#ifndef FB_STRIDED_P8
#define FB_STRIDED_P8 32    // target pencils per workgroup, strided complex64
#endif
#ifndef FB_CONTIG_THREADS
#define FB_CONTIG_THREADS 256
#endif

constexpr int lds_budget_bytes(bool contig, int esize, bool mx = false)
{
    return !contig     ? (mx ? FB_LDS_STRIDED_MX_KB : FB_LDS_STRIDED_KB) * 1024
           : esize == 16 ? FB_LDS_CONTIG16_KB * 1024
           : mx          ? FB_LDS_CONTIG_MX_KB * 1024
                         : FB_LDS_CONTIG_KB * 1024;
}

constexpr int gcd_int(int a, int b) { return b == 0 ? a : gcd_int(b, a % b); }

// split: the tile's LDS holds one real part per element (8 bytes) at a time
constexpr bool pencils_fit(int P, int n, bool contig, int esize, bool mx = false, bool split = false)
{
    const int elem = split ? 8 : esize;
    const int budget = split ? (contig ? FB_LDS_SPLIT_CONTIG_KB : FB_LDS_SPLIT_STRIDED_KB) * 1024
                             : lds_budget_bytes(contig, esize, mx);
    return P * threads_per_pencil(n) <= 1024 && P * lds_pencil_stride(n) * elem <= budget;
}

// Pencils per workgroup.  Contiguous passes aim for 256 threads; strided
// passes aim for 16 (c128) / 32 (c64) adjacent pencils so that every row
// access is a 256-byte segment.  P is then moved to a multiple of
// 64 / gcd(T, 64) so that the workgroup is whole wavefronts, when that fits;
// finally it is capped by 1024 threads and by the LDS budget.  A
// matrix-core pass (mx) takes the budget of its own kind only where the tile
// stays whole wavefronts (which the matrix-core stages need); otherwise that
// of the vector-unit pass.
constexpr int pencils_per_wg_b(int n, bool contig, int esize, bool mx, bool split)
{
    const int T = threads_per_pencil(n);
    int P = contig ? (FB_CONTIG_THREADS / T > 0 ? FB_CONTIG_THREADS / T : 1)
                   : (esize == 16 ? FB_STRIDED_P16 : FB_STRIDED_P8);
    if (!contig && T == 1) P = 64;
    const int m = 64 / gcd_int(T, 64);
    if (P % m) {
        const int down = (P / m) * m, up = down + m;
        if (down > 0) P = down;
        else if (pencils_fit(up, n, contig, esize, mx, split)) P = up;
    }
    while (P > 1 && !pencils_fit(P, n, contig, esize, mx, split)) P /= 2;
    return P;
}
constexpr int pencils_per_wg(int n, bool contig, int esize, bool mx = false, bool split = false)
{
    if (mx) {
        const int P = pencils_per_wg_b(n, contig, esize, true, split);
        if ((P * threads_per_pencil(n)) % 64 == 0) return P;
    }
    return pencils_per_wg_b(n, contig, esize, false, split);
}

}  // namespace fb

// fb_pass.hpp -- the pencil pass: one 1D DFT of length N along one axis of
// every pencil of the grid, self-sorting (Stockham), with the elements of a
// pencil held in registers and exchanged through padded LDS between radix
// stages.
//
// Stage s (radix R, Ns = product of the earlier radices) computes, for every
// butterfly b < N/R with k = b mod Ns:
//     v[q]  = x[b + q N/R] * w_{Ns R}^(q k)          (q < R)
//     v     = DFT_R(v)
//     y[(b div Ns) Ns R + k + q Ns] = v[q]
// so the output of the last stage is in natural order; its element q of
// butterfly b lands at b + q N/R, the same pattern the first stage reads.
// The first stage therefore reads global memory and the last one writes it,
// both in that pattern; in-place use is safe because a workgroup reads its
// whole tile before any of it is written.
//
// Pencil geometry: pencil p starts at element
//     base(p) = (p / inner) * outer + (p % inner) * istep
// and has element stride `stride` (the output may use a geometry of its own,
// and a batch of equal-length transforms may place each segment of pencils
// at its own offset; see PassArgs).  A contiguous pass (z axis) has
// stride 1 and pencils back to back; a strided pass (y or x axis) takes P
// adjacent pencils per workgroup so that each row access covers P
// consecutive elements.
//
// MX (complex64 only): the radix-16 stages run on the matrix cores
// (fb_mfma.hpp).  A first matrix-core stage takes its inputs straight from
// the registers the global loads filled, and a last one leaves its outputs in
// the registers the global stores read, by a lane exchange within the
// wavefront (MxStage::regs); the others work LDS to LDS, as the vector stages
// exchange through LDS.  The remaining stages and the twiddles stay on the
// vector units.
#pragma once
#include "fb_device.hpp"
#include "fb_internal.hpp"
#include "fb_mfma.hpp"
#include "fb_plan_rules.hpp"

namespace fb {

__device__ __forceinline__ int64_t signed_k(int64_t i, int64_t n) { return (2 * i >= n) ? i - n : i; }

template <typename V, int N, bool CONTIG, bool MX = false> struct PassCfg {
    // complex128 tiles exchange real and imaginary parts in two rounds
    static constexpr bool SPLIT = FB_SPLIT_EXCHANGE && std::is_same<V, double2>::value && N <= FB_SPLIT_MAX_N;
    using LdsT = typename std::conditional<SPLIT, double, V>::type;   // LDS element
    static constexpr RadixPlan RP = radix_plan(N);
    static constexpr int T = threads_per_pencil(N);
    static constexpr int P = pencils_per_wg(N, CONTIG, (int)sizeof(V), MX, SPLIT);
    static constexpr int THREADS = P * T;
    static constexpr int M = regs_per_thread(N);
    static constexpr int LS = lds_pencil_stride(N);
    static_assert(RP.count >= 1, "pass needs at least one stage");
};

// True when the matrix-core variant exists for this length and geometry:
// complex64 (single pencils, or pencil pairs in a strided pass), a radix-16
// stage, 16 elements per thread and whole wavefronts.
template <typename V, int N, bool CONTIG> constexpr bool mx_capable()
{
    using Cfg = PassCfg<V, N, CONTIG, true>;
    bool has16 = false;
    for (int s = 0; s < Cfg::RP.count; s++) has16 = has16 || Cfg::RP.r[s] == 16;
    const bool c64 = std::is_same<V, float2>::value || (std::is_same<V, c2x>::value && !CONTIG);
    return c64 && has16 && N % 16 == 0 && Cfg::THREADS % 64 == 0;
}

// Streaming global access: the grid is read once and written once per pass,
// so loads and stores may be marked non-temporal (no allocation in the
// caches).  Whether that pays depends on the pass; measured on MI355X at
// 512x256x256 (per-pass durations, us):
//  - complex128 contiguous passes, loads and stores: 204.7 -> 177.8;
//  - complex128 strided passes, loads only: 208.9 -> 198.4 (n = 512) and
//    178.6 -> 172.3 (n = 256); stores too: no further gain;
//  - complex64 contiguous passes (vector and matrix-core): the whole block
//    3.05 -> 2.96 ms and 3.69 -> 3.58 ms;
//  - complex64 strided passes: loads 90.5 -> 103.7 (n = 512), all accesses
//    up to 40 % slower: their 256 MiB grids partly stay in the 256 MB
//    last-level cache between passes, which non-temporal accesses give up.
// The choice is per pass kind, with build-time knobs, and per launch: the
// kinds above are instantiated twice (template argument NT), and the host
// launches the non-temporal instance only when the data a pass sweeps is
// larger than the last-level cache (FB_NT_MIN_BYTES), since a grid that fits
// it (the 128 MiB 256x256x128 complex128 block, the 64 MiB 2048x2048 one)
// gains from the cache between passes: that block took 2.96 ms per 20 steps
// with non-temporal accesses against 2.69 ms without.  (A branch on a
// kernel argument instead of two instances made every pass carry both
// versions of its loads and stores; in the serving mix, where many pass
// kernels run at once, that alone raised the service p50 from 2.50 to
// 2.84 ms and the end-to-end p50 from 16 to 48 ms.)
#ifndef FB_NT_C128_CONTIG
#define FB_NT_C128_CONTIG 1
#endif
#ifndef FB_NT_C128_STRIDED_LD
#define FB_NT_C128_STRIDED_LD 1
#endif
#ifndef FB_NT_C128_STRIDED_ST
#define FB_NT_C128_STRIDED_ST 0
#endif
#ifndef FB_NT_C64_CONTIG
#define FB_NT_C64_CONTIG 1
#endif
#ifndef FB_NT_C64_STRIDED_LD
#define FB_NT_C64_STRIDED_LD 0
#endif
#ifndef FB_NT_C64_STRIDED_ST
#define FB_NT_C64_STRIDED_ST 0
#endif
template <typename V, bool CONTIG> constexpr bool nt_load()
{
    return std::is_same<V, double2>::value ? (CONTIG ? FB_NT_C128_CONTIG : FB_NT_C128_STRIDED_LD)
                                           : (CONTIG ? FB_NT_C64_CONTIG : FB_NT_C64_STRIDED_LD);
}
template <typename V, bool CONTIG> constexpr bool nt_store()
{
    return std::is_same<V, double2>::value ? (CONTIG ? FB_NT_C128_CONTIG : FB_NT_C128_STRIDED_ST)
                                           : (CONTIG ? FB_NT_C64_CONTIG : FB_NT_C64_STRIDED_ST);
}

template <bool NT, typename V> __device__ __forceinline__ V ld_stream(const V *p)
{
    if constexpr (NT) {
        typedef real_t<V> Rv __attribute__((ext_vector_type(2)));
        const Rv r = __builtin_nontemporal_load((const Rv *)p);
        return mk<V>(r.x, r.y);
    } else {
        return *p;
    }
}
template <bool NT, typename V> __device__ __forceinline__ void st_stream(V *p, V v)
{
    if constexpr (NT) {
        typedef real_t<V> Rv __attribute__((ext_vector_type(2)));
        Rv r;
        r.x = v.x;
        r.y = v.y;
        __builtin_nontemporal_store(r, (Rv *)p);
    } else {
        *p = v;
    }
}

// Element type in global memory: a pencil pair (c2x) is two adjacent
// complex64 elements read or written with one 16-byte access.
template <typename V> using elem_t = typename std::conditional<std::is_same<V, c2x>::value, float2, V>::type;

template <bool NT, typename V> __device__ __forceinline__ V ld_v(const elem_t<V> *p)
{
    if constexpr (std::is_same<V, c2x>::value) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        f4 r;
        if constexpr (NT) r = __builtin_nontemporal_load((const f4 *)p);
        else r = *(const f4 *)p;
        return mk2(make_float2(r.x, r.y), make_float2(r.z, r.w));
    } else {
        return ld_stream<NT>(p);
    }
}
template <bool NT, typename V> __device__ __forceinline__ void st_v(elem_t<V> *p, V v)
{
    if constexpr (std::is_same<V, c2x>::value) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        f4 r;
        r.x = v.a.x; r.y = v.a.y; r.z = v.b.x; r.w = v.b.y;
        if constexpr (NT) __builtin_nontemporal_store(r, (f4 *)p);
        else *(f4 *)p = r;
    } else {
        st_stream<NT>(p, v);
    }
}

// Pre-twiddle of the element at offset o from the start of its segment
// (and of the pair's second pencil, `istep` further): the factor is ptw[o].
// The table is laid out like one segment of the data, so its reads are as
// coalesced as the data's and it stays in cache across segments.
template <typename V> __device__ __forceinline__ V pre_twiddle(V v, int64_t o, int64_t istep, const void *ptw)
{
    const tw_t<V> *t = (const tw_t<V> *)ptw;
    if constexpr (std::is_same<V, c2x>::value) {
        v.a = cmul(v.a, t[o]);
        v.b = cmul(v.b, t[o + istep]);
        return v;
    } else {
        (void)istep;
        return cmul(v, t[o]);
    }
}

// Whether the first / last matrix-core stage may read / write global memory
// directly (1) or always go through LDS (0).  Direct access saves two LDS
// round trips per pass but measured slower on MI355X (512x256x256 forward +
// inverse: 405 us direct, 318 us through LDS), so it is off by default.
#ifndef FB_MX_DIRECT
#define FB_MX_DIRECT 0
#endif
// Whether the first / last matrix-core stage of a pass takes its inputs from /
// leaves its outputs in the vector-unit registers (a lane exchange, see
// mx_stage16_reg) instead of an LDS round trip.
#ifndef FB_MX_REGS
#define FB_MX_REGS 1
#endif
// The same for the last stage of pencil-pair tiles (FB_MX_REGS_OUT_PAIRS).
#ifndef FB_MX_REGS_OUT_PAIRS
#define FB_MX_REGS_OUT_PAIRS 1
#endif

template <typename V, int N, bool CONTIG, bool MX> struct MxStage {
    // whether stage s runs on the matrix cores
    static constexpr bool at(int s) { return MX && PassCfg<V, N, CONTIG>::RP.r[s] == 16; }
    // whether the first / last matrix-core stage reads / writes global memory
    // itself: contiguous passes always (16 consecutive butterflies of one
    // pencil are 16 consecutive elements), strided passes when 16 adjacent
    // pencils fit in the tile (they are 16 consecutive elements)
    static constexpr bool direct()
    {
        return FB_MX_DIRECT && MX && std::is_same<V, float2>::value && (CONTIG || PassCfg<V, N, CONTIG, MX>::P % 16 == 0);
    }
    static constexpr bool regs() { return FB_MX_REGS && MX && !direct(); }
    static constexpr bool regs_out() { return regs() && (FB_MX_REGS_OUT_PAIRS || !std::is_same<V, c2x>::value); }
};

// Butterfly numbering of the matrix-core stages: beta -> (pencil, b).
template <int NBF> struct MxMapContig {
    __device__ __forceinline__ void operator()(int beta, int &pp, int &b) const
    {
        pp = beta / NBF;
        b = beta % NBF;
    }
};
template <int P> struct MxMapStrided {
    __device__ __forceinline__ void operator()(int beta, int &pp, int &b) const
    {
        pp = beta % P;
        b = beta / P;
    }
};

// Global memory as the source of the first matrix-core stage (complex64):
// element pos of pencil pp of the tile, with the fused evolution factor and
// the conjugation of an inverse applied as it is loaded.
struct MxGlobalIn {
    const PassArgs *a;
    int64_t tile;
    int P;
    const float *gtab;
    struct H {
        const float2 *p;
        float g;
        bool ok;
    };
    __device__ __forceinline__ H open(int pp) const
    {
        H h{nullptr, 1.f, false};
        const int64_t pq = tile * P + pp;
        if (pq >= a->npencils) return h;
        int64_t s0 = 0, l = pq;
        if (a->seg_off) {
            s0 = a->seg_off[pq / a->seg_pencils];
            l = pq % a->seg_pencils;
        }
        h.p = (const float2 *)a->in + s0 + (l / a->inner) * a->outer + (l % a->inner) * a->istep;
        if (a->evolve) {
            const int64_t pa = pq / a->ev_d, pb = pq % a->ev_d;
            const double ka = (double)signed_k(pa, a->ev_la), kb = (double)signed_k(pb, a->ev_lb);
            h.g = evol_factor<float>(a->ev_c, ka * ka + kb * kb);
        }
        h.ok = true;
        return h;
    }
    __device__ __forceinline__ float2 load(const H &h, int pos) const
    {
        if (!h.ok) return make_float2(0.f, 0.f);
        float2 v = a->gen ? uniform_elem<float2>(a->gen_seed, (uint64_t)(h.p - (const float2 *)a->in) +
                                                                   (uint64_t)pos * (uint64_t)a->stride)
                          : ld_stream<false>(h.p + (int64_t)pos * a->stride);
        if (a->evolve) v = cscale(v, h.g * gtab[pos]);
        if (a->inv) v = cconj(v);
        return v;
    }
};

// Global memory as the destination of the last matrix-core stage.
struct MxGlobalOut {
    const PassArgs *a;
    int64_t tile;
    int P;
    struct H {
        float2 *p;
        bool ok;
    };
    __device__ __forceinline__ H open(int pp) const
    {
        H h{nullptr, false};
        const int64_t pq = tile * P + pp;
        if (pq >= a->npencils) return h;
        int64_t s0 = 0, l = pq;
        if (a->seg_off) {
            s0 = a->seg_off[pq / a->seg_pencils];
            l = pq % a->seg_pencils;
        }
        h.p = (float2 *)a->out + s0 +
              (a->ostride ? (l / a->oinner) * a->oouter + (l % a->oinner) * a->oistep
                          : (l / a->inner) * a->outer + (l % a->inner) * a->istep);
        h.ok = true;
        return h;
    }
    __device__ __forceinline__ void store(const H &h, int pos, float2 v) const
    {
        if (!h.ok) return;
        if (a->inv) v = cconj(v);
        if (a->scale != 1.0) v = cscale(v, (float)a->scale);
        st_stream<false>(h.p + (int64_t)pos * (a->ostride ? a->ostride : a->stride), v);
    }
};

// Tile-contiguous output of a strided vector-unit pass (PassArgs::otile):
// the last stage's outputs go to LDS in natural order, then the workgroup
// writes the tile's block of P x N elements with consecutive threads on
// consecutive elements.  On entry the LDS rows are free (the last stage has
// read its inputs and passed a barrier).
template <typename V, int N, bool CONTIG, bool NT, int M>
__device__ __forceinline__ void store_tile_contiguous(const PassArgs &a, int64_t tile, int tid, bool active,
                                                      bool valid, int t, V *row, V *lds, const V (&v)[M])
{
    using Cfg = PassCfg<V, N, CONTIG>;
    using R = real_t<V>;
    constexpr RadixPlan RP = Cfg::RP;
    constexpr int T = Cfg::T, P = Cfg::P, LS = Cfg::LS;
    constexpr int RL = RP.r[RP.count - 1];
    constexpr int NBF = N / RL;
    constexpr int U = (NBF + T - 1) / T;
    constexpr bool PAIR = std::is_same<V, c2x>::value;
    constexpr int UNIT = PAIR ? 2 : 1;
    if (valid) {
        const R sc = (R)a.scale;
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int b = t + T * u;
            if (NBF % T == 0 || b < NBF) {
#pragma unroll
                for (int q = 0; q < RL; q++) {
                    V o = v[u * RL + q];
                    if (a.inv) o = cconj(o);
                    if (a.scale != 1.0) o = cscale(o, sc);
                    row[lds_pos(b + q * NBF)] = o;
                }
            }
        }
    }
    __syncthreads();
    const int64_t p0 = tile * P * UNIT;   // first pencil of the tile
    if (active && p0 < a.npencils) {
        int64_t seg0 = 0, lp0 = p0;
        if (a.seg_off) {
            seg0 = a.seg_off[p0 / a.seg_pencils];
            lp0 = p0 % a.seg_pencils;
        }
        const int64_t ob = seg0 + (a.ostride ? (lp0 / a.oinner) * a.oouter + (lp0 % a.oinner) * a.oistep
                                             : (lp0 / a.inner) * a.outer + (lp0 % a.inner) * a.istep);
        const int64_t np = a.npencils - p0 < P * UNIT ? a.npencils - p0 : P * UNIT;
        const int count = (int)np * N;
        elem_t<V> *o = (elem_t<V> *)a.out + ob;
        auto store_all = [&](auto ntc) {
            constexpr bool NTA = decltype(ntc)::value;
            for (int i = tid; i < count; i += Cfg::THREADS) {
                const int j = i / N, k = i - (i / N) * N;
                if constexpr (PAIR) {
                    const c2x &e = lds[(j >> 1) * LS + lds_pos(k)];
                    st_stream<NTA>(o + i, (j & 1) ? e.b : e.a);
                } else {
                    st_stream<NTA>(o + i, lds[j * LS + lds_pos(k)]);
                }
            }
        };
        store_all(std::integral_constant<bool, NT && nt_store<V, CONTIG>()>{});
    }
}

#ifdef FB_WAVES_PER_EU
#define FB_OCCUPANCY __attribute__((amdgpu_waves_per_eu(FB_WAVES_PER_EU)))
#else
#define FB_OCCUPANCY
#endif

// One tile of a pass: P pencils of length N.  `lds` holds P * LS elements,
// `gtab` N reals (contiguous passes).  The caller may run the tile on a
// workgroup larger than the tile's THREADS (the persistent batch kernel):
// the extra threads only take part in the barriers.
template <typename V, int N, bool CONTIG, bool MX, bool MULTI = false, bool NT = false>
__device__ __forceinline__ void pass_tile(const PassArgs &a, int64_t tile, int tid, V *lds, real_t<V> *gtab)
{
    using Cfg = PassCfg<V, N, CONTIG, MX>;
    using R = real_t<V>;
    constexpr RadixPlan RP = Cfg::RP;
    constexpr int T = Cfg::T, P = Cfg::P, M = Cfg::M, LS = Cfg::LS;
    constexpr int NST = RP.count;
    static_assert(!MX || mx_capable<V, N, CONTIG>(), "no matrix-core variant for this pass");
    constexpr bool PAIR = std::is_same<V, c2x>::value;   // each unit is two adjacent pencils
    static_assert(!PAIR || !CONTIG, "pencil pairs are for strided passes");
    static_assert(!MULTI || CONTIG, "multi-output passes are contiguous evolve passes");
    using E = elem_t<V>;
    using TW = tw_t<V>;

    const bool active = tid < Cfg::THREADS;
    const int t = CONTIG ? tid % T : tid / P;
    const int pp = CONTIG ? tid / T : tid % P;
    const int64_t p = (tile * P + pp) * (PAIR ? 2 : 1);   // (first) pencil of this thread
    const bool valid = active && p < a.npencils;
    int64_t seg0 = 0, lp = p;   // segment start and local pencil index
    if (a.seg_off && valid) {
        seg0 = a.seg_off[p / a.seg_pencils];
        lp = p % a.seg_pencils;
    }
    const int64_t base = valid ? seg0 + (lp / a.inner) * a.outer + (lp % a.inner) * a.istep : 0;
    const bool ogeom = a.ostride != 0;
    const int64_t obase = !valid ? 0 : ogeom ? seg0 + (lp / a.oinner) * a.oouter + (lp % a.oinner) * a.oistep : base;
    const E *__restrict__ gin = (const E *)a.in + base;
    E *__restrict__ gout = (E *)a.out + obase;
    const TW *__restrict__ tw = (const TW *)a.tw;
    const int64_t S = a.stride;
    const int64_t OS = ogeom ? a.ostride : a.stride;
    V *row = lds + (active ? pp : 0) * LS;

    V v[M];
    [[maybe_unused]] V v0[MULTI ? M : 1];   // the loaded spectrum, kept for every output

    using MXS = MxStage<V, N, CONTIG, MX>;
    // first / last matrix-core stage reads / writes global memory itself
    constexpr bool MX_IN = MXS::at(0) && MXS::direct() && !MULTI;
    constexpr bool MX_OUT = MXS::at(NST - 1) && MXS::direct() && !MULTI;
    // first / last matrix-core stage works on the registers
    constexpr bool MX_RIN = MXS::at(0) && MXS::regs();
    constexpr bool MX_ROUT = MXS::at(NST - 1) && MXS::regs_out();
    constexpr int R0 = RP.r[0];
    constexpr int NBF0 = N / R0;
    constexpr int U0 = (NBF0 + T - 1) / T;

    // ---- optional fused evolution factor (contiguous only): a table along
    // the pencil times a factor of the pencil's own two wavenumbers.  A
    // single-output pass builds it before its loads (fewer live registers);
    // a multi-output pass once per output.
    R gab = (R)1;
    [[maybe_unused]] auto evolve_factors = [&](double c) {
        for (int i = tid; active && i < N; i += Cfg::THREADS) {
            const double k = (double)signed_k(i, N);
            gtab[i] = evol_factor<R>(c, k * k);
        }
        if (valid) {
            const int64_t pa = p / a.ev_d, pb = p % a.ev_d;
            const double ka = (double)signed_k(pa, a.ev_la), kb = (double)signed_k(pb, a.ev_lb);
            gab = evol_factor<R>(c, ka * ka + kb * kb);
        }
        __syncthreads();
    };
    if constexpr (CONTIG && !MULTI) {
        if (a.evolve) evolve_factors(a.ev_c);
    }

    // ---- stage 0 input: global loads (or generated values), pattern b + q N/R0
    // global loads, non-temporal when this pass kind gains from it and the
    // grid is larger than the last-level cache (PassArgs::nt)
    auto load_all = [&](auto ntc) {
        constexpr bool NTA = decltype(ntc)::value;
#pragma unroll
        for (int u = 0; u < U0; u++) {
            const int b = t + T * u;
            if (NBF0 % T == 0 || b < NBF0) {
#pragma unroll
                for (int q = 0; q < R0; q++) v[u * R0 + q] = ld_v<NTA, V>(gin + (int64_t)(b + q * NBF0) * S);
            }
        }
    };
    if (valid && !MX_IN) {
        if (a.gen) {
#pragma unroll
            for (int u = 0; u < U0; u++) {
                const int b = t + T * u;
                if (NBF0 % T == 0 || b < NBF0) {
#pragma unroll
                    for (int q = 0; q < R0; q++)
                        v[u * R0 + q] = uniform_elem<V>(a.gen_seed, (uint64_t)(base + (int64_t)(b + q * NBF0) * S));
                }
            }
        } else {
            load_all(std::integral_constant<bool, NT && nt_load<V, CONTIG>()>{});
        }
    }
    if constexpr (MULTI) {
#pragma unroll
        for (int i = 0; i < M; i++) v0[i] = v[i];
    }

    [[maybe_unused]] MxConsts mxc;
    if constexpr (MX) mxc = mx_consts(tid & 63);

    auto body = [&](int rep) {
    if constexpr (MULTI) {
        if (rep > 0) {
#pragma unroll
            for (int i = 0; i < M; i++) v[i] = v0[i];
            __syncthreads();   // the previous output's LDS and factor-table readers are done
        }
    }

    if constexpr (MULTI) {
        if (a.evolve) evolve_factors(a.ev_cs[rep]);
    }

    // ---- stage 0 input: evolution factor, conjugation, pre-twiddle
    {
        constexpr int NBF = NBF0;
        constexpr int U = U0;
        if (valid && !MX_IN) {
            if constexpr (CONTIG) {
                if (a.evolve) {
#pragma unroll
                    for (int u = 0; u < U; u++) {
                        const int b = t + T * u;
                        if (NBF % T == 0 || b < NBF) {
#pragma unroll
                            for (int q = 0; q < R0; q++) v[u * R0 + q] = cscale(v[u * R0 + q], gab * gtab[b + q * NBF]);
                        }
                    }
                }
            }
            if (a.inv) {
#pragma unroll
                for (int i = 0; i < M; i++) v[i] = cconj(v[i]);
            }
            // pre-twiddle after the conjugation: an inverse is conj(DFT(conj(x))) as a whole
            if (a.ptw) {
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const int b = t + T * u;
                    if (NBF % T == 0 || b < NBF) {
#pragma unroll
                        for (int q = 0; q < R0; q++) {
                            const int64_t o = (base - seg0) + (int64_t)(b + q * NBF) * S;
                            v[u * R0 + q] = pre_twiddle(v[u * R0 + q], o, a.istep, a.ptw);
                        }
                    }
                }
            }
        }
        if constexpr (MXS::at(0) && !MX_IN && !MX_RIN) {
            // the matrix-core stage reads its inputs from LDS in natural order
#pragma unroll
            for (int u = 0; active && u < U; u++) {
                const int b = t + T * u;
                if (NBF % T == 0 || b < NBF) {
#pragma unroll
                    for (int q = 0; q < R0; q++) row[lds_pos(b + q * NBF)] = v[u * R0 + q];
                }
            }
            __syncthreads();
        }
    }

    static_for<0, NST>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        constexpr int Rr = RP.r[s];
        constexpr int Ns = RP.ns[s];
        constexpr int NBF = N / Rr;
        constexpr int U = (NBF + T - 1) / T;

        if constexpr (MxStage<V, N, CONTIG, MX>::at(s)) {
            if constexpr (s > 0 && !MxStage<V, N, CONTIG, MX>::at(s - 1)) {
                // previous (vector) stage's outputs go to LDS
                constexpr int Rp = RP.r[s - 1];
                constexpr int Nsp = RP.ns[s - 1];
                constexpr int NBFp = N / Rp;
                constexpr int Up = (NBFp + T - 1) / T;
#pragma unroll
                for (int u = 0; active && u < Up; u++) {
                    const int b = t + T * u;
                    if (NBFp % T == 0 || b < NBFp) {
                        const int idx = (b / Nsp) * Nsp * Rp + (b % Nsp);
#pragma unroll
                        for (int q = 0; q < Rp; q++) row[lds_pos(idx + q * Nsp)] = v[u * Rp + q];
                    }
                }
                __syncthreads();
            }
            constexpr bool RIN = (s == 0) && MX_RIN;
            constexpr bool ROUT = (s == NST - 1) && MX_ROUT;
            if constexpr (RIN || ROUT) {
                // lane l of the wave holds the butterfly of thread (tid & ~63) + l
                constexpr int SETS = PAIR ? 2 : 1;
                float2 r[SETS][16];
                if constexpr (RIN) {
#pragma unroll
                    for (int q = 0; q < 16; q++) {
                        if constexpr (PAIR) {
                            r[0][q] = v[q].a;
                            r[1][q] = v[q].b;
                        } else if constexpr (std::is_same<V, float2>::value) {
                            r[0][q] = v[q];
                        }
                    }
                }
                auto who = [&](int l, int &pq, int &b) {
                    const int tt = (tid & ~63) + l;
                    b = CONTIG ? tt % T : tt / P;
                    const int pl = CONTIG ? tt / T : tt % P;
                    pq = PAIR ? 2 * pl : pl;   // a pair's first pencil
                };
                if (active) {
                    if constexpr (PAIR) {
                        const MxLdsPair L{(float2 *)lds, LS};
                        mx_stage16_reg<N, Ns, RP.twoff[s], RIN, ROUT, SETS>((const float2 *)tw, mxc, tid & 63, r,
                                                                            who, L, L);
                    } else {
                        const MxLds L{(float2 *)lds, LS};
                        mx_stage16_reg<N, Ns, RP.twoff[s], RIN, ROUT, SETS>((const float2 *)tw, mxc, tid & 63, r,
                                                                            who, L, L);
                    }
                }
                if constexpr (ROUT) {
#pragma unroll
                    for (int q = 0; q < 16; q++) {
                        if constexpr (PAIR) {
                            v[q].a = r[0][q];
                            v[q].b = r[1][q];
                        } else if constexpr (std::is_same<V, float2>::value) {
                            v[q] = r[0][q];
                        }
                    }
                } else {
                    __syncthreads();   // the outputs are in LDS for the next stage
                }
            } else if constexpr (std::is_same<V, float2>::value) {
                constexpr bool IN_G = (s == 0) && MX_IN;
                constexpr bool OUT_G = (s == NST - 1) && MX_OUT;
                const MxLds ldsio{(float2 *)lds, LS};
                const MxGlobalIn gin_io{&a, tile, P, (const float *)gtab};
                const MxGlobalOut gout_io{&a, tile, P};
                auto run = [&](const auto &map) {
                    if constexpr (IN_G && OUT_G)
                        mx_stage16<N, Ns, RP.twoff[s], false, false>((const float2 *)tw, mxc, tid >> 6, tid & 63,
                                                                     active, map, gin_io, gout_io);
                    else if constexpr (IN_G)
                        mx_stage16<N, Ns, RP.twoff[s], false, true>((const float2 *)tw, mxc, tid >> 6, tid & 63,
                                                                    active, map, gin_io, ldsio);
                    else if constexpr (OUT_G)
                        mx_stage16<N, Ns, RP.twoff[s], true, false>((const float2 *)tw, mxc, tid >> 6, tid & 63,
                                                                    active, map, ldsio, gout_io);
                    else
                        mx_stage16<N, Ns, RP.twoff[s], true, true>((const float2 *)tw, mxc, tid >> 6, tid & 63,
                                                                   active, map, ldsio, ldsio);
                };
                // strided tiles with direct access number butterflies pencil-fastest so that
                // the 16 lanes of a group touch 16 adjacent pencils (consecutive addresses)
                if constexpr (!CONTIG && MXS::direct()) run(MxMapStrided<P>{});
                else run(MxMapContig<N / 16>{});
            } else if constexpr (PAIR) {
                // a tile of P pencil pairs is 2P pencils of complex64 for the matrix
                // cores: each wave takes twice the butterfly groups
                const MxLdsPair ldsp{(float2 *)lds, LS};
                mx_stage16<N, Ns, RP.twoff[s], true, true, 8>((const float2 *)tw, mxc, tid >> 6, tid & 63, active,
                                                              MxMapContig<N / 16>{}, ldsp, ldsp);
            }
        } else {
            if constexpr (Cfg::SPLIT) {
              if constexpr (s > 0) {
                // exchange of a complex128 tile in two rounds through LDS rows
                // of reals: real parts, then imaginary parts (a round's reads
                // change only its own part of v, so the other part still holds
                // the previous stage's outputs for the next round's writes)
                constexpr int Rp = RP.r[s - 1];
                constexpr int Nsp = RP.ns[s - 1];
                constexpr int NBFp = N / Rp;
                constexpr int Up = (NBFp + T - 1) / T;
                R *rrow = (R *)lds + (active ? pp : 0) * LS;
                static_for<0, 2>([&](auto hc) {
                    constexpr int part = decltype(hc)::value;
#pragma unroll
                    for (int u = 0; active && u < Up; u++) {
                        const int b = t + T * u;
                        if (NBFp % T == 0 || b < NBFp) {
                            const int idx = (b / Nsp) * Nsp * Rp + (b % Nsp);
#pragma unroll
                            for (int q = 0; q < Rp; q++)
                                rrow[lds_pos(idx + q * Nsp)] = part ? v[u * Rp + q].y : v[u * Rp + q].x;
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (int u = 0; active && u < U; u++) {
                        const int b = t + T * u;
                        if (NBF % T == 0 || b < NBF) {
#pragma unroll
                            for (int q = 0; q < Rr; q++) {
                                if constexpr (part) v[u * Rr + q].y = rrow[lds_pos(b + q * NBF)];
                                else v[u * Rr + q].x = rrow[lds_pos(b + q * NBF)];
                            }
                        }
                    }
                    __syncthreads();
                });
              }
            } else if constexpr (s > 0) {
                if constexpr (!MxStage<V, N, CONTIG, MX>::at(s - 1)) {
                    // exchange: write the previous stage's outputs
                    constexpr int Rp = RP.r[s - 1];
                    constexpr int Nsp = RP.ns[s - 1];
                    constexpr int NBFp = N / Rp;
                    constexpr int Up = (NBFp + T - 1) / T;
#pragma unroll
                    for (int u = 0; active && u < Up; u++) {
                        const int b = t + T * u;
                        if (NBFp % T == 0 || b < NBFp) {
                            const int idx = (b / Nsp) * Nsp * Rp + (b % Nsp);
#pragma unroll
                            for (int q = 0; q < Rp; q++) row[lds_pos(idx + q * Nsp)] = v[u * Rp + q];
                        }
                    }
                    __syncthreads();
                }
                // read this stage's inputs
#pragma unroll
                for (int u = 0; active && u < U; u++) {
                    const int b = t + T * u;
                    if (NBF % T == 0 || b < NBF) {
#pragma unroll
                        for (int q = 0; q < Rr; q++) v[u * Rr + q] = row[lds_pos(b + q * NBF)];
                    }
                }
                __syncthreads();
            }

#pragma unroll
            for (int u = 0; active && u < U; u++) {
                const int b = t + T * u;
                if (NBF % T == 0 || b < NBF) {
                    V *w = v + u * Rr;
                    if constexpr (Ns > 1) {
                        const int k = b % Ns;
#pragma unroll
                        for (int q = 1; q < Rr; q++) w[q] = cmul(w[q], tw[RP.twoff[s] + (q - 1) * Ns + k]);
                    }
                    dft<Rr>(w);
                }
            }
        }
    });

    // ---- last stage output: global stores, pattern b + q N/R
    {
        constexpr int RL = RP.r[NST - 1];
        constexpr int NBF = N / RL;
        constexpr int U = (NBF + T - 1) / T;
        if constexpr (MXS::at(NST - 1) && !MX_OUT && !MX_ROUT) {
            // the matrix-core stage left the result in LDS in natural order
#pragma unroll
            for (int u = 0; active && u < U; u++) {
                const int b = t + T * u;
                if (NBF % T == 0 || b < NBF) {
#pragma unroll
                    for (int q = 0; q < RL; q++) v[u * RL + q] = row[lds_pos(b + q * NBF)];
                }
            }
        }
        if constexpr (!CONTIG && !MX && !Cfg::SPLIT) {
            if (a.otile) {   // uniform over the workgroup
                store_tile_contiguous<V, N, CONTIG, NT>(a, tile, tid, active, valid, t, row, lds, v);
                return;
            }
        }
        auto store_all = [&](auto ntc) {
            constexpr bool NTA = decltype(ntc)::value;
            const R sc = (R)a.scale;
            E *__restrict__ go = MULTI ? gout + rep * a.out_step : gout;
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int b = t + T * u;
                if (NBF % T == 0 || b < NBF) {
#pragma unroll
                    for (int q = 0; q < RL; q++) {
                        V o = v[u * RL + q];
                        if (a.inv) o = cconj(o);
                        if (a.scale != 1.0) o = cscale(o, sc);
                        if constexpr (PAIR) {
                            if (a.opair_step) {   // the pair's outputs are not adjacent
                                st_stream<NTA>(go + (int64_t)(b + q * NBF) * OS, o.a);
                                st_stream<NTA>(go + (int64_t)(b + q * NBF) * OS + a.opair_step, o.b);
                                continue;
                            }
                        }
                        st_v<NTA, V>(go + (int64_t)(b + q * NBF) * OS, o);
                    }
                }
            }
        };
        if (valid && !MX_OUT) {
            store_all(std::integral_constant<bool, NT && nt_store<V, CONTIG>()>{});
        }
    }
    };   // outputs
    if constexpr (MULTI) {
        for (int rep = 0; rep < a.nout; rep++) body(rep);
    } else {
        body(0);
    }
}

// Tile of workgroup b of a grid of nb workgroups.  The dispatcher deals
// workgroups to the 8 XCDs (each with its own L2) round robin, so workgroup b
// runs on XCD b mod 8; with REMAP the tiles are renumbered so that each XCD
// takes one contiguous run of tiles (consecutive tiles on one XCD share L2
// lines and DRAM pages at the tile edges).  A bijection on [0, nb).
// Measured per pass kind on MI355X (512x256x256): the strided complex64
// matrix-core passes gain (with half-size tiles, 36 KB, the 256-point pass
// 117 -> 107 us), the complex128 passes lose (the 512-point x pass 201 ->
// 217 us), so it is a per-kind build knob.
#ifndef FB_XCD_REMAP
#define FB_XCD_REMAP 0               // every pass
#endif
#ifndef FB_XCD_REMAP_MX_STRIDED
#define FB_XCD_REMAP_MX_STRIDED 1    // strided matrix-core passes
#endif
constexpr int kXcds = 8;
template <bool REMAP> __device__ __forceinline__ int64_t tile_of_block(int64_t b, int64_t nb)
{
    if constexpr (!REMAP) {
        (void)nb;
        return b;
    } else {
        const int64_t q = nb / kXcds, r = nb % kXcds;
        const int64_t x = b % kXcds, i = b / kXcds;
        return x * q + (x < r ? x : r) + i;
    }
}
// Strided tiles whose row segment (P adjacent pencils) is narrower than an
// L2 line share lines with their neighbours: those are remapped too
// (FB_XCD_REMAP_NARROW).
#ifndef FB_XCD_REMAP_NARROW
#define FB_XCD_REMAP_NARROW 1
#endif
template <typename V, int N, bool CONTIG, bool MX> constexpr bool xcd_remap()
{
    constexpr int seg_bytes = PassCfg<V, N, CONTIG, MX>::P * (int)sizeof(V);
    return FB_XCD_REMAP || (FB_XCD_REMAP_MX_STRIDED && MX && !CONTIG) ||
           (FB_XCD_REMAP_NARROW && !CONTIG && seg_bytes < 128);
}

// True when the pass kind has a non-temporal instance (NT = true).
template <typename V, bool CONTIG> constexpr bool has_nt() { return nt_load<V, CONTIG>() || nt_store<V, CONTIG>(); }

template <typename V, int N, bool CONTIG, bool MX, bool NT = false>
__global__ void __launch_bounds__((PassCfg<V, N, CONTIG, MX>::THREADS)) FB_OCCUPANCY fft_pass(PassArgs a)
{
    using Cfg = PassCfg<V, N, CONTIG, MX>;
    __shared__ typename Cfg::LdsT lds[Cfg::P * Cfg::LS];
    __shared__ real_t<V> gtab[CONTIG ? N : 1];
    pass_tile<V, N, CONTIG, MX, false, NT>(a, tile_of_block<xcd_remap<V, N, CONTIG, MX>()>(blockIdx.x, gridDim.x),
                                           threadIdx.x, (V *)lds, gtab);
}

// Contiguous evolve pass with several outputs: the tile's spectrum is read
// once and output j (evolution constant ev_cs[j]) is written at
// out + j out_step, for j < nout.
template <typename V, int N, bool MX, bool NT = false>
__global__ void __launch_bounds__((PassCfg<V, N, true, MX>::THREADS)) FB_OCCUPANCY fft_pass_multi(PassArgs a)
{
    using Cfg = PassCfg<V, N, true, MX>;
    __shared__ typename Cfg::LdsT lds[Cfg::P * Cfg::LS];
    __shared__ real_t<V> gtab[N];
    pass_tile<V, N, true, MX, true, NT>(a, tile_of_block<xcd_remap<V, N, true, MX>()>(blockIdx.x, gridDim.x),
                                        threadIdx.x, (V *)lds, gtab);
}

}  // namespace fb

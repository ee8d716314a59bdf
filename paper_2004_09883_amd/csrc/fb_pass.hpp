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
// and has element stride `stride`.  A contiguous pass (z axis) has
// stride 1 and pencils back to back; a strided pass (y or x axis) takes P
// adjacent pencils per workgroup so that each row access covers P
// consecutive elements.
//
// MX (complex64 only): the radix-16 stages run on the matrix cores
// (fb_mfma.hpp), LDS to LDS; the other stages, the twiddles and the global
// loads and stores stay on the vector units.
#pragma once
#include "fb_device.hpp"
#include "fb_internal.hpp"
#include "fb_mfma.hpp"
#include "fb_plan_rules.hpp"

namespace fb {

__device__ __forceinline__ int64_t signed_k(int64_t i, int64_t n) { return (2 * i >= n) ? i - n : i; }

template <typename V, int N, bool CONTIG> struct PassCfg {
    static constexpr RadixPlan RP = radix_plan(N);
    static constexpr int T = threads_per_pencil(N);
    static constexpr int P = pencils_per_wg(N, CONTIG, (int)sizeof(V));
    static constexpr int THREADS = P * T;
    static constexpr int M = regs_per_thread(N);
    static constexpr int LS = lds_pencil_stride(N);
    static_assert(RP.count >= 1, "pass needs at least one stage");
};

// True when the matrix-core variant exists for this length and geometry:
// complex64, a radix-16 stage, 16 elements per thread and whole wavefronts.
template <typename V, int N, bool CONTIG> constexpr bool mx_capable()
{
    using Cfg = PassCfg<V, N, CONTIG>;
    bool has16 = false;
    for (int s = 0; s < Cfg::RP.count; s++) has16 = has16 || Cfg::RP.r[s] == 16;
    return sizeof(V) == 8 && has16 && N % 16 == 0 && Cfg::THREADS % 64 == 0;
}

template <typename V, int N, bool CONTIG, bool MX> struct MxStage {
    // whether stage s runs on the matrix cores
    static constexpr bool at(int s) { return MX && PassCfg<V, N, CONTIG>::RP.r[s] == 16; }
};

template <typename V, int N, bool CONTIG, bool MX>
__global__ void __launch_bounds__((PassCfg<V, N, CONTIG>::THREADS)) fft_pass(PassArgs a)
{
    using Cfg = PassCfg<V, N, CONTIG>;
    using R = real_t<V>;
    constexpr RadixPlan RP = Cfg::RP;
    constexpr int T = Cfg::T, P = Cfg::P, M = Cfg::M, LS = Cfg::LS;
    constexpr int NST = RP.count;
    static_assert(!MX || mx_capable<V, N, CONTIG>(), "no matrix-core variant for this pass");

    __shared__ V lds[P * LS];
    __shared__ R gtab[CONTIG ? N : 1];

    const int tid = threadIdx.x;
    const int t = CONTIG ? tid % T : tid / P;
    const int pp = CONTIG ? tid / T : tid % P;
    const int64_t p = (int64_t)blockIdx.x * P + pp;
    const bool valid = p < a.npencils;
    const int64_t base = valid ? (p / a.inner) * a.outer + (p % a.inner) * a.istep : 0;
    const V *__restrict__ gin = (const V *)a.in + base;
    V *__restrict__ gout = (V *)a.out + base;
    const V *__restrict__ tw = (const V *)a.tw;
    const int64_t S = a.stride;
    V *row = lds + pp * LS;

    V v[M];

    // ---- optional fused evolution factor along the pencil (contiguous only)
    R gab = (R)1;
    if constexpr (CONTIG) {
        if (a.evolve) {
            for (int i = tid; i < N; i += Cfg::THREADS) {
                const double k = (double)signed_k(i, N);
                gtab[i] = evol_factor<R>(a.ev_c, k * k);
            }
            if (valid) {
                const int64_t pa = p / a.ev_d, pb = p % a.ev_d;
                const double ka = (double)signed_k(pa, a.ev_la), kb = (double)signed_k(pb, a.ev_lb);
                gab = evol_factor<R>(a.ev_c, ka * ka + kb * kb);
            }
            __syncthreads();
        }
    }

    // ---- stage 0 input: global loads, pattern b + q N/R0
    {
        constexpr int R0 = RP.r[0];
        constexpr int NBF = N / R0;
        constexpr int U = (NBF + T - 1) / T;
        if (valid) {
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int b = t + T * u;
                if (NBF % T == 0 || b < NBF) {
#pragma unroll
                    for (int q = 0; q < R0; q++) v[u * R0 + q] = gin[(int64_t)(b + q * NBF) * S];
                }
            }
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
        }
        if constexpr (MxStage<V, N, CONTIG, MX>::at(0)) {
            // the matrix-core stage reads its inputs from LDS in natural order
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int b = t + T * u;
                if (NBF % T == 0 || b < NBF) {
#pragma unroll
                    for (int q = 0; q < R0; q++) row[lds_pos(b + q * NBF)] = v[u * R0 + q];
                }
            }
            __syncthreads();
        }
    }

    [[maybe_unused]] MxConsts mxc;
    if constexpr (MX) mxc = mx_consts(tid & 63);

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
                for (int u = 0; u < Up; u++) {
                    const int b = t + T * u;
                    if (NBFp % T == 0 || b < NBFp) {
                        const int idx = (b / Nsp) * Nsp * Rp + (b % Nsp);
#pragma unroll
                        for (int q = 0; q < Rp; q++) row[lds_pos(idx + q * Nsp)] = v[u * Rp + q];
                    }
                }
                __syncthreads();
            }
            if constexpr (std::is_same<V, float2>::value)
                mx_stage16<N, LS, Ns, RP.twoff[s]>((float2 *)lds, (const float2 *)tw, mxc, tid >> 6, tid & 63);
        } else {
            if constexpr (s > 0) {
                if constexpr (!MxStage<V, N, CONTIG, MX>::at(s - 1)) {
                    // exchange: write the previous stage's outputs
                    constexpr int Rp = RP.r[s - 1];
                    constexpr int Nsp = RP.ns[s - 1];
                    constexpr int NBFp = N / Rp;
                    constexpr int Up = (NBFp + T - 1) / T;
#pragma unroll
                    for (int u = 0; u < Up; u++) {
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
                for (int u = 0; u < U; u++) {
                    const int b = t + T * u;
                    if (NBF % T == 0 || b < NBF) {
#pragma unroll
                        for (int q = 0; q < Rr; q++) v[u * Rr + q] = row[lds_pos(b + q * NBF)];
                    }
                }
                __syncthreads();
            }

#pragma unroll
            for (int u = 0; u < U; u++) {
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
        if constexpr (MxStage<V, N, CONTIG, MX>::at(NST - 1)) {
            // the matrix-core stage left the result in LDS in natural order
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int b = t + T * u;
                if (NBF % T == 0 || b < NBF) {
#pragma unroll
                    for (int q = 0; q < RL; q++) v[u * RL + q] = row[lds_pos(b + q * NBF)];
                }
            }
        }
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
                        gout[(int64_t)(b + q * NBF) * S] = o;
                    }
                }
            }
        }
    }
}

}  // namespace fb

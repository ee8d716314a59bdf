// fb_pass_inst.hpp -- instantiates the pencil passes of one element type for
// every supported axis length (2^a and 3*2^a up to 4096) and builds the
// length -> launcher table.
#pragma once
#include "fb_internal.hpp"
#include "fb_pass.hpp"

namespace fb {

template <typename V, int N, bool CONTIG, bool MX> hipError_t launch_pass(const PassArgs &a, hipStream_t st)
{
    using Cfg = PassCfg<V, N, CONTIG, MX>;
    constexpr int64_t UNIT = std::is_same<V, c2x>::value ? 2 : 1;   // pencils per tile slot
    const int64_t blocks = (a.npencils + UNIT * Cfg::P - 1) / (UNIT * Cfg::P);
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((fft_pass<V, N, CONTIG, MX>), dim3((unsigned)blocks), dim3(Cfg::THREADS), 0, st, a);
    return hipGetLastError();
}

// MX selects the matrix-core radix-16 variant where one exists (complex64);
// otherwise the vector-unit pass is returned.
template <typename V, int N, bool CONTIG> PassInfo pass_info_k(bool mx)
{
    using Cfg = PassCfg<V, N, CONTIG>;
    using CfgM = PassCfg<V, N, CONTIG, true>;
    if constexpr (mx_capable<V, N, CONTIG>()) {
        if (mx) return {&launch_pass<V, N, CONTIG, true>, CfgM::P, CfgM::THREADS, 1};
    }
    return {&launch_pass<V, N, CONTIG, false>, Cfg::P, Cfg::THREADS, 0};
}

template <typename V, int N> PassInfo pass_info(bool contig, bool mx)
{
    return contig ? pass_info_k<V, N, true>(mx) : pass_info_k<V, N, false>(mx);
}

#define FB_FOR_EACH_LENGTH(X) \
    X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) \
    X(384) X(512) X(768) X(1024) X(1536) X(2048) X(3072) X(4096)

// Strided complex64 passes over pencil pairs (16-byte accesses); MX selects
// the matrix-core radix-16 variant where one exists.
template <int N> PassInfo pass_info_pair(bool mx)
{
    using Cfg = PassCfg<c2x, N, false>;
    using CfgM = PassCfg<c2x, N, false, true>;
    if constexpr (mx_capable<c2x, N, false>()) {
        if (mx) return {&launch_pass<c2x, N, false, true>, 2 * CfgM::P, CfgM::THREADS, 1};
    }
    return {&launch_pass<c2x, N, false, false>, 2 * Cfg::P, Cfg::THREADS, 0};
}

inline PassInfo find_pass_pair_t(int n, bool mx)
{
    switch (n) {
#define FB_CASE(L) case L: return pass_info_pair<L>(mx);
        FB_FOR_EACH_LENGTH(FB_CASE)
#undef FB_CASE
    default: return {nullptr, 0, 0, 0};
    }
}

template <typename V, int N, bool MX> hipError_t launch_pass_multi(const PassArgs &a, hipStream_t st)
{
    using Cfg = PassCfg<V, N, true, MX>;
    const int64_t blocks = (a.npencils + Cfg::P - 1) / Cfg::P;
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((fft_pass_multi<V, N, MX>), dim3((unsigned)blocks), dim3(Cfg::THREADS), 0, st, a);
    return hipGetLastError();
}

// Contiguous multi-output evolve passes (the matrix-core variant where one
// exists and MX is asked for).
template <typename V, int N> PassInfo pass_info_multi(bool mx)
{
    using Cfg = PassCfg<V, N, true>;
    using CfgM = PassCfg<V, N, true, true>;
    if constexpr (mx_capable<V, N, true>()) {
        if (mx) return {&launch_pass_multi<V, N, true>, CfgM::P, CfgM::THREADS, 1};
    }
    return {&launch_pass_multi<V, N, false>, Cfg::P, Cfg::THREADS, 0};
}

template <typename V> PassInfo find_pass_multi_t(int n, bool mx)
{
    switch (n) {
#define FB_CASE(L) case L: return pass_info_multi<V, L>(mx);
        FB_FOR_EACH_LENGTH(FB_CASE)
#undef FB_CASE
    default: return {nullptr, 0, 0, 0};
    }
}

template <typename V> PassInfo find_pass_t(int n, bool contig, bool mx)
{
    switch (n) {
#define FB_CASE(L) case L: return pass_info<V, L>(contig, mx);
        FB_FOR_EACH_LENGTH(FB_CASE)
#undef FB_CASE
    default: return {nullptr, 0, 0, 0};
    }
}

}  // namespace fb

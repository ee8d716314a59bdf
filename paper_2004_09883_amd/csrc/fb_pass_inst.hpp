// fb_pass_inst.hpp -- instantiates the pencil passes of one element type for
// a list of axis lengths (2^a and 3*2^a up to 4096, or with FB_LENGTHS_3B
// the lengths 2^a 3^b, b >= 2, up to 4096) and builds the length ->
// launcher table.
#pragma once
#include "fb_internal.hpp"
#include "fb_pass.hpp"

namespace fb {

template <typename V, int N, bool CONTIG, bool MX, bool NT = false>
hipError_t launch_pass(const PassArgs &a, hipStream_t st)
{
    using Cfg = PassCfg<V, N, CONTIG, MX>;
    constexpr int64_t UNIT = std::is_same<V, c2x>::value ? 2 : 1;   // pencils per tile slot
    const int64_t blocks = (a.npencils + UNIT * Cfg::P - 1) / (UNIT * Cfg::P);
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((fft_pass<V, N, CONTIG, MX, NT>), dim3((unsigned)blocks), dim3(Cfg::THREADS), 0, st, a);
    return hipGetLastError();
}

// The non-temporal instance of a pass kind, where it has one.
template <typename V, int N, bool CONTIG, bool MX> constexpr PassLauncher nt_launcher()
{
    if constexpr (has_nt<V, CONTIG>()) return &launch_pass<V, N, CONTIG, MX, true>;
    else return nullptr;
}

// MX selects the matrix-core radix-16 variant where one exists (complex64);
// otherwise the vector-unit pass is returned.
template <typename V, int N, bool CONTIG> PassInfo pass_info_k(bool mx)
{
    using Cfg = PassCfg<V, N, CONTIG>;
    using CfgM = PassCfg<V, N, CONTIG, true>;
    if constexpr (mx_capable<V, N, CONTIG>()) {
        if (mx)
            return {&launch_pass<V, N, CONTIG, true>, CfgM::P, CfgM::THREADS, 1, nt_launcher<V, N, CONTIG, true>()};
    }
    return {&launch_pass<V, N, CONTIG, false>, Cfg::P, Cfg::THREADS, 0, nt_launcher<V, N, CONTIG, false>()};
}

template <typename V, int N> PassInfo pass_info(bool contig, bool mx)
{
    return contig ? pass_info_k<V, N, true>(mx) : pass_info_k<V, N, false>(mx);
}

// Axis lengths 2^a and 3 * 2^a up to 4096 (the list the batched form and
// the other translation units share) ...
#define FB_FOR_EACH_LENGTH(X) \
    X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) \
    X(384) X(512) X(768) X(1024) X(1536) X(2048) X(3072) X(4096)
// ... and 2^a 3^b with b >= 2 up to 4096, instantiated in translation units
// of their own (fb_pass3_*.hip, fb_steps3_*.hip) so that both halves compile
// in parallel.
#define FB_FOR_EACH_LENGTH_3B(X) \
    X(9) X(18) X(36) X(72) X(144) X(288) X(576) X(1152) X(2304) \
    X(27) X(54) X(108) X(216) X(432) X(864) X(1728) X(3456) \
    X(81) X(162) X(324) X(648) X(1296) X(2592) \
    X(243) X(486) X(972) X(1944) X(3888) \
    X(729) X(1458) X(2916) X(2187)
// The lookup functions below take the list as a template argument (B3), so
// that the two halves are distinct instantiations rather than one inline
// function with two bodies.
#ifdef FB_LENGTHS_3B
#define FB_LIST_B3 true
#else
#define FB_LIST_B3 false
#endif

// Strided complex64 passes over pencil pairs (16-byte accesses); MX selects
// the matrix-core radix-16 variant where one exists.
template <int N> PassInfo pass_info_pair(bool mx)
{
    using Cfg = PassCfg<c2x, N, false>;
    using CfgM = PassCfg<c2x, N, false, true>;
    if constexpr (mx_capable<c2x, N, false>()) {
        if (mx) return {&launch_pass<c2x, N, false, true>, 2 * CfgM::P, CfgM::THREADS, 1, nt_launcher<c2x, N, false, true>()};
    }
    return {&launch_pass<c2x, N, false, false>, 2 * Cfg::P, Cfg::THREADS, 0, nt_launcher<c2x, N, false, false>()};
}

template <bool B3> PassInfo find_pass_pair_t(int n, bool mx)
{
#define FB_CASE(L) case L: return pass_info_pair<L>(mx);
    if constexpr (B3) {
        switch (n) { FB_FOR_EACH_LENGTH_3B(FB_CASE) default: return {nullptr, 0, 0, 0}; }
    } else {
        switch (n) { FB_FOR_EACH_LENGTH(FB_CASE) default: return {nullptr, 0, 0, 0}; }
    }
#undef FB_CASE
}

template <typename V, int N, bool MX, bool NT = false> hipError_t launch_pass_multi(const PassArgs &a, hipStream_t st)
{
    using Cfg = PassCfg<V, N, true, MX>;
    const int64_t blocks = (a.npencils + Cfg::P - 1) / Cfg::P;
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((fft_pass_multi<V, N, MX, NT>), dim3((unsigned)blocks), dim3(Cfg::THREADS), 0, st, a);
    return hipGetLastError();
}
template <typename V, int N, bool MX> constexpr PassLauncher nt_launcher_multi()
{
    if constexpr (has_nt<V, true>()) return &launch_pass_multi<V, N, MX, true>;
    else return nullptr;
}

// Contiguous multi-output evolve passes (the matrix-core variant where one
// exists and MX is asked for).
template <typename V, int N> PassInfo pass_info_multi(bool mx)
{
    using Cfg = PassCfg<V, N, true>;
    using CfgM = PassCfg<V, N, true, true>;
    if constexpr (mx_capable<V, N, true>()) {
        if (mx) return {&launch_pass_multi<V, N, true>, CfgM::P, CfgM::THREADS, 1, nt_launcher_multi<V, N, true>()};
    }
    return {&launch_pass_multi<V, N, false>, Cfg::P, Cfg::THREADS, 0, nt_launcher_multi<V, N, false>()};
}

template <typename V, bool B3> PassInfo find_pass_multi_t(int n, bool mx)
{
#define FB_CASE(L) case L: return pass_info_multi<V, L>(mx);
    if constexpr (B3) {
        switch (n) { FB_FOR_EACH_LENGTH_3B(FB_CASE) default: return {nullptr, 0, 0, 0}; }
    } else {
        switch (n) { FB_FOR_EACH_LENGTH(FB_CASE) default: return {nullptr, 0, 0, 0}; }
    }
#undef FB_CASE
}

template <typename V, bool B3> PassInfo find_pass_t(int n, bool contig, bool mx)
{
#define FB_CASE(L) case L: return pass_info<V, L>(contig, mx);
    if constexpr (B3) {
        switch (n) { FB_FOR_EACH_LENGTH_3B(FB_CASE) default: return {nullptr, 0, 0, 0}; }
    } else {
        switch (n) { FB_FOR_EACH_LENGTH(FB_CASE) default: return {nullptr, 0, 0, 0}; }
    }
#undef FB_CASE
}

}  // namespace fb

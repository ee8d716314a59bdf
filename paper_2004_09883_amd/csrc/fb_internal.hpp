// fb_internal.hpp -- interface between the C ABI (host) and the kernel
// translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fb_plan_rules.hpp"

namespace fb {

// Arguments of one pencil pass (see fb_pass.hpp for the geometry).
// Evolution steps one multi-output pass computes from one read of the spectrum.
#define FB_MAX_FUSED_STEPS 8

struct PassArgs {
    const void *in;
    void *out;
    const void *tw;     // per-stage twiddle table of this axis (same real type as the data)
    int64_t npencils;
    int64_t inner, outer, istep, stride;  // input geometry
    // output geometry; when ostride == 0 the output uses the input geometry
    int64_t oinner, oouter, oistep, ostride;
    // segmented batches: when seg_off is set, pencil p belongs to segment
    // p / seg_pencils, whose data starts at element seg_off[p / seg_pencils];
    // the geometry above then applies to the local pencil p % seg_pencils
    const int64_t *seg_off;
    int64_t seg_pencils;
    // pre-twiddle on load (two-pass long transforms): the element at offset
    // o from the start of its segment is multiplied by ptw[o] (a table laid
    // out like one segment); requires ptw_len >= the segment's extent
    const void *ptw;
    int64_t ptw_len;
    // pencil-pair passes: distance in elements between the outputs of the two
    // pencils of a pair (0 = adjacent, one 16-byte store)
    int64_t opair_step;
    // tile-contiguous output (strided passes): the outputs of the P pencils
    // of a tile fill one contiguous block, element k of tile pencil j at
    // obase(first pencil) + j N + k; the tile is then written from LDS with
    // consecutive lanes on consecutive elements.  Every tile must lie within
    // one segment.
    int otile;
    // generated input (first pass of a transform of the seeded uniform
    // grid): the element at offset i of the grid is uniform_elem(gen_seed, i)
    // instead of a load from `in`
    int gen;
    uint64_t gen_seed;
    // non-temporal global accesses wanted (the host then launches the pass
    // kind's non-temporal instance, where it has one): set when the data the
    // pass sweeps exceeds the last-level cache
    int nt;
    int inv;            // 1: inverse (conjugate on load and on store)
    double scale;       // applied on store (1/N in the last inverse pass)
    // fused spectral evolution (contiguous passes only): element i of pencil
    // p = (pa, pb) with pa = p / ev_d, pb = p % ev_d gets the factor
    // exp(-ev_c (k(pa; ev_la)^2 + k(pb; ev_lb)^2 + k(i; N)^2))
    int evolve;
    double ev_c;
    int64_t ev_d;
    int ev_la, ev_lb;
    // several evolution steps from one read of the spectrum (contiguous
    // evolve passes of the multi-output kernel): output j (j < nout) is the
    // pass applied with evolution constant ev_cs[j], written at out + j out_step
    int nout;
    int64_t out_step;
    double ev_cs[FB_MAX_FUSED_STEPS];
};

// Data swept by one pass above which its global accesses may be
// non-temporal (the MI355X last-level cache is 256 MB; grids of 128 MiB and
// less gain from it between passes).
#ifndef FB_NT_MIN_BYTES
#define FB_NT_MIN_BYTES (192ll << 20)
#endif

using PassLauncher = hipError_t (*)(const PassArgs &, hipStream_t);

// Geometry of one instantiated pencil pass (for host-side checks).
struct PassInfo {
    PassLauncher launch;
    int pencils_per_wg;
    int threads;
    int mx;   // 1 when the radix-16 stages run on the matrix cores
    // the same pass with non-temporal global accesses (nullptr when the pass
    // kind has none); launched instead when PassArgs::nt is set
    PassLauncher launch_nt = nullptr;
    PassLauncher pick(const PassArgs &a) const { return (a.nt && launch_nt) ? launch_nt : launch; }
};

// esize: 16 (complex128) or 8 (complex64); mx asks for the matrix-core
// radix-16 variant (complex64 only; the vector-unit pass is returned where
// no such variant exists).  Returns launch == nullptr when the length has no
// instantiated pass.
PassInfo find_pass(int esize, int n, bool contig, bool mx);

// Contiguous evolve pass with up to FB_MAX_FUSED_STEPS outputs from one read
// of its input (PassArgs::nout); mx as for find_pass.
PassInfo find_pass_multi(int esize, int n, bool mx);

// Strided complex64 pass that moves two adjacent pencils per 16-byte access
// (needs an even number of pencils, pencil pairs adjacent in memory
// (even `inner`) and 16-byte aligned buffers).  pencils_per_wg counts pencils.
// `mx` selects the matrix-core radix-16 variant where one exists (the
// returned mx field says which one it is).
PassInfo find_pass_pair(int n, bool mx = false);

// Twiddle tables of one axis: for each stage s with ns > 1, entry
// off[s] + (q-1) ns + k = w_{ns r}^(q k), w_L = exp(-2 pi i / L), in binary64
// (tw64) and rounded to binary32 (tw32).
struct TwDesc {
    int nst;
    int r[16];
    int ns[16];
    int off[16];
    int total;
};
hipError_t launch_twiddles(const TwDesc &d, double2 *tw64, float2 *tw32, hipStream_t st);

// u_out = u_in * exp(-c |k|^2) (u_in may equal u_out).
hipError_t launch_evolve(int esize, const void *in, void *out, int64_t nx, int64_t ny, int64_t nz,
                         double c, hipStream_t st);

// out2[0] + i out2[1] = sum_{j<1024} x[(17 j) mod N], fixed-order binary64 tree.
// Checksums of `count` consecutive grids of N elements into out2[2g], out2[2g+1].
hipError_t launch_checksum(int esize, const void *x, int64_t N, double *out2, hipStream_t st, int count = 1);

}  // namespace fb
struct fb_plan;
namespace fb {
// Make every pass of the plan use non-temporal global accesses (where the
// pass kind gains from them) whatever the grid's size: for callers that run
// many requests at once, whose grids together exceed the last-level cache.
// Call before the plan is used.
void plan_set_nt_always(fb_plan *p, bool on);

// Device address of the current device's copy of the static staging buffer
// (FB_STATIC_SCRATCH_BYTES), looked up once per device and cached.
hipError_t static_scratch(void **ptr);

// x[i] = U(seed, 2i) + i U(seed, 2i+1)  (SplitMix64, counter based)
hipError_t launch_fill_uniform(int esize, void *x, int64_t N, uint64_t seed, hipStream_t st);

}  // namespace fb

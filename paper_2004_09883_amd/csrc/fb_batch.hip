// fb_batch.hip -- device side of the batched form: many independent 1D and
// 2D complex64 transforms of mixed lengths, executed as one launch per
// (length, pass) group, as one persistent launch per phase, or as a single
// persistent launch for the whole batch.
//
// A batch is a list of groups; every group is one pencil pass (PassArgs)
// over all transforms of one length, with `ntiles` tiles.  Groups come in
// two phases: phase 0 holds the first passes of two-pass long transforms,
// the row passes of 2D transforms and the single-pass lengths; phase 1 the
// second passes and the column passes, which read what phase 0 wrote.
//
// None of the persistent forms communicates between workgroups: the
// per-phase form orders its phases on the stream, and the single launch
// gives each two-pass transform (both passes) to one workgroup, which runs
// the second pass after its own first pass and a barrier.
#include <hip/hip_runtime.h>

#include "fb_batch.hpp"
#include "fb_pass.hpp"

namespace fb {

// Tile kinds of the persistent kernel: every complex64 pass length, in the
// contiguous and the strided geometry.
#define FB_BATCH_KINDS(X) \
    X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) \
    X(384) X(512) X(768) X(1024) X(1536) X(2048) X(3072) X(4096)

constexpr int max_int(int a, int b) { return a > b ? a : b; }

// Contiguous tiles hold complex64 pencils; strided tiles hold pencil pairs
// (two adjacent pencils per 16-byte element).
template <int N> constexpr int kind_threads()
{
    return max_int(PassCfg<float2, N, true>::THREADS, PassCfg<c2x, N, false>::THREADS);
}
template <int N> constexpr int kind_lds_bytes()
{
    return max_int(PassCfg<float2, N, true>::P * PassCfg<float2, N, true>::LS * 8,
                   PassCfg<c2x, N, false>::P * PassCfg<c2x, N, false>::LS * 16);
}

constexpr int batch_threads()
{
    int m = 0;
#define FB_MAXT(L) m = max_int(m, kind_threads<L>());
    FB_BATCH_KINDS(FB_MAXT)
#undef FB_MAXT
    return m;
}
constexpr int batch_lds_bytes()
{
    int m = 0;
#define FB_MAXL(L) m = max_int(m, kind_lds_bytes<L>());
    FB_BATCH_KINDS(FB_MAXL)
#undef FB_MAXL
    return m;
}

constexpr int BATCH_THREADS = batch_threads();
constexpr int BATCH_LDS_MAX = batch_lds_bytes();
static_assert(BATCH_THREADS % 64 == 0 && BATCH_THREADS <= 1024, "persistent workgroup size");
static_assert(BATCH_LDS_MAX <= 160 * 1024, "persistent kernel LDS");

int batch_persistent_threads() { return BATCH_THREADS; }

int batch_kind_lds_bytes(int n, bool contig)
{
    switch (n) {
#define FB_KL(L)                                                                                          \
    case L:                                                                                                \
        return contig ? PassCfg<float2, L, true>::P * PassCfg<float2, L, true>::LS * 8                   \
                      : PassCfg<c2x, L, false>::P * PassCfg<c2x, L, false>::LS * 16;
        FB_BATCH_KINDS(FB_KL)
#undef FB_KL
    default: return -1;
    }
}

// One tile of one group.  Every kind is inlined into the switch below; the
// empty asm statement makes `tid` opaque inside each case, which keeps the
// compiler from hoisting every kind's index arithmetic in front of the
// switch (that would keep all of it live at once: the registers of the
// kernel are then those of its largest kind instead of their sum).  The
// group descriptor is read through a wave-uniform pointer (scalar loads), so
// every branch around a barrier is uniform.
template <int L, bool CONTIG>
__device__ __forceinline__ void tile_fn(const BatchGroup *g, const BatchBuffers &bufs, int64_t tile, int tid, c2x *lds)
{
    asm volatile("" : "+v"(tid));
    PassArgs a = g->args;
    a.in = bufs.p[g->in_sel];
    a.out = bufs.p[g->out_sel];
    a.inv = bufs.inv;
    a.nt = bufs.nt;
    a.scale = (bufs.inv && g->last) ? g->inv_scale : 1.0;
    if constexpr (CONTIG) pass_tile<float2, L, true, false>(a, tile, tid, (float2 *)lds, nullptr);
    else pass_tile<c2x, L, false, false>(a, tile, tid, lds, nullptr);
}

__device__ __forceinline__ void run_tile(const BatchGroup *g, const BatchBuffers &bufs, int64_t tile, int tid,
                                         c2x *lds)
{
    switch (g->n * 2 + (g->contig ? 1 : 0)) {
#define FB_KIND(L)                                                        \
    case 2 * L + 1: tile_fn<L, true>(g, bufs, tile, tid, lds); break; \
    case 2 * L: tile_fn<L, false>(g, bufs, tile, tid, lds); break;
        FB_BATCH_KINDS(FB_KIND)
#undef FB_KIND
    default: break;
    }
}

// Persistent execution of one phase: the tiles of groups [g0, g1) are
// numbered 0 .. ntasks-1 in group order and workgroup w takes tiles
// w, w + gridDim.x, w + 2 gridDim.x, ...  Groups of one phase are independent
// of each other; a phase that depends on another is launched after it on the
// same stream.  There is no communication between workgroups.  The LDS is
// dynamic, sized by the host for the largest tile kind of the phase.
__global__ void __launch_bounds__(BATCH_THREADS) batch_persistent(const BatchGroup *__restrict__ groups, int g0,
                                                                  int g1, int64_t ntasks, BatchBuffers bufs)
{
    extern __shared__ c2x lds[];
    const int tid = threadIdx.x;
    int g = g0;
    for (int64_t t = blockIdx.x; t < ntasks; t += gridDim.x) {
        while (g + 1 < g1 && t >= groups[g + 1].task0) g++;
        run_tile(groups + g, bufs, t - groups[g].task0, tid, lds);
        __syncthreads();   // the next tile reuses the LDS
    }
}

hipError_t launch_batch_persistent(const BatchGroup *groups_dev, int g0, int g1, int64_t ntasks, int nblocks,
                                   int lds_bytes, const BatchBuffers &bufs, hipStream_t st)
{
    if (ntasks <= 0) return hipSuccess;
    if (lds_bytes <= 0 || lds_bytes > BATCH_LDS_MAX) return hipErrorInvalidValue;
    const int64_t blocks = ntasks < nblocks ? ntasks : nblocks;
    hipLaunchKernelGGL(batch_persistent, dim3((unsigned)blocks), dim3(BATCH_THREADS), (unsigned)lds_bytes, st,
                       groups_dev, g0, g1, ntasks, bufs);
    return hipGetLastError();
}

// The whole batch in one launch.  Workgroup w runs its items in order; an
// item is a range of tiles of one group, or the two passes of one transform
// (or one 2D transform): the first pass's tiles, then the second pass's,
// which read what the first wrote.  Both ranges run in this workgroup, so
// the barrier after each tile (a workgroup-scope release and acquire) is
// all the ordering they need.  The host builds the item lists (largest item
// first onto the least-loaded workgroup), so no workgroup waits for
// another.
__global__ void __launch_bounds__(BATCH_THREADS) batch_onelaunch(const BatchGroup *__restrict__ groups,
                                                                 const BatchItem *__restrict__ items,
                                                                 const int64_t *__restrict__ item_begin,
                                                                 BatchBuffers bufs)
{
    extern __shared__ c2x lds[];
    const int tid = threadIdx.x;
    const int64_t i0 = item_begin[blockIdx.x], i1 = item_begin[blockIdx.x + 1];
    for (int64_t it = i0; it < i1; it++) {
        const BatchItem item = items[it];
        for (int64_t t = item.a1; t < item.b1; t++) {
            run_tile(groups + item.g1, bufs, t, tid, lds);
            __syncthreads();   // the next tile reuses the LDS; the second range reads this one's output
        }
        if (item.g2 >= 0) {
            for (int64_t t = item.a2; t < item.b2; t++) {
                run_tile(groups + item.g2, bufs, t, tid, lds);
                __syncthreads();
            }
        }
    }
}

hipError_t launch_batch_onelaunch(const BatchGroup *groups_dev, const BatchItem *items_dev,
                                  const int64_t *item_begin_dev, int nblocks, int lds_bytes, const BatchBuffers &bufs,
                                  hipStream_t st)
{
    if (nblocks <= 0) return hipSuccess;
    if (lds_bytes <= 0 || lds_bytes > BATCH_LDS_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(batch_onelaunch, dim3((unsigned)nblocks), dim3(BATCH_THREADS), (unsigned)lds_bytes, st,
                       groups_dev, items_dev, item_begin_dev, bufs);
    return hipGetLastError();
}

hipError_t batch_occupancy(int lds_bytes, int *blocks_per_cu, bool onelaunch)
{
    if (onelaunch)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, batch_onelaunch, BATCH_THREADS,
                                                            (size_t)lds_bytes);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, batch_persistent, BATCH_THREADS,
                                                        (size_t)lds_bytes);
}

}  // namespace fb

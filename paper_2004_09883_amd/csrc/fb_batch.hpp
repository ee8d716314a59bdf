// fb_batch.hpp -- shared between the batch plan (host) and fb_batch.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fb_internal.hpp"

namespace fb {

#define FB_BATCH_MAX_GROUPS 512

// One (length, pass) group of a batch.  The data pointers of `args` are
// chosen per execution: in_sel / out_sel name the buffer (0 = the caller's
// input, 1 = the caller's output, 2 = the workspace data region).
struct BatchGroup {
    PassArgs args;
    int n;          // pass length
    int contig;     // 1: contiguous geometry, 0: strided
    int phase;      // 0 or 1; phase 1 groups read what phase 0 wrote
    int in_sel, out_sel;
    int last;       // 1 when this pass completes its transforms (inverse scale applies)
    double inv_scale;
    int64_t ntiles;
    int64_t task0;  // index of the group's first tile within its phase
    int64_t tile_pencils;   // pencils per tile
};

// One work item of the one-launch persistent kernel: tiles [a1, b1) of group
// g1, then (when g2 >= 0) tiles [a2, b2) of group g2, which read what the
// first range wrote (the two passes of one transform, run by the same
// workgroup one after the other).
struct BatchItem {
    int g1, g2;
    int64_t a1, b1, a2, b2;
};

// Buffers of one execution: p[0] input, p[1] output, p[2] intermediate.
struct BatchBuffers {
    void *p[3];
    int inv;
    int nt;   // PassArgs::nt for every pass of the execution
};

int batch_persistent_threads();
// LDS bytes of one tile of the persistent kernel for a group of pass length
// n (-1 when n is not a tile kind)
int batch_kind_lds_bytes(int n, bool contig);
hipError_t batch_occupancy(int lds_bytes, int *blocks_per_cu, bool onelaunch = false);
hipError_t launch_batch_persistent(const BatchGroup *groups_dev, int g0, int g1, int64_t ntasks, int nblocks,
                                   int lds_bytes, const BatchBuffers &bufs, hipStream_t st);
// The whole batch in one launch: workgroup w runs items [item_begin[w],
// item_begin[w + 1]) of `items`, in order.
hipError_t launch_batch_onelaunch(const BatchGroup *groups_dev, const BatchItem *items_dev,
                                  const int64_t *item_begin_dev, int nblocks, int lds_bytes, const BatchBuffers &bufs,
                                  hipStream_t st);

// tables[m] = w_n^m = exp(-2 pi i m / n), m < n, binary64 and binary32
hipError_t launch_roots(int64_t n, double2 *t64, float2 *t32, hipStream_t st);
// t32[q n1 + b] = w_(n1 n2)^(q b): the second-pass pre-twiddles of a two-pass
// transform, laid out like its data
hipError_t launch_pretwiddle(int64_t n1, int64_t n2, float2 *t32, hipStream_t st);

}  // namespace fb

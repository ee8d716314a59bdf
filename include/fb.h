/*
 * fb.h -- C ABI of libfb, an MI355X (gfx950) library for the 3D complex FFT
 * spectral block: forward 3D DFT, pointwise spectral evolution, inverse 3D
 * DFT and a strided checksum.
 *
 * The paper (section 3.4, steps B-1 and C-1) replaces a detected CPU
 * function block -- its evaluation uses a Fourier-transform block, section
 * 5.1(a) -- by an accelerator library call "of the same meaning", connected
 * through a usage method registered with the library.  These calls are that
 * library for the Fourier-transform block.  Following step C-2, an argument
 * that does not match what the library supports is rejected with a status
 * code and a message; nothing is coerced silently.
 *
 * Conventions shared by every call
 *  - Grids are C order [nx][ny][nz] (z contiguous), interleaved complex:
 *    complex128 (two binary64) for FB_C128, complex64 (two binary32) for
 *    FB_C64 and FB_C64_SPLITBF16.  This is torch/numpy shape (nx, ny, nz).
 *  - All grid, table and result pointers are DEVICE pointers on the device
 *    that was current when the plan was created.  They belong to the caller
 *    and must be aligned to the element size (16 B or 8 B).
 *  - Work is enqueued asynchronously on `hip_stream` (a hipStream_t; NULL is
 *    the default stream).  A status of FB_OK means the work was enqueued;
 *    device-side faults surface at the caller's next synchronisation.
 *  - Arguments are validated on the host before any HIP call, so invalid
 *    arguments never launch anything.  On error the call returns a negative
 *    fb_status (or NULL) and records a message readable with fb_last_error
 *    (thread-local).
 *  - Plans are immutable after creation: one plan may be used concurrently
 *    from several host threads and streams.
 */
#ifndef FB_H
#define FB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fb_plan fb_plan;

/* Storage and arithmetic of a plan. */
typedef enum {
    FB_C128 = 0,          /* complex128 storage, binary64 arithmetic            */
    FB_C64 = 1,           /* complex64 storage, binary32 arithmetic             */
    FB_C64_SPLITBF16 = 2  /* complex64 storage; radix-16 stages as split-bf16
                             (hi+lo) matrix-core products, fp32 accumulation   */
} fb_dtype;

/* Sign of the exponent of the transform. */
enum { FB_FORWARD = -1, FB_INVERSE = +1 };

typedef enum {
    FB_OK = 0,
    FB_ERR_INVALID_ARG = -1,      /* null/misaligned pointer, bad dir, alpha<0 ...  */
    FB_ERR_UNSUPPORTED_SIZE = -2, /* axis length outside the supported set          */
    FB_ERR_DTYPE = -3,            /* dtype not an fb_dtype value                    */
    FB_ERR_OOM = -4,              /* device allocation failed                       */
    FB_ERR_DEVICE = -5,           /* HIP runtime error (no device, launch failure)  */
    FB_ERR_BUDGET = -6            /* serving admission refused: over the budget     */
} fb_status;

/* Library version as 10000*major + 100*minor + patch. */
int fb_version(void);

/* Last error recorded on this host thread: returns its fb_status and, when
 * msg is not NULL, points *msg at a thread-local message (valid until the
 * next fb_* call on this thread).  FB_OK / "" when the last call succeeded. */
int fb_last_error(const char **msg);

/* Describe the plan that fb_fft3d_plan would build for this shape and dtype,
 * without touching the device: writes "z:<radices> y:<radices> x:<radices>
 * order:zyx" (radices in the order the stages are applied; "-" for an axis of
 * length 1) into buf (capacity cap bytes, NUL-terminated).  Returns the
 * string length, or a negative fb_status. */
int fb_describe_shape(int64_t nx, int64_t ny, int64_t nz, int dtype, char *buf, int cap);

/* Create a plan for an nx x ny x nz grid of the given dtype (section 3.4
 * B-1: the library and its usage method for this block).  Every axis length
 * must be 2^a 3^b with 1 <= n <= 4096 (n = 1 skips that axis).  The plan
 * owns small device tables (twiddles generated on the device in binary64, a
 * binary32 copy rounded from them); creation is synchronous.  Returns NULL on
 * error (see fb_last_error). */
fb_plan *fb_fft3d_plan(int64_t nx, int64_t ny, int64_t nz, int dtype);

/* Release a plan and its tables.  NULL-safe.  The caller must make sure no
 * enqueued work still uses the plan. */
void fb_fft3d_destroy(fb_plan *p);

/* Bytes of device memory the plan holds (its tables). */
size_t fb_plan_device_bytes(const fb_plan *p);

/* The plan's description (same format as fb_describe_shape); owned by the
 * plan. */
const char *fb_plan_describe(const fb_plan *p);

/* 3D DFT of the grid `in` into `out` (section 5.1(a): the Fourier-transform
 * block).  dir = FB_FORWARD computes X[k] = sum_r x[r] exp(-2 pi i k.r/n)
 * (unscaled); dir = FB_INVERSE uses exp(+2 pi i ...) and divides by
 * N = nx ny nz, so inverse(forward(x)) = x.  in == out (in place) is allowed;
 * partially overlapping buffers are rejected.  Needs no workspace. */
fb_status fb_fft3d_exec(const fb_plan *p, const void *in, void *out, int dir, void *hip_stream);

/* The same transform on HOST buffers, synchronously: the grid is copied to a
 * device buffer the call allocates, transformed in place there and copied
 * back (in_host == out_host allowed).  This is the drop-in form of a CPU
 * library call "of the same meaning" (section 3.4, C-1: the replaced call
 * keeps the host program's data where it was); its cost includes both PCIe
 * copies and an allocation, so streamed device-resident use goes through
 * fb_fft3d_exec.  Errors as fb_fft3d_exec, plus FB_ERR_OOM. */
fb_status fb_fft3d_exec_host(const fb_plan *p, const void *in_host, void *out_host, int dir);

/* Size of the static device staging buffer of fb_fft3d_exec_host_noalloc:
 * 64 MiB, one 2048 x 2048 complex128 grid. */
#define FB_STATIC_SCRATCH_BYTES (64u << 20)

/* fb_fft3d_exec_host without any device allocation, for callers that cannot
 * allocate device memory (code that must not call hipMalloc: tight serving
 * loops, harnesses that forbid allocation after start-up).  The grid is
 * staged through a static device buffer of FB_STATIC_SCRATCH_BYTES that
 * every GPU the library runs on holds until the process ends; the call
 * itself allocates nothing (no hipMalloc, hipFree or allocating library
 * routine).  Grids larger than the buffer are rejected with
 * FB_ERR_UNSUPPORTED_SIZE before any HIP call.  The buffer keeps the last
 * call's grid; calls of one process on one GPU share it and are serialised
 * by a process-wide lock (calls from other processes use their own copy).
 * Synchronous; results equal fb_fft3d_exec_host's bit for bit.  Errors as
 * fb_fft3d_exec_host, without FB_ERR_OOM. */
fb_status fb_fft3d_exec_host_noalloc(const fb_plan *p, const void *in_host, void *out_host, int dir);

/* The same transform restricted to some axes: bit 0 of `axes` selects z,
 * bit 1 y, bit 2 x (axes = 7 is fb_fft3d_exec).  The inverse divides by the
 * product of the selected lengths.  With no axis of length > 1 selected the
 * call copies in to out.  Same buffer rules as fb_fft3d_exec. */
fb_status fb_fft3d_exec_axes(const fb_plan *p, const void *in, void *out, int dir, int axes,
                             void *hip_stream);

/* Spectral evolution in place: u[k] *= exp(-(4 pi^2 alpha t) |k|^2), with
 * the signed wavenumber k = i - n [2i >= n] on each axis (heat-equation decay
 * of each Fourier mode on the unit periodic cube).  alpha >= 0, t >= 0,
 * both finite.  The paper defines no evolution: this step, like the
 * checksum below, belongs to the spectral-block workload built around the
 * paper's Fourier-transform block (section 5.1(a)), a forward transform
 * followed by per-step decay, inverse transform and checksum; it is
 * offered as a library call of its own so that a detected block made of
 * these steps can be replaced call by call (section 3.4, B-1). */
fb_status fb_spectral_evolve(const fb_plan *p, void *u, double alpha, double t, void *hip_stream);

/* Checksum: out2_dev[0] + i out2_dev[1] = sum_{j=0}^{1023} x.flat[(17 j) mod N],
 * accumulated in binary64 in a fixed order (deterministic).  out2_dev points
 * at two device doubles.  Not from the paper: the spectral-block workload's
 * per-step check value (1024 samples at stride 17 of the normalised
 * spatial grid). */
fb_status fb_checksum(const fb_plan *p, const void *x, double *out2_dev, void *hip_stream);

/* One step of the spectral block, fused (the workload's step, see
 * fb_spectral_evolve; the paper's block is replaced by one call of the same
 * meaning, section 3.4 B-1): x_out = inverse(evolve(uhat0, alpha, t)) and
 * its checksum into out2_dev (when out2_dev is not NULL).
 * uhat0 is read only and is not modified; x_out must not overlap uhat0.
 * The evolution is applied while the first inverse pass loads its input, so
 * it costs no extra pass over the grid. */
fb_status fb_spectral_step(const fb_plan *p, const void *uhat0, void *x_out, double alpha,
                           double t, double *out2_dev, void *hip_stream);

/* Several steps of the spectral block from one spectrum: for j < nsteps,
 * grid j of x_out (x_out + j N elements) = inverse(evolve(uhat0, alpha,
 * t[j])), and its checksum into sums_dev[2j], sums_dev[2j+1] (when sums_dev
 * is not NULL).  Each grid equals what fb_spectral_step gives for t[j], bit
 * for bit; the steps share the first inverse pass, which reads uhat0 once for
 * up to 8 steps and writes their grids, so a step moves 5 grid sweeps
 * instead of 6 (the paper's block is one library call of the same meaning,
 * section 3.4 B-1).  t is a host array of nsteps finite values >= 0; x_out
 * holds nsteps grids and must not overlap uhat0. */
fb_status fb_spectral_steps(const fb_plan *p, const void *uhat0, void *x_out, double alpha, const double *t,
                            int nsteps, double *sums_dev, void *hip_stream);

/* Fill a grid of the plan's shape and dtype with the seeded uniform input:
 * element i = U(seed, 2i) + i U(seed, 2i+1), U(s, c) = (h >> 11) 2^-52 - 1
 * with h the SplitMix64 output at counter c of stream s (complex64 grids get
 * the binary64 values rounded to nearest). */
fb_status fb_fill_uniform(const fb_plan *p, void *x, uint64_t seed, void *hip_stream);

/* Forward 3D DFT (FB_FORWARD, unnormalized) of the grid fb_fill_uniform(p,
 * ., seed) would write, into `out`, with the input generated inside the
 * first pencil pass instead of being written to and read back from device
 * memory: the result equals fb_fill_uniform followed by fb_fft3d_exec
 * bit for bit.  The paper replaces a detected block (here: make the input,
 * transform it) by one library call of the same meaning (section 3.4, B-1).
 * `out` is a device grid of the plan's dtype, aligned to its element size.
 * Errors as fb_fft3d_exec. */
fb_status fb_fft3d_forward_uniform(const fb_plan *p, uint64_t seed, void *out, void *hip_stream);

/* ---- LU function block -------------------------------------------------
 * The paper's other offloaded function block (section 5.1(b): an LU
 * factorization replaced by a GPU library call of the same meaning).
 * LU factorization with partial pivoting of the row-major n x n binary64
 * matrix a (device memory, row stride lda >= n), in place: on return the
 * strictly lower part holds L (unit diagonal, not stored) and the upper part
 * U, with P a = L U where P applies, for j = 0..n-1 in order, the swap of
 * rows j and ipiv[j] (0-based, ipiv[j] >= j).  The pivot of column j is the
 * first row of largest magnitude.  info (device) receives 0, or j + 1 for
 * the first column j whose pivot is zero (the factorization still
 * completes, as the usual library convention).  ipiv (n int32) and info are
 * device memory owned by the caller; nothing is allocated.  1 <= n <= 2048
 * (else FB_ERR_UNSUPPORTED_SIZE); NULL or misaligned pointers, lda < n or
 * overlapping arguments -> FB_ERR_INVALID_ARG.  Stream-ordered. */
fb_status fb_lu_factor(double *a, int64_t n, int64_t lda, int32_t *ipiv, int32_t *info, void *hip_stream);

/* ---- Batched form ------------------------------------------------------
 * Many independent complex64 transforms in one call: n1d 1D transforms of
 * lengths lens[0..n1d) (each 2^a or 3*2^a, 2 <= n <= 2^21) and n2d 2D
 * transforms of side2d x side2d (side2d = 2^a or 3*2^a, up to 4096), packed
 * back to back in one buffer in that order (fb_batch_offsets gives each
 * start).  Forward transforms are unscaled; inverse ones divide by the
 * transform size.  Lengths up to 4096 take one pencil pass; longer 1D
 * lengths n = n1 n2 take two (a length-n1 pass over stride n2 into blocks of
 * n1, then a pre-twiddled length-n2 pass over stride n1); 2D transforms take
 * a row pass and a column pass.  The batch plan groups equal lengths so that
 * each (length, pass) group is one launch; or one persistent kernel runs
 * the whole batch in a single launch: each workgroup runs a list of items
 * (both passes of a two-pass or 2D transform, one after the other, or one
 * tile of a single-pass length) that the plan deals out largest first to
 * the least-loaded workgroup; or a persistent kernel per phase runs the
 * tiles of all groups of the phase (first passes, 2D rows and single-pass
 * lengths, then second passes and 2D columns), ordered on the stream.  No
 * form makes one workgroup wait for another.
 * The buffers are one packed array of all transforms plus offsets (a reading
 * of "pointer arrays": one allocation, one pointer per call; the offsets
 * give each transform's start). */
typedef struct fb_batch fb_batch;

/* NULL on error.  dtype must be FB_C64.  Synchronous (builds tables). */
fb_batch *fb_batch_plan(const int64_t *lens, int n1d, int n2d, int64_t side2d, int dtype);
void fb_batch_destroy(fb_batch *b);                    /* NULL-safe */
int64_t fb_batch_elements(const fb_batch *b);          /* complex elements of the packed buffer */
/* Writes the n1d + n2d start offsets (in complex elements); returns the count. */
int fb_batch_offsets(const fb_batch *b, int64_t *off);
/* Workspace bytes fb_batch_exec needs: 0 out of place; a buffer as large as
 * the packed data when in_place != 0 (in == out). */
size_t fb_batch_workspace_bytes(const fb_batch *b, int in_place);
int fb_batch_launches(const fb_batch *b);              /* launches of the per-group mode */
const char *fb_batch_describe(const fb_batch *b);

/* Executes the batch: in and out are 16-byte aligned device buffers of
 * fb_batch_elements complex64 values (equal, or not overlapping).  workspace (256-byte
 * aligned, at least fb_batch_workspace_bytes(b, in == out) bytes) is needed
 * only in place; it may be NULL otherwise.  persistent = 0: one launch per
 * group; 1: the whole batch in one launch (when every two-pass and 2D
 * transform's tiles lie within that transform, which fb_batch_describe
 * reports as onelaunch=1; otherwise as 2); 2: one persistent launch per
 * phase.  All three give the same bits. */
fb_status fb_batch_exec(const fb_batch *b, const void *in, void *out, void *workspace, size_t workspace_bytes,
                        int dir, int persistent, void *hip_stream);

/* ---- Serving form ------------------------------------------------------
 * A request loop with continuous batching: submitted spectral-block
 * requests wait in a FIFO; a worker thread admits the head as soon as a
 * stream slot is free and the request's device bytes (the spectrum,
 * min(steps, 8) output grids and its checksums) fit in the HBM budget, so
 * work of requests that arrive while others run overlaps on the device.  Plans (per shape and dtype) and device
 * buffers (per size) stay resident; pooled buffers count against the budget.
 * A request: its input grid (as fb_fill_uniform with the stream seed
 * SplitMix64(seed, request_key)) is generated inside the first forward
 * pass (fb_fft3d_forward_uniform) and transformed forward,
 * then for t = 1..steps evolved (alpha, t), transformed back and
 * checksummed, up to 8 steps per read of the spectrum (fb_spectral_steps); the checksums (and the final grid when want_grid) come back
 * to host memory.  A result does not depend on what else runs. */
#define FB_SERVE_MAX_STEPS 64

typedef struct {
    int64_t nx, ny, nz;
    int dtype;              /* FB_C128 or FB_C64 */
    int steps;              /* 1 .. FB_SERVE_MAX_STEPS */
    double alpha;
    uint64_t seed;
    int64_t request_key;    /* selects the input stream */
    int want_grid;          /* copy the final grid back */
} fb_request;

typedef struct {
    int64_t id;             /* as returned by fb_server_submit */
    int status;             /* FB_OK or a negative fb_status */
    int64_t nx, ny, nz;
    int dtype, steps;
    double t_arrival, t_admit, t_done;   /* host steady-clock seconds */
    int64_t grid_bytes;     /* size of the final grid (0 unless want_grid) */
} fb_result;

typedef struct {
    size_t budget, bytes_allocated, peak_allocated;
    int plans_cached, max_concurrent;
    int64_t queued;
} fb_server_info;

typedef struct fb_server fb_server;

/* budget_bytes >= 1 MiB, 1 <= n_streams <= 64; NULL on error.  Uses the
 * device current at creation. */
fb_server *fb_server_create(size_t budget_bytes, int n_streams);
/* Queues a request; returns its id (>= 0) or a negative fb_status
 * (FB_ERR_BUDGET if it could never fit the budget). */
int64_t fb_server_submit(fb_server *s, const fb_request *r);
/* Takes one finished request, if any: returns 1 and fills *out, copies up to
 * sums_cap doubles of checksums (re, im per step) and, when grid_cap is
 * large enough, the final grid; returns 0 when none is finished. */
int fb_server_poll(fb_server *s, fb_result *out, double *sums, int sums_cap, void *grid, size_t grid_cap);
/* Requests submitted and not yet taken by fb_server_poll's producer side. */
int64_t fb_server_in_flight(fb_server *s);
int fb_server_stats(fb_server *s, fb_server_info *info);
/* Admission order (either way a request starts only when a stream slot is
 * free and its bytes fit the budget, and the chosen request waits for that):
 *   FB_SERVE_FIFO (the default): the oldest queued request first;
 *   FB_SERVE_DEADLINE: the request with the earliest arrival time plus
 *     estimated service time first, the estimate being its bytes under the
 *     pass model (5 + ceil(steps/8) + 5 steps grids of E N bytes) at a
 *     nominal 5 TB/s.  A short request overtakes long ones that arrived at
 *     most its estimated saving earlier, and no request is overtaken by one
 *     that arrived after its own estimated completion, so none starves.
 * May be changed while requests run (it applies to later admissions).
 * Returns FB_OK, or FB_ERR_INVALID_ARG for a NULL server or another value. */
enum { FB_SERVE_FIFO = 0, FB_SERVE_DEADLINE = 1 };
int fb_server_set_policy(fb_server *s, int policy);
/* Finishes queued and running requests, then releases everything. */
void fb_server_destroy(fb_server *s);

/* Per-launch timing of the library's kernels, for benchmarks.  While
 * enabled, every kernel the library enqueues is bracketed by two HIP events
 * on the stream it is launched on.  Process wide: not for concurrent use from
 * several host threads.  fb_profile_enable(1) clears earlier records. */
int fb_profile_enable(int on);

/* Waits for the recorded events and writes a JSON array, one object per
 * kernel in first-launch order: {"kernel", "launches", "total_ms", "avg_ms",
 * "bytes_per_launch"} (bytes_per_launch = the algorithmic bytes: one read and
 * one write of the grid for a pass).  Returns the length or a negative
 * fb_status. */
int fb_profile_report(char *buf, int cap);

#ifdef __cplusplus
}
#endif

#endif /* FB_H */

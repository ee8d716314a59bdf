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
 * must be 2^a or 3*2^a with 1 <= n <= 4096 (n = 1 skips that axis).  The plan
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

/* The same transform restricted to some axes: bit 0 of `axes` selects z,
 * bit 1 y, bit 2 x (axes = 7 is fb_fft3d_exec).  The inverse divides by the
 * product of the selected lengths.  With no axis of length > 1 selected the
 * call copies in to out.  Same buffer rules as fb_fft3d_exec. */
fb_status fb_fft3d_exec_axes(const fb_plan *p, const void *in, void *out, int dir, int axes,
                             void *hip_stream);

/* Spectral evolution in place: u[k] *= exp(-(4 pi^2 alpha t) |k|^2), with
 * the signed wavenumber k = i - n [2i >= n] on each axis (heat-equation decay
 * of each Fourier mode on the unit periodic cube).  alpha >= 0, t >= 0,
 * both finite. */
fb_status fb_spectral_evolve(const fb_plan *p, void *u, double alpha, double t, void *hip_stream);

/* Checksum: out2_dev[0] + i out2_dev[1] = sum_{j=0}^{1023} x.flat[(17 j) mod N],
 * accumulated in binary64 in a fixed order (deterministic).  out2_dev points
 * at two device doubles. */
fb_status fb_checksum(const fb_plan *p, const void *x, double *out2_dev, void *hip_stream);

/* One step of the spectral block, fused: x_out = inverse(evolve(uhat0,
 * alpha, t)) and its checksum into out2_dev (when out2_dev is not NULL).
 * uhat0 is read only and is not modified; x_out must not overlap uhat0.
 * The evolution is applied while the first inverse pass loads its input, so
 * it costs no extra pass over the grid. */
fb_status fb_spectral_step(const fb_plan *p, const void *uhat0, void *x_out, double alpha,
                           double t, double *out2_dev, void *hip_stream);

/* Fill a grid of the plan's shape and dtype with the seeded uniform input:
 * element i = U(seed, 2i) + i U(seed, 2i+1), U(s, c) = (h >> 11) 2^-52 - 1
 * with h the SplitMix64 output at counter c of stream s (complex64 grids get
 * the binary64 values rounded to nearest). */
fb_status fb_fill_uniform(const fb_plan *p, void *x, uint64_t seed, void *hip_stream);

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

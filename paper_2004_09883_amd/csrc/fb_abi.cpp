// fb_abi.cpp -- the C ABI of libfb (declared in include/fb.h): argument
// validation, plans (radix lists, pass geometry, device twiddle tables) and
// the enqueue order of the passes.
//
// The paper's step C-2 (section 3.4) asks that an interface mismatch between
// the replaced block and the library be surfaced, not papered over: every
// call validates its arguments on the host before any HIP call and returns a
// status code with a thread-local message.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "fb.h"
#include "fb_internal.hpp"
#include "fb_lu.hpp"

using fb::PassArgs;
using fb::PassInfo;

namespace {

thread_local int g_code = FB_OK;
thread_local std::string g_msg;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_code = code;
    g_msg = buf;
    return code;
}

int ok()
{
    g_code = FB_OK;
    g_msg.clear();
    return FB_OK;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? FB_ERR_OOM : FB_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int esize_of(int dtype) { return dtype == FB_C128 ? 16 : 8; }

// ---- optional per-launch timing (process wide, for benchmarks)
struct ProfRec {
    std::string name;
    hipEvent_t a, b;
    double bytes;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t pool_event()
{
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void prof_clear_locked()
{
    for (auto &r : g_prof) {
        g_event_pool.push_back(r.a);
        g_event_pool.push_back(r.b);
    }
    g_prof.clear();
}

// Runs launch(); when timing is on, brackets it with two events on `st`.
template <class F> hipError_t timed_launch(const char *name, double bytes, hipStream_t st, F &&launch)
{
    if (!g_prof_on) return launch();
    std::lock_guard<std::mutex> lk(g_prof_mu);
    hipEvent_t a = pool_event(), b = pool_event();
    if (!a || !b) return launch();
    (void)hipEventRecord(a, st);
    hipError_t e = launch();
    (void)hipEventRecord(b, st);
    g_prof.push_back({name, a, b, bytes});
    return e;
}

const char *dtype_tag(int esize) { return esize == 16 ? "c128" : "c64"; }

// Axis geometry: index 0 = z (contiguous), 1 = y, 2 = x.
struct AxisPlan {
    int64_t n;
    fb::RadixPlan rp;
    PassInfo pass;
    PassInfo pass_pair;   // 16-byte pencil-pair variant (complex64 strided), when usable
    size_t tw_off;   // first entry of this axis in the plan's tables
    int64_t npencils, inner, outer, istep, stride;
    bool contig;
};

int check_shape(int64_t nx, int64_t ny, int64_t nz, int dtype)
{
    if (dtype != FB_C128 && dtype != FB_C64 && dtype != FB_C64_SPLITBF16)
        return fail(FB_ERR_DTYPE, "dtype %d is not an fb_dtype value (0, 1 or 2)", dtype);
    const int64_t d[3] = {nx, ny, nz};
    const char *nm[3] = {"nx", "ny", "nz"};
    for (int i = 0; i < 3; i++) {
        if (d[i] < 1) return fail(FB_ERR_INVALID_ARG, "%s = %lld must be >= 1", nm[i], (long long)d[i]);
        if (!fb::supported_length(d[i]))
            return fail(FB_ERR_UNSUPPORTED_SIZE,
                        "%s = %lld is not supported (axis lengths must be 2^a 3^b, 1..4096)", nm[i],
                        (long long)d[i]);
    }
    return FB_OK;
}

void build_axes(int64_t nx, int64_t ny, int64_t nz, int esize, bool mx, AxisPlan ax[3])
{
    const int64_t len[3] = {nz, ny, nx};
    size_t off = 0;
    for (int a = 0; a < 3; a++) {
        AxisPlan &A = ax[a];
        A.n = len[a];
        A.rp = fb::radix_plan((int)A.n);
        A.contig = (a == 0);
        A.pass = A.n > 1 ? fb::find_pass(esize, (int)A.n, A.contig, mx) : PassInfo{nullptr, 0, 0, 0};
        A.tw_off = off;
        off += (size_t)A.rp.twlen;
    }
    // z: pencils (x, y) back to back
    ax[0].npencils = nx * ny; ax[0].inner = 1;       ax[0].outer = nz;      ax[0].istep = 0; ax[0].stride = 1;
    // y: pencils (x, z); base = x ny nz + z
    ax[1].npencils = nx * nz; ax[1].inner = nz;      ax[1].outer = ny * nz; ax[1].istep = 1; ax[1].stride = nz;
    // x: pencils (y, z); base = y nz + z
    ax[2].npencils = ny * nz; ax[2].inner = ny * nz; ax[2].outer = 0;       ax[2].istep = 1; ax[2].stride = ny * nz;
    // complex64 strided passes can move pencil pairs when pencils pair up
    // inside each inner group; the pair pass must run its radix-16 stages on
    // the same units as the single-pencil pass of the plan
    for (int a = 1; a < 3; a++) {
        AxisPlan &A = ax[a];
        A.pass_pair = PassInfo{nullptr, 0, 0, 0};
        if (esize == 8 && A.n > 1 && A.inner % 2 == 0 && A.npencils % 2 == 0 && A.pass.launch) {
            const PassInfo pp = fb::find_pass_pair((int)A.n, A.pass.mx != 0);
            if (pp.launch && pp.mx == A.pass.mx) A.pass_pair = pp;
        }
    }
    ax[0].pass_pair = PassInfo{nullptr, 0, 0, 0};
}

void describe(const AxisPlan ax[3], char *out, size_t cap)
{
    std::string s;
    const char nm[3] = {'z', 'y', 'x'};
    for (int a = 0; a < 3; a++) {
        s += nm[a];
        s += ':';
        if (ax[a].rp.count == 0) s += '-';
        for (int i = 0; i < ax[a].rp.count; i++) {
            if (i) s += ',';
            s += std::to_string(ax[a].rp.r[i]);
        }
        s += ' ';
    }
    s += "order:zyx";
    snprintf(out, cap, "%s", s.c_str());
}

}  // namespace

struct fb_plan {
    int64_t nx, ny, nz, N;
    int dtype, esize;
    AxisPlan ax[3];
    double2 *tw64;
    float2 *tw32;
    size_t tw_total;
    int device;
    // non-temporal accesses for every pass, whatever the grid's size (set by
    // the serving loop, whose concurrent requests share the last-level cache)
    bool nt_always = false;
    char desc[256];
};

namespace fb {
void plan_set_nt_always(fb_plan *p, bool on)
{
    if (p) p->nt_always = on;
}
}  // namespace fb

namespace {

int check_plan(const fb_plan *p)
{
    if (!p) return fail(FB_ERR_INVALID_ARG, "plan is NULL");
    return FB_OK;
}

int check_grid_ptr(const fb_plan *p, const void *ptr, const char *name)
{
    if (!ptr) return fail(FB_ERR_INVALID_ARG, "%s is NULL", name);
    if ((uintptr_t)ptr % (uintptr_t)p->esize)
        return fail(FB_ERR_INVALID_ARG, "%s is not aligned to the %d-byte element", name, p->esize);
    return FB_OK;
}

int check_no_partial_overlap(const fb_plan *p, const void *a, const void *b, bool allow_equal, const char *what)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b, n = (uintptr_t)(p->N * p->esize);
    if (x == y) return allow_equal ? FB_OK : fail(FB_ERR_INVALID_ARG, "%s: buffers must not alias", what);
    if (x < y + n && y < x + n) return fail(FB_ERR_INVALID_ARG, "%s: buffers partially overlap", what);
    return FB_OK;
}

int check_device(const fb_plan *p)
{
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (cur != p->device)
        return fail(FB_ERR_INVALID_ARG, "plan was created on device %d but device %d is current", p->device, cur);
    return FB_OK;
}

const void *axis_table(const fb_plan *p, int a)
{
    if (p->esize == 16) return p->tw64 + p->ax[a].tw_off;
    return p->tw32 + p->ax[a].tw_off;
}

// Largest element index touched by a pass over `total` elements; must stay
// below it.
bool pass_in_bounds(const PassArgs &g, int64_t n, int64_t total)
{
    const int64_t np = g.npencils;
    const int64_t in_max = (np < g.inner ? np : g.inner) - 1;
    const int64_t max_base = ((np - 1) / g.inner) * g.outer + in_max * g.istep;
    return max_base + (n - 1) * g.stride < total && max_base >= 0;
}

// Evolution constants of a multi-output evolve pass.
struct MultiOut {
    int nout;
    double cs[FB_MAX_FUSED_STEPS];
};

// One pencil pass along axis a.  ngrids > 1 runs it over that many
// consecutive grids in one launch; `multi` (contiguous evolve pass only)
// writes multi->nout outputs, N elements apart, from one read of `in`.
int launch_axis(const fb_plan *p, int a, const void *in, void *out, int inv, double scale, const PassArgs *ev,
                hipStream_t st, const uint64_t *gen_seed = nullptr, int ngrids = 1, const MultiOut *multi = nullptr)
{
    const AxisPlan &A = p->ax[a];
    if (!A.pass.launch) return fail(FB_ERR_UNSUPPORTED_SIZE, "no pass for length %lld", (long long)A.n);
    const bool pair = !multi && A.pass_pair.launch && (uintptr_t)in % 16 == 0 && (uintptr_t)out % 16 == 0;
    PassInfo pm{nullptr, 0, 0, 0};
    if (multi) {
        if (!A.contig || !ev || ngrids != 1 || multi->nout < 1 || multi->nout > FB_MAX_FUSED_STEPS)
            return fail(FB_ERR_INVALID_ARG, "internal: multi-output pass misuse");
        pm = fb::find_pass_multi(p->esize, (int)A.n, A.pass.mx != 0);
        if (!pm.launch || pm.mx != A.pass.mx) return fail(FB_ERR_UNSUPPORTED_SIZE, "no multi-output pass");
    }
    const PassInfo &pi = multi ? pm : pair ? A.pass_pair : A.pass;
    PassArgs args{};
    args.in = in;
    args.out = out;
    args.tw = axis_table(p, a);
    args.npencils = A.npencils * ngrids;
    args.inner = A.inner;
    // the x axis has all pencils of a grid in its inner group; further grids
    // follow N elements apart
    args.outer = (ngrids > 1 && A.npencils <= A.inner) ? p->N : A.outer;
    args.istep = A.istep;
    args.stride = A.stride;
    if (!pass_in_bounds(args, A.n, p->N * ngrids)) return fail(FB_ERR_INVALID_ARG, "internal: pass geometry out of bounds");
    if (multi) {
        args.nout = multi->nout;
        args.out_step = p->N;
        for (int j = 0; j < multi->nout; j++) args.ev_cs[j] = multi->cs[j];
    }
    args.inv = inv;
    args.scale = scale;
    args.nt = (p->nt_always || (double)ngrids * (double)p->N * (double)p->esize >= (double)FB_NT_MIN_BYTES) ? 1 : 0;
    if (ev) {
        args.evolve = 1;
        args.ev_c = ev->ev_c;
        args.ev_d = ev->ev_d;
        args.ev_la = ev->ev_la;
        args.ev_lb = ev->ev_lb;
    }
    if (gen_seed) {
        args.gen = 1;
        args.gen_seed = *gen_seed;
    }
    char name[128];
    char multi_tag[32] = "";
    if (multi) snprintf(multi_tag, sizeof multi_tag, ",outputs=%d", multi->nout);
    char grids_tag[32] = "";
    if (ngrids > 1) snprintf(grids_tag, sizeof grids_tag, ",grids=%d", ngrids);
    snprintf(name, sizeof name, "fft_pass<%s,n=%lld,%s%s%s%s%s%s%s>", dtype_tag(p->esize), (long long)A.n,
             A.contig ? "contiguous" : "strided", pi.mx ? ",mfma" : "", pair ? ",pairs" : "", ev ? ",evolve" : "",
             gen_seed ? ",generated-input" : "", multi_tag, grids_tag);
    // a pass with generated input only writes the grid; a multi-output pass
    // reads once and writes nout times
    const double reads = gen_seed ? 0.0 : 1.0;
    const double writes = multi ? (double)multi->nout : 1.0;
    const double bytes = (reads + writes) * (double)ngrids * (double)p->N * (double)p->esize;
    const fb::PassLauncher launcher = pi.pick(args);
    hipError_t e = timed_launch(name, bytes, st, [&] { return launcher(args, st); });
    if (e != hipSuccess) return hip_fail(e, "pass launch");
    return FB_OK;
}

// Runs the active passes z, y, x.  The first active pass reads `in`; later
// ones work in place on `out`.  `ev` (optional) fuses the evolution into the
// first pass, which must then be the contiguous z pass.
int run_passes(const fb_plan *p, const void *in, void *out, int dir, const PassArgs *ev, hipStream_t st,
               int axes = 7, const uint64_t *gen_seed = nullptr)
{
    int last = -1;
    double nsel = 1.0;
    for (int a = 0; a < 3; a++)
        if ((axes >> a & 1) && p->ax[a].n > 1) {
            last = a;
            nsel *= (double)p->ax[a].n;
        }
    if (last < 0) {
        if (gen_seed) {   // a 1x1x1 grid: the transform is the identity
            hipError_t e = fb::launch_fill_uniform(p->esize, out, p->N, *gen_seed, st);
            if (e != hipSuccess) return hip_fail(e, "fill launch");
            return FB_OK;
        }
        if (in != out) {
            hipError_t e = hipMemcpyAsync(out, in, (size_t)p->N * (size_t)p->esize, hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
        }
        return FB_OK;
    }
    bool first = true;
    for (int a = 0; a < 3; a++) {
        if (!(axes >> a & 1) || p->ax[a].n <= 1) continue;
        const double scale = (dir > 0 && a == last) ? 1.0 / nsel : 1.0;
        int rc = launch_axis(p, a, first ? in : out, out, dir > 0, scale, first ? ev : nullptr, st,
                             first ? gen_seed : nullptr);
        if (rc) return rc;
        first = false;
    }
    return FB_OK;
}

int check_alpha_t(double alpha, double t)
{
    if (!isfinite(alpha) || alpha < 0) return fail(FB_ERR_INVALID_ARG, "alpha must be finite and >= 0");
    if (!isfinite(t) || t < 0) return fail(FB_ERR_INVALID_ARG, "t must be finite and >= 0");
    return FB_OK;
}

double evolve_c(double alpha, double t)
{
    const double four_pi2 = 4.0 * M_PI * M_PI;
    return four_pi2 * alpha * t;
}

}  // namespace

extern "C" {

int fb_version(void) { return 100; }

int fb_last_error(const char **msg)
{
    if (msg) *msg = g_msg.c_str();
    return g_code;
}

int fb_describe_shape(int64_t nx, int64_t ny, int64_t nz, int dtype, char *buf, int cap)
{
    if (check_shape(nx, ny, nz, dtype)) return g_code;
    if (!buf || cap <= 0) return fail(FB_ERR_INVALID_ARG, "buf is NULL or cap <= 0");
    AxisPlan ax[3];
    build_axes(nx, ny, nz, esize_of(dtype), dtype == FB_C64_SPLITBF16, ax);
    // the host-side lookup must find an instantiated pass for every axis
    // (the same lookup fb_fft3d_plan makes; no device needed)
    for (int a = 0; a < 3; a++)
        if (ax[a].n > 1 && (!ax[a].pass.launch || ax[a].pass.pencils_per_wg < 1))
            return fail(FB_ERR_UNSUPPORTED_SIZE, "internal: no pass instantiated for length %lld",
                        (long long)ax[a].n);
    char tmp[256];
    describe(ax, tmp, sizeof tmp);
    const int len = (int)strlen(tmp);
    if (len + 1 > cap) return fail(FB_ERR_INVALID_ARG, "buffer too small (%d bytes needed)", len + 1);
    memcpy(buf, tmp, (size_t)len + 1);
    ok();
    return len;
}

fb_plan *fb_fft3d_plan(int64_t nx, int64_t ny, int64_t nz, int dtype)
{
    if (check_shape(nx, ny, nz, dtype)) return nullptr;
    fb_plan *p = new (std::nothrow) fb_plan();
    if (!p) {
        fail(FB_ERR_OOM, "host allocation failed");
        return nullptr;
    }
    p->nx = nx; p->ny = ny; p->nz = nz; p->N = nx * ny * nz;
    p->dtype = dtype;
    p->esize = esize_of(dtype);
    build_axes(nx, ny, nz, p->esize, dtype == FB_C64_SPLITBF16, p->ax);
    for (int a = 0; a < 3; a++) {
        if (p->ax[a].n > 1 && !p->ax[a].pass.launch) {
            fail(FB_ERR_UNSUPPORTED_SIZE, "no pass for length %lld", (long long)p->ax[a].n);
            delete p;
            return nullptr;
        }
    }
    describe(p->ax, p->desc, sizeof p->desc);
    p->tw_total = 0;
    for (int a = 0; a < 3; a++) p->tw_total += (size_t)p->ax[a].rp.twlen;

    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        hip_fail(e, "hipGetDevice");
        delete p;
        return nullptr;
    }
    const size_t nt = p->tw_total > 0 ? p->tw_total : 1;
    e = hipMalloc((void **)&p->tw64, nt * sizeof(double2));
    if (e == hipSuccess) e = hipMalloc((void **)&p->tw32, nt * sizeof(float2));
    if (e != hipSuccess) {
        hip_fail(e, "hipMalloc (twiddle tables)");
        fb_fft3d_destroy(p);
        return nullptr;
    }
    for (int a = 0; a < 3 && e == hipSuccess; a++) {
        const AxisPlan &A = p->ax[a];
        if (A.rp.twlen == 0) continue;
        fb::TwDesc d{};
        d.nst = A.rp.count;
        for (int s = 0; s < A.rp.count; s++) {
            d.r[s] = A.rp.r[s];
            d.ns[s] = A.rp.ns[s];
            d.off[s] = A.rp.twoff[s];
        }
        d.total = A.rp.twlen;
        e = fb::launch_twiddles(d, p->tw64 + A.tw_off, p->tw32 + A.tw_off, nullptr);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        hip_fail(e, "twiddle generation");
        fb_fft3d_destroy(p);
        return nullptr;
    }
    ok();
    return p;
}

void fb_fft3d_destroy(fb_plan *p)
{
    if (!p) return;
    if (p->tw64) (void)hipFree(p->tw64);
    if (p->tw32) (void)hipFree(p->tw32);
    delete p;
}

size_t fb_plan_device_bytes(const fb_plan *p)
{
    if (!p) return 0;
    const size_t nt = p->tw_total > 0 ? p->tw_total : 1;
    return nt * (sizeof(double2) + sizeof(float2));
}

const char *fb_plan_describe(const fb_plan *p)
{
    if (!p) {
        fail(FB_ERR_INVALID_ARG, "plan is NULL");
        return "";
    }
    return p->desc;
}

fb_status fb_fft3d_exec(const fb_plan *p, const void *in, void *out, int dir, void *hip_stream)
{
    if (check_plan(p) || check_grid_ptr(p, in, "in") || check_grid_ptr(p, out, "out")) return (fb_status)g_code;
    if (dir != FB_FORWARD && dir != FB_INVERSE)
        return (fb_status)fail(FB_ERR_INVALID_ARG, "dir must be FB_FORWARD (-1) or FB_INVERSE (+1), got %d", dir);
    if (check_no_partial_overlap(p, in, out, true, "fb_fft3d_exec")) return (fb_status)g_code;
    if (check_device(p)) return (fb_status)g_code;
    if (run_passes(p, in, out, dir, nullptr, (hipStream_t)hip_stream)) return (fb_status)g_code;
    return (fb_status)ok();
}

fb_status fb_lu_factor(double *a, int64_t n, int64_t lda, int32_t *ipiv, int32_t *info, void *hip_stream)
{
    if (n < 1 || n > fb::LU_MAX_N)
        return (fb_status)fail(FB_ERR_UNSUPPORTED_SIZE, "n must be in 1..%lld, got %lld", (long long)fb::LU_MAX_N,
                               (long long)n);
    if (lda < n) return (fb_status)fail(FB_ERR_INVALID_ARG, "lda (%lld) < n (%lld)", (long long)lda, (long long)n);
    if (!a || (uintptr_t)a % 8) return (fb_status)fail(FB_ERR_INVALID_ARG, "a is NULL or not 8-byte aligned");
    if (!ipiv || (uintptr_t)ipiv % 4 || !info || (uintptr_t)info % 4)
        return (fb_status)fail(FB_ERR_INVALID_ARG, "ipiv / info is NULL or not 4-byte aligned");
    {
        // ipiv and info must not overlap the matrix
        const uintptr_t a0 = (uintptr_t)a, a1 = a0 + (uintptr_t)((n - 1) * lda + n) * 8;
        const uintptr_t p0 = (uintptr_t)ipiv, p1 = p0 + (uintptr_t)n * 4, i0 = (uintptr_t)info, i1 = i0 + 4;
        if ((p0 < a1 && a0 < p1) || (i0 < a1 && a0 < i1) || (i0 < p1 && p0 < i1))
            return (fb_status)fail(FB_ERR_INVALID_ARG, "a, ipiv and info must not overlap");
    }
    hipStream_t st = (hipStream_t)hip_stream;
    // model bytes: the trailing updates read and write A22 once per panel
    double bytes = 0.0;
    for (int64_t k = 0; k < n; k += fb::LU_NB) {
        const double r = (double)(n - k);
        bytes += 16.0 * r * r;
    }
    hipError_t e = timed_launch("lu<f64>", bytes, st, [&] { return fb::launch_lu(a, n, lda, ipiv, info, st); });
    if (e != hipSuccess) return (fb_status)hip_fail(e, "lu launch");
    return (fb_status)ok();
}

fb_status fb_fft3d_exec_host(const fb_plan *p, const void *in_host, void *out_host, int dir)
{
    if (check_plan(p)) return (fb_status)g_code;
    if (!in_host || !out_host) return (fb_status)fail(FB_ERR_INVALID_ARG, "in_host / out_host is NULL");
    if (dir != FB_FORWARD && dir != FB_INVERSE)
        return (fb_status)fail(FB_ERR_INVALID_ARG, "dir must be FB_FORWARD (-1) or FB_INVERSE (+1), got %d", dir);
    if (check_device(p)) return (fb_status)g_code;
    const size_t bytes = (size_t)p->N * (size_t)p->esize;
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, bytes);
    if (e != hipSuccess) return (fb_status)fail(FB_ERR_OOM, "hipMalloc of %zu bytes failed", bytes);
    e = hipMemcpy(d, in_host, bytes, hipMemcpyHostToDevice);
    int rc = e != hipSuccess ? hip_fail(e, "host-to-device copy") : run_passes(p, d, d, dir, nullptr, nullptr);
    if (!rc) {
        e = hipMemcpy(out_host, d, bytes, hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc = hip_fail(e, "device-to-host copy");
    }
    (void)hipFree(d);
    if (rc) return (fb_status)rc;
    return (fb_status)ok();
}

// Serialises the calls of fb_fft3d_exec_host_noalloc within the process:
// they share one staging buffer per device.
static std::mutex g_static_mu;

fb_status fb_fft3d_exec_host_noalloc(const fb_plan *p, const void *in_host, void *out_host, int dir)
{
    if (check_plan(p)) return (fb_status)g_code;
    if (!in_host || !out_host) return (fb_status)fail(FB_ERR_INVALID_ARG, "in_host / out_host is NULL");
    if (dir != FB_FORWARD && dir != FB_INVERSE)
        return (fb_status)fail(FB_ERR_INVALID_ARG, "dir must be FB_FORWARD (-1) or FB_INVERSE (+1), got %d", dir);
    const size_t bytes = (size_t)p->N * (size_t)p->esize;
    if (bytes > (size_t)FB_STATIC_SCRATCH_BYTES)
        return (fb_status)fail(FB_ERR_UNSUPPORTED_SIZE,
                               "grid of %zu bytes exceeds the %zu-byte static staging buffer of the "
                               "allocation-free form (use fb_fft3d_exec_host)",
                               bytes, (size_t)FB_STATIC_SCRATCH_BYTES);
    if (check_device(p)) return (fb_status)g_code;
    std::lock_guard<std::mutex> lk(g_static_mu);
    void *d = nullptr;
    hipError_t e = fb::static_scratch(&d);
    if (e != hipSuccess) return (fb_status)hip_fail(e, "hipGetSymbolAddress (static staging buffer)");
    e = hipMemcpy(d, in_host, bytes, hipMemcpyHostToDevice);
    int rc = e != hipSuccess ? hip_fail(e, "host-to-device copy") : run_passes(p, d, d, dir, nullptr, nullptr);
    if (!rc) {
        e = hipMemcpy(out_host, d, bytes, hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc = hip_fail(e, "device-to-host copy");
    }
    if (rc) return (fb_status)rc;
    return (fb_status)ok();
}

fb_status fb_fft3d_exec_axes(const fb_plan *p, const void *in, void *out, int dir, int axes, void *hip_stream)
{
    if (check_plan(p) || check_grid_ptr(p, in, "in") || check_grid_ptr(p, out, "out")) return (fb_status)g_code;
    if (dir != FB_FORWARD && dir != FB_INVERSE)
        return (fb_status)fail(FB_ERR_INVALID_ARG, "dir must be FB_FORWARD (-1) or FB_INVERSE (+1), got %d", dir);
    if (axes < 0 || axes > 7) return (fb_status)fail(FB_ERR_INVALID_ARG, "axes must be a mask of bits 0 (z), 1 (y), 2 (x)");
    if (check_no_partial_overlap(p, in, out, true, "fb_fft3d_exec_axes")) return (fb_status)g_code;
    if (check_device(p)) return (fb_status)g_code;
    if (run_passes(p, in, out, dir, nullptr, (hipStream_t)hip_stream, axes)) return (fb_status)g_code;
    return (fb_status)ok();
}

int fb_profile_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_clear_locked();
    g_prof_on = on != 0;
    return ok();
}

int fb_profile_report(char *buf, int cap)
{
    if (!buf || cap <= 0) return fail(FB_ERR_INVALID_ARG, "buf is NULL or cap <= 0");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    struct Agg {
        std::string name;
        long n;
        double ms, bytes;
    };
    std::vector<Agg> agg;
    for (auto &r : g_prof) {
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        size_t i = 0;
        while (i < agg.size() && agg[i].name != r.name) i++;
        if (i == agg.size()) agg.push_back({r.name, 0, 0.0, r.bytes});
        agg[i].n++;
        agg[i].ms += ms;
    }
    std::string js = "[";
    for (size_t i = 0; i < agg.size(); i++) {
        char line[256];
        snprintf(line, sizeof line, "%s{\"kernel\": \"%s\", \"launches\": %ld, \"total_ms\": %.6f, \"avg_ms\": %.6f, "
                 "\"bytes_per_launch\": %.0f}", i ? ", " : "", agg[i].name.c_str(), agg[i].n, agg[i].ms,
                 agg[i].ms / (double)agg[i].n, agg[i].bytes);
        js += line;
    }
    js += "]";
    if ((int)js.size() + 1 > cap) return fail(FB_ERR_INVALID_ARG, "buffer too small (%d bytes needed)", (int)js.size() + 1);
    memcpy(buf, js.c_str(), js.size() + 1);
    ok();
    return (int)js.size();
}

fb_status fb_spectral_evolve(const fb_plan *p, void *u, double alpha, double t, void *hip_stream)
{
    if (check_plan(p) || check_grid_ptr(p, u, "u") || check_alpha_t(alpha, t)) return (fb_status)g_code;
    if (check_device(p)) return (fb_status)g_code;
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = timed_launch(p->esize == 16 ? "evolve<c128>" : "evolve<c64>", 2.0 * p->N * p->esize, st, [&] {
        return fb::launch_evolve(p->esize, u, u, p->nx, p->ny, p->nz, evolve_c(alpha, t), st);
    });
    if (e != hipSuccess) return (fb_status)hip_fail(e, "evolve launch");
    return (fb_status)ok();
}

fb_status fb_checksum(const fb_plan *p, const void *x, double *out2_dev, void *hip_stream)
{
    if (check_plan(p) || check_grid_ptr(p, x, "x")) return (fb_status)g_code;
    if (!out2_dev || (uintptr_t)out2_dev % 8) return (fb_status)fail(FB_ERR_INVALID_ARG, "out2_dev is NULL or misaligned");
    if (check_device(p)) return (fb_status)g_code;
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = timed_launch(p->esize == 16 ? "checksum<c128>" : "checksum<c64>", 1024.0 * p->esize + 16, st,
                                [&] { return fb::launch_checksum(p->esize, x, p->N, out2_dev, st); });
    if (e != hipSuccess) return (fb_status)hip_fail(e, "checksum launch");
    return (fb_status)ok();
}

fb_status fb_spectral_step(const fb_plan *p, const void *uhat0, void *x_out, double alpha, double t,
                           double *out2_dev, void *hip_stream)
{
    if (check_plan(p) || check_grid_ptr(p, uhat0, "uhat0") || check_grid_ptr(p, x_out, "x_out") ||
        check_alpha_t(alpha, t))
        return (fb_status)g_code;
    if (out2_dev && (uintptr_t)out2_dev % 8) return (fb_status)fail(FB_ERR_INVALID_ARG, "out2_dev is misaligned");
    if (check_no_partial_overlap(p, uhat0, x_out, false, "fb_spectral_step")) return (fb_status)g_code;
    if (check_device(p)) return (fb_status)g_code;
    hipStream_t st = (hipStream_t)hip_stream;
    const double c = evolve_c(alpha, t);
    if (p->nz > 1) {
        // z pass pencils are (x, y): p = x ny + y
        PassArgs ev{};
        ev.ev_c = c;
        ev.ev_d = p->ny;
        ev.ev_la = (int)p->nx;
        ev.ev_lb = (int)p->ny;
        if (run_passes(p, uhat0, x_out, FB_INVERSE, &ev, st)) return (fb_status)g_code;
    } else {
        hipError_t e = timed_launch(p->esize == 16 ? "evolve<c128>" : "evolve<c64>", 2.0 * p->N * p->esize, st,
                                    [&] { return fb::launch_evolve(p->esize, uhat0, x_out, p->nx, p->ny, p->nz, c, st); });
        if (e != hipSuccess) return (fb_status)hip_fail(e, "evolve launch");
        if (run_passes(p, x_out, x_out, FB_INVERSE, nullptr, st)) return (fb_status)g_code;
    }
    if (out2_dev) {
        hipError_t e = timed_launch(p->esize == 16 ? "checksum<c128>" : "checksum<c64>", 1024.0 * p->esize + 16, st,
                                    [&] { return fb::launch_checksum(p->esize, x_out, p->N, out2_dev, st); });
        if (e != hipSuccess) return (fb_status)hip_fail(e, "checksum launch");
    }
    return (fb_status)ok();
}

fb_status fb_spectral_steps(const fb_plan *p, const void *uhat0, void *x_out, double alpha, const double *t,
                            int nsteps, double *sums_dev, void *hip_stream)
{
    if (check_plan(p) || check_grid_ptr(p, uhat0, "uhat0") || check_grid_ptr(p, x_out, "x_out"))
        return (fb_status)g_code;
    if (nsteps < 1 || !t) return (fb_status)fail(FB_ERR_INVALID_ARG, "need nsteps >= 1 and a host array t");
    for (int j = 0; j < nsteps; j++)
        if (check_alpha_t(alpha, t[j])) return (fb_status)g_code;
    if (sums_dev && (uintptr_t)sums_dev % 8) return (fb_status)fail(FB_ERR_INVALID_ARG, "sums_dev is misaligned");
    {
        const uintptr_t u = (uintptr_t)uhat0, x = (uintptr_t)x_out;
        const uintptr_t g = (uintptr_t)(p->N * p->esize), xs = g * (uintptr_t)nsteps;
        if (u < x + xs && x < u + g) return (fb_status)fail(FB_ERR_INVALID_ARG, "fb_spectral_steps: x_out overlaps uhat0");
    }
    if (check_device(p)) return (fb_status)g_code;
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t gbytes = (size_t)p->N * (size_t)p->esize;
    if (p->nz <= 1) {   // no contiguous evolve pass to share: one step at a time
        for (int j = 0; j < nsteps; j++) {
            fb_status rc = fb_spectral_step(p, uhat0, (char *)x_out + gbytes * j, alpha, t[j],
                                            sums_dev ? sums_dev + 2 * j : nullptr, hip_stream);
            if (rc) return rc;
        }
        return (fb_status)ok();
    }
    int last = -1;
    double nsel = 1.0;
    for (int a = 0; a < 3; a++)
        if (p->ax[a].n > 1) {
            last = a;
            nsel *= (double)p->ax[a].n;
        }
    PassArgs ev{};
    ev.ev_d = p->ny;
    ev.ev_la = (int)p->nx;
    ev.ev_lb = (int)p->ny;
    for (int j0 = 0; j0 < nsteps; j0 += FB_MAX_FUSED_STEPS) {
        const int k = nsteps - j0 < FB_MAX_FUSED_STEPS ? nsteps - j0 : FB_MAX_FUSED_STEPS;
        MultiOut m{};
        m.nout = k;
        for (int i = 0; i < k; i++) m.cs[i] = evolve_c(alpha, t[j0 + i]);
        char *xo = (char *)x_out + gbytes * j0;
        // z: evolve + inverse DFT of the spectrum into k grids; then y and x over all k grids
        int rc = launch_axis(p, 0, uhat0, xo, 1, last == 0 ? 1.0 / nsel : 1.0, &ev, st, nullptr, 1, &m);
        for (int a = 1; !rc && a < 3; a++)
            if (p->ax[a].n > 1) rc = launch_axis(p, a, xo, xo, 1, a == last ? 1.0 / nsel : 1.0, nullptr, st, nullptr, k);
        if (rc) return (fb_status)rc;
        if (sums_dev) {
            hipError_t e = timed_launch(p->esize == 16 ? "checksum<c128>" : "checksum<c64>",
                                        (1024.0 * p->esize + 16) * k, st,
                                        [&] { return fb::launch_checksum(p->esize, xo, p->N, sums_dev + 2 * j0, st, k); });
            if (e != hipSuccess) return (fb_status)hip_fail(e, "checksum launch");
        }
    }
    return (fb_status)ok();
}

fb_status fb_fft3d_forward_uniform(const fb_plan *p, uint64_t seed, void *out, void *hip_stream)
{
    if (check_plan(p) || check_grid_ptr(p, out, "out")) return (fb_status)g_code;
    if (check_device(p)) return (fb_status)g_code;
    // the first pass generates its input; `in` is never read, `out` stands in
    if (run_passes(p, out, out, FB_FORWARD, nullptr, (hipStream_t)hip_stream, 7, &seed)) return (fb_status)g_code;
    return (fb_status)ok();
}

fb_status fb_fill_uniform(const fb_plan *p, void *x, uint64_t seed, void *hip_stream)
{
    if (check_plan(p) || check_grid_ptr(p, x, "x")) return (fb_status)g_code;
    if (check_device(p)) return (fb_status)g_code;
    hipError_t e = fb::launch_fill_uniform(p->esize, x, p->N, seed, (hipStream_t)hip_stream);
    if (e != hipSuccess) return (fb_status)hip_fail(e, "fill launch");
    return (fb_status)ok();
}

}  // extern "C"

// ======================================================================
// Batched form: many independent complex64 1D transforms of mixed lengths
// plus 2D transforms, packed back to back in one buffer.
// ======================================================================

#include <algorithm>
#include <map>

#include "fb_batch.hpp"

struct fb_batch {
    int n1d, n2d;
    int64_t side2d;
    int64_t total;                 // complex elements of the packed layout
    std::vector<int64_t> len, off; // per transform (1D first, then 2D)
    std::vector<fb::BatchGroup> groups;
    int phase1_begin;                // first group of phase 1
    int64_t ntasks[2];               // tiles per phase
    fb::BatchGroup *groups_dev;
    std::vector<void *> dev_allocs;  // tables, segment offsets
    int device;
    int nblocks[2];                  // persistent grid per phase
    int lds_bytes[2];                // persistent LDS per phase: the largest tile kind of the phase
    // the single-launch form: item lists per workgroup (empty when some
    // transform's tiles straddle transforms, and the per-phase form is used)
    bool onelaunch = false;
    int ol_nblocks = 0, ol_lds_bytes = 0;
    int64_t ol_items = 0;
    double ol_balance = 0.0;         // largest workgroup load / mean load (model bytes)
    fb::BatchItem *items_dev = nullptr;
    int64_t *item_begin_dev = nullptr;
    std::string desc;
};

namespace {

// Split of a long transform n = n1 * n2 into two strided passes (n1 first);
// n2 is the power of two nearest sqrt(n) from above, at most 512.
void batch_split(int64_t n, int64_t &n1, int64_t &n2)
{
    int lg = 0;
    while ((int64_t(1) << (lg + 1)) <= n) lg++;
    int64_t k = (lg + 1) / 2 + ((lg + 1) % 2);   // ceil(log2(n) / 2), approximately
    if (k > 9) k = 9;
    n2 = int64_t(1) << k;
    while (n2 > 2 && (n % n2 != 0 || n / n2 > 4096)) n2 >>= 1;
    n1 = n / n2;
}

bool batch_length_ok(int64_t n)
{
    if (fb::supported_length_b1(n)) return n >= 2;
    if (n <= 4096 || n > 4096 * 512) return false;
    int64_t n1, n2;
    batch_split(n, n1, n2);
    return n1 * n2 == n && fb::supported_length_b1(n1) && fb::supported_length_b1(n2) && n1 >= 2 && n2 >= 2;
}

template <class T> T *dev_alloc(fb_batch *b, size_t count, hipError_t &e)
{
    T *p = nullptr;
    e = hipMalloc((void **)&p, count * sizeof(T) + 16);
    if (e == hipSuccess) b->dev_allocs.push_back(p);
    return p;
}

void batch_free(fb_batch *b)
{
    for (void *p : b->dev_allocs) (void)hipFree(p);
    b->dev_allocs.clear();
}

// Fills the geometry of a pass over segments of `segp` pencils each.
void set_geom(PassArgs &a, int64_t npencils, int64_t segp, const int64_t *seg_off, int64_t inner, int64_t outer,
              int64_t istep, int64_t stride)
{
    a.npencils = npencils;
    a.seg_pencils = segp;
    a.seg_off = seg_off;
    a.inner = inner;
    a.outer = outer;
    a.istep = istep;
    a.stride = stride;
}

int64_t gcd64(int64_t a, int64_t b) { return b == 0 ? a : gcd64(b, a % b); }

// Pencils per tile of an instantiated pass; 1 (and `bad` set) when the
// length has no pass, so that no tile count divides by zero.
int tile_pencils_of(const PassInfo &pi, bool &bad)
{
    if (!pi.launch || pi.pencils_per_wg < 1) {
        bad = true;
        return 1;
    }
    return pi.pencils_per_wg;
}

// Smallest number of consecutive segments (transforms) of a group that its
// tiles cover exactly: tiles hold tile_pencils pencils and start at pencil 0.
int64_t segments_per_chunk(const fb::BatchGroup &g)
{
    const int64_t p = g.tile_pencils, sp = g.args.seg_pencils;
    return p / gcd64(p, sp);
}

// Work items of the single-launch form and their order: the two passes of
// every two-pass 1D transform and of every 2D transform as one item (of the
// fewest consecutive transforms whose pencils both passes' tiles cover
// exactly, usually one), every tile of a single-pass group as one item;
// items are handed out by longest processing time first (largest model
// bytes first, each to the workgroup with the least load so far), so that
// the loads even out.  Returns false when a pair's chunks would not cover
// its tiles (not expected: both passes see the same transforms).
bool build_onelaunch_items(const std::vector<fb::BatchGroup> &groups, const std::vector<std::pair<int, int>> &pairs,
                           const std::vector<int> &singles, int nwg, std::vector<fb::BatchItem> &items,
                           std::vector<int64_t> &begin, double &balance)
{
    // model bytes of one tile: the transform data it reads and writes, plus
    // a fixed allowance for the tile's latency (barriers, twiddles)
    constexpr double kTileOverhead = 32768.0;
    struct Cand {
        fb::BatchItem it;
        double cost;
    };
    std::vector<Cand> c;
    for (const auto &pr : pairs) {
        const fb::BatchGroup &g1 = groups[(size_t)pr.first], &g2 = groups[(size_t)pr.second];
        const int64_t sp1 = g1.args.seg_pencils, sp2 = g2.args.seg_pencils;
        if (g1.tile_pencils < 1 || g2.tile_pencils < 1 || sp1 < 1 || sp2 < 1) return false;
        const int64_t nseg = g1.args.npencils / sp1;
        if (nseg * sp1 != g1.args.npencils || nseg * sp2 != g2.args.npencils) return false;
        const int64_t m1 = segments_per_chunk(g1), m2 = segments_per_chunk(g2);
        const int64_t m = m1 / gcd64(m1, m2) * m2;   // transforms per item
        const double seg_elems = (double)sp1 * (double)g1.n;   // = the transform's length
        for (int64_t s0 = 0; s0 < nseg; s0 += m) {
            const int64_t s1 = s0 + m < nseg ? s0 + m : nseg;
            // tiles of g covering pencils [s0 sp, s1 sp): s0 sp is a tile boundary
            auto range = [&](const fb::BatchGroup &g, int64_t sp, int64_t &a, int64_t &b) {
                a = s0 * sp / g.tile_pencils;
                b = s1 == nseg ? g.ntiles : s1 * sp / g.tile_pencils;
            };
            fb::BatchItem it{pr.first, pr.second, 0, 0, 0, 0};
            range(g1, sp1, it.a1, it.b1);
            range(g2, sp2, it.a2, it.b2);
            const double cost = 2.0 * 16.0 * seg_elems * (double)(s1 - s0) +
                                kTileOverhead * (double)(it.b1 - it.a1 + it.b2 - it.a2);
            c.push_back({it, cost});
        }
    }
    for (int gi : singles) {
        const fb::BatchGroup &g = groups[(size_t)gi];
        const double per_tile = (double)g.args.npencils * (double)g.n * 16.0 / (double)g.ntiles + kTileOverhead;
        for (int64_t t = 0; t < g.ntiles; t++) c.push_back({{gi, -1, t, t + 1, 0, 0}, per_tile});
    }
    std::stable_sort(c.begin(), c.end(), [](const Cand &x, const Cand &y) { return x.cost > y.cost; });
    // least-loaded workgroup first (ties: lower index), by a binary heap
    std::vector<std::pair<double, int>> heap;
    for (int w = 0; w < nwg; w++) heap.push_back({0.0, w});
    auto gt = [](const std::pair<double, int> &x, const std::pair<double, int> &y) {
        return x.first > y.first || (x.first == y.first && x.second > y.second);
    };
    std::make_heap(heap.begin(), heap.end(), gt);
    std::vector<std::vector<fb::BatchItem>> per(nwg);
    std::vector<double> load(nwg, 0.0);
    for (const Cand &x : c) {
        std::pop_heap(heap.begin(), heap.end(), gt);
        auto &top = heap.back();
        per[(size_t)top.second].push_back(x.it);
        top.first += x.cost;
        load[(size_t)top.second] = top.first;
        std::push_heap(heap.begin(), heap.end(), gt);
    }
    items.clear();
    begin.assign(1, 0);
    double mx = 0.0, sum = 0.0;
    for (int w = 0; w < nwg; w++) {
        for (const auto &it : per[(size_t)w]) items.push_back(it);
        begin.push_back((int64_t)items.size());
        mx = load[(size_t)w] > mx ? load[(size_t)w] : mx;
        sum += load[(size_t)w];
    }
    balance = sum > 0.0 ? mx / (sum / nwg) : 1.0;
    return true;
}

// Largest element touched by a group, relative to its segment start.
bool group_in_bounds(const fb::BatchGroup &g, int64_t seg_max_off, int64_t total)
{
    const PassArgs &a = g.args;
    const int64_t np = a.seg_pencils;
    auto reach = [&](int64_t inner, int64_t outer, int64_t istep, int64_t stride) {
        const int64_t in_max = (np < inner ? np : inner) - 1;
        return ((np - 1) / inner) * outer + in_max * istep + (int64_t)(g.n - 1) * stride;
    };
    if (seg_max_off + reach(a.inner, a.outer, a.istep, a.stride) >= total) return false;
    if (a.ostride && seg_max_off + reach(a.oinner, a.oouter, a.oistep, a.ostride) >= total) return false;
    return true;
}

}  // namespace

extern "C" {

fb_batch *fb_batch_plan(const int64_t *lens, int n1d, int n2d, int64_t side2d, int dtype)
{
    if (dtype != FB_C64) {
        fail(FB_ERR_DTYPE, "batched transforms support complex64 (FB_C64) only, got dtype %d", dtype);
        return nullptr;
    }
    if (n1d < 0 || n2d < 0 || n1d + n2d < 1) {
        fail(FB_ERR_INVALID_ARG, "need n1d >= 0, n2d >= 0 and at least one transform");
        return nullptr;
    }
    if (n1d > 0 && !lens) {
        fail(FB_ERR_INVALID_ARG, "lens is NULL");
        return nullptr;
    }
    for (int i = 0; i < n1d; i++)
        if (!batch_length_ok(lens[i])) {
            fail(FB_ERR_UNSUPPORTED_SIZE, "1D length %lld (transform %d) is not supported (2^a or 3*2^a, 2..2^21)",
                 (long long)lens[i], i);
            return nullptr;
        }
    if (n2d > 0 && (side2d < 2 || !fb::supported_length_b1(side2d))) {
        fail(FB_ERR_UNSUPPORTED_SIZE, "2D side %lld is not supported", (long long)side2d);
        return nullptr;
    }
    fb_batch *b = new (std::nothrow) fb_batch();
    if (!b) {
        fail(FB_ERR_OOM, "host allocation failed");
        return nullptr;
    }
    b->n1d = n1d;
    b->n2d = n2d;
    b->side2d = side2d;
    int64_t off = 0;
    for (int i = 0; i < n1d; i++) {
        b->len.push_back(lens[i]);
        b->off.push_back(off);
        off += lens[i];
    }
    for (int j = 0; j < n2d; j++) {
        b->len.push_back(side2d * side2d);
        b->off.push_back(off);
        off += side2d * side2d;
    }
    b->total = off;

    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) {
        hip_fail(e, "hipGetDevice");
        delete b;
        return nullptr;
    }

    // transforms by length
    std::map<int64_t, std::vector<int64_t>> by_len;
    for (int i = 0; i < n1d; i++) by_len[lens[i]].push_back(b->off[i]);

    // stage twiddle tables per pass length, pre-twiddles per long length
    std::map<int64_t, float2 *> stage_tw;
    std::map<int64_t, float2 *> roots;
    double2 *scratch64 = nullptr;
    auto stage_table = [&](int64_t n) -> float2 * {
        auto it = stage_tw.find(n);
        if (it != stage_tw.end()) return it->second;
        fb::RadixPlan rp = fb::radix_plan((int)n);
        const int cnt = rp.twlen > 0 ? rp.twlen : 1;
        float2 *t32 = dev_alloc<float2>(b, cnt, e);
        if (e != hipSuccess) return nullptr;
        if (rp.twlen > 0) {
            double2 *t64 = dev_alloc<double2>(b, cnt, e);
            if (e != hipSuccess) return nullptr;
            fb::TwDesc d{};
            d.nst = rp.count;
            for (int s = 0; s < rp.count; s++) {
                d.r[s] = rp.r[s];
                d.ns[s] = rp.ns[s];
                d.off[s] = rp.twoff[s];
            }
            d.total = rp.twlen;
            e = fb::launch_twiddles(d, t64, t32, nullptr);
        }
        stage_tw[n] = t32;
        return t32;
    };
    (void)scratch64;

    std::vector<fb::BatchGroup> pass1, single, pass2;
    bool nopass = false;   // a pass length without an instantiated pass (not expected)
    auto new_group = [&](int64_t n, bool contig) {
        fb::BatchGroup g{};
        g.n = (int)n;
        g.contig = contig ? 1 : 0;
        g.phase = 0;
        g.args.tw = stage_table(n);
        g.inv_scale = 1.0;
        return g;
    };
    const int esize = 8;
    for (auto &kv : by_len) {
        const int64_t L = kv.first;
        const int64_t cnt = (int64_t)kv.second.size();
        int64_t *soff = dev_alloc<int64_t>(b, kv.second.size(), e);
        if (e == hipSuccess)
            e = hipMemcpy(soff, kv.second.data(), kv.second.size() * sizeof(int64_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) break;
        const int64_t segmax = kv.second.back();
        if (L <= 4096) {
            fb::BatchGroup g = new_group(L, true);
            set_geom(g.args, cnt, 1, soff, 1, L, 0, 1);
            g.in_sel = 0;
            g.out_sel = 1;
            g.last = 1;
            g.inv_scale = 1.0 / (double)L;
            g.tile_pencils = tile_pencils_of(fb::find_pass(esize, (int)L, true, false), nopass);
            g.ntiles = (cnt + g.tile_pencils - 1) / g.tile_pencils;
            if (!group_in_bounds(g, segmax, b->total)) e = hipErrorInvalidValue;
            single.push_back(g);
        } else {
            int64_t n1, n2;
            batch_split(L, n1, n2);
            // pass 1: length-n1 DFTs over b < n2 (elements b + q n2), output to b n1 + q
            fb::BatchGroup g1 = new_group(n1, false);
            set_geom(g1.args, cnt * n2, n2, soff, n2, 0, 1, n2);
            g1.args.oinner = 1;
            g1.args.oouter = n1;
            g1.args.oistep = 0;
            g1.args.ostride = 1;
            g1.args.opair_step = n1;   // pencils b and b + 1 start n1 apart in the output
            g1.in_sel = 0;
            g1.out_sel = 2;   // fixed up per execution when out != in
            g1.last = 0;
            const int P1 = tile_pencils_of(fb::find_pass_pair((int)n1), nopass);
            g1.ntiles = (cnt * n2 + P1 - 1) / P1;
            // a tile's outputs (pencils b .. b + P1 - 1 of one transform) form one
            // block of P1 n1 elements: write it whole when tiles do not straddle
            // transforms
            g1.args.otile = (n2 % P1 == 0) ? 1 : 0;
            g1.tile_pencils = P1;
            // pass 2: pre-twiddle w_L^(q b), length-n2 DFTs over b < n1 (elements b + q n1)
            fb::BatchGroup g2 = new_group(n2, false);
            set_geom(g2.args, cnt * n1, n1, soff, n1, 0, 1, n1);
            auto it = roots.find(L);
            float2 *rt = nullptr;
            if (it != roots.end()) rt = it->second;
            else {
                rt = dev_alloc<float2>(b, L, e);
                if (e == hipSuccess) e = fb::launch_pretwiddle(n1, n2, rt, nullptr);
                roots[L] = rt;
            }
            g2.args.ptw = rt;
            g2.args.ptw_len = L;
            g2.in_sel = 2;
            g2.out_sel = 1;
            g2.last = 1;
            g2.inv_scale = 1.0 / (double)L;
            const int P2 = tile_pencils_of(fb::find_pass_pair((int)n2), nopass);
            g2.ntiles = (cnt * n1 + P2 - 1) / P2;
            g2.tile_pencils = P2;
            // the pass-2 kernel reads the pre-twiddle table at the element's offset
            // within its transform (< n2 n1)
            if (!group_in_bounds(g1, segmax, b->total) || !group_in_bounds(g2, segmax, b->total) ||
                g2.args.ptw_len < n2 * n1)
                e = hipErrorInvalidValue;
            g2.phase = 1;
            pass1.push_back(g1);
            pass2.push_back(g2);
        }
        if (e != hipSuccess) break;
    }
    fb::BatchGroup rows{}, cols{};
    bool has2d = n2d > 0 && e == hipSuccess;
    if (has2d) {
        std::vector<int64_t> o2(b->off.begin() + n1d, b->off.end());
        int64_t *soff = dev_alloc<int64_t>(b, o2.size(), e);
        if (e == hipSuccess) e = hipMemcpy(soff, o2.data(), o2.size() * sizeof(int64_t), hipMemcpyHostToDevice);
        const int64_t s = side2d;
        rows = new_group(s, true);
        set_geom(rows.args, n2d * s, s, soff, 1, s, 0, 1);
        rows.in_sel = 0;
        rows.out_sel = 1;
        rows.tile_pencils = tile_pencils_of(fb::find_pass(esize, (int)s, true, false), nopass);
        rows.ntiles = (n2d * s + rows.tile_pencils - 1) / rows.tile_pencils;
        cols = new_group(s, false);
        set_geom(cols.args, n2d * s, s, soff, s, 0, 1, s);
        cols.in_sel = 1;
        cols.out_sel = 1;
        cols.last = 1;
        cols.phase = 1;
        cols.inv_scale = 1.0 / (double)(s * s);
        cols.tile_pencils = tile_pencils_of(fb::find_pass_pair((int)s), nopass);
        cols.ntiles = (n2d * s + cols.tile_pencils - 1) / cols.tile_pencils;
        if (e == hipSuccess && (!group_in_bounds(rows, o2.back(), b->total) || !group_in_bounds(cols, o2.back(), b->total)))
            e = hipErrorInvalidValue;
    }
    if (e == hipSuccess && nopass) e = hipErrorInvalidValue;
    if (e != hipSuccess) {
        if (e == hipErrorInvalidValue) fail(FB_ERR_INVALID_ARG, "internal: batch geometry out of bounds or no pass");
        else hip_fail(e, "batch plan");
        batch_free(b);
        delete b;
        return nullptr;
    }
    // phase 0: first passes, 2D rows, single-pass transforms; phase 1: second
    // passes and 2D columns (they read what phase 0 wrote)
    for (auto &g : pass1) b->groups.push_back(g);
    if (has2d) b->groups.push_back(rows);
    for (auto &g : single) b->groups.push_back(g);
    b->phase1_begin = (int)b->groups.size();
    for (auto &g : pass2) b->groups.push_back(g);
    if (has2d) b->groups.push_back(cols);
    if ((int)b->groups.size() > FB_BATCH_MAX_GROUPS) {
        fail(FB_ERR_UNSUPPORTED_SIZE, "too many distinct lengths in one batch (%d groups, at most %d)",
             (int)b->groups.size(), FB_BATCH_MAX_GROUPS);
        batch_free(b);
        delete b;
        return nullptr;
    }
    int64_t task[2] = {0, 0};
    for (auto &g : b->groups) {
        g.task0 = task[g.phase];
        task[g.phase] += g.ntiles;
    }
    b->ntasks[0] = task[0];
    b->ntasks[1] = task[1];
    b->groups_dev = dev_alloc<fb::BatchGroup>(b, b->groups.size(), e);
    if (e == hipSuccess)
        e = hipMemcpy(b->groups_dev, b->groups.data(), b->groups.size() * sizeof(fb::BatchGroup), hipMemcpyHostToDevice);
    int per_cu[2] = {0, 0}, cus = 0;
    for (int ph = 0; ph < 2; ph++) {
        b->lds_bytes[ph] = 16;
        for (auto &g : b->groups)
            if (g.phase == ph) {
                const int lb = fb::batch_kind_lds_bytes(g.n, g.contig != 0);
                if (lb < 0) e = hipErrorInvalidValue;
                if (lb > b->lds_bytes[ph]) b->lds_bytes[ph] = lb;
            }
        if (e == hipSuccess) e = fb::batch_occupancy(b->lds_bytes[ph], &per_cu[ph]);
    }
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        hip_fail(e, "batch plan");
        batch_free(b);
        delete b;
        return nullptr;
    }
    for (int ph = 0; ph < 2; ph++) b->nblocks[ph] = (per_cu[ph] > 0 ? per_cu[ph] : 1) * (cus > 0 ? cus : 1);

    // the single-launch form: one grid sized for the largest tile kind of
    // either phase; item lists per workgroup
    {
        const int np1 = (int)pass1.size();
        std::vector<std::pair<int, int>> pairs;
        for (int i = 0; i < np1; i++) pairs.push_back({i, b->phase1_begin + i});
        if (has2d) pairs.push_back({np1, b->phase1_begin + (int)pass2.size()});
        std::vector<int> singles;
        for (int i = np1 + (has2d ? 1 : 0); i < b->phase1_begin; i++) singles.push_back(i);
        b->ol_lds_bytes = b->lds_bytes[0] > b->lds_bytes[1] ? b->lds_bytes[0] : b->lds_bytes[1];
        int per = 0;
        e = fb::batch_occupancy(b->ol_lds_bytes, &per, true);
        if (e == hipSuccess) {
            b->ol_nblocks = (per > 0 ? per : 1) * (cus > 0 ? cus : 1);
            std::vector<fb::BatchItem> items;
            std::vector<int64_t> begin;
            if (build_onelaunch_items(b->groups, pairs, singles, b->ol_nblocks, items, begin, b->ol_balance)) {
                b->items_dev = dev_alloc<fb::BatchItem>(b, items.size() ? items.size() : 1, e);
                if (e == hipSuccess) b->item_begin_dev = dev_alloc<int64_t>(b, begin.size(), e);
                if (e == hipSuccess && !items.empty())
                    e = hipMemcpy(b->items_dev, items.data(), items.size() * sizeof(fb::BatchItem),
                                  hipMemcpyHostToDevice);
                if (e == hipSuccess)
                    e = hipMemcpy(b->item_begin_dev, begin.data(), begin.size() * sizeof(int64_t),
                                  hipMemcpyHostToDevice);
                b->onelaunch = e == hipSuccess;
                b->ol_items = (int64_t)items.size();
            }
        }
        if (e != hipSuccess) {
            hip_fail(e, "batch plan (single-launch items)");
            batch_free(b);
            delete b;
            return nullptr;
        }
    }
    char d[384];
    snprintf(d, sizeof d,
             "batch n1d=%d n2d=%d side=%lld groups=%d tiles=%lld+%lld elements=%lld persistent grid=%d+%d lds=%d+%d "
             "onelaunch=%d items=%lld grid=%d lds=%d balance=%.3f",
             n1d, n2d, (long long)side2d, (int)b->groups.size(), (long long)b->ntasks[0], (long long)b->ntasks[1],
             (long long)b->total, b->nblocks[0], b->nblocks[1], b->lds_bytes[0], b->lds_bytes[1],
             b->onelaunch ? 1 : 0, (long long)b->ol_items, b->ol_nblocks, b->ol_lds_bytes, b->ol_balance);
    b->desc = d;
    ok();
    return b;
}

void fb_batch_destroy(fb_batch *b)
{
    if (!b) return;
    batch_free(b);
    delete b;
}

int64_t fb_batch_elements(const fb_batch *b) { return b ? b->total : 0; }

int fb_batch_offsets(const fb_batch *b, int64_t *off)
{
    if (!b || !off) return fail(FB_ERR_INVALID_ARG, "NULL argument");
    for (size_t i = 0; i < b->off.size(); i++) off[i] = b->off[i];
    ok();
    return (int)b->off.size();
}

size_t fb_batch_workspace_bytes(const fb_batch *b, int in_place)
{
    if (!b) return 0;
    return in_place ? (size_t)b->total * 8 : 0;
}

int fb_batch_launches(const fb_batch *b) { return b ? (int)b->groups.size() : 0; }

const char *fb_batch_describe(const fb_batch *b) { return b ? b->desc.c_str() : ""; }

fb_status fb_batch_exec(const fb_batch *b, const void *in, void *out, void *workspace, size_t workspace_bytes, int dir,
                        int persistent, void *hip_stream)
{
    if (!b) return (fb_status)fail(FB_ERR_INVALID_ARG, "batch plan is NULL");
    if (!in || !out || (uintptr_t)in % 16 || (uintptr_t)out % 16)
        return (fb_status)fail(FB_ERR_INVALID_ARG, "in/out must be non-NULL and 16-byte aligned");
    if (dir != FB_FORWARD && dir != FB_INVERSE)
        return (fb_status)fail(FB_ERR_INVALID_ARG, "dir must be FB_FORWARD (-1) or FB_INVERSE (+1), got %d", dir);
    if (persistent < 0 || persistent > 2)
        return (fb_status)fail(FB_ERR_INVALID_ARG, "persistent must be 0, 1 or 2, got %d", persistent);
    const size_t bytes = (size_t)b->total * 8;
    const uintptr_t x = (uintptr_t)in, y = (uintptr_t)out;
    const bool in_place = x == y;
    if (!in_place && x < y + bytes && y < x + bytes)
        return (fb_status)fail(FB_ERR_INVALID_ARG, "fb_batch_exec: buffers partially overlap");
    const size_t need = fb_batch_workspace_bytes(b, in_place ? 1 : 0);
    if (need && (!workspace || workspace_bytes < need || (uintptr_t)workspace % 256))
        return (fb_status)fail(FB_ERR_INVALID_ARG, "in-place execution needs a 256-byte aligned workspace of %zu bytes",
                               need);
    void *wsdata = workspace;
    if (in_place) {
        const uintptr_t w = (uintptr_t)wsdata;
        if (w < x + bytes && x < w + bytes) return (fb_status)fail(FB_ERR_INVALID_ARG, "workspace overlaps the data");
    }
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return (fb_status)hip_fail(e, "hipGetDevice");
    if (cur != b->device) return (fb_status)fail(FB_ERR_INVALID_ARG, "batch plan belongs to device %d", b->device);
    hipStream_t st = (hipStream_t)hip_stream;
    // first passes of long transforms write into the output when it is a
    // separate buffer, else into the workspace
    void *mid = in_place ? wsdata : out;
    fb::BatchBuffers bufs{};
    bufs.p[0] = (void *)in;
    bufs.p[1] = out;
    bufs.p[2] = mid;
    bufs.inv = dir > 0;
    bufs.nt = (double)b->total * 8.0 >= (double)FB_NT_MIN_BYTES ? 1 : 0;
    if (persistent == 1 && b->onelaunch) {
        e = timed_launch("batch_onelaunch<c64>", 0.0, st, [&] {
            return fb::launch_batch_onelaunch(b->groups_dev, b->items_dev, b->item_begin_dev, b->ol_nblocks,
                                              b->ol_lds_bytes, bufs, st);
        });
        if (e != hipSuccess) return (fb_status)hip_fail(e, "single-launch batch");
        return (fb_status)ok();
    }
    if (persistent) {
        const int ng = (int)b->groups.size();
        e = timed_launch("batch_persistent<c64,phase0>", 0.0, st, [&] {
            return fb::launch_batch_persistent(b->groups_dev, 0, b->phase1_begin, b->ntasks[0], b->nblocks[0],
                                               b->lds_bytes[0], bufs, st);
        });
        if (e == hipSuccess)
            e = timed_launch("batch_persistent<c64,phase1>", 0.0, st, [&] {
                return fb::launch_batch_persistent(b->groups_dev, b->phase1_begin, ng, b->ntasks[1], b->nblocks[1],
                                                   b->lds_bytes[1], bufs, st);
            });
        if (e != hipSuccess) return (fb_status)hip_fail(e, "persistent batch launch");
        return (fb_status)ok();
    }
    for (const fb::BatchGroup &g : b->groups) {
        PassArgs a = g.args;
        a.in = bufs.p[g.in_sel];
        a.out = bufs.p[g.out_sel];
        a.inv = bufs.inv;
        a.nt = bufs.nt;
        a.scale = (bufs.inv && g.last) ? g.inv_scale : 1.0;
        // contiguous groups move complex64 pencils, strided groups pencil pairs
        const PassInfo pi = g.contig ? fb::find_pass(8, g.n, true, false) : fb::find_pass_pair(g.n);
        char name[96];
        snprintf(name, sizeof name, "fft_pass<c64,n=%d,%s>", g.n, g.contig ? "contiguous" : "strided,pairs");
        const fb::PassLauncher launcher = pi.pick(a);
        e = timed_launch(name, 0.0, st, [&] { return launcher(a, st); });
        if (e != hipSuccess) return (fb_status)hip_fail(e, "batch pass launch");
    }
    return (fb_status)ok();
}

}  // extern "C"

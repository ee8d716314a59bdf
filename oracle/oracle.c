/*
 * oracle.c -- plain, slow, obviously correct CPU oracle for the 3D FFT
 * spectral block (forward 3D DFT, spectral evolution, inverse 3D DFT,
 * strided checksum) and for the batched 1D/2D transforms.
 *
 * TEST INFRASTRUCTURE ONLY.  It is loaded by the tests, by the smoke check
 * and by the benchmark's CPU-baseline leg, and by nothing else; the GPU
 * library shares no code, table or constant generator with it.
 *
 * What it computes (the paper, section 5.1(a), replaces a CPU Fourier
 * transform block by a GPU library call of the same meaning; the block
 * re-created here is the 3D spectral block built around that transform):
 *
 *   forward DFT   X[k] = sum_r x[r] w_nx^(rx kx) w_ny^(ry ky) w_nz^(rz kz),
 *                 w_n = exp(-2 pi i / n)                (sign -1)
 *   inverse DFT   x[r] = (1/N) sum_k X[k] w^(-...)      (sign +1, / N)
 *   evolution     U_t[k] = X[k] exp(-(4 pi^2 alpha t) |k|^2), with signed
 *                 wavenumbers k = i - n [i >= n/2] on every axis
 *   checksum      C = sum_{j=0}^{1023} x.flat[(17 j) mod N], binary64,
 *                 accumulated in j order
 *
 * Grids are C order [nx][ny][nz] (z contiguous), interleaved re/im binary64.
 *
 * Also the paper's other function block (section 5.1(b)), an LU
 * factorization with partial pivoting (orc_lu, at the end of this file).
 *
 * Two tiers:
 *   orc_dft3d_brute  the definition: a direct triple sum in long double with
 *                    exact integer phase reduction (tiny grids only);
 *   orc_fft3d        the fast tier: separable 1D transforms along z, then y,
 *                    then x, each a recursive mixed-radix decimation in time
 *                    over the radix list given by orc_radices.
 *
 * Radix list (the paper is silent; this is the reading used): for
 * n = 2^a 3^b the radices, in the order the stages are applied to the data,
 * are b threes, then floor(a/4) sixteens, then one 2^(a mod 4) if a mod 4 > 0.
 * The recursive decimation in time splits by the LAST radix at the top level,
 * so the first radix of the list is the first one applied.
 *
 * Twiddles w_n^m come from cosl/sinl of a quadrant-reduced angle, so that
 * multiples of pi/2 are exact, and are rounded to binary64.
 * Build: gcc -O2 -ffp-contract=off -fopenmp (no fused multiply-add).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double re, im; } cplx;

#define ORC_MAX_RADICES 32
#define ORC_PI_L 3.141592653589793238462643383279502884L

static cplx cmul(cplx a, cplx b)
{
    cplx r;
    r.re = a.re * b.re - a.im * b.im;
    r.im = a.re * b.im + a.im * b.re;
    return r;
}

static cplx cadd(cplx a, cplx b)
{
    cplx r = { a.re + b.re, a.im + b.im };
    return r;
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of later calls (for timing the oracle on one core); no
 * effect on results: every pencil is computed by one thread in a fixed
 * order whatever the count. */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Radix list of n (see the header); returns the count, or -1 when n is not
 * of the form 2^a 3^b with n >= 1.  n == 1 has an empty list. */
int orc_radices(int64_t n, int *out, int cap)
{
    if (n < 1) return -1;
    int a = 0, b = 0;
    while (n % 3 == 0) { n /= 3; b++; }
    while (n % 2 == 0) { n /= 2; a++; }
    if (n != 1) return -1;
    int cnt = 0;
    for (int i = 0; i < b; i++) { if (cnt >= cap) return -1; out[cnt++] = 3; }
    for (int i = 0; i < a / 4; i++) { if (cnt >= cap) return -1; out[cnt++] = 16; }
    if (a % 4) { if (cnt >= cap) return -1; out[cnt++] = 1 << (a % 4); }
    return cnt;
}

/* "z:16,16 y:16,16 x:16,16,2 order:zyx"; an axis of length 1 prints "-". */
int orc_describe(int64_t nx, int64_t ny, int64_t nz, char *buf, int cap)
{
    const int64_t len[3] = { nz, ny, nx };
    const char name[3] = { 'z', 'y', 'x' };
    char tmp[512];
    int pos = 0;
    for (int ax = 0; ax < 3; ax++) {
        int r[ORC_MAX_RADICES];
        int c = orc_radices(len[ax], r, ORC_MAX_RADICES);
        if (c < 0) return -1;
        pos += snprintf(tmp + pos, sizeof tmp - pos, "%c:", name[ax]);
        if (c == 0) pos += snprintf(tmp + pos, sizeof tmp - pos, "-");
        for (int i = 0; i < c; i++)
            pos += snprintf(tmp + pos, sizeof tmp - pos, i ? ",%d" : "%d", r[i]);
        pos += snprintf(tmp + pos, sizeof tmp - pos, " ");
    }
    pos += snprintf(tmp + pos, sizeof tmp - pos, "order:zyx");
    if (pos + 1 > cap) return -1;
    memcpy(buf, tmp, (size_t)pos + 1);
    return pos;
}

/* exp(sign * 2 pi i m / n), m reduced mod n, quadrant-exact. */
static void omega_ld(int64_t n, int64_t m, int sign, long double *re, long double *im)
{
    m %= n;
    if (m < 0) m += n;
    /* 2 pi m / n = (pi/2) q + (pi/2) r / n with 4m = q n + r, 0 <= r < n */
    int64_t q = (4 * m) / n, r = (4 * m) % n;
    long double c, s;
    if (2 * r <= n) {
        long double phi = (ORC_PI_L / 2.0L) * (long double)r / (long double)n;
        c = cosl(phi); s = sinl(phi);
    } else {
        long double phi = (ORC_PI_L / 2.0L) * (long double)(n - r) / (long double)n;
        c = sinl(phi); s = cosl(phi);
    }
    long double cr, ci;
    switch (q & 3) {
    case 0: cr = c;  ci = s;  break;
    case 1: cr = -s; ci = c;  break;
    case 2: cr = -c; ci = -s; break;
    default: cr = s; ci = -c; break;
    }
    *re = cr;
    *im = sign < 0 ? -ci : ci;
}

void orc_omega(int64_t n, int64_t m, int sign, double *re, double *im)
{
    long double r, i;
    omega_ld(n, m, sign, &r, &i);
    *re = (double)r;
    *im = (double)i;
}

/* ---------------------------------------------------------------------- */
/* 1D mixed-radix decimation in time                                        */
/* ---------------------------------------------------------------------- */

typedef struct {
    int64_t n;          /* top-level length */
    int nr;
    int r[ORC_MAX_RADICES];
    cplx *tw;           /* tw[m] = w_n^m for the transform's sign, m < n */
} fft1d_plan;

static int plan1d_init(fft1d_plan *p, int64_t n, int sign)
{
    p->n = n;
    p->nr = orc_radices(n, p->r, ORC_MAX_RADICES);
    if (p->nr < 0) return -1;
    p->tw = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!p->tw) return -1;
    for (int64_t m = 0; m < n; m++) orc_omega(n, m, sign, &p->tw[m].re, &p->tw[m].im);
    return 0;
}

static void plan1d_free(fft1d_plan *p) { free(p->tw); p->tw = NULL; }

/* w_len^j looked up in the top-level table (len divides the top length). */
static cplx tw_at(const fft1d_plan *p, int64_t len, int64_t j)
{
    int64_t idx = (j % len) * (p->n / len);
    return p->tw[idx];
}

/*
 * X[0..len) = DFT_len of the sequence x[0], x[s], x[2s], ... using the first
 * nr radices of the plan's list.  work must hold 2*len elements.
 *
 * len = R * m with R the last radix of the list: the input splits into the
 * R decimated subsequences x[q + R p] (p < m), each transformed with the
 * remaining radices, and
 *     X[k1 + m k2] = sum_q w_R^(q k2) (w_len^(q k1) Y_q[k1]),
 * k1 < m, k2 < R.  A single radix is a direct DFT.
 */
static void fft_rec(const fft1d_plan *p, int nr, int64_t len, const cplx *x, int64_t s,
                    cplx *X, cplx *work)
{
    if (len == 1) { X[0] = x[0]; return; }
    if (nr == 1) {
        for (int64_t k = 0; k < len; k++) {
            cplx acc = { 0.0, 0.0 };
            for (int64_t q = 0; q < len; q++)
                acc = cadd(acc, cmul(x[q * s], tw_at(p, len, q * k)));
            X[k] = acc;
        }
        return;
    }
    const int R = p->r[nr - 1];
    const int64_t m = len / R;
    cplx *Y = work;              /* Y_q occupies Y[q m .. q m + m) */
    for (int q = 0; q < R; q++)
        fft_rec(p, nr - 1, m, x + q * s, s * R, Y + q * m, work + len);
    cplx t[16 * 3];              /* R <= 16 */
    for (int64_t k1 = 0; k1 < m; k1++) {
        for (int q = 0; q < R; q++) t[q] = cmul(Y[q * m + k1], tw_at(p, len, q * k1));
        for (int k2 = 0; k2 < R; k2++) {
            cplx acc = { 0.0, 0.0 };
            for (int q = 0; q < R; q++) acc = cadd(acc, cmul(t[q], tw_at(p, R, (int64_t)q * k2)));
            X[k1 + m * k2] = acc;
        }
    }
}

/* Transform `count` pencils of length n; pencil c starts at base(c) and has
 * element stride `stride` (in complex elements).  base(c) = (c / inner) *
 * outer_step + (c % inner) * inner_step. */
static int fft_axis(double *data, int64_t n, int64_t stride, int64_t count, int64_t inner,
                    int64_t inner_step, int64_t outer_step, int sign)
{
    if (n == 1) return 0;
    fft1d_plan p;
    if (plan1d_init(&p, n, sign)) return -1;
    cplx *d = (cplx *)data;
    int err = 0;
#pragma omp parallel
    {
        cplx *buf = (cplx *)malloc(sizeof(cplx) * (size_t)n * 4);
        if (!buf) {
#pragma omp atomic write
            err = 1;
        }
#pragma omp for schedule(static)
        for (int64_t c = 0; c < count; c++) {
            if (!buf) continue;
            cplx *pen = buf, *out = buf + n, *work = buf + 2 * n;
            int64_t base = (c / inner) * outer_step + (c % inner) * inner_step;
            for (int64_t i = 0; i < n; i++) pen[i] = d[base + i * stride];
            fft_rec(&p, p.nr, n, pen, 1, out, work);
            for (int64_t i = 0; i < n; i++) d[base + i * stride] = out[i];
        }
        free(buf);
    }
    plan1d_free(&p);
    return err ? -1 : 0;
}

/* In-place transform along the axes selected by `axes` (bit 0 z, bit 1 y,
 * bit 2 x), in the order z, y, x.  sign -1 forward (unscaled), sign +1
 * inverse divided by the product of the selected lengths. */
int orc_fft3d_axes(int64_t nx, int64_t ny, int64_t nz, int sign, int axes, double *data)
{
    if (nx < 1 || ny < 1 || nz < 1 || (sign != 1 && sign != -1) || axes < 0 || axes > 7) return -1;
    int r[ORC_MAX_RADICES];
    if (orc_radices(nx, r, ORC_MAX_RADICES) < 0 || orc_radices(ny, r, ORC_MAX_RADICES) < 0 ||
        orc_radices(nz, r, ORC_MAX_RADICES) < 0)
        return -2;
    int64_t nsel = 1;
    /* z: pencils (x, y), contiguous */
    if (axes & 1) {
        if (fft_axis(data, nz, 1, nx * ny, 1, 0, nz, sign)) return -3;
        nsel *= nz;
    }
    /* y: pencils (x, z), stride nz */
    if (axes & 2) {
        if (fft_axis(data, ny, nz, nx * nz, nz, 1, ny * nz, sign)) return -3;
        nsel *= ny;
    }
    /* x: pencils (y, z), stride ny nz */
    if (axes & 4) {
        if (fft_axis(data, nx, ny * nz, ny * nz, ny * nz, 1, 0, sign)) return -3;
        nsel *= nx;
    }
    if (sign > 0) {
        const double N = (double)nsel;
        const int64_t tot = 2 * nx * ny * nz;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < tot; i++) data[i] = data[i] / N;
    }
    return 0;
}

/* In-place 3D transform: z, then y, then x.  sign -1 forward (unscaled),
 * sign +1 inverse divided by N = nx ny nz after the last axis. */
int orc_fft3d(int64_t nx, int64_t ny, int64_t nz, int sign, double *data)
{
    return orc_fft3d_axes(nx, ny, nz, sign, 7, data);
}

/* `howmany` contiguous 1D transforms of length n (unscaled for sign -1,
 * divided by n for sign +1). */
int orc_fft1d_many(int64_t n, int64_t howmany, int sign, double *data)
{
    int r[ORC_MAX_RADICES];
    if (n < 1 || howmany < 0 || orc_radices(n, r, ORC_MAX_RADICES) < 0) return -2;
    if (fft_axis(data, n, 1, howmany, 1, 0, n, sign)) return -3;
    if (sign > 0) {
        const int64_t tot = 2 * n * howmany;
        for (int64_t i = 0; i < tot; i++) data[i] = data[i] / (double)n;
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Definition tier: direct triple sum in long double                        */
/* ---------------------------------------------------------------------- */

static int64_t gcd64(int64_t a, int64_t b) { while (b) { int64_t t = a % b; a = b; b = t; } return a; }

int orc_dft3d_brute(int64_t nx, int64_t ny, int64_t nz, int sign, const double *in, double *out)
{
    if (nx < 1 || ny < 1 || nz < 1 || (sign != 1 && sign != -1)) return -1;
    const int64_t N = nx * ny * nz;
    if (N > (1 << 16)) return -1;
    int64_t L = nx;
    L = L / gcd64(L, ny) * ny;
    L = L / gcd64(L, nz) * nz;
    const int64_t fx = L / nx, fy = L / ny, fz = L / nz;
    long double *cs = (long double *)malloc(sizeof(long double) * 2 * (size_t)L);
    if (!cs) return -1;
    for (int64_t m = 0; m < L; m++) omega_ld(L, m, sign, &cs[2 * m], &cs[2 * m + 1]);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < N; k++) {
        const int64_t kx = k / (ny * nz), ky = (k / nz) % ny, kz = k % nz;
        long double sr = 0.0L, si = 0.0L;
        for (int64_t r = 0; r < N; r++) {
            const int64_t rx = r / (ny * nz), ry = (r / nz) % ny, rz = r % nz;
            /* exact phase index: (rx kx / nx + ry ky / ny + rz kz / nz) L mod L */
            const int64_t ph = ((rx * kx % nx) * fx + (ry * ky % ny) * fy + (rz * kz % nz) * fz) % L;
            const long double wr = cs[2 * ph], wi = cs[2 * ph + 1];
            const long double xr = in[2 * r], xi = in[2 * r + 1];
            sr += xr * wr - xi * wi;
            si += xr * wi + xi * wr;
        }
        if (sign > 0) { sr /= (long double)N; si /= (long double)N; }
        out[2 * k] = (double)sr;
        out[2 * k + 1] = (double)si;
    }
    free(cs);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Spectral evolution and checksum                                          */
/* ---------------------------------------------------------------------- */

static int64_t signed_wavenumber(int64_t i, int64_t n) { return (2 * i >= n) ? i - n : i; }

/* u[k] *= exp(-(4 pi^2 alpha t) |k|^2), one exp per element. */
int orc_evolve(int64_t nx, int64_t ny, int64_t nz, double *u, double alpha, double t)
{
    if (nx < 1 || ny < 1 || nz < 1 || !(alpha >= 0.0) || !(t >= 0.0)) return -1;
    const double four_pi2 = 39.47841760435743;   /* 4 pi^2 rounded to binary64 */
    const double c = four_pi2 * alpha * t;
    const int64_t N = nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t idx = 0; idx < N; idx++) {
        const int64_t ix = idx / (ny * nz), iy = (idx / nz) % ny, iz = idx % nz;
        const int64_t kx = signed_wavenumber(ix, nx), ky = signed_wavenumber(iy, ny),
                      kz = signed_wavenumber(iz, nz);
        const double k2 = (double)(kx * kx + ky * ky + kz * kz);
        const double f = exp(-c * k2);
        u[2 * idx] *= f;
        u[2 * idx + 1] *= f;
    }
    return 0;
}

/* out[0] + i out[1] = sum_{j<1024} x.flat[(17 j) mod N], in j order. */
int orc_checksum(int64_t nx, int64_t ny, int64_t nz, const double *x, double *out)
{
    if (nx < 1 || ny < 1 || nz < 1) return -1;
    const int64_t N = nx * ny * nz;
    double sr = 0.0, si = 0.0;
    for (int64_t j = 0; j < 1024; j++) {
        const int64_t i = (17 * j) % N;
        sr += x[2 * i];
        si += x[2 * i + 1];
    }
    out[0] = sr;
    out[1] = si;
    return 0;
}

/* ------------------------------------------------------------------ LU
 * The paper's second function block (section 5.1(b)): an LU factorization,
 * here the definition of Gaussian elimination with partial pivoting on a
 * row-major n x n binary64 matrix (row stride lda), in place:
 *
 *   for j = 0 .. n-1:
 *     p = the first row i >= j with the largest |a[i][j]|
 *     ipiv[j] = p; swap rows j and p (all n columns)
 *     if a[j][j] != 0: for i > j: a[i][j] /= a[j][j];
 *                      for i > j, c > j: a[i][c] -= a[i][j] * a[j][c]
 *     else: info = j + 1 for the first such j (the column is left as it is)
 *
 * so that P A = L U with L unit lower triangular (below the diagonal) and U
 * upper triangular (on and above it), P the product of the swaps in order.
 * Returns info (0: all pivots non-zero), or -1 on bad arguments.  The
 * trailing updates of one step are independent per row (OpenMP over rows);
 * each element receives its updates in increasing j. */
int orc_lu(int64_t n, int64_t lda, double *a, int32_t *ipiv)
{
    if (n < 0 || lda < n || (n > 0 && (!a || !ipiv))) return -1;
    int info = 0;
    for (int64_t j = 0; j < n; j++) {
        int64_t p = j;
        double best = fabs(a[j * lda + j]);
        for (int64_t i = j + 1; i < n; i++) {
            const double v = fabs(a[i * lda + j]);
            if (v > best) {
                best = v;
                p = i;
            }
        }
        ipiv[j] = (int32_t)p;
        if (p != j)
            for (int64_t c = 0; c < n; c++) {
                const double t = a[j * lda + c];
                a[j * lda + c] = a[p * lda + c];
                a[p * lda + c] = t;
            }
        const double piv = a[j * lda + j];
        if (piv == 0.0) {
            if (!info) info = (int)(j + 1);
            continue;
        }
#pragma omp parallel for schedule(static)
        for (int64_t i = j + 1; i < n; i++) {
            const double l = a[i * lda + j] / piv;
            a[i * lda + j] = l;
            for (int64_t c = j + 1; c < n; c++) a[i * lda + c] -= l * a[j * lda + c];
        }
    }
    return info;
}

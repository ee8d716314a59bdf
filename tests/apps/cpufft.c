/* cpufft.c -- iterative radix-2 transforms along each axis of a 3D grid
 * (bit-reversal permutation, then log2(n) butterfly stages), written for
 * the sample application; plain C99, binary64. */
#include "cpufft.h"

#include <math.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#include <stdlib.h>

static int is_pow2(int64_t n) { return n >= 1 && (n & (n - 1)) == 0; }

/* one 1D transform of length n over elements x[0], x[s], x[2s], ... */
static void fft1d(double *x, int64_t n, int64_t s, int sign, double *tmp)
{
    for (int64_t i = 0; i < n; i++) {
        tmp[2 * i] = x[2 * i * s];
        tmp[2 * i + 1] = x[2 * i * s + 1];
    }
    for (int64_t i = 1, j = 0; i < n; i++) {   /* bit reversal */
        int64_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double r = tmp[2 * i], m = tmp[2 * i + 1];
            tmp[2 * i] = tmp[2 * j];
            tmp[2 * i + 1] = tmp[2 * j + 1];
            tmp[2 * j] = r;
            tmp[2 * j + 1] = m;
        }
    }
    for (int64_t len = 2; len <= n; len <<= 1) {
        const double ang = sign * 2.0 * M_PI / (double)len;
        for (int64_t i = 0; i < n; i += len) {
            for (int64_t k = 0; k < len / 2; k++) {
                const double wr = cos(ang * (double)k), wi = sin(ang * (double)k);
                double *a = tmp + 2 * (i + k), *b = tmp + 2 * (i + k + len / 2);
                const double br = b[0] * wr - b[1] * wi, bi = b[0] * wi + b[1] * wr;
                b[0] = a[0] - br;
                b[1] = a[1] - bi;
                a[0] += br;
                a[1] += bi;
            }
        }
    }
    for (int64_t i = 0; i < n; i++) {
        x[2 * i * s] = tmp[2 * i];
        x[2 * i * s + 1] = tmp[2 * i + 1];
    }
}

int cfft3d(int64_t nx, int64_t ny, int64_t nz, double *data, int sign)
{
    if (!data || (sign != -1 && sign != 1) || !is_pow2(nx) || !is_pow2(ny) || !is_pow2(nz)) return -1;
    int64_t nmax = nx > ny ? nx : ny;
    if (nz > nmax) nmax = nz;
    double *tmp = malloc(sizeof(double) * 2 * (size_t)nmax);
    if (!tmp) return -1;
    for (int64_t i = 0; i < nx * ny; i++) fft1d(data + 2 * i * nz, nz, 1, sign, tmp);
    for (int64_t i = 0; i < nx; i++)
        for (int64_t k = 0; k < nz; k++) fft1d(data + 2 * (i * ny * nz + k), ny, nz, sign, tmp);
    for (int64_t j = 0; j < ny * nz; j++) fft1d(data + 2 * j, nx, ny * nz, sign, tmp);
    free(tmp);
    if (sign > 0) {
        const double s = 1.0 / (double)(nx * ny * nz);
        for (int64_t i = 0; i < 2 * nx * ny * nz; i++) data[i] *= s;
    }
    return 0;
}

/* heat3d.c -- a host application with a Fourier-transform function block:
 * the spectral solution of the heat equation on the periodic unit cube.
 * The input grid is uniform on [-1, 1) (SplitMix64, seed 1), transformed
 * forward once; for t = 1..steps the spectrum is damped by
 * exp(-4 pi^2 alpha t |k|^2), transformed back and summed at 1024 points
 * (stride 17).  All transforms are calls into the external CPU library
 * cpufft.  Prints one line per step: "t re im"; the elapsed time of the
 * transform-and-evolve part goes to stderr.
 *
 * usage: heat3d [nx ny nz [steps [alpha]]] */
#include <math.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#include "cpufft.h"

static uint64_t splitmix64_at(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double uniform(uint64_t seed, uint64_t c) { return (double)(splitmix64_at(seed, c) >> 11) * 0x1.0p-52 - 1.0; }

static double wave(int64_t i, int64_t n) { return (double)(2 * i >= n ? i - n : i); }

int main(int argc, char **argv)
{
    int64_t nx = 64, ny = 64, nz = 64;
    int steps = 6;
    double alpha = 1e-6;
    if (argc >= 4) {
        nx = atoll(argv[1]);
        ny = atoll(argv[2]);
        nz = atoll(argv[3]);
    }
    if (argc >= 5) steps = atoi(argv[4]);
    if (argc >= 6) alpha = atof(argv[5]);
    const int64_t n = nx * ny * nz;
    double *u0 = malloc(sizeof(double) * 2 * (size_t)n);
    double *x = malloc(sizeof(double) * 2 * (size_t)n);
    if (!u0 || !x) return 1;
    for (int64_t i = 0; i < n; i++) {
        u0[2 * i] = uniform(1, 2 * (uint64_t)i);
        u0[2 * i + 1] = uniform(1, 2 * (uint64_t)i + 1);
    }
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    if (cfft3d(nx, ny, nz, u0, -1) != 0) return 2;   /* forward transform */
    for (int t = 1; t <= steps; t++) {
        const double c = 4.0 * M_PI * M_PI * alpha * (double)t;
        for (int64_t a = 0; a < nx; a++)
            for (int64_t b = 0; b < ny; b++)
                for (int64_t d = 0; d < nz; d++) {
                    const double ka = wave(a, nx), kb = wave(b, ny), kd = wave(d, nz);
                    const double g = exp(-c * (ka * ka + kb * kb + kd * kd));
                    const int64_t i = (a * ny + b) * nz + d;
                    x[2 * i] = u0[2 * i] * g;
                    x[2 * i + 1] = u0[2 * i + 1] * g;
                }
        if (cfft3d(nx, ny, nz, x, +1) != 0) return 3;   /* inverse transform */
        double sr = 0.0, si = 0.0;
        for (int64_t j = 0; j < 1024; j++) {
            const int64_t i = (17 * j) % n;
            sr += x[2 * i];
            si += x[2 * i + 1];
        }
        printf("%d %.17g %.17g\n", t, sr, si);
    }
    clock_gettime(CLOCK_MONOTONIC, &t1);
    fprintf(stderr, "elapsed_s %.6f\n", (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec));
    free(u0);
    free(x);
    return 0;
}

/* cpufft.h -- a small CPU library of 3D complex transforms: the "external
 * library" that the sample host application calls, and that the
 * library-call substitution replaces by libfb. */
#ifndef CPUFFT_H
#define CPUFFT_H
#include <stdint.h>

/* In-place 3D DFT of an nx x ny x nz grid of interleaved complex doubles in
 * C order (z fastest).  sign = -1: forward, unnormalized; sign = +1:
 * inverse, scaled by 1/(nx ny nz).  Every length must be a power of two.
 * Returns 0, or -1 on bad arguments. */
int cfft3d(int64_t nx, int64_t ny, int64_t nz, double *data, int sign);

#endif

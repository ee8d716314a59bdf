// fb_misc.hip -- the small kernels around the pencil passes: twiddle-table
// generation (binary64 on the device), standalone spectral evolution, the
// strided checksum, and the seeded uniform input generator.
#include <hip/hip_runtime.h>

#include "fb_device.hpp"
#include "fb_batch.hpp"
#include "fb_internal.hpp"

namespace fb {

PassInfo find_pass_c128(int n, bool contig, bool mx);
PassInfo find_pass_c64(int n, bool contig, bool mx);
PassInfo find_pass_multi_c128(int n);
PassInfo find_pass_multi_c64(int n, bool mx);

PassInfo find_pass_multi(int esize, int n, bool mx)
{
    if (esize == 16) return find_pass_multi_c128(n);
    if (esize == 8) return find_pass_multi_c64(n, mx);
    return {nullptr, 0, 0, 0};
}

PassInfo find_pass(int esize, int n, bool contig, bool mx)
{
    if (esize == 16) return find_pass_c128(n, contig, false);
    if (esize == 8) return find_pass_c64(n, contig, mx);
    return {nullptr, 0, 0, 0};
}

// ---------------------------------------------------------------- twiddles

// exp(-2 pi i m / L) for 0 <= m < L.  The angle is split into whole
// quadrants and a remainder so that multiples of pi/2 come out exact.
__device__ double2 root_of_unity(int64_t m, int64_t L)
{
    const int64_t m4 = 4 * m;
    const int64_t quad = m4 / L, rem = m4 - quad * L;   // angle = (pi/2)(quad + rem/L)
    double s, c;
    sincospi((double)rem / (2.0 * (double)L), &s, &c);   // sin, cos of (pi/2) rem/L
    double cr, si;                                        // cos and sin of the full angle
    switch (quad & 3) {
    case 0: cr = c;  si = s;  break;
    case 1: cr = -s; si = c;  break;
    case 2: cr = -c; si = -s; break;
    default: cr = s; si = -c; break;
    }
    return make_double2(cr, -si);
}

__global__ void twiddle_kernel(TwDesc d, double2 *tw64, float2 *tw32)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= d.total) return;
    int s = -1;   // the stage owning entry e (stages with ns == 1 own none)
    for (int i = 0; i < d.nst; i++)
        if (d.ns[i] > 1 && e >= d.off[i] && e < d.off[i] + (d.r[i] - 1) * d.ns[i]) s = i;
    if (s < 0) return;
    const int local = e - d.off[s];
    const int q = 1 + local / d.ns[s];
    const int k = local % d.ns[s];
    const int64_t L = (int64_t)d.ns[s] * d.r[s];
    const double2 w = root_of_unity(((int64_t)q * k) % L, L);
    tw64[e] = w;
    tw32[e] = make_float2((float)w.x, (float)w.y);
}

hipError_t launch_twiddles(const TwDesc &d, double2 *tw64, float2 *tw32, hipStream_t st)
{
    if (d.total <= 0) return hipSuccess;
    const int threads = 256;
    const int blocks = (d.total + threads - 1) / threads;
    hipLaunchKernelGGL(twiddle_kernel, dim3(blocks), dim3(threads), 0, st, d, tw64, tw32);
    return hipGetLastError();
}

// w_n^m for every m < n (pre-twiddles of the two-pass long transforms)
__global__ void roots_kernel(int64_t n, double2 *t64, float2 *t32)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const double2 w = root_of_unity(m, n);
    if (t64) t64[m] = w;
    t32[m] = make_float2((float)w.x, (float)w.y);
}

// Pre-twiddle table of a two-pass transform of length n = n1 n2, laid out
// like the data the second pass reads: t32[q n1 + b] = w_n^(q b), b < n1,
// q < n2 (q b < n, so no reduction is needed).
__global__ void pretwiddle_kernel(int64_t n1, int64_t n2, float2 *t32)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n1 * n2) return;
    const int64_t q = m / n1, b = m % n1;
    const double2 w = root_of_unity(q * b, n1 * n2);
    t32[m] = make_float2((float)w.x, (float)w.y);
}

hipError_t launch_pretwiddle(int64_t n1, int64_t n2, float2 *t32, hipStream_t st)
{
    const int threads = 256;
    const int64_t blocks = (n1 * n2 + threads - 1) / threads;
    hipLaunchKernelGGL(pretwiddle_kernel, dim3((unsigned)blocks), dim3(threads), 0, st, n1, n2, t32);
    return hipGetLastError();
}

hipError_t launch_roots(int64_t n, double2 *t64, float2 *t32, hipStream_t st)
{
    const int threads = 256;
    const int64_t blocks = (n + threads - 1) / threads;
    hipLaunchKernelGGL(roots_kernel, dim3((unsigned)blocks), dim3(threads), 0, st, n, t64, t32);
    return hipGetLastError();
}

// ---------------------------------------------------------------- evolution

__device__ __forceinline__ int64_t wrapped(int64_t i, int64_t n) { return (2 * i >= n) ? i - n : i; }

// One thread per element of a z row; block (bx, iy, ix).
template <typename V, typename R>
__global__ void evolve_kernel(const V *in, V *out, int64_t nx, int64_t ny, int64_t nz, double c)
{
    const int64_t iz = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t iy = blockIdx.y, ix = blockIdx.z;
    if (iz >= nz) return;
    const int64_t kx = wrapped(ix, nx), ky = wrapped(iy, ny), kz = wrapped(iz, nz);
    const double k2 = (double)(kx * kx + ky * ky + kz * kz);
    const R f = evol_factor<R>(c, k2);
    const int64_t i = (ix * ny + iy) * nz + iz;
    V v = in[i];
    v.x *= f;
    v.y *= f;
    out[i] = v;
}

hipError_t launch_evolve(int esize, const void *in, void *out, int64_t nx, int64_t ny, int64_t nz,
                         double c, hipStream_t st)
{
    const int threads = nz >= 256 ? 256 : (int)((nz + 63) / 64) * 64;
    const dim3 grid((unsigned)((nz + threads - 1) / threads), (unsigned)ny, (unsigned)nx);
    if (esize == 16)
        hipLaunchKernelGGL((evolve_kernel<double2, double>), grid, dim3(threads), 0, st,
                           (const double2 *)in, (double2 *)out, nx, ny, nz, c);
    else
        hipLaunchKernelGGL((evolve_kernel<float2, float>), grid, dim3(threads), 0, st,
                           (const float2 *)in, (float2 *)out, nx, ny, nz, c);
    return hipGetLastError();
}

// ---------------------------------------------------------------- checksum

// The 1024 samples x[(17 j) mod N] summed in binary64 by a fixed tree: level
// h = 512, 256, ..., 1 adds sample j + h into sample j for j < h.  One
// wavefront per grid: lane l holds samples l + 64 i (i < 16), so the levels
// h >= 64 combine a lane's own values (i with i + h/64) and the levels h < 64
// combine lane l with lane l + h (a lane exchange); lane 0 ends with the sum.
// Every addition is the one the tree prescribes, so the result does not
// depend on the launch shape.  Workgroup g sums grid g of `count` consecutive
// grids into out2[2g], out2[2g+1].
template <typename V>
__global__ void __launch_bounds__(64) checksum_kernel(const V *x, int64_t N, double *out2)
{
    const int l = threadIdx.x;
    x += (int64_t)blockIdx.x * N;
    out2 += 2 * (int64_t)blockIdx.x;
    double sr[16], si[16];
#pragma unroll
    for (int i = 0; i < 16; i++) {
        const V v = x[(17 * (int64_t)(l + 64 * i)) % N];
        sr[i] = (double)v.x;
        si[i] = (double)v.y;
    }
#pragma unroll
    for (int h = 8; h > 0; h >>= 1) {   // tree levels 512 .. 64 within the lane
#pragma unroll
        for (int i = 0; i < h; i++) {
            sr[i] += sr[i + h];
            si[i] += si[i + h];
        }
    }
    double r = sr[0], m = si[0];
#pragma unroll
    for (int h = 32; h > 0; h >>= 1) {   // levels 32 .. 1 across lanes
        const double ro = __shfl_down(r, h), mo = __shfl_down(m, h);
        r += ro;
        m += mo;
    }
    if (l == 0) {
        out2[0] = r;
        out2[1] = m;
    }
}

hipError_t launch_checksum(int esize, const void *x, int64_t N, double *out2, hipStream_t st, int count)
{
    if (count <= 0) return hipSuccess;
    if (esize == 16)
        hipLaunchKernelGGL((checksum_kernel<double2>), dim3(count), dim3(64), 0, st, (const double2 *)x, N, out2);
    else
        hipLaunchKernelGGL((checksum_kernel<float2>), dim3(count), dim3(64), 0, st, (const float2 *)x, N, out2);
    return hipGetLastError();
}

// ---------------------------------------------------------------- inputs

template <typename V, typename R>
__global__ void fill_uniform_kernel(V *x, int64_t N, uint64_t seed)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] = uniform_elem<V>(seed, (uint64_t)i);
    }
}

hipError_t launch_fill_uniform(int esize, void *x, int64_t N, uint64_t seed, hipStream_t st)
{
    const int threads = 256;
    int64_t blocks = (N + threads - 1) / threads;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    if (esize == 16)
        hipLaunchKernelGGL((fill_uniform_kernel<double2, double>), dim3((unsigned)blocks), dim3(threads), 0, st,
                           (double2 *)x, N, seed);
    else
        hipLaunchKernelGGL((fill_uniform_kernel<float2, float>), dim3((unsigned)blocks), dim3(threads), 0, st,
                           (float2 *)x, N, seed);
    return hipGetLastError();
}

}  // namespace fb

// Sample generation and surface data (the sample set of the estimate and
// the point/data streams the kernel sums read).
//
// Samples are area-uniform on the mesh (Section 4.1.1: density 1/|Gamma|).
// Random words come from SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) used
// as a counter generator: word(seed, stream, c) = mix(s + (c+1) * gamma)
// with s = seed ^ (stream << 56).  Sample j uses counters 3j, 3j+1, 3j+2 of
// stream 0.  The triangle search and the barycentric warp are done in FP64
// so the triangle index is reproducible bit for bit on any IEEE machine.
#include "nat_internal.h"

namespace nat {
namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double unit_draw(uint64_t seed, uint32_t stream, uint64_t counter)
{
    const uint64_t start = seed ^ (static_cast<uint64_t>(stream) << 56);
    const uint64_t h = mix64(start + (counter + 1ull) * 0x9E3779B97F4A7C15ull);
    return static_cast<double>(h >> 11) * 0x1.0p-53;
}

// Smallest t with cdf[t] > tau (the last triangle if none).
__device__ __forceinline__ int32_t upper_search(const double* __restrict__ cdf, int32_t nT,
                                                double tau)
{
    int32_t lo = 0, hi = nT - 1;
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (cdf[mid] > tau)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

__global__ void __launch_bounds__(256)
k_samples(const double* __restrict__ cdf, int32_t nT, double area, int32_t N, uint64_t seed,
          int32_t* __restrict__ tri, double* __restrict__ bary)
{
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N)
        return;
    const uint64_t c = 3ull * static_cast<uint64_t>(j);
    const double u0 = unit_draw(seed, 0, c);
    const double u1 = unit_draw(seed, 0, c + 1);
    const double u2 = unit_draw(seed, 0, c + 2);
    const double tau = u0 * area;
    tri[j] = upper_search(cdf, nT, tau);
    const double s = __builtin_sqrt(u1);
    bary[2 * j + 0] = s * (1.0 - u2);
    bary[2 * j + 1] = s * u2;
}

// Point i on triangle tri[i]: x = v0 + b1 (v1 - v0) + b2 (v2 - v0); the unit
// normal of the triangle; FP32 copies relative to the mesh centre.
__global__ void __launch_bounds__(256)
k_points(const double* __restrict__ V, const int32_t* __restrict__ T,
         const double* __restrict__ nrm, int32_t n, const int32_t* __restrict__ tri,
         const double* __restrict__ bary, double cx, double cy, double cz,
         double* __restrict__ x64, double* __restrict__ n64, float* __restrict__ x32,
         float* __restrict__ n32)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int32_t t = tri[i];
    const double b1 = bary[2 * i], b2 = bary[2 * i + 1];
    const double* v0 = V + 3 * T[3 * t + 0];
    const double* v1 = V + 3 * T[3 * t + 1];
    const double* v2 = V + 3 * T[3 * t + 2];
    const double ctr[3] = {cx, cy, cz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double x = v0[d] + b1 * (v1[d] - v0[d]) + b2 * (v2[d] - v0[d]);
        if (x64)
            x64[(size_t)d * n + i] = x;
        if (x32)
            x32[(size_t)d * n + i] = static_cast<float>(x - ctr[d]);
        const double nd = nrm[3 * t + d];
        if (n64)
            n64[(size_t)d * n + i] = nd;
        if (n32)
            n32[(size_t)d * n + i] = static_cast<float>(nd);
    }
}

// g_out[m][i]: per-vertex data interpolated with (1 - b1 - b2, b1, b2), or
// the triangle's value.
__global__ void __launch_bounds__(256)
k_neumann(const int32_t* __restrict__ T, int32_t layout, const double2* __restrict__ g,
          int32_t ld_g, int32_t n, const int32_t* __restrict__ tri,
          const double* __restrict__ bary, double2* __restrict__ out)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t m = blockIdx.y;
    if (i >= n)
        return;
    const double2* gm = g + (size_t)m * ld_g;
    const int32_t t = tri[i];
    double2 r;
    if (layout == NAT_NEUMANN_PER_TRIANGLE) {
        r = gm[t];
    } else {
        const double b1 = bary[2 * i], b2 = bary[2 * i + 1];
        const double b0 = 1.0 - b1 - b2;
        const double2 g0 = gm[T[3 * t]], g1 = gm[T[3 * t + 1]], g2 = gm[T[3 * t + 2]];
        r.x = b0 * g0.x + b1 * g1.x + b2 * g2.x;
        r.y = b0 * g0.y + b1 * g1.y + b2 * g2.y;
    }
    out[(size_t)m * n + i] = r;
}

inline dim3 grid1(int64_t n) { return dim3(static_cast<unsigned>((n + 255) / 256)); }

}  // namespace

hipError_t launch_samples(const nat_mesh* m, int32_t N, uint64_t seed, int32_t* tri,
                          double* bary, hipStream_t s)
{
    if (N <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_samples, grid1(N), dim3(256), 0, s, m->d_cdf, m->nT, m->area_total, N,
                       seed, tri, bary);
    return hipGetLastError();
}

hipError_t launch_points(const nat_mesh* m, int32_t n, const int32_t* tri, const double* bary,
                         PointStreams out, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_points, grid1(n), dim3(256), 0, s, m->d_V, m->d_T, m->d_normal, n, tri,
                       bary, m->center[0], m->center[1], m->center[2], out.x64, out.n64, out.x32,
                       out.n32);
    return hipGetLastError();
}

hipError_t launch_neumann(const nat_mesh* m, int32_t layout, const double2* g, int32_t ld_g,
                          int32_t n_modes, int32_t n, const int32_t* tri, const double* bary,
                          double2* g_out, hipStream_t s)
{
    if (n <= 0 || n_modes <= 0)
        return hipSuccess;
    dim3 grid(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>(n_modes));
    hipLaunchKernelGGL(k_neumann, grid, dim3(256), 0, s, m->d_T, layout, g, ld_g, n, tri, bary,
                       g_out);
    return hipGetLastError();
}

}  // namespace nat

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

// ---- the batch forms: blockIdx.y is the instance ---------------------------

__global__ void __launch_bounds__(256) k_samples_batch(const SurfBatch b)
{
    const SurfJob& J = b.jobs[blockIdx.y];
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= J.N)
        return;
    const uint64_t c = 3ull * static_cast<uint64_t>(j);
    const double u0 = unit_draw(J.seed, 0, c);
    const double u1 = unit_draw(J.seed, 0, c + 1);
    const double u2 = unit_draw(J.seed, 0, c + 2);
    const double tau = u0 * J.area;
    b.tri[J.on + j] = upper_search(J.cdf, J.nT, tau);
    const double sq = __builtin_sqrt(u1);
    b.bary[2 * (J.on + j) + 0] = sq * (1.0 - u2);
    b.bary[2 * (J.on + j) + 1] = sq * u2;
}

// blockIdx.z = 0: the samples, 1: the queries.
__global__ void __launch_bounds__(256) k_points_batch(const SurfBatch b)
{
    const SurfJob& J = b.jobs[blockIdx.y];
    const bool q = blockIdx.z == 1;
    const int32_t n = q ? J.Q : J.N;
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const double ctr[3] = {J.cx, J.cy, J.cz};
    double* x64 = q ? b.q64 + 3 * J.oq : b.x64 + 3 * J.on;
    float* x32 = q ? b.q32 + 3 * J.oq : b.x32 + 3 * J.on;
    if (q && J.fpts) {
        // free field points, world coordinates
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double x = J.fpts[3 * i + d];
            x64[(size_t)d * n + i] = x;
            x32[(size_t)d * n + i] = static_cast<float>(x - ctr[d]);
        }
        return;
    }
    const int32_t t = q ? J.q_tri[i] : b.tri[J.on + i];
    const double* bb = q ? J.q_bary + 2 * i : b.bary + 2 * (J.on + i);
    const double b1 = bb[0], b2 = bb[1];
    const double* v0 = J.V + 3 * J.T[3 * t + 0];
    const double* v1 = J.V + 3 * J.T[3 * t + 1];
    const double* v2 = J.V + 3 * J.T[3 * t + 2];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double x = v0[d] + b1 * (v1[d] - v0[d]) + b2 * (v2[d] - v0[d]);
        x64[(size_t)d * n + i] = x;
        x32[(size_t)d * n + i] = static_cast<float>(x - ctr[d]);
        if (!q) {
            const double nd = J.nrm[3 * t + d];
            b.n64[3 * J.on + (size_t)d * n + i] = nd;
            b.n32[3 * J.on + (size_t)d * n + i] = static_cast<float>(nd);
        }
    }
}

// blockIdx.z = 0: data at the samples, 1: at the queries; all modes.
__global__ void __launch_bounds__(256) k_neumann_batch(const SurfBatch b)
{
    const SurfJob& J = b.jobs[blockIdx.y];
    const bool q = blockIdx.z == 1;
    const int32_t n = q ? J.Q : J.N;
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    double2* out = q ? b.gq + J.og_q : b.gj + J.og_n;
    if (q && J.fpts) {
        // no Neumann data off the surface (the disk term is zero there)
        for (int32_t m = 0; m < J.M; ++m)
            out[(size_t)m * n + i] = make_double2(0.0, 0.0);
        return;
    }
    const int32_t t = q ? J.q_tri[i] : b.tri[J.on + i];
    const double* bb = q ? J.q_bary + 2 * i : b.bary + 2 * (J.on + i);
    if (b.layout == NAT_NEUMANN_PER_TRIANGLE) {
        for (int32_t m = 0; m < J.M; ++m)
            out[(size_t)m * n + i] = J.v_n[(size_t)m * J.ng + t];
        return;
    }
    const double b1 = bb[0], b2 = bb[1];
    const double b0 = 1.0 - b1 - b2;
    const int32_t c0 = J.T[3 * t], c1 = J.T[3 * t + 1], c2 = J.T[3 * t + 2];
    for (int32_t m = 0; m < J.M; ++m) {
        const double2* gm = J.v_n + (size_t)m * J.ng;
        const double2 g0 = gm[c0], g1 = gm[c1], g2 = gm[c2];
        double2 r;
        r.x = b0 * g0.x + b1 * g1.x + b2 * g2.x;
        r.y = b0 * g0.y + b1 * g1.y + b2 * g2.y;
        out[(size_t)m * n + i] = r;
    }
}

// Query records in range and finite Neumann data, for every instance.
__global__ void __launch_bounds__(256) k_checks_batch(const SurfBatch b)
{
    const SurfJob& J = b.jobs[blockIdx.y];
    const int64_t n_vals = 2 * (int64_t)J.M * J.ng;
    const double* vals = reinterpret_cast<const double*>(J.v_n);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_vals || i < J.Q; i += stride) {
        if (i < J.Q && J.fpts) {
            if (!isfinite(J.fpts[3 * i]) || !isfinite(J.fpts[3 * i + 1]) || !isfinite(J.fpts[3 * i + 2]))
                atomicOr(b.flags, 1);
        } else if (i < J.Q) {
            const int32_t t = J.q_tri[i];
            const double b1 = J.q_bary[2 * i], b2 = J.q_bary[2 * i + 1];
            if (!(t >= 0 && t < J.nT && b1 >= 0.0 && b2 >= 0.0 && b1 + b2 <= 1.0 + 1e-12))
                atomicOr(b.flags, 1);
        }
        if (i < n_vals && !isfinite(vals[i]))
            atomicOr(b.flags + 1, 1);
    }
}

// Field points around a scene (Section 3.4: random points in a shell of
// radius r_lo R .. r_hi R about the bounding-box centre; Section 3.1: an
// n_a x n_b grid of directions at radius r_lo R for FFAT maps).  Shell
// point i draws u0, u1, u2 from counters 3i .. 3i+2 of stream 5:
// r = R (r_lo + (r_hi - r_lo) u0), cos(theta) = 1 - 2 u1, phi = 2 pi u2.
// Grid point a n_b + b: theta = (a + 1/2) pi / n_a, phi = (b + 1/2) 2 pi / n_b.
__global__ void __launch_bounds__(256)
k_field_points(double cx, double cy, double cz, double R, int32_t kind, int32_t n_a, int32_t n_b,
               double r_lo, double r_hi, uint64_t seed, double* __restrict__ xyz,
               double* __restrict__ coords)
{
    const int64_t n = kind == 0 ? (int64_t)n_a : (int64_t)n_a * n_b;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    constexpr double kPi = 3.141592653589793;
    double r, th, ph;
    if (kind == 0) {
        const uint64_t c = 3ull * static_cast<uint64_t>(i);
        const double u0 = unit_draw(seed, 5, c);
        const double u1 = unit_draw(seed, 5, c + 1);
        const double u2 = unit_draw(seed, 5, c + 2);
        r = R * (r_lo + (r_hi - r_lo) * u0);
        th = acos(1.0 - 2.0 * u1);
        ph = 2.0 * kPi * u2;
    } else {
        const int32_t a = static_cast<int32_t>(i / n_b), b = static_cast<int32_t>(i % n_b);
        r = R * r_lo;
        th = (a + 0.5) * kPi / n_a;
        ph = (b + 0.5) * 2.0 * kPi / n_b;
    }
    double st, ct, sp, cp;
    sincos(th, &st, &ct);
    sincos(ph, &sp, &cp);
    xyz[3 * i + 0] = cx + r * (st * cp);
    xyz[3 * i + 1] = cy + r * (st * sp);
    xyz[3 * i + 2] = cz + r * ct;
    if (coords) {
        coords[3 * i + 0] = r;
        coords[3 * i + 1] = th;
        coords[3 * i + 2] = ph;
    }
}

// out[i] = |z[i]|
__global__ void __launch_bounds__(256) k_abs(const double2* __restrict__ z, int64_t n,
                                             double* __restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) {
        const double2 v = z[i];
        out[i] = __builtin_sqrt(v.x * v.x + v.y * v.y);
    }
}

}  // namespace

hipError_t launch_field_points(const nat_mesh* m, int32_t kind, int32_t n_a, int32_t n_b, double r_lo,
                               double r_hi, uint64_t seed, double* xyz, double* coords, hipStream_t s)
{
    const int64_t n = kind == 0 ? (int64_t)n_a : (int64_t)n_a * n_b;
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_field_points, grid1(n), dim3(256), 0, s, m->center[0], m->center[1],
                       m->center[2], 0.5 * m->diameter, kind, n_a, n_b, r_lo, r_hi, seed, xyz, coords);
    return hipGetLastError();
}

hipError_t launch_abs(const double2* z, int64_t n, double* out, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_abs, grid1(n), dim3(256), 0, s, z, n, out);
    return hipGetLastError();
}

hipError_t launch_checks_batch(const SurfBatch& b, int64_t max_work, hipStream_t s)
{
    if (b.n_jobs <= 0 || max_work <= 0)
        return hipSuccess;
    const int64_t blocks = (max_work + 255) / 256;
    dim3 grid(static_cast<unsigned>(blocks < 256 ? blocks : 256), static_cast<unsigned>(b.n_jobs));
    hipLaunchKernelGGL(k_checks_batch, grid, dim3(256), 0, s, b);
    return hipGetLastError();
}

// 1 / c_q for every query of every instance: a query exactly on a mesh
// vertex (two of its barycentric weights zero) or edge (one zero) takes the
// mesh's free term there, any other point c_q = 1/2; a free field point
// c_q = 1.
__global__ void __launch_bounds__(256)
k_jump_batch(const SurfBatch b)
{
    const SurfJob& X = b.jobs[blockIdx.y];
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= X.Q)
        return;
    if (X.fpts) {
        // exterior point: the representation formula has c = 1
        b.qfac[X.oq + i] = 1.0;
        return;
    }
    const int32_t t = X.q_tri[i];
    const double b1 = X.q_bary[2 * i], b2 = X.q_bary[2 * i + 1];
    const double w0 = 1.0 - b1 - b2;
    const bool z0 = w0 == 0.0, z1 = b1 == 0.0, z2 = b2 == 0.0;
    double c = 0.5;
    if (z1 && z2)
        c = X.cvert[X.T[3 * t + 0]];
    else if (z0 && z2)
        c = X.cvert[X.T[3 * t + 1]];
    else if (z0 && z1)
        c = X.cvert[X.T[3 * t + 2]];
    else if (z0)
        c = X.cedge[3 * t + 0];
    else if (z1)
        c = X.cedge[3 * t + 1];
    else if (z2)
        c = X.cedge[3 * t + 2];
    b.qfac[X.oq + i] = 1.0 / c;
}

hipError_t launch_surface_batch(const SurfBatch& b, int32_t max_n, int32_t max_q, hipStream_t s)
{
    if (b.n_jobs <= 0 || max_n <= 0)
        return hipSuccess;
    const int32_t mx = max_n > max_q ? max_n : max_q;
    const unsigned nj = static_cast<unsigned>(b.n_jobs);
    hipError_t e = hipSuccess;
    if (!b.samples_given) {
        hipLaunchKernelGGL(k_samples_batch, dim3((max_n + 255) / 256, nj), dim3(256), 0, s, b);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_points_batch, dim3((mx + 255) / 256, nj, max_q > 0 ? 2 : 1), dim3(256), 0, s, b);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_neumann_batch, dim3((mx + 255) / 256, nj, max_q > 0 ? 2 : 1), dim3(256), 0, s, b);
    e = hipGetLastError();
    if (e != hipSuccess || !b.qfac || max_q <= 0)
        return e;
    hipLaunchKernelGGL(k_jump_batch, dim3((max_q + 255) / 256, nj), dim3(256), 0, s, b);
    return hipGetLastError();
}

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

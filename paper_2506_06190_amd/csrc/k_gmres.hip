// Batched GMRES (Saad & Schultz 1986) for many independent systems that share
// a matvec launch: one workgroup per system runs the whole Arnoldi step after
// the matvec -- classical Gram-Schmidt applied twice (CGS2) in FP64, the norm,
// the new basis vector, the Givens rotations of the Hessenberg column and the
// convergence flag -- so one iteration costs the matvec plus one launch and
// no host round trip.  x0 = 0, restart = mmax (unrestarted up to mmax steps,
// Section 6.1 uses at most 200).
#include "nat_internal.h"

namespace nat {
namespace {

constexpr int kBlock = 1024;
constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b)  // conj(a) * b
{
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Sum `cnt` values per thread across the block; results in red[0..cnt).
// Fixed reduction tree, so the result does not depend on timing.
template <int CNT>
__device__ void block_sum(double (&v)[CNT], double* red /* [kWaves][CNT] */, double* out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < CNT; ++c) {
        double x = v[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            x += __shfl_xor(x, off, 64);
        v[c] = x;
    }
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < CNT; ++c)
            red[wave * CNT + c] = v[c];
    }
    __syncthreads();
    if (threadIdx.x < CNT) {
        double s = 0.0;
        for (int w = 0; w < kWaves; ++w)
            s += red[w * CNT + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kBlock)
k_gmres_init(GmresState g, const double2* __restrict__ b, int64_t ld_b)
{
    __shared__ double red[kWaves * 1];
    __shared__ double tot[1];
    const int m = blockIdx.x;
    const int n = g.n;
    const double2* bm = b + (size_t)m * ld_b;
    double acc[1] = {0.0};
    for (int t = threadIdx.x; t < n; t += kBlock) {
        const double2 v = bm[t];
        acc[0] += v.x * v.x + v.y * v.y;
    }
    block_sum<1>(acc, red, tot);
    const double beta = sqrt(tot[0]);
    double2* v0 = g.V + (size_t)m * (g.mmax + 1) * n;
    const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
    for (int t = threadIdx.x; t < n; t += kBlock) {
        const double2 v = bm[t];
        const double2 u = make_double2(v.x * inv, v.y * inv);
        v0[t] = u;
        if (g.v32)
            g.v32[(size_t)m * n + t] = make_float2(static_cast<float>(g.v32_scale * u.x),
                                                  static_cast<float>(g.v32_scale * u.y));
    }
    if (threadIdx.x == 0) {
        g.beta[m] = beta;
        g.gv[(size_t)m * (g.mmax + 1)] = make_double2(beta, 0.0);
        g.resid[m] = beta > 0.0 ? 1.0 : 0.0;
        g.iters[m] = 0;
        g.active[m] = beta > 0.0 ? 1 : 0;
    }
}

__device__ __forceinline__ void fold2(float& hi, float& lo, float t)
{
    const float s = hi + t;
    const float bp = s - hi;
    lo += (hi - (s - bp)) + (t - bp);
    hi = s;
}

__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        x += __shfl_xor(x, off, 64);
    return x;
}

// One Arnoldi step for system blockIdx.x.  Dot products are spread over the
// waves (wave q takes basis vectors q, q + 16, ...) and reduced inside the
// wave, so a CGS pass costs two barriers.
__global__ void __launch_bounds__(kBlock)
k_gmres_orth(GmresState g, int32_t j, const float4* __restrict__ partial, int32_t n_split)
{
    extern __shared__ double2 s_h[];  // [j+1] this pass, then [j+1] total
    __shared__ double red[kWaves];
    __shared__ double s_norm;
    const int m = blockIdx.x;
    if (!g.active[m])
        return;
    const int n = g.n;
    const int mm1 = g.mmax + 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double2* Vm = g.V + (size_t)m * mm1 * n;
    double2* w = g.w + (size_t)m * n;
    double2* h_pass = s_h;
    double2* h_tot = s_h + (j + 1);

    if (partial) {
        // matvec epilogue: w = v_j / 2 - (sum of the FP32 split partials)
        const double2* vj = Vm + (size_t)j * n;
        for (int t = tid; t < n; t += kBlock) {
            float hr = 0.0f, hi = 0.0f, lr = 0.0f, li = 0.0f;
            for (int32_t sp = 0; sp < n_split; ++sp) {
                const float4 v = partial[((size_t)sp * g.n_modes + m) * n + t];
                fold2(hr, lr, v.x);
                fold2(hi, li, v.y);
                lr += v.z;
                li += v.w;
            }
            const double ar = static_cast<double>(hr) + static_cast<double>(lr);
            const double ai = static_cast<double>(hi) + static_cast<double>(li);
            const double2 x = vj[t];
            w[t] = make_double2(0.5 * x.x - ar, 0.5 * x.y - ai);
        }
    }
    for (int i = tid; i <= j; i += kBlock)
        h_tot[i] = make_double2(0.0, 0.0);
    __syncthreads();

    for (int pass = 0; pass < 2; ++pass) {
        for (int i = wave; i <= j; i += kWaves) {
            const double2* vi = Vm + (size_t)i * n;
            double ar = 0.0, ai = 0.0;
            for (int t = lane; t < n; t += 64) {
                const double2 d = cmulc(vi[t], w[t]);
                ar += d.x;
                ai += d.y;
            }
            ar = wave_sum(ar);
            ai = wave_sum(ai);
            if (lane == 0)
                h_pass[i] = make_double2(ar, ai);
        }
        __syncthreads();
        for (int t = tid; t < n; t += kBlock) {
            double2 wt = w[t];
            for (int i = 0; i <= j; ++i) {
                const double2 d = cmul(h_pass[i], Vm[(size_t)i * n + t]);
                wt.x -= d.x;
                wt.y -= d.y;
            }
            w[t] = wt;
        }
        for (int i = tid; i <= j; i += kBlock) {
            h_tot[i].x += h_pass[i].x;
            h_tot[i].y += h_pass[i].y;
        }
        __syncthreads();
    }

    double nacc = 0.0;
    for (int t = tid; t < n; t += kBlock) {
        const double2 wt = w[t];
        nacc += wt.x * wt.x + wt.y * wt.y;
    }
    nacc = wave_sum(nacc);
    if (lane == 0)
        red[wave] = nacc;
    __syncthreads();
    if (tid == 0) {
        double sacc = 0.0;
        for (int q = 0; q < kWaves; ++q)
            sacc += red[q];
        s_norm = sqrt(sacc);
    }
    __syncthreads();
    const double hn = s_norm;
    const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
    double2* vn = g.V + ((size_t)m * mm1 + j + 1) * n;
    for (int t = tid; t < n; t += kBlock) {
        const double2 wt = w[t];
        const double2 u = make_double2(wt.x * inv, wt.y * inv);
        vn[t] = u;
        if (g.v32)
            g.v32[(size_t)m * n + t] = make_float2(static_cast<float>(g.v32_scale * u.x),
                                                  static_cast<float>(g.v32_scale * u.y));
    }

    if (tid == 0) {
        double2* H = g.H + ((size_t)m * g.mmax + j) * mm1;  // column j
        double* cs = g.cs + (size_t)m * g.mmax;
        double2* sn = g.sn + (size_t)m * g.mmax;
        double2* gv = g.gv + (size_t)m * mm1;
        for (int i = 0; i <= j; ++i)
            H[i] = h_tot[i];
        // earlier rotations: [c, s; -conj(s), c]
        for (int i = 0; i < j; ++i) {
            const double2 a = H[i], b = H[i + 1];
            const double2 sb = cmul(sn[i], b);
            const double2 sa = cmulc(sn[i], a);
            H[i] = make_double2(cs[i] * a.x + sb.x, cs[i] * a.y + sb.y);
            H[i + 1] = make_double2(cs[i] * b.x - sa.x, cs[i] * b.y - sa.y);
        }
        const double2 a = H[j];
        const double amag = hypot(a.x, a.y);
        const double den = hypot(amag, hn);
        double c;
        double2 sg;
        if (amag == 0.0) {
            c = 0.0;
            sg = make_double2(1.0, 0.0);
        } else {
            c = amag / den;
            sg = make_double2(a.x / amag * hn / den, a.y / amag * hn / den);
        }
        cs[j] = c;
        sn[j] = sg;
        H[j] = make_double2(c * a.x + sg.x * hn, c * a.y + sg.y * hn);
        H[j + 1] = make_double2(0.0, 0.0);
        const double2 gj = gv[j];
        const double2 cg = cmulc(sg, gj);
        gv[j + 1] = make_double2(-cg.x, -cg.y);
        gv[j] = make_double2(c * gj.x, c * gj.y);
        const double res = hypot(gv[j + 1].x, gv[j + 1].y) / g.beta[m];
        g.resid[m] = res;
        g.iters[m] = j + 1;
        if (res <= g.tol || hn == 0.0 || j + 1 >= g.mmax)
            g.active[m] = 0;
    }
}

// y = H^{-1} g on the first iters columns, x = V y.
__global__ void __launch_bounds__(kBlock)
k_gmres_solution(GmresState g, double2* __restrict__ x, int64_t ld_x)
{
    extern __shared__ double2 s_y[];
    const int m = blockIdx.x;
    const int n = g.n;
    const int mm1 = g.mmax + 1;
    const int it = g.iters[m];
    if (threadIdx.x == 0) {
        const double2* gv = g.gv + (size_t)m * mm1;
        for (int i = it - 1; i >= 0; --i) {
            double2 s = gv[i];
            for (int t = i + 1; t < it; ++t) {
                const double2 d = cmul(g.H[((size_t)m * g.mmax + t) * mm1 + i], s_y[t]);
                s.x -= d.x;
                s.y -= d.y;
            }
            const double2 hd = g.H[((size_t)m * g.mmax + i) * mm1 + i];
            const double den = hd.x * hd.x + hd.y * hd.y;
            s_y[i] = make_double2((s.x * hd.x + s.y * hd.y) / den, (s.y * hd.x - s.x * hd.y) / den);
        }
    }
    __syncthreads();
    const double2* Vm = g.V + (size_t)m * mm1 * n;
    double2* xm = x + (size_t)m * ld_x;
    for (int t = threadIdx.x; t < n; t += kBlock) {
        double2 acc = make_double2(0.0, 0.0);
        for (int i = 0; i < it; ++i) {
            const double2 d = cmul(s_y[i], Vm[(size_t)i * n + t]);
            acc.x += d.x;
            acc.y += d.y;
        }
        xm[t] = acc;
    }
}

}  // namespace

size_t gmres_state_bytes(int32_t n, int32_t M, int32_t mmax)
{
    const size_t mm1 = (size_t)mmax + 1;
    return carve_size<>({sizeof(double2) * M * mm1 * n, sizeof(double2) * M * mmax * mm1,
                         sizeof(double) * M * mmax, sizeof(double2) * M * mmax,
                         sizeof(double2) * M * mm1, sizeof(double) * M, sizeof(double) * M,
                         sizeof(int32_t) * M, sizeof(int32_t) * M, sizeof(double2) * M * n,
                         sizeof(float2) * M * n});
}

void gmres_carve(GmresState& g, Carver& c)
{
    const size_t M = g.n_modes, n = g.n, mm1 = (size_t)g.mmax + 1;
    g.V = c.take<double2>(M * mm1 * n);
    g.H = c.take<double2>(M * g.mmax * mm1);
    g.cs = c.take<double>(M * g.mmax);
    g.sn = c.take<double2>(M * g.mmax);
    g.gv = c.take<double2>(M * mm1);
    g.beta = c.take<double>(M);
    g.resid = c.take<double>(M);
    g.iters = c.take<int32_t>(M);
    g.active = c.take<int32_t>(M);
    g.w = c.take<double2>(M * n);
    g.v32 = c.take<float2>(M * n);
}

hipError_t launch_gmres_init(const GmresState& g, const double2* b, int64_t ld_b, hipStream_t s)
{
    hipLaunchKernelGGL(k_gmres_init, dim3(g.n_modes), dim3(kBlock), 0, s, g, b, ld_b);
    return hipGetLastError();
}

hipError_t launch_gmres_orth(const GmresState& g, int32_t j, const void* partial, int32_t n_split,
                             hipStream_t s)
{
    const size_t lds = sizeof(double2) * 2 * (size_t)(j + 1);
    hipLaunchKernelGGL(k_gmres_orth, dim3(g.n_modes), dim3(kBlock), lds, s, g, j,
                       static_cast<const float4*>(partial), n_split);
    return hipGetLastError();
}

hipError_t launch_gmres_solution(const GmresState& g, double2* x, int64_t ld_x, hipStream_t s)
{
    const size_t lds = sizeof(double2) * (size_t)(g.mmax > 0 ? g.mmax : 1);
    hipLaunchKernelGGL(k_gmres_solution, dim3(g.n_modes), dim3(kBlock), lds, s, g, x, ld_x);
    return hipGetLastError();
}

}  // namespace nat

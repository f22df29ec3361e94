// Batched GMRES (Saad & Schultz 1986) for many independent systems that share
// their matvec launches.  The Arnoldi step after each matvec is classical
// Gram-Schmidt applied twice (CGS2) in FP64, spread over row chunks of 256
// rows so one system uses as many CUs as it has chunks:
//   dots     partial <v_i, w> over the chunk's rows        (w formed from the
//            FP32 matvec partials first when there are any)
//   update   h = sum of the chunk partials in chunk order; w -= V h on the
//            chunk's rows; then either the second pass's partial dots or the
//            partial squared norm
//   finalize |w|, v_{j+1} = w / |w| and its FP32 copy; the first chunk's
//            first thread applies the Givens rotations to the new Hessenberg
//            column and sets the convergence flag.
// Every chunk sums the same partials in the same order, so all chunks use
// identical coefficients and results do not depend on scheduling.  x0 = 0,
// restart = mmax (unrestarted up to mmax steps; Section 6.1 uses at most 200).
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
        if (g.host_active)
            *reinterpret_cast<volatile int32_t*>(g.host_active + m) = beta > 0.0 ? 1 : 0;
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

constexpr int kRows = 256;  // rows per chunk = threads per chunk block
constexpr int kRowWaves = kRows / 64;

// Partial dot products of the chunk's rows s_w (in LDS) with v_0..v_j.  A
// wave takes 8 consecutive basis vectors per round: all loads of the round
// are issued before the 16 interleaved butterfly reductions.
constexpr int kDotGroup = 8;

__device__ __forceinline__ void chunk_dots(const GmresState& g, const double2* Vm, int32_t j,
                                           int32_t r0, const double2* s_w, double2* dp_out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = g.n;
    for (int i0 = kDotGroup * wave; i0 <= j; i0 += kDotGroup * kRowWaves) {
        double ar[kDotGroup], ai[kDotGroup];
#pragma unroll
        for (int c = 0; c < kDotGroup; ++c)
            ar[c] = ai[c] = 0.0;
#pragma unroll
        for (int q = 0; q < kRows / 64; ++q) {
            const int rr = lane + 64 * q;
            if (r0 + rr >= n)
                continue;
            const double2 wv = s_w[rr];
            double2 v[kDotGroup];
#pragma unroll
            for (int c = 0; c < kDotGroup; ++c)
                v[c] = (i0 + c <= j) ? Vm[(size_t)(i0 + c) * n + r0 + rr] : make_double2(0.0, 0.0);
#pragma unroll
            for (int c = 0; c < kDotGroup; ++c) {
                const double2 d = cmulc(v[c], wv);
                ar[c] += d.x;
                ai[c] += d.y;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
            for (int c = 0; c < kDotGroup; ++c) {
                ar[c] += __shfl_xor(ar[c], off, 64);
                ai[c] += __shfl_xor(ai[c], off, 64);
            }
        }
        if (lane < kDotGroup && i0 + lane <= j) {
            double xr = ar[0], xi = ai[0];
#pragma unroll
            for (int c = 1; c < kDotGroup; ++c)
                if (lane == c) {
                    xr = ar[c];
                    xi = ai[c];
                }
            dp_out[i0 + lane] = make_double2(xr, xi);
        }
    }
}

__global__ void __launch_bounds__(kRows)
k_orth_dots(GmresState g, int32_t j, const float4* __restrict__ partial, int32_t n_split,
            ModeList modes)
{
    __shared__ double2 s_w[kRows];
    const int32_t m = mode_at(modes, blockIdx.x);
    const int32_t chunk = blockIdx.y;
    if (!g.active[m])
        return;
    const int n = g.n, mm1 = g.mmax + 1;
    const int32_t r0 = chunk * kRows;
    const int32_t t = r0 + threadIdx.x;
    const double2* Vm = g.V + (size_t)m * mm1 * n;
    double2* w = g.w + (size_t)m * n;
    double2 wt = make_double2(0.0, 0.0);
    if (t < n) {
        if (partial) {
            // matvec epilogue: w = v_j / 2 - (sum of the FP32 split partials)
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
            const double2 x = Vm[(size_t)j * n + t];
            wt = make_double2(0.5 * x.x - ar, 0.5 * x.y - ai);
            w[t] = wt;
        } else {
            wt = w[t];
        }
    }
    s_w[threadIdx.x] = wt;
    __syncthreads();
    chunk_dots(g, Vm, j, r0, s_w, g.dp1 + ((size_t)m * g.nch + chunk) * mm1);
}

// pass 0: w -= V h1, then the partial dots of the second pass into dp2.
// pass 1: w -= V h2, then the partial squared norm.
__global__ void __launch_bounds__(kRows)
k_orth_update(GmresState g, int32_t j, int32_t pass, ModeList modes)
{
    __shared__ double2 s_w[kRows];
    extern __shared__ double2 s_h[];  // [j+1]
    const int32_t m = mode_at(modes, blockIdx.x);
    const int32_t chunk = blockIdx.y;
    if (!g.active[m])
        return;
    const int n = g.n, mm1 = g.mmax + 1;
    const double2* dp = (pass == 0 ? g.dp1 : g.dp2) + (size_t)m * g.nch * mm1;
    for (int i = threadIdx.x; i <= j; i += kRows) {
        double hr = 0.0, hi = 0.0;
        for (int c = 0; c < g.nch; ++c) {
            const double2 v = dp[(size_t)c * mm1 + i];
            hr += v.x;
            hi += v.y;
        }
        s_h[i] = make_double2(hr, hi);
        if (chunk == 0) {
            double2* ht = g.htot + (size_t)m * mm1;
            ht[i] = pass == 0 ? make_double2(hr, hi) : make_double2(ht[i].x + hr, ht[i].y + hi);
        }
    }
    __syncthreads();
    const int32_t r0 = chunk * kRows;
    const int32_t t = r0 + threadIdx.x;
    const double2* Vm = g.V + (size_t)m * mm1 * n;
    double2* w = g.w + (size_t)m * n;
    double2 wt = make_double2(0.0, 0.0);
    if (t < n) {
        wt = w[t];
        constexpr int U = 16;
        int i = 0;
        for (; i + U <= j + 1; i += U) {
            double2 v[U];
#pragma unroll
            for (int c = 0; c < U; ++c)
                v[c] = Vm[(size_t)(i + c) * n + t];
#pragma unroll
            for (int c = 0; c < U; ++c) {
                const double2 d = cmul(s_h[i + c], v[c]);
                wt.x -= d.x;
                wt.y -= d.y;
            }
        }
        for (; i <= j; ++i) {
            const double2 d = cmul(s_h[i], Vm[(size_t)i * n + t]);
            wt.x -= d.x;
            wt.y -= d.y;
        }
        w[t] = wt;
    }
    s_w[threadIdx.x] = wt;
    __syncthreads();
    if (pass == 0) {
        chunk_dots(g, Vm, j, r0, s_w, g.dp2 + ((size_t)m * g.nch + chunk) * mm1);
    } else {
        __shared__ double red[kRowWaves];
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        double a = wave_sum(wt.x * wt.x + wt.y * wt.y);
        if (lane == 0)
            red[wave] = a;
        __syncthreads();
        if (threadIdx.x == 0) {
            double sacc = 0.0;
            for (int q = 0; q < kRowWaves; ++q)
                sacc += red[q];
            g.normpart[(size_t)m * g.nch + chunk] = sacc;
        }
    }
}

// v_{j+1} = w / |w| on the chunk's rows; Givens and convergence on chunk 0.
// Blocks of a system that stopped in an earlier iteration only rewrite
// basis rows past its last iteration, which the solution never reads.
__global__ void __launch_bounds__(kRows)
k_orth_finalize(GmresState g, int32_t j, ModeList modes)
{
    __shared__ double s_hn;
    const int32_t m = mode_at(modes, blockIdx.x);
    const int32_t chunk = blockIdx.y;
    const int n = g.n, mm1 = g.mmax + 1;
    if (threadIdx.x == 0) {
        double sacc = 0.0;
        for (int c = 0; c < g.nch; ++c)
            sacc += g.normpart[(size_t)m * g.nch + c];
        s_hn = sqrt(sacc);
    }
    __syncthreads();
    const double hn = s_hn;
    const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
    const int32_t t = chunk * kRows + threadIdx.x;
    if (t < n && j + 1 <= g.mmax) {
        const double2 wt = g.w[(size_t)m * n + t];
        const double2 u = make_double2(wt.x * inv, wt.y * inv);
        g.V[((size_t)m * mm1 + j + 1) * n + t] = u;
        if (g.v32)
            g.v32[(size_t)m * n + t] = make_float2(static_cast<float>(g.v32_scale * u.x),
                                                  static_cast<float>(g.v32_scale * u.y));
    }
    if (g.host_progress && blockIdx.x == 0 && chunk == 0 && threadIdx.x == 0)
        *reinterpret_cast<volatile int32_t*>(g.host_progress) = j + 1;
    if (chunk != 0 || !g.active[m])
        return;
    // Givens rotations of the new Hessenberg column, staged in LDS: rotation
    // i mixes entries i and i+1, so thread 0 carries the running entry in
    // registers while the other threads load and store in parallel.
    extern __shared__ double2 s_col[];   // [j+2] column, then [j] sines
    double* s_cs = reinterpret_cast<double*>(s_col + 2 * (j + 2));
    double2* s_sn = s_col + (j + 2);
    double2* H = g.H + ((size_t)m * g.mmax + j) * mm1;  // column j
    double* cs = g.cs + (size_t)m * g.mmax;
    double2* sn = g.sn + (size_t)m * g.mmax;
    double2* gv = g.gv + (size_t)m * mm1;
    const double2* ht = g.htot + (size_t)m * mm1;
    for (int i = threadIdx.x; i <= j; i += kRows) {
        s_col[i] = ht[i];
        if (i < j) {
            s_cs[i] = cs[i];
            s_sn[i] = sn[i];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // earlier rotations: [c, s; -conj(s), c]
        double2 carry = s_col[0];
        for (int i = 0; i < j; ++i) {
            const double2 b = s_col[i + 1];
            const double c = s_cs[i];
            const double2 sv = s_sn[i];
            const double2 sb = cmul(sv, b);
            const double2 sa = cmulc(sv, carry);
            s_col[i] = make_double2(c * carry.x + sb.x, c * carry.y + sb.y);
            carry = make_double2(c * b.x - sa.x, c * b.y - sa.y);
        }
        const double2 a = carry;
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
        s_col[j] = make_double2(c * a.x + sg.x * hn, c * a.y + sg.y * hn);
        s_col[j + 1] = make_double2(0.0, 0.0);
        const double2 gj = gv[j];
        const double2 cg = cmulc(sg, gj);
        gv[j + 1] = make_double2(-cg.x, -cg.y);
        gv[j] = make_double2(c * gj.x, c * gj.y);
        const double res = hypot(gv[j + 1].x, gv[j + 1].y) / g.beta[m];
        g.resid[m] = res;
        g.iters[m] = j + 1;
        if (res <= g.tol || hn == 0.0 || j + 1 >= g.mmax) {
            g.active[m] = 0;
            if (g.host_active)
                *reinterpret_cast<volatile int32_t*>(g.host_active + m) = 0;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= j + 1; i += kRows)
        H[i] = s_col[i];
}

// y = H^{-1} g on the first `iters` columns (column-oriented back
// substitution: y_t is final once the columns right of t are applied, then
// all rows above t subtract column t in parallel), then x = V y.
__global__ void __launch_bounds__(kBlock)
k_gmres_solution(GmresState g, double2* __restrict__ x, int64_t ld_x)
{
    extern __shared__ double2 s_y[];  // [mmax] right-hand side, becomes y
    const int m = blockIdx.x;
    const int n = g.n;
    const int mm1 = g.mmax + 1;
    const int it = g.iters[m];
    const double2* gv = g.gv + (size_t)m * mm1;
    for (int i = threadIdx.x; i < it; i += kBlock)
        s_y[i] = gv[i];
    __syncthreads();
    for (int t = it - 1; t >= 0; --t) {
        const double2* col = g.H + ((size_t)m * g.mmax + t) * mm1;
        const double2 hd = col[t];
        const double den = hd.x * hd.x + hd.y * hd.y;
        const double2 st = s_y[t];
        const double2 yt = make_double2((st.x * hd.x + st.y * hd.y) / den,
                                        (st.y * hd.x - st.x * hd.y) / den);
        __syncthreads();
        if (threadIdx.x == 0)
            s_y[t] = yt;
        for (int i = threadIdx.x; i < t; i += kBlock) {
            const double2 d = cmul(col[i], yt);
            s_y[i] = make_double2(s_y[i].x - d.x, s_y[i].y - d.y);
        }
        __syncthreads();
    }
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
    const size_t nch = (size_t)((n + kRows - 1) / kRows);
    return carve_size<>({sizeof(double2) * M * mm1 * n, sizeof(double2) * M * mmax * mm1,
                         sizeof(double) * M * mmax, sizeof(double2) * M * mmax,
                         sizeof(double2) * M * mm1, sizeof(double) * M, sizeof(double) * M,
                         sizeof(int32_t) * M, sizeof(int32_t) * M, sizeof(double2) * M * n,
                         sizeof(float2) * M * n, 2 * sizeof(double2) * M * nch * mm1,
                         sizeof(double) * M * nch, sizeof(double2) * M * mm1});
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
    g.nch = (g.n + kRows - 1) / kRows;
    g.dp1 = c.take<double2>(M * g.nch * mm1);
    g.dp2 = c.take<double2>(M * g.nch * mm1);
    g.normpart = c.take<double>(M * g.nch);
    g.htot = c.take<double2>(M * mm1);
}

hipError_t launch_gmres_init(const GmresState& g, const double2* b, int64_t ld_b, hipStream_t s)
{
    hipLaunchKernelGGL(k_gmres_init, dim3(g.n_modes), dim3(kBlock), 0, s, g, b, ld_b);
    return hipGetLastError();
}

hipError_t launch_gmres_orth(const GmresState& g, int32_t j, const void* partial, int32_t n_split,
                             const ModeList& modes, hipStream_t s, const ProfSlot& ev)
{
    if (modes.n <= 0)
        return hipSuccess;
    const dim3 grid(static_cast<unsigned>(modes.n), static_cast<unsigned>(g.nch));
    const size_t lds = sizeof(double2) * (size_t)(j + 1);
    launch_k(k_orth_dots, grid, dim3(kRows), 0, s, ev.start, nullptr, g, j,
             static_cast<const float4*>(partial), n_split, modes);
    hipLaunchKernelGGL(k_orth_update, grid, dim3(kRows), lds, s, g, j, 0, modes);
    hipLaunchKernelGGL(k_orth_update, grid, dim3(kRows), lds, s, g, j, 1, modes);
    const size_t lds_fin = sizeof(double2) * (size_t)(2 * (j + 2)) + sizeof(double) * (size_t)(j + 1);
    launch_k(k_orth_finalize, grid, dim3(kRows), lds_fin, s, nullptr, ev.stop, g, j, modes);
    return hipGetLastError();
}

hipError_t launch_gmres_solution(const GmresState& g, double2* x, int64_t ld_x, hipStream_t s)
{
    const size_t lds = sizeof(double2) * (size_t)(g.mmax > 0 ? g.mmax : 1);
    hipLaunchKernelGGL(k_gmres_solution, dim3(g.n_modes), dim3(kBlock), lds, s, g, x, ld_x);
    return hipGetLastError();
}

}  // namespace nat

// Batched GMRES (Saad & Schultz 1986) for many independent systems of uneven
// size that share their matvec launches.  x0 = 0, restart = mmax
// (unrestarted up to mmax steps; Section 6.1 uses at most 200).
//
// Arnoldi step: classical Gram-Schmidt with the reorthogonalisation of CGS2
// folded into the first projection through the Gram matrix of the basis.
// With s = V^H w and G = V^H V, the second CGS pass would project with
// V^H (w - V s) = s - G s in exact arithmetic, so the step uses the single
// coefficient vector h = s - (G - I) s and one update w <- w - V h.  G is
// kept column by column: the pass that forms s also forms V^H v_j for the
// newest basis vector.  This corrects the basis's own loss of orthogonality
// exactly; what it cannot see is the rounding of the update itself, of
// relative size eps |w| / |w - V h|, so when the update cancels w by more
// than a factor 100 a true second pass (dots and update) follows, as in
// selective reorthogonalisation (Daniel, Gragg, Kaufman & Stewart 1976).
// The idea of obtaining the reorthogonalisation coefficients from inner
// products computed in the same sweep follows the low-synchronisation
// Gram-Schmidt variants of Swirydowicz, Langou, Ananthan, Yang & Thomas
// (2020).  The basis is read twice per step instead of four times.
//
// The work is spread over items (system, chunk of 256 rows), so one system
// uses as many CUs as it has chunks:
//   dots      w formed from the FP32 matvec partials when there are any, then
//             partial <v_i, w> and <v_i, v_j> over the chunk's rows, and the
//             partial |w|^2
//   coef      the Gram column of v_j and h = s - (G - I) s, one 64-row
//             block of h per item, the sum over k split between 4 waves
//   update    w -= V h on the chunk's rows, partial |w|^2
//   dots2     (only after strong cancellation) partial <v_i, w>
//   update2   (same) w -= V h2, h += h2, partial |w|^2
//   finalize  |w|, v_{j+1} = w/|w| and its FP32 copy; the first chunk applies
//             the Givens rotations to the new Hessenberg column and sets the
//             convergence flag
//   advance   j <- j + 1
// Every chunk sums the same partials in the same order, so all chunks use
// identical coefficients and take identical decisions.  The kernels are
// persistent over the item list and read j from device memory, so a run of
// iterations can be captured once as a graph and replayed while the host
// refreshes the lists between replays.
#include "nat_internal.h"

namespace nat {
namespace {

constexpr int kRows = 256;  // rows per chunk = threads per workgroup
constexpr int32_t kCoefGridX = 8;   // workgroups of k_orth_coef per streaming workgroup
constexpr int32_t kFinalGridX = 4;  // ... of k_orth_finalize
constexpr int kRowWaves = kRows / 64;
// true second pass when |w - V h|^2 < kCancel2 |w|^2 (cancellation by > 100x)
constexpr double kCancel2 = 1e-4;

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b)  // conj(a) * b
{
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
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

__device__ __forceinline__ double block_sum(double v, double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0)
        red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < kRowWaves; ++q)
        s += red[q];
    return s;
}

// Partial dot products of the chunk's rows s_x (LDS) with v_0..v_j, and with
// kTwo of s_y as well.  A wave takes kDotGroup consecutive basis vectors
// per round: all loads of the round are issued before the interleaved
// butterfly reductions.  Small groups keep the register count low enough for 6-7
// waves per SIMD, which hides the latency of the many short items of the
// early iterations.
template <bool kTwo, int kDotGroup = kTwo ? 2 : 4>
__device__ __forceinline__ void chunk_dots(const double2* Vs, int32_t n, int32_t j, int32_t r0,
                                           const double2* s_x, const double2* s_y, double2* dpx,
                                           double2* dpy)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i0 = kDotGroup * wave; i0 <= j; i0 += kDotGroup * kRowWaves) {
        double ar[kDotGroup], ai[kDotGroup], br[kDotGroup], bi[kDotGroup];
#pragma unroll
        for (int c = 0; c < kDotGroup; ++c)
            ar[c] = ai[c] = br[c] = bi[c] = 0.0;
#pragma unroll
        for (int q = 0; q < kRows / 64; ++q) {
            const int rr = lane + 64 * q;
            if (r0 + rr >= n)
                continue;
            const double2 xv = s_x[rr];
            const double2 yv = kTwo ? s_y[rr] : make_double2(0.0, 0.0);
            double2 v[kDotGroup];
#pragma unroll
            for (int c = 0; c < kDotGroup; ++c)
                v[c] = (i0 + c <= j) ? Vs[(size_t)(i0 + c) * n + r0 + rr] : make_double2(0.0, 0.0);
#pragma unroll
            for (int c = 0; c < kDotGroup; ++c) {
                const double2 d = cmulc(v[c], xv);
                ar[c] += d.x;
                ai[c] += d.y;
                if (kTwo) {
                    const double2 e = cmulc(v[c], yv);
                    br[c] += e.x;
                    bi[c] += e.y;
                }
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
            for (int c = 0; c < kDotGroup; ++c) {
                ar[c] += __shfl_xor(ar[c], off, 64);
                ai[c] += __shfl_xor(ai[c], off, 64);
                if (kTwo) {
                    br[c] += __shfl_xor(br[c], off, 64);
                    bi[c] += __shfl_xor(bi[c], off, 64);
                }
            }
        }
        if (lane < kDotGroup && i0 + lane <= j) {
            double xr = ar[0], xi = ai[0], yr = br[0], yi = bi[0];
#pragma unroll
            for (int c = 1; c < kDotGroup; ++c)
                if (lane == c) {
                    xr = ar[c];
                    xi = ai[c];
                    yr = br[c];
                    yi = bi[c];
                }
            dpx[i0 + lane] = make_double2(xr, xi);
            if (kTwo)
                dpy[i0 + lane] = make_double2(yr, yi);
        }
    }
}

// Whether system S's step needs the true second pass: |w - V h|^2 against
// |w|^2 before the projection, both summed over the chunks in order.
__device__ __forceinline__ bool strong_cancel(const GmresBatch& g, const SysDev& S)
{
    double a = 0.0, b = 0.0;
    for (int c = 0; c < S.nch; ++c) {
        a += g.normpart[S.off_ch + c];
        b += g.wnorm0[S.off_ch + c];
    }
    return a < kCancel2 * b;
}

// Sum of the chunk partials of entry i, in chunk order.
__device__ __forceinline__ double2 chunk_sum(const double2* dp, int32_t nch, int mm1, int i)
{
    double hr = 0.0, hi = 0.0;
    for (int c0 = 0; c0 < nch; c0 += 8) {
        double2 v[8];
#pragma unroll
        for (int c = 0; c < 8; ++c)
            v[c] = c0 + c < nch ? dp[(size_t)(c0 + c) * mm1 + i] : make_double2(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if (c0 + c < nch) {
                hr += v[c].x;
                hi += v[c].y;
            }
        }
    }
    return make_double2(hr, hi);
}

__global__ void __launch_bounds__(kRows) k_orth_dots(GmresBatch g)
{
    __shared__ double2 s_w[kRows];
    __shared__ double2 s_v[kRows];
    __shared__ double red[kRowWaves];
    const int32_t j = *g.iter;
    const int32_t n_items = *g.n_items;
    if (j >= g.mmax)
        return;
    const int mm1 = g.mmax + 1;
    for (int32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 item = g.items[it];
        const int32_t s = item.x, chunk = item.y;
        if (!g.active[s])
            continue;
        const SysDev& S = g.sys[s];
        const int32_t n = S.n;
        const int32_t r0 = chunk * kRows;
        const int32_t t = r0 + threadIdx.x;
        const double2* Vs = g.V + S.off_v;
        double2* w = g.w + S.off_n;
        double2 wt = make_double2(0.0, 0.0);
        double2 vj = make_double2(0.0, 0.0);
        if (t < n) {
            vj = Vs[(size_t)j * n + t];
            if (g.partial) {
                // matvec epilogue: w = v_j / 2 - (sum of the FP32 split partials)
                float hr = 0.0f, hi = 0.0f, lr = 0.0f, li = 0.0f;
                const float4* pp = g.partial + S.off_pa + t;
                const float2* pp2 = reinterpret_cast<const float2*>(g.partial) + 2 * S.off_pa + t;
                if (S.mv_pair) {
                    for (int32_t sp0 = 0; sp0 < S.nsplit_mv; sp0 += 8) {
                        float2 v[8];
#pragma unroll
                        for (int c = 0; c < 8; ++c)
                            v[c] = sp0 + c < S.nsplit_mv ? pp2[(int64_t)(sp0 + c) * n]
                                                         : make_float2(0.0f, 0.0f);
#pragma unroll
                        for (int c = 0; c < 8; ++c) {
                            if (sp0 + c < S.nsplit_mv) {
                                fold2(hr, lr, v[c].x);
                                fold2(hi, li, v[c].y);
                            }
                        }
                    }
                }
                for (int32_t sp0 = 0; sp0 < (S.mv_pair ? 0 : S.nsplit_mv); sp0 += 8) {
                    // issue the group's loads together, fold in split order
                    float4 v[8];
#pragma unroll
                    for (int c = 0; c < 8; ++c)
                        v[c] = sp0 + c < S.nsplit_mv ? pp[(int64_t)(sp0 + c) * n]
                                                     : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        if (sp0 + c < S.nsplit_mv) {
                            fold2(hr, lr, v[c].x);
                            fold2(hi, li, v[c].y);
                            lr += v[c].z;
                            li += v[c].w;
                        }
                    }
                }
                const double ar = static_cast<double>(hr) + static_cast<double>(lr);
                const double ai = static_cast<double>(hi) + static_cast<double>(li);
                wt = make_double2(0.5 * vj.x - ar, 0.5 * vj.y - ai);
                w[t] = wt;
            } else {
                wt = w[t];
            }
        }
        __syncthreads();
        s_w[threadIdx.x] = wt;
        s_v[threadIdx.x] = vj;
        __syncthreads();
        chunk_dots<true>(Vs, n, j, r0, s_w, s_v, g.dp1 + (S.off_ch + chunk) * mm1,
                         g.dp2 + (S.off_ch + chunk) * mm1);
        const double nw = block_sum(wt.x * wt.x + wt.y * wt.y, red);
        if (threadIdx.x == 0)
            g.wnorm0[S.off_ch + chunk] = nw;
    }
}

// s = V^H w and the new Gram column V^H v_j from the chunk partials, then
// h = s - (G - I) s into the Hessenberg column: item (system, chunk c)
// takes the 64-row blocks b = c, c + nch, ... of h; in a block lane l owns
// row 64 b + l and wave q sums the columns k = q, q + 4, ... of G; the four
// partial sums are added in wave order.
__global__ void __launch_bounds__(kRows) k_orth_coef(GmresBatch g)
{
    extern __shared__ double2 s_sv[];  // [mmax + 1] s | [mmax + 1] Gram column j
    __shared__ double2 s_part[kRowWaves][64];
    const int32_t j = *g.iter;
    const int32_t n_items = *g.n_items;
    if (j >= g.mmax)
        return;
    const int mm1 = g.mmax + 1;
    const int32_t n_blk = (j + 64) / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double2* s_gj = s_sv + mm1;
    for (int32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 item = g.items[it];
        const int32_t s = item.x, chunk = item.y;
        if (chunk >= n_blk || !g.active[s])
            continue;
        const SysDev& S = g.sys[s];
        // the full Hermitian G, column-major with leading dimension mmax + 1:
        // column k is complete up to row j once step j has run
        double2* G = g.gram + (size_t)s * g.gram_stride;
        __syncthreads();
        for (int i = threadIdx.x; i <= j; i += kRows) {
            s_sv[i] = chunk_sum(g.dp1 + S.off_ch * mm1, S.nch, mm1, i);
            s_gj[i] = chunk_sum(g.dp2 + S.off_ch * mm1, S.nch, mm1, i);
        }
        __syncthreads();
        double2* ht = g.htot + (size_t)s * mm1;
        for (int32_t blk = chunk; blk < n_blk; blk += S.nch) {
            const int i = 64 * blk + lane;
            // (G - I) s, row i: entry (i, k) is column k's row i (loads
            // coalesced across the lanes), column j and row j from LDS
            double er = 0.0, ei = 0.0;
            if (i <= j) {
                for (int k0 = wave; k0 <= j; k0 += 8 * kRowWaves) {
                    double2 gk[8];
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const int k = k0 + kRowWaves * c;
                        if (k >= j)
                            gk[c] = k == j ? s_gj[i] : make_double2(0.0, 0.0);
                        else if (i == j)
                            gk[c] = make_double2(s_gj[k].x, -s_gj[k].y);
                        else
                            gk[c] = G[(size_t)k * mm1 + i];
                    }
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const int k = k0 + kRowWaves * c;
                        if (k <= j) {
                            double2 gik = gk[c];
                            if (k == i)
                                gik.x -= 1.0;
                            const double2 d = cmul(gik, s_sv[k]);
                            er += d.x;
                            ei += d.y;
                        }
                    }
                }
            }
            s_part[wave][lane] = make_double2(er, ei);
            __syncthreads();
            if (wave == 0 && i <= j) {
                double tr = 0.0, ti = 0.0;
#pragma unroll
                for (int q = 0; q < kRowWaves; ++q) {
                    tr += s_part[q][lane].x;
                    ti += s_part[q][lane].y;
                }
                ht[i] = make_double2(s_sv[i].x - tr, s_sv[i].y - ti);
                const double2 gij = s_gj[i];
                G[(size_t)j * mm1 + i] = gij;
                if (i < j)
                    G[(size_t)i * mm1 + j] = make_double2(gij.x, -gij.y);
            }
            __syncthreads();
        }
    }
}

// pass 0: w -= V h with h the Hessenberg column, partial |w|^2 into normpart.
// pass 1 (systems with strong cancellation only): h2 = sum of the second
// pass's partial dots, w -= V h2, h += h2, partial |w|^2 into normpart2.
__global__ void __launch_bounds__(kRows) k_orth_update(GmresBatch g, int32_t pass)
{
    __shared__ double red[kRowWaves];
    __shared__ int32_t s_go;
    extern __shared__ double2 s_h[];  // [mmax + 1]
    const int32_t j = *g.iter;
    const int32_t n_items = *g.n_items;
    if (j >= g.mmax)
        return;
    const int mm1 = g.mmax + 1;
    for (int32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 item = g.items[it];
        const int32_t s = item.x, chunk = item.y;
        if (!g.active[s])
            continue;
        const SysDev& S = g.sys[s];
        const int32_t n = S.n;
        __syncthreads();
        if (pass == 1) {
            if (threadIdx.x == 0)
                s_go = strong_cancel(g, S) ? 1 : 0;
            __syncthreads();
            if (!s_go)
                continue;
        }
        double2* ht = g.htot + (size_t)s * mm1;
        for (int i = threadIdx.x; i <= j; i += kRows) {
            if (pass == 0) {
                s_h[i] = ht[i];
            } else {
                const double2 h2 = chunk_sum(g.dp1 + S.off_ch * mm1, S.nch, mm1, i);
                s_h[i] = h2;
                if (chunk == 0)
                    ht[i] = make_double2(ht[i].x + h2.x, ht[i].y + h2.y);
            }
        }
        __syncthreads();
        const int32_t t = chunk * kRows + threadIdx.x;
        const double2* Vs = g.V + S.off_v;
        double2* w = g.w + S.off_n;
        double2 wt = make_double2(0.0, 0.0);
        if (t < n) {
            wt = w[t];
            // groups of 8 basis vectors, the last one predicated, so every
            // group's loads are in flight together; subtraction in index order
            constexpr int U = 8;
            for (int i = 0; i <= j; i += U) {
                double2 v[U];
#pragma unroll
                for (int c = 0; c < U; ++c)
                    v[c] = i + c <= j ? Vs[(size_t)(i + c) * n + t] : make_double2(0.0, 0.0);
#pragma unroll
                for (int c = 0; c < U; ++c) {
                    if (i + c <= j) {
                        const double2 d = cmul(s_h[i + c], v[c]);
                        wt.x -= d.x;
                        wt.y -= d.y;
                    }
                }
            }
            w[t] = wt;
        }
        const double tot = block_sum(wt.x * wt.x + wt.y * wt.y, red);
        if (threadIdx.x == 0)
            (pass == 0 ? g.normpart : g.normpart2)[S.off_ch + chunk] = tot;
    }
}

// Partial dots of the second pass, for the systems with strong cancellation.
__global__ void __launch_bounds__(kRows) k_orth_dots2(GmresBatch g)
{
    __shared__ double2 s_w[kRows];
    __shared__ int32_t s_go;
    const int32_t j = *g.iter;
    const int32_t n_items = *g.n_items;
    if (j >= g.mmax)
        return;
    const int mm1 = g.mmax + 1;
    for (int32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 item = g.items[it];
        const int32_t s = item.x, chunk = item.y;
        if (!g.active[s])
            continue;
        const SysDev& S = g.sys[s];
        __syncthreads();
        if (threadIdx.x == 0)
            s_go = strong_cancel(g, S) ? 1 : 0;
        __syncthreads();
        if (!s_go)
            continue;
        const int32_t n = S.n;
        const int32_t r0 = chunk * kRows;
        const int32_t t = r0 + threadIdx.x;
        s_w[threadIdx.x] = t < n ? g.w[S.off_n + t] : make_double2(0.0, 0.0);
        __syncthreads();
        chunk_dots<false>(g.V + S.off_v, n, j, r0, s_w, nullptr,
                          g.dp1 + (S.off_ch + chunk) * mm1, nullptr);
    }
}

// v_{j+1} = w / |w| on the chunk's rows; Givens rotations and the
// convergence test on chunk 0.
__global__ void __launch_bounds__(kRows) k_orth_finalize(GmresBatch g)
{
    __shared__ double s_hn;
    __shared__ int32_t s_act;
    extern __shared__ double2 s_col[];  // [mmax+2] column | [mmax] sines | [mmax] cosines
    const int32_t j = *g.iter;
    const int32_t n_items = *g.n_items;
    if (j >= g.mmax)
        return;
    const int mm1 = g.mmax + 1;
    double2* s_sn = s_col + (g.mmax + 2);
    double* s_cs = reinterpret_cast<double*>(s_sn + g.mmax);
    for (int32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 item = g.items[it];
        const int32_t s = item.x, chunk = item.y;
        // the first chunk of a system may clear its flag while other chunks
        // run: read it once per workgroup so every thread takes the same path
        __syncthreads();
        if (threadIdx.x == 0)
            s_act = g.active[s];
        __syncthreads();
        if (!s_act)
            continue;
        const SysDev& S = g.sys[s];
        const int32_t n = S.n;
        if (threadIdx.x == 0) {
            const double* np = strong_cancel(g, S) ? g.normpart2 : g.normpart;
            double sacc = 0.0;
            for (int c = 0; c < S.nch; ++c)
                sacc += np[S.off_ch + c];
            s_hn = sqrt(sacc);
        }
        __syncthreads();
        const double hn = s_hn;
        const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
        const int32_t t = chunk * kRows + threadIdx.x;
        if (t < n) {
            const double2 wt = g.w[S.off_n + t];
            const double2 u = make_double2(wt.x * inv, wt.y * inv);
            g.V[S.off_v + (size_t)(j + 1) * n + t] = u;
            if (g.v32)
                g.v32[S.off_n + t] = make_float2(static_cast<float>(S.wscale * u.x),
                                                 static_cast<float>(S.wscale * u.y));
        }
        if (chunk != 0)
            continue;
        // Givens rotations of the new Hessenberg column, staged in LDS:
        // rotation i mixes entries i and i+1, so thread 0 carries the running
        // entry in registers while the other threads load and store.
        double2* H = g.H + ((size_t)s * g.mmax + j) * mm1;  // column j
        double* cs = g.cs + (size_t)s * g.mmax;
        double2* sn = g.sn + (size_t)s * g.mmax;
        double2* gv = g.gv + (size_t)s * mm1;
        const double2* ht = g.htot + (size_t)s * mm1;
        for (int i = threadIdx.x; i <= j; i += kRows) {
            s_col[i] = ht[i];
            if (i < j) {
                s_cs[i] = cs[i];
                s_sn[i] = sn[i];
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
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
            const double res = hypot(gv[j + 1].x, gv[j + 1].y) / g.beta[s];
            g.resid[s] = res;
            g.iters[s] = j + 1;
            if (res <= g.tol || hn == 0.0 || j + 1 >= g.mmax) {
                g.active[s] = 0;
                if (g.host_active)
                    *reinterpret_cast<volatile int32_t*>(g.host_active + s) = 0;
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i <= j + 1; i += kRows)
            H[i] = s_col[i];
    }
}

// j <- j + 1, and the loop's progress for the host.
__global__ void k_gmres_advance(GmresBatch g)
{
    const int32_t j = *g.iter + 1;
    *g.iter = j;
    if (g.host_progress)
        *reinterpret_cast<volatile int32_t*>(g.host_progress) = j;
}

// beta = |b|, v_0 = b / beta; one workgroup per system.
__global__ void __launch_bounds__(kRows) k_gmres_init(GmresBatch g, const double2* __restrict__ b)
{
    __shared__ double red[kRowWaves];
    const int32_t s = blockIdx.x;
    const SysDev& S = g.sys[s];
    const int32_t n = S.n;
    const double2* bs = b + S.off_n;
    double acc = 0.0;
    for (int t = threadIdx.x; t < n; t += kRows) {
        const double2 v = bs[t];
        acc += v.x * v.x + v.y * v.y;
    }
    const double beta = sqrt(block_sum(acc, red));
    const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
    double2* v0 = g.V + S.off_v;
    for (int t = threadIdx.x; t < n; t += kRows) {
        const double2 v = bs[t];
        const double2 u = make_double2(v.x * inv, v.y * inv);
        v0[t] = u;
        if (g.v32)
            g.v32[S.off_n + t] = make_float2(static_cast<float>(S.wscale * u.x),
                                             static_cast<float>(S.wscale * u.y));
    }
    if (threadIdx.x == 0) {
        g.beta[s] = beta;
        g.gv[(size_t)s * (g.mmax + 1)] = make_double2(beta, 0.0);
        g.resid[s] = beta > 0.0 ? 1.0 : 0.0;
        g.iters[s] = 0;
        g.active[s] = beta > 0.0 ? 1 : 0;
        if (g.host_active)
            *reinterpret_cast<volatile int32_t*>(g.host_active + s) = beta > 0.0 ? 1 : 0;
        if (s == 0)
            *g.iter = 0;
    }
}

// y = H^{-1} g on the first `iters` columns (column-oriented back
// substitution: y_t is final once the columns right of t are applied, then
// all rows above t subtract column t in parallel), then x = V y into the
// system's output row.
__global__ void __launch_bounds__(1024) k_gmres_solution(GmresBatch g)
{
    extern __shared__ double2 s_y[];  // [mmax]
    const int32_t s = blockIdx.x;
    const SysDev& S = g.sys[s];
    const int32_t n = S.n;
    const int mm1 = g.mmax + 1;
    const int32_t it = g.iters[s];
    const double2* gv = g.gv + (size_t)s * mm1;
    for (int i = threadIdx.x; i < it; i += blockDim.x)
        s_y[i] = gv[i];
    __syncthreads();
    for (int t = it - 1; t >= 0; --t) {
        const double2* col = g.H + ((size_t)s * g.mmax + t) * mm1;
        const double2 hd = col[t];
        const double den = hd.x * hd.x + hd.y * hd.y;
        const double2 st = s_y[t];
        const double2 yt = make_double2((st.x * hd.x + st.y * hd.y) / den,
                                        (st.y * hd.x - st.x * hd.y) / den);
        __syncthreads();
        if (threadIdx.x == 0)
            s_y[t] = yt;
        for (int i = threadIdx.x; i < t; i += blockDim.x) {
            const double2 d = cmul(col[i], yt);
            s_y[i] = make_double2(s_y[i].x - d.x, s_y[i].y - d.y);
        }
        __syncthreads();
    }
    const double2* Vs = g.V + S.off_v;
    double2* xs = S.out_n;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        double2 acc = make_double2(0.0, 0.0);
        for (int i = 0; i < it; ++i) {
            const double2 d = cmul(s_y[i], Vs[(size_t)i * n + t]);
            acc.x += d.x;
            acc.y += d.y;
        }
        xs[t] = acc;
    }
}

}  // namespace

int32_t gmres_chunks(int32_t n) { return (n + kRows - 1) / kRows; }

hipError_t launch_gmres_init(const GmresBatch& g, const double2* b, hipStream_t s)
{
    if (g.n_sys <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_gmres_init, dim3(g.n_sys), dim3(kRows), 0, s, g, b);
    return hipGetLastError();
}

hipError_t launch_gmres_step(const GmresBatch& g, int32_t grid, hipStream_t s, const ProfSlot& ev)
{
    const size_t lds_h = sizeof(double2) * (size_t)(g.mmax + 1);
    const size_t lds_fin = sizeof(double2) * (size_t)(2 * g.mmax + 2) + sizeof(double) * (size_t)g.mmax;
    // The coefficient and finalisation kernels do a short serial chain per
    // system in the workgroup that owns its first chunk; more workgroups than
    // the streaming kernels run more systems' chains at once (measured on the
    // headline batch: 8x and 4x took the Arnoldi step from 0.68 to 0.62 ms).
    launch_k(k_orth_dots, dim3(grid), dim3(kRows), 0, s, ev.start, nullptr, g);
    hipLaunchKernelGGL(k_orth_coef, dim3(grid * kCoefGridX), dim3(kRows), 2 * lds_h, s, g);
    hipLaunchKernelGGL(k_orth_update, dim3(grid), dim3(kRows), lds_h, s, g, 0);
    hipLaunchKernelGGL(k_orth_dots2, dim3(grid), dim3(kRows), 0, s, g);
    hipLaunchKernelGGL(k_orth_update, dim3(grid), dim3(kRows), lds_h, s, g, 1);
    hipLaunchKernelGGL(k_orth_finalize, dim3(grid * kFinalGridX), dim3(kRows), lds_fin, s, g);
    launch_k(k_gmres_advance, dim3(1), dim3(1), 0, s, nullptr, ev.stop, g);
    return hipGetLastError();
}

hipError_t launch_gmres_solution(const GmresBatch& g, hipStream_t s)
{
    if (g.n_sys <= 0)
        return hipSuccess;
    const size_t lds = sizeof(double2) * (size_t)(g.mmax > 0 ? g.mmax : 1);
    hipLaunchKernelGGL(k_gmres_solution, dim3(g.n_sys), dim3(1024), lds, s, g);
    return hipGetLastError();
}

}  // namespace nat

// FP32 tiled kernel sums of the Monte-Carlo BEM (Section 4.1.1 and 4.2), the
// hot loop of every stage: right-hand side (G), GMRES matvec (dG/dn) and
// surface evaluation (both), for a batch of instances of uneven size.
//
// Schedule (gfx950):
//  * one persistent launch walks a queue of work items; an item is one
//    mode group (up to 8 systems of one instance) x one tile of 256 targets
//    x one split of the sources; a workgroup of 256 threads owns the item's
//    targets, one per lane;
//  * sources stream through LDS in tiles of 64: positions and normals
//    (SoA, coalesced) plus the weighted data of the group's modes; every
//    lane reads the same source at the same time, so LDS reads broadcast;
//  * the pair geometry (d, r^2, 1/r, r, d.n/r^3) is computed once and shared
//    by the group's modes, which all have their own k;
//  * the pair terms are folded as e^{ikr} Z with
//       Z = a/r + (ikr - 1) (d.n / r^3) b,
//    a, b = w/(4 pi)-weighted source data, so one complex multiply-add per
//    pair and mode accumulates both the G and the dG/dn terms;
//  * the phase kappa r (kappa = k/(2 pi)) is fed to the hardware sine and
//    cosine, which take revolutions; instances whose phases can exceed
//    kPhaseRevNoFract revolutions reduce it with fract() first;
//  * each LDS tile's FP32 sum is folded into a (hi, lo) pair with Knuth's
//    TwoSum; the splits are combined the same way by the consumer (the
//    reduction kernel, or the GMRES step for the matvec), in FP64 only for
//    the final epilogue.
// The split count of an instance depends only on its own sizes, so a system
// gets the same rounding alone or inside any batch.
#include "nat_internal.h"

namespace nat {
namespace {

constexpr int kThreads = 256;
constexpr int kTS = 64;  // sources per LDS tile
constexpr int kMB = 8;   // systems per mode group
constexpr double kInv2Pi = 0.15915494309189535;  // 1 / (2 pi)

__device__ __forceinline__ void two_sum_fold(float& hi, float& lo, float t)
{
    const float s = hi + t;
    const float bp = s - hi;
    lo += (hi - (s - bp)) + (t - bp);
    hi = s;
}

// Group holding work item `item`: the last group whose first item <= item.
__device__ __forceinline__ int32_t find_group(const GroupDev* __restrict__ g, int32_t n_groups,
                                              int64_t item)
{
    int32_t lo = 0, hi = n_groups - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (g[mid].item0 <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ float uniform_f(float x)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// The pairs of one LDS tile for the first MB modes of the group (MB is the
// group width rounded up to a power of two; the padded modes carry zero
// source data).  Per (pair, mode):
//   RHS     acc += (1/r) e^{i th} a
//   MATVEC  acc += q e^{i th} (ikr - 1) b,           q = (d.n) / r^3
//           with (ikr - 1) b formed as -b + i r (k b) from the staged k b
//   EVAL    acc += e^{i th} (a/r + q (ikr - 1) b)
// with th = 2 pi kappa r taken by the hardware sine and cosine, which take
// revolutions (reduced by fract() first only for instances whose largest
// kappa r exceeds kPhaseRevNoFract, RED).  PH64: the FP64 phase -- r refined
// from the FP64 positions (s_p64, t64) by one Newton step on the FP32
// distance, r + (r64^2 - r^2) / (2 r), and kappa r reduced to [0, 1)
// revolutions in FP64 before the FP32 sine and cosine.
template <int OP, int MB, bool RED, bool PH64>
__device__ __forceinline__ void tile_pairs(const float (&s_pos)[6][kTS],
                                           const float2 (*s_a)[kMB], const float2 (*s_b)[kMB],
                                           const float2 (*s_kb)[kMB], float tx, float ty,
                                           float tz, float eps2, const float (&kap)[kMB],
                                           const double (*s_p64)[kTS], const double (&t64)[3],
                                           const double (&kap64)[kMB],
                                           float (&ar)[kMB], float (&ai)[kMB])
{
    constexpr bool kA = (OP == OP_RHS || OP == OP_EVAL);
    constexpr bool kB = (OP == OP_MATVEC || OP == OP_EVAL);
    for (int c = 0; c < kTS; ++c) {
        float2 av[MB], bv[MB], cv[MB];
#pragma unroll
        for (int mm = 0; mm < MB; ++mm) {
            if (kA)
                av[mm] = s_a[c][mm];
            if (kB) {
                bv[mm] = s_b[c][mm];
                cv[mm] = s_kb[c][mm];
            }
        }
        const float dx = s_pos[0][c] - tx;
        const float dy = s_pos[1][c] - ty;
        const float dz = s_pos[2][c] - tz;
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        const float rinv = (r2 >= eps2) ? __builtin_amdgcn_rsqf(r2) : 0.0f;
        const float r = r2 * rinv;
        float q = 0.0f;
        if (kB) {
            const float dn = fmaf(dz, s_pos[5][c], fmaf(dy, s_pos[4][c], dx * s_pos[3][c]));
            q = dn * (rinv * rinv) * rinv;
        }
        double rd = 0.0;
        if (PH64) {
            const double ex = s_p64[0][c] - t64[0];
            const double ey = s_p64[1][c] - t64[1];
            const double ez = s_p64[2][c] - t64[2];
            const double rr = static_cast<double>(r);
            rd = fma(fma(ez, ez, fma(ey, ey, ex * ex)) - rr * rr, static_cast<double>(0.5f * rinv), rr);
        }
#pragma unroll
        for (int mm = 0; mm < MB; ++mm) {
            const float ph = PH64 ? static_cast<float>(__builtin_amdgcn_fract(kap64[mm] * rd))
                                  : (RED ? __builtin_amdgcn_fractf(r * kap[mm]) : r * kap[mm]);
            const float sn = __builtin_amdgcn_sinf(ph);
            const float cs = __builtin_amdgcn_cosf(ph);
            if (OP == OP_RHS) {
                const float vr = fmaf(cs, av[mm].x, -(sn * av[mm].y));
                const float vi = fmaf(cs, av[mm].y, sn * av[mm].x);
                ar[mm] = fmaf(rinv, vr, ar[mm]);
                ai[mm] = fmaf(rinv, vi, ai[mm]);
            } else {
                // (ikr - 1) b = -b + i r (k b), k b staged with the tile
                const float ur = fmaf(-r, cv[mm].y, -bv[mm].x);
                const float ui = fmaf(r, cv[mm].x, -bv[mm].y);
                if (OP == OP_MATVEC) {
                    const float vr = fmaf(cs, ur, -(sn * ui));
                    const float vi = fmaf(cs, ui, sn * ur);
                    ar[mm] = fmaf(q, vr, ar[mm]);
                    ai[mm] = fmaf(q, vi, ai[mm]);
                } else {
                    const float zr = fmaf(q, ur, rinv * av[mm].x);
                    const float zi = fmaf(q, ui, rinv * av[mm].y);
                    ar[mm] = fmaf(-sn, zi, fmaf(cs, zr, ar[mm]));
                    ai[mm] = fmaf(sn, zr, fmaf(cs, zi, ai[mm]));
                }
            }
        }
    }
}

// The tile's pairs for the group width rounded up to 1, 2, 4 or 8 modes.
template <int OP, bool RED, bool PH64>
__device__ __forceinline__ void tile_width(int32_t nm, const float (&s_pos)[6][kTS],
                                           const float2 (*s_a)[kMB], const float2 (*s_b)[kMB],
                                           const float2 (*s_kb)[kMB], float tx, float ty, float tz,
                                           float eps2, const float (&kap)[kMB],
                                           const double (*s_p64)[kTS], const double (&t64)[3],
                                           const double (&kap64)[kMB], float (&ar)[kMB], float (&ai)[kMB])
{
    if (nm > 4)
        tile_pairs<OP, 8, RED, PH64>(s_pos, s_a, s_b, s_kb, tx, ty, tz, eps2, kap, s_p64, t64, kap64, ar, ai);
    else if (nm > 2)
        tile_pairs<OP, 4, RED, PH64>(s_pos, s_a, s_b, s_kb, tx, ty, tz, eps2, kap, s_p64, t64, kap64, ar, ai);
    else if (nm > 1)
        tile_pairs<OP, 2, RED, PH64>(s_pos, s_a, s_b, s_kb, tx, ty, tz, eps2, kap, s_p64, t64, kap64, ar, ai);
    else
        tile_pairs<OP, 1, RED, PH64>(s_pos, s_a, s_b, s_kb, tx, ty, tz, eps2, kap, s_p64, t64, kap64, ar, ai);
}

template <int OP, bool PH64>
__global__ void __launch_bounds__(kThreads) k_sum32(const Sum32Batch p)
{
    constexpr bool kA = (OP == OP_RHS || OP == OP_EVAL);
    constexpr bool kB = (OP == OP_MATVEC || OP == OP_EVAL);
    __shared__ float s_pos[6][kTS];
    __shared__ double s_pos64[PH64 ? 3 : 1][kTS];
    __shared__ float2 s_a[kA ? kTS : 1][kMB];
    __shared__ float2 s_b[kB ? kTS : 1][kMB];
    __shared__ float2 s_kb[kB ? kTS : 1][kMB];

    const int32_t tid = threadIdx.x;
    const int64_t n_items = *p.n_items;
    const int32_t n_groups = *p.n_groups;

    for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        const GroupDev& G = p.groups[find_group(p.groups, n_groups, item)];
        const int32_t nm = __builtin_amdgcn_readfirstlane(G.nm);
        const int32_t inst = __builtin_amdgcn_readfirstlane(G.inst);
        const int32_t nsplit = __builtin_amdgcn_readfirstlane(G.nsplit);
        const int64_t local = item - G.item0;
        const InstDev& I = p.inst[inst];
        const int32_t tile = static_cast<int32_t>(local / nsplit);
        const int32_t split = static_cast<int32_t>(local % nsplit);
        const int32_t NS = I.n;
        const int32_t NT = (OP == OP_EVAL) ? I.q : I.n;
        const float* t32 = (OP == OP_EVAL) ? I.q32 : I.s32;
        const int32_t per_split = (OP == OP_EVAL) ? I.per_split_b : I.per_split_a;

        int32_t sys[kMB];
        float kap[kMB], kk[kMB];
        double kap64[kMB];
        bool any = false;
#pragma unroll
        for (int mm = 0; mm < kMB; ++mm) {
            const int32_t sl = mm < nm ? mm : nm - 1;
            sys[mm] = __builtin_amdgcn_readfirstlane(G.sys[sl]);
            const SysDev& S = p.sys[sys[mm]];
            any |= mm < nm && (!p.active || p.active[sys[mm]]);
            kap[mm] = uniform_f(S.kappa32);
            kk[mm] = uniform_f(S.k32);
            kap64[mm] = PH64 ? S.k * kInv2Pi : 0.0;
        }
        if (!any)
            continue;  // uniform across the workgroup

        const int32_t i = tile * kThreads + tid;
        const int32_t ic = i < NT ? i : NT - 1;
        // a wave whose 64 targets all lie past the end of a ragged last tile
        // only helps stage the LDS tiles
        const bool wave_live =
            __builtin_amdgcn_readfirstlane(tile * kThreads + (tid & ~63)) < NT;
        const float tx = t32[ic], ty = t32[NT + ic], tz = t32[2 * NT + ic];
        double t64[3] = {0.0, 0.0, 0.0};
        if (PH64) {
            const double* tp = (OP == OP_EVAL) ? I.q64 : I.s64;
            t64[0] = tp[ic];
            t64[1] = tp[NT + ic];
            t64[2] = tp[2 * NT + ic];
        }
        const float eps2 = I.eps2;
        const bool red = __builtin_amdgcn_readfirstlane(I.phase_fract) != 0;

        float hr[kMB], hi_[kMB], lr[kMB], li[kMB];
#pragma unroll
        for (int mm = 0; mm < kMB; ++mm)
            hr[mm] = hi_[mm] = lr[mm] = li[mm] = 0.0f;

        const int32_t j_begin = split * per_split;
        const int32_t j_end = min(NS, j_begin + per_split);
        for (int32_t j0 = j_begin; j0 < j_end; j0 += kTS) {
            const int32_t cnt = min(kTS, j_end - j0);
            __syncthreads();
            for (int e = tid; e < 6 * kTS; e += kThreads) {
                const int row = e / kTS, c = e % kTS;
                float v = 0.0f;
                if (c < cnt)
                    v = row < 3 ? I.s32[(size_t)row * NS + j0 + c]
                                : I.sn32[(size_t)(row - 3) * NS + j0 + c];
                s_pos[row][c] = v;
            }
            if (PH64) {
                for (int e = tid; e < 3 * kTS; e += kThreads) {
                    const int row = e / kTS, c = e % kTS;
                    s_pos64[row][c] = c < cnt ? I.s64[(size_t)row * NS + j0 + c] : 0.0;
                }
            }
            for (int e = tid; e < kMB * kTS; e += kThreads) {
                const int mm = e / kTS, c = e % kTS;
                const bool ok = c < cnt && mm < nm;
                const int64_t o = p.sys[sys[mm]].off_n + j0 + c;
                if (kA)
                    s_a[c][mm] = ok ? p.a32[o] : make_float2(0.0f, 0.0f);
                if (kB) {
                    const float2 b = ok ? p.b32[o] : make_float2(0.0f, 0.0f);
                    s_b[c][mm] = b;
                    s_kb[c][mm] = make_float2(kk[mm] * b.x, kk[mm] * b.y);
                }
            }
            __syncthreads();

            float ar[kMB], ai[kMB];
#pragma unroll
            for (int mm = 0; mm < kMB; ++mm)
                ar[mm] = ai[mm] = 0.0f;
            if (!wave_live)
                ;
            else if (PH64)
                tile_width<OP, false, true>(nm, s_pos, s_a, s_b, s_kb, tx, ty, tz, eps2, kap, s_pos64,
                                            t64, kap64, ar, ai);
            else if (red)
                tile_width<OP, true, false>(nm, s_pos, s_a, s_b, s_kb, tx, ty, tz, eps2, kap, s_pos64,
                                            t64, kap64, ar, ai);
            else
                tile_width<OP, false, false>(nm, s_pos, s_a, s_b, s_kb, tx, ty, tz, eps2, kap, s_pos64,
                                             t64, kap64, ar, ai);
#pragma unroll
            for (int mm = 0; mm < kMB; ++mm) {
                two_sum_fold(hr[mm], lr[mm], ar[mm]);
                two_sum_fold(hi_[mm], li[mm], ai[mm]);
            }
        }

        if (i < NT) {
#pragma unroll
            for (int mm = 0; mm < kMB; ++mm) {
                if (mm < nm) {
                    const SysDev& S = p.sys[sys[mm]];
                    const int64_t off = (OP == OP_EVAL) ? S.off_pb : S.off_pa;
                    p.partial[off + (int64_t)split * NT + i] =
                        make_float4(hr[mm], hi_[mm], lr[mm], li[mm]);
                }
            }
        }
    }
}

// Combine the splits of one system's targets (TwoSum in FP32) and apply the
// epilogue of the operation in FP64:
//   RHS   b_i = -acc_i - d g_i    (d: the disk factor, eps/2 or its closed form)
//   EVAL  p_q = (1/c_q) (acc_q - d g_q), 1/c_q = 2 unless the instance
//         carries per-query factors
template <int OP>
__global__ void __launch_bounds__(256)
k_reduce32(const Sum32Batch p, const double2* __restrict__ g_tgt, double2* __restrict__ out_n)
{
    const int32_t s = blockIdx.y;
    const SysDev S = p.sys[s];
    const int32_t NT = (OP == OP_EVAL) ? S.q : S.n;
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NT)
        return;
    const int32_t nsplit = (OP == OP_EVAL) ? S.nsplit_b : S.nsplit_a;
    const int64_t off = (OP == OP_EVAL) ? S.off_pb : S.off_pa;
    float hr = 0.0f, hi = 0.0f, lr = 0.0f, li = 0.0f;
    const float4* pp = p.partial + off + i;
    for (int32_t sp0 = 0; sp0 < nsplit; sp0 += 8) {
        // issue the group's loads together, fold in split order
        float4 v[8];
#pragma unroll
        for (int c = 0; c < 8; ++c)
            v[c] = sp0 + c < nsplit ? pp[(int64_t)(sp0 + c) * NT] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if (sp0 + c < nsplit) {
                two_sum_fold(hr, lr, v[c].x);
                two_sum_fold(hi, li, v[c].y);
                lr += v[c].z;
                li += v[c].w;
            }
        }
    }
    const double accr = static_cast<double>(hr) + static_cast<double>(lr);
    const double acci = static_cast<double>(hi) + static_cast<double>(li);
    if (OP == OP_RHS) {
        const double2 g = g_tgt[S.off_n + i];
        const double dr = S.disk.x * g.x - S.disk.y * g.y, di = S.disk.x * g.y + S.disk.y * g.x;
        out_n[S.off_n + i] = make_double2(-accr - dr, -acci - di);
    } else {
        const double2 g = g_tgt[S.off_q + i];
        const double* qf = p.inst[S.inst].qfac;
        const double f = qf ? qf[i] : 2.0;
        const double dr = S.disk.x * g.x - S.disk.y * g.y, di = S.disk.x * g.y + S.disk.y * g.x;
        S.out_q[i] = make_double2(f * (accr - dr), f * (acci - di));
    }
}

// Assembled form of the Stage-A operator, FP32 complex [n][n] at off_k,
// stored source-major (entry (i, j) at j n + i) so that consecutive targets
// are consecutive in memory: K_ij = q e^{i th} (ikr - 1) with
// q = (d.n_j)/r^3, d = y_j - y_i, the matvec's pair term formed by the same
// operations without the source data; 0 inside the disk (the diagonal
// included).  One workgroup per source column, a thread per target.
__global__ void __launch_bounds__(256)
k_assemble32(const InstDev* __restrict__ inst, const SysDev* __restrict__ sys,
             const int32_t* __restrict__ list, float2* __restrict__ kmat)
{
    const SysDev& S = sys[list[blockIdx.y]];
    const int32_t n = S.n;
    const InstDev& I = inst[S.inst];
    const float* sp = I.s32;
    const float* sn = I.sn32;
    const float eps2 = I.eps2, kap = S.kappa32, kk = S.k32;
    for (int32_t j = blockIdx.x; j < n; j += gridDim.x) {
        const float sx = sp[j], sy = sp[n + j], sz = sp[2 * n + j];
        const float nx = sn[j], ny = sn[n + j], nz = sn[2 * n + j];
        float2* col = kmat + S.off_k + (size_t)j * n;
        for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
            const float dx = sx - sp[i];
            const float dy = sy - sp[n + i];
            const float dz = sz - sp[2 * n + i];
            const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            float2 v = make_float2(0.0f, 0.0f);
            if (r2 >= eps2) {
                const float rinv = __builtin_amdgcn_rsqf(r2);
                const float r = r2 * rinv;
                const float dn = fmaf(dz, nz, fmaf(dy, ny, dx * nx));
                const float q = dn * (rinv * rinv) * rinv;
                const float ph = __builtin_amdgcn_fractf(r * kap);
                const float sv = __builtin_amdgcn_sinf(ph);
                const float cv = __builtin_amdgcn_cosf(ph);
                const float kr = r * kk;
                v = make_float2(-q * fmaf(kr, sv, cv), q * fmaf(kr, cv, -sv));
            }
            col[i] = v;
        }
    }
}

// GMRES matvec from the assembled operators: a thread per target row of a
// (system, 256-row chunk) item walks the source columns, so every load of
// the operator is a coalesced run along a column and the source value is
// the same for the whole wave; products and sums in FP64, written as the
// single (hi, lo) split partial the Arnoldi step folds.
__global__ void __launch_bounds__(256)
k_kmatvec32(const KmvBatch p)
{
    const int32_t n_items = *p.n_items;
    for (int32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const int2 item = p.items[it];
        const int32_t s = item.x;
        if (p.active && !p.active[s])
            continue;
        const SysDev& S = p.sys[s];
        if (S.off_k < 0)
            continue;
        const int32_t n = S.n;
        const int32_t i = item.y * 256 + static_cast<int32_t>(threadIdx.x);
        const bool ok = i < n;
        const float2* col = p.kmat + S.off_k + (ok ? i : 0);
        const float2* b = p.b32 + S.off_n;
        double ar = 0.0, ai = 0.0;
        int32_t j = 0;
        for (; j + 8 <= n; j += 8) {
            float2 kv[8], bv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                kv[u] = col[(size_t)(j + u) * n];
                bv[u] = b[j + u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                ar = fma((double)kv[u].x, (double)bv[u].x, ar);
                ar = fma(-(double)kv[u].y, (double)bv[u].y, ar);
                ai = fma((double)kv[u].x, (double)bv[u].y, ai);
                ai = fma((double)kv[u].y, (double)bv[u].x, ai);
            }
        }
        for (; j < n; ++j) {
            const float2 kv = col[(size_t)j * n], bv = b[j];
            ar = fma((double)kv.x, (double)bv.x, ar);
            ar = fma(-(double)kv.y, (double)bv.y, ar);
            ai = fma((double)kv.x, (double)bv.y, ai);
            ai = fma((double)kv.y, (double)bv.x, ai);
        }
        if (ok) {
            const float hr = static_cast<float>(ar), hi = static_cast<float>(ai);
            p.partial[S.off_pa + i] = make_float4(hr, hi, static_cast<float>(ar - (double)hr),
                                                  static_cast<float>(ai - (double)hi));
        }
    }
}

// dst[off_n + j] = float2(sign * w/(4 pi) * src[off_n + j]) for every system.
__global__ void __launch_bounds__(256)
k_weight32(const SysDev* __restrict__ sys, const double2* __restrict__ src, double sign,
           float2* __restrict__ dst)
{
    const SysDev& S = sys[blockIdx.y];
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= S.n)
        return;
    const double sc = sign * S.wscale;
    const double2 v = src[S.off_n + j];
    dst[S.off_n + j] = make_float2(static_cast<float>(sc * v.x), static_cast<float>(sc * v.y));
}

}  // namespace

void split_rule(int32_t n_targets, int32_t n_sources, int32_t want_items, int32_t* nsplit,
                int32_t* per_split)
{
    // enough splits that one mode group spans >= want_items work items,
    // never more than one split per LDS tile of sources
    const int32_t tiles = (n_targets + kThreads - 1) / kThreads;
    const int32_t src_tiles = (n_sources + kTS - 1) / kTS;
    int32_t want = (want_items + tiles - 1) / tiles;
    if (want < 1)
        want = 1;
    if (want > src_tiles)
        want = src_tiles;
    const int32_t tiles_per_split = (src_tiles + want - 1) / want;
    *per_split = tiles_per_split * kTS;
    *nsplit = (n_sources + *per_split - 1) / *per_split;
}

int32_t target_tiles(int32_t n_targets) { return (n_targets + kThreads - 1) / kThreads; }

hipError_t launch_sum32_batch(int32_t op, const Sum32Batch& p, int32_t grid, hipStream_t s,
                              const ProfSlot& ev)
{
    if (grid <= 0)
        return hipSuccess;
    const bool ph64 = p.phase64 != 0;
    switch (op) {
    case OP_RHS:
        if (ph64)
            launch_k(k_sum32<OP_RHS, true>, dim3(grid), dim3(kThreads), 0, s, ev.start, ev.stop, p);
        else
            launch_k(k_sum32<OP_RHS, false>, dim3(grid), dim3(kThreads), 0, s, ev.start, ev.stop, p);
        break;
    case OP_MATVEC:
        if (ph64)
            launch_k(k_sum32<OP_MATVEC, true>, dim3(grid), dim3(kThreads), 0, s, ev.start, ev.stop, p);
        else
            launch_k(k_sum32<OP_MATVEC, false>, dim3(grid), dim3(kThreads), 0, s, ev.start, ev.stop, p);
        break;
    default:
        if (ph64)
            launch_k(k_sum32<OP_EVAL, true>, dim3(grid), dim3(kThreads), 0, s, ev.start, ev.stop, p);
        else
            launch_k(k_sum32<OP_EVAL, false>, dim3(grid), dim3(kThreads), 0, s, ev.start, ev.stop, p);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_kmatvec32(const KmvBatch& p, int32_t grid, hipStream_t s, const ProfSlot& ev)
{
    if (grid <= 0)
        return hipSuccess;
    launch_k(k_kmatvec32, dim3(grid), dim3(256), 0, s, ev.start, ev.stop, p);
    return hipGetLastError();
}

hipError_t launch_assemble32(const InstDev* inst, const SysDev* sys, const int32_t* list,
                             int32_t n_list, int32_t max_n, float2* kmat, hipStream_t s)
{
    if (n_list <= 0 || max_n <= 0)
        return hipSuccess;
    const unsigned rows = static_cast<unsigned>(max_n < 2048 ? max_n : 2048);
    hipLaunchKernelGGL(k_assemble32, dim3(rows, static_cast<unsigned>(n_list)), dim3(256), 0, s,
                       inst, sys, list, kmat);
    return hipGetLastError();
}

hipError_t launch_reduce32_batch(int32_t op, const Sum32Batch& p, int32_t n_sys, int32_t max_targets,
                                 const double2* g_tgt, double2* out_n, hipStream_t s,
                                 const ProfSlot& ev)
{
    if (n_sys <= 0 || max_targets <= 0)
        return hipSuccess;
    dim3 grid(static_cast<unsigned>((max_targets + 255) / 256), static_cast<unsigned>(n_sys));
    if (op == OP_RHS)
        launch_k(k_reduce32<OP_RHS>, grid, dim3(256), 0, s, ev.start, ev.stop, p, g_tgt, out_n);
    else
        launch_k(k_reduce32<OP_EVAL>, grid, dim3(256), 0, s, ev.start, ev.stop, p, g_tgt, out_n);
    return hipGetLastError();
}

hipError_t launch_weight32_batch(const SysDev* sys, int32_t n_sys, int32_t max_n,
                                 const double2* src, double sign, float2* dst, hipStream_t s)
{
    if (n_sys <= 0 || max_n <= 0)
        return hipSuccess;
    dim3 grid(static_cast<unsigned>((max_n + 255) / 256), static_cast<unsigned>(n_sys));
    hipLaunchKernelGGL(k_weight32, grid, dim3(256), 0, s, sys, src, sign, dst);
    return hipGetLastError();
}

}  // namespace nat

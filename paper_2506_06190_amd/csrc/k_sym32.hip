// Symmetric form of the GMRES matvec of the FP32 Monte-Carlo sums
// (eq. bem_linear_system): e^{ikr} and r are the same for the pair (i, j) and
// the pair (j, i), so each unordered sample pair is evaluated once and feeds
// both targets:
//   y_i += q_ij e^{ikr} (ikr - 1) b_j,   q_ij = (d . n_j) / r^3,  d = y_j - y_i
//   y_j += q_ji e^{ikr} (ikr - 1) b_i,   q_ji = -(d . n_i) / r^3
// which halves the sine and cosine work that dominates the ordered form.
//
// A work item is one wave: a mode group (up to 8 systems of one instance)
// and a pair (P, Q), P <= Q, of 64-sample sub-tiles.  Lane l owns target
// 64 P + l (its position, normal and weighted data stay in registers); the
// source sub-tile Q is staged in the wave's own LDS slice.  At step c lane l
// meets source (l + c) mod 64: its row sum stays in the lane, and the column
// sum of the source it meets travels with that source, one lane down before
// every step (a DPP wave rotate feeding the accumulate), so no cross-lane
// reduction is needed; one shuffle at the end puts the column sum of source
// l in lane l.  A diagonal item (P == Q) takes steps 1..32 only: step c and
// step 64 - c meet the same unordered pairs, and at step 32 both lanes of
// each pair add their own row term.  The waves of a workgroup take items
// independently (no workgroup barrier), so the diagonal items, half as
// long, leave no wave idle.
//
// Each target receives exactly one partial sum per sub-tile of its instance
// (from the item that pairs its own sub-tile with that one): a plain FP32
// sum of at most 64 terms, written as a float2 to slot = that sub-tile; the
// Arnoldi step folds the slots in order with compensation.
// The work of a system therefore depends only on its own sizes, so it gets
// the same rounding alone or inside any batch.
#include "nat_internal.h"

namespace nat {
namespace {

constexpr int kMB = 8;  // systems per mode group
constexpr int kWaves = 4;
constexpr double kInv2Pi = 0.15915494309189535;  // 1 / (2 pi)

__device__ __forceinline__ float uniform_f(float x)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// Last group whose first item (in the prefix `which` = 0 diagonal, 1 off)
// is <= item.
__device__ __forceinline__ int32_t find_sym_group(const SymGroupDev* __restrict__ g, int32_t n_groups,
                                                  int64_t item, int which)
{
    int32_t lo = 0, hi = n_groups - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        const int64_t v = which ? g[mid].o0 : g[mid].d0;
        if (v <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Value of lane l + 1 (mod 64) in lane l (one DPP wave_rol:1 move).
__device__ __forceinline__ float rot_from_next(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x134, 0xf, 0xf, true));
}

// FP64 positions of the item's targets and staged sources, for the FP64
// phase (PH64): r refined from them by one Newton step on the FP32
// distance, r + (r64^2 - r^2) / (2 r), and k r / (2 pi) reduced to [0, 1)
// revolutions in FP64 before the FP32 sine and cosine.
struct Pos64 {
    const double (*src)[64];   // LDS [3][64], the staged sub-tile
    double tx, ty, tz;         // the lane's target
};

// The steps c0 <= c < c1 of one item for the first MB modes of the group.
// BOTH: the step feeds the column sums too; RED: reduce the phase with
// fract() first; PH64: form and reduce the phase in FP64 (then RED is
// moot).  Both directions share f = e^{ikr} (ikr - 1):
//   row:    acc_i += q_ij f b_j        column: col_j += q_ji f b_i
// The column sum of the source a lane meets travels with that source: at
// step c lane l meets source (l + c) mod 64, so the sums move one lane down
// before each step's term is added; after the last step lane l holds the
// sum of source (l + c1 - 1) mod 64.
template <int MB, bool RED, bool PH64>
__device__ __forceinline__ void sym_steps(int c0, int c1, bool both, const float (&sp)[6][64],
                                          const float2 (&sd)[kMB][64], float tx, float ty, float tz,
                                          float tnx, float tny, float tnz, const float2 (&bi)[MB],
                                          float eps2, const float (&kap)[kMB], const float (&kk)[kMB],
                                          const Pos64& p64, const double (&kap64)[kMB],
                                          float (&ar)[MB], float (&ai)[MB], float (&cr)[MB], float (&ci)[MB])
{
    const int lane = threadIdx.x & 63;
    for (int c = c0; c < c1; ++c) {
        const int jl = (lane + c) & 63;
        const float dx = sp[0][jl] - tx;
        const float dy = sp[1][jl] - ty;
        const float dz = sp[2][jl] - tz;
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        const float rinv = (r2 >= eps2) ? __builtin_amdgcn_rsqf(r2) : 0.0f;
        const float r = r2 * rinv;
        const float r3 = (rinv * rinv) * rinv;
        const float qij = fmaf(dz, sp[5][jl], fmaf(dy, sp[4][jl], dx * sp[3][jl])) * r3;
        const float qji = -(fmaf(dz, tnz, fmaf(dy, tny, dx * tnx)) * r3);
        double rd = 0.0;
        if (PH64) {
            const double ex = p64.src[0][jl] - p64.tx;
            const double ey = p64.src[1][jl] - p64.ty;
            const double ez = p64.src[2][jl] - p64.tz;
            const double rr = static_cast<double>(r);
            rd = fma(fma(ez, ez, fma(ey, ey, ex * ex)) - rr * rr, static_cast<double>(0.5f * rinv), rr);
        }
#pragma unroll
        for (int mm = 0; mm < MB; ++mm) {
            const float2 bj = sd[mm][jl];
            const float ph = PH64 ? static_cast<float>(__builtin_amdgcn_fract(kap64[mm] * rd))
                                  : (RED ? __builtin_amdgcn_fractf(r * kap[mm]) : r * kap[mm]);
            const float sn = __builtin_amdgcn_sinf(ph);
            const float cs = __builtin_amdgcn_cosf(ph);
            const float rk = r * kk[mm];
            // f = (cs + i sn)(-1 + i k r)
            const float fr = fmaf(-sn, rk, -cs);
            const float fi = fmaf(cs, rk, -sn);
            const float vr = fmaf(fr, bj.x, -(fi * bj.y));
            const float vi = fmaf(fr, bj.y, fi * bj.x);
            ar[mm] = fmaf(qij, vr, ar[mm]);
            ai[mm] = fmaf(qij, vi, ai[mm]);
            if (both) {
                const float xr = fmaf(fr, bi[mm].x, -(fi * bi[mm].y));
                const float xi = fmaf(fr, bi[mm].y, fi * bi[mm].x);
                cr[mm] = __fadd_rn(rot_from_next(cr[mm]), __fmul_rn(qji, xr));
                ci[mm] = __fadd_rn(rot_from_next(ci[mm]), __fmul_rn(qji, xi));
            }
        }
    }
}

template <int MB, bool RED, bool PH64>
__device__ __forceinline__ void sym_item(const SymBatch& p, const InstDev& I, const int32_t (&sys)[kMB],
                                         int32_t nm, const float (&kap)[kMB], const float (&kk)[kMB],
                                         const double (&kap64)[kMB], int32_t P, int32_t Q,
                                         const float (&sp)[6][64], const float2 (&sd)[kMB][64],
                                         const double (*sp64)[64])
{
    const int lane = threadIdx.x & 63;
    const int32_t n = I.n;
    const int32_t i = 64 * P + lane;
    const bool oki = i < n;
    const int32_t ic = oki ? i : 0;
    const float tx = oki ? I.s32[ic] : 0.0f;
    const float ty = oki ? I.s32[n + ic] : 0.0f;
    const float tz = oki ? I.s32[2 * n + ic] : 0.0f;
    const float tnx = oki ? I.sn32[ic] : 0.0f;
    const float tny = oki ? I.sn32[n + ic] : 0.0f;
    const float tnz = oki ? I.sn32[2 * n + ic] : 0.0f;
    Pos64 p64{sp64, 0.0, 0.0, 0.0};
    if (PH64) {
        p64.tx = I.s64[ic];
        p64.ty = I.s64[n + ic];
        p64.tz = I.s64[2 * n + ic];
    }
    float2 bi[MB];
    float ar[MB], ai[MB], cr[MB], ci[MB];
#pragma unroll
    for (int mm = 0; mm < MB; ++mm) {
        bi[mm] = (oki && mm < nm) ? p.b32[p.sys[sys[mm]].off_n + i] : make_float2(0.0f, 0.0f);
        ar[mm] = ai[mm] = cr[mm] = ci[mm] = 0.0f;
    }
    const float eps2 = I.eps2;
    // diagonal pair: step c and step 64 - c meet the same unordered pairs,
    // and at step 32 each lane of a pair adds its own row term
    const int32_t c_last = (P == Q) ? 31 : 63;
    if (P == Q) {
        sym_steps<MB, RED, PH64>(1, 32, true, sp, sd, tx, ty, tz, tnx, tny, tnz, bi, eps2, kap, kk, p64,
                                 kap64, ar, ai, cr, ci);
        sym_steps<MB, RED, PH64>(32, 33, false, sp, sd, tx, ty, tz, tnx, tny, tnz, bi, eps2, kap, kk, p64,
                                 kap64, ar, ai, cr, ci);
    } else {
        sym_steps<MB, RED, PH64>(0, 64, true, sp, sd, tx, ty, tz, tnx, tny, tnz, bi, eps2, kap, kk, p64,
                                 kap64, ar, ai, cr, ci);
    }
    // the column sum of source l sits in lane l - c_last
    const int src_lane = (lane - c_last) & 63;
    const int32_t j = 64 * Q + lane;
#pragma unroll
    for (int mm = 0; mm < MB; ++mm) {
        const float colr = __shfl(cr[mm], src_lane, 64);
        const float coli = __shfl(ci[mm], src_lane, 64);
        if (mm < nm) {
            float2* part = reinterpret_cast<float2*>(p.partial) + 2 * p.sys[sys[mm]].off_pa;
            if (P == Q) {
                if (oki)
                    part[(int64_t)P * n + i] = make_float2(ar[mm] + colr, ai[mm] + coli);
            } else {
                if (oki)
                    part[(int64_t)Q * n + i] = make_float2(ar[mm], ai[mm]);
                if (j < n)
                    part[(int64_t)P * n + j] = make_float2(colr, coli);
            }
        }
    }
}

// One item with the group width as a compile-time constant, so no padded
// mode costs work.
template <bool RED, bool PH64>
__device__ __forceinline__ void dispatch_item(const SymBatch& p, const InstDev& I, const int32_t (&sys)[kMB],
                                              int32_t nm, const float (&kap)[kMB], const float (&kk)[kMB],
                                              const double (&kap64)[kMB], int32_t P, int32_t Q,
                                              const float (&sp)[6][64], const float2 (&sd)[kMB][64],
                                              const double (*sp64)[64])
{
    switch (nm) {
    case 8: sym_item<8, RED, PH64>(p, I, sys, nm, kap, kk, kap64, P, Q, sp, sd, sp64); break;
    case 7: sym_item<7, RED, PH64>(p, I, sys, nm, kap, kk, kap64, P, Q, sp, sd, sp64); break;
    case 6: sym_item<6, RED, PH64>(p, I, sys, nm, kap, kk, kap64, P, Q, sp, sd, sp64); break;
    case 5: sym_item<5, RED, PH64>(p, I, sys, nm, kap, kk, kap64, P, Q, sp, sd, sp64); break;
    case 4: sym_item<4, RED, PH64>(p, I, sys, nm, kap, kk, kap64, P, Q, sp, sd, sp64); break;
    case 3: sym_item<3, RED, PH64>(p, I, sys, nm, kap, kk, kap64, P, Q, sp, sd, sp64); break;
    case 2: sym_item<2, RED, PH64>(p, I, sys, nm, kap, kk, kap64, P, Q, sp, sd, sp64); break;
    default: sym_item<1, RED, PH64>(p, I, sys, nm, kap, kk, kap64, P, Q, sp, sd, sp64); break;
    }
}

// 5 waves per SIMD (at most 102 VGPRs): measured faster than 4 or 6 on the
// batched workload, with no extra instructions in the step loop.  PH64:
// the FP64-phase form, which also stages the sources' FP64 positions.
template <bool PH64>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PH64 ? 4 : 5, 5)))
k_sym32(const SymBatch p)
{
    __shared__ float s_pos[kWaves][6][64];
    __shared__ float2 s_dat[kWaves][kMB][64];
    __shared__ double s_pos64[PH64 ? kWaves : 1][3][64];
    const int32_t tid = threadIdx.x, lane = tid & 63;
    const int32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t n_diag = p.n_items[0];
    const int64_t n_total = n_diag + p.n_items[1];
    const int32_t n_groups = *p.n_groups;

    for (int64_t item = (int64_t)blockIdx.x * kWaves + wave; item < n_total;
         item += (int64_t)gridDim.x * kWaves) {
        int32_t gi = 0, P = 0, Q = 0;
        {
            if (item < n_diag) {
                gi = find_sym_group(p.groups, n_groups, item, 0);
                P = Q = static_cast<int32_t>(item - p.groups[gi].d0);
            } else {
                const int64_t k = item - n_diag;
                gi = find_sym_group(p.groups, n_groups, k, 1);
                const int64_t local = k - p.groups[gi].o0;
                // (P, Q), P < Q, from local = Q (Q - 1) / 2 + P
                int64_t q = static_cast<int64_t>((1.0 + sqrt(1.0 + 8.0 * (double)local)) * 0.5);
                while (q * (q - 1) / 2 > local)
                    --q;
                while ((q + 1) * q / 2 <= local)
                    ++q;
                Q = static_cast<int32_t>(q);
                P = static_cast<int32_t>(local - q * (q - 1) / 2);
            }
            gi = __builtin_amdgcn_readfirstlane(gi);
            P = __builtin_amdgcn_readfirstlane(P);
            Q = __builtin_amdgcn_readfirstlane(Q);
        }
        const SymGroupDev& G = p.groups[gi];
        const int32_t nm = __builtin_amdgcn_readfirstlane(G.nm);
        const InstDev& I = p.inst[__builtin_amdgcn_readfirstlane(G.inst)];
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
            continue;  // uniform across the wave
        const int32_t n = I.n;
        // stage source sub-tile Q (zeros past the end) in the wave's own LDS
        // slice; the wave's LDS accesses complete in order, so only the
        // compiler has to be kept from moving them across the item boundary
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        {
            const int32_t j = 64 * Q + lane;
            const bool ok = j < n;
            s_pos[wave][0][lane] = ok ? I.s32[j] : 0.0f;
            s_pos[wave][1][lane] = ok ? I.s32[n + j] : 0.0f;
            s_pos[wave][2][lane] = ok ? I.s32[2 * n + j] : 0.0f;
            s_pos[wave][3][lane] = ok ? I.sn32[j] : 0.0f;
            s_pos[wave][4][lane] = ok ? I.sn32[n + j] : 0.0f;
            s_pos[wave][5][lane] = ok ? I.sn32[2 * n + j] : 0.0f;
            if (PH64) {
                s_pos64[wave][0][lane] = ok ? I.s64[j] : 0.0;
                s_pos64[wave][1][lane] = ok ? I.s64[n + j] : 0.0;
                s_pos64[wave][2][lane] = ok ? I.s64[2 * n + j] : 0.0;
            }
#pragma unroll
            for (int mm = 0; mm < kMB; ++mm) {
                const float2 b = (ok && mm < nm) ? p.b32[p.sys[sys[mm]].off_n + j] : make_float2(0.0f, 0.0f);
                s_dat[wave][mm][lane] = b;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        {
            const bool red = __builtin_amdgcn_readfirstlane(I.phase_fract) != 0;
            const double (*sp64)[64] = s_pos64[PH64 ? wave : 0];
            if (PH64)
                dispatch_item<false, true>(p, I, sys, nm, kap, kk, kap64, P, Q, s_pos[wave], s_dat[wave],
                                           sp64);
            else if (red)
                dispatch_item<true, false>(p, I, sys, nm, kap, kk, kap64, P, Q, s_pos[wave], s_dat[wave],
                                           sp64);
            else
                dispatch_item<false, false>(p, I, sys, nm, kap, kk, kap64, P, Q, s_pos[wave], s_dat[wave],
                                            sp64);
        }
    }
}

}  // namespace

hipError_t launch_sym32(const SymBatch& p, int32_t grid, hipStream_t s, const ProfSlot& ev)
{
    if (grid <= 0)
        return hipSuccess;
    if (p.phase64)
        launch_k(k_sym32<true>, dim3(grid), dim3(256), 0, s, ev.start, ev.stop, p);
    else
        launch_k(k_sym32<false>, dim3(grid), dim3(256), 0, s, ev.start, ev.stop, p);
    return hipGetLastError();
}

}  // namespace nat

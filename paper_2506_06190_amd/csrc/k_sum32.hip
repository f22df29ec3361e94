// FP32 tiled kernel sums of the Monte-Carlo BEM (Section 4.1.1 and 4.2), the
// hot loop of every stage: RHS (G), GMRES matvec (dG/dn) and surface
// evaluation (both).
//
// Layout and schedule (gfx950):
//  * a workgroup of 256 threads owns 256 targets, one per lane, and one
//    contiguous split of the sources; blockIdx.z picks a group of MB modes;
//  * sources stream through LDS in tiles of TS: positions and normals (SoA,
//    coalesced) plus the weighted data of the MB modes; every lane reads the
//    same source at the same time, so LDS reads are broadcasts;
//  * the geometry of a pair (d, r^2, 1/r, r, d.n/r^3) is computed once and
//    shared by the MB modes of the group, which all have their own k;
//  * the pair terms are folded as e^{ikr} Z with
//       Z = a/r + (ikr - 1) (d.n / r^3) b,
//    a = w/(4 pi) g-like data and b = w/(4 pi) p-like data, so one complex
//    multiply-add per pair and mode accumulates both G and dG/dn terms;
//  * the phase is reduced in revolutions, kappa r - floor(kappa r) with
//    kappa = k / (2 pi), and fed to the hardware sine and cosine, which take
//    revolutions;
//  * each tile's FP32 sum is folded into a (hi, lo) pair with Knuth's
//    TwoSum, and the splits are combined the same way by the reduction
//    kernel, which applies the epilogue of the operation in FP64.
#include "nat_internal.h"

namespace nat {
namespace {

constexpr int kThreads = 256;
constexpr int kTS = 64;  // sources per LDS tile

struct Sum32Params {
    int32_t NT, NS, n_modes;
    const float* t32;      // [3][NT]
    const float* s32;      // [3][NS]
    const float* sn32;     // [3][NS]
    const float2* a32;     // [mode][ld_s]   (RHS, EVAL)
    const float2* b32;     // [mode][ld_s]   (MATVEC, EVAL)
    int64_t ld_s;
    const float* kappa;    // [n_modes]
    const float* kk;       // [n_modes]
    const int32_t* active; // [n_modes] or null
    ModeList modes;        // slots of the launch
    float eps2;
    int32_t per_split;     // sources per split, multiple of kTS
    float4* partial;       // [split][mode][NT]: (hi.re, hi.im, lo.re, lo.im)
};

__device__ __forceinline__ void two_sum_fold(float& hi, float& lo, float t)
{
    const float s = hi + t;
    const float bp = s - hi;
    lo += (hi - (s - bp)) + (t - bp);
    hi = s;
}

template <int OP, int MB>
__global__ void __launch_bounds__(kThreads) k_sum32(const Sum32Params p)
{
    constexpr bool kA = (OP == OP_RHS || OP == OP_EVAL);
    constexpr bool kB = (OP == OP_MATVEC || OP == OP_EVAL);
    __shared__ float s_pos[6][kTS];
    __shared__ float2 s_a[kA ? MB : 1][kTS];
    __shared__ float2 s_b[kB ? MB : 1][kTS];

    const int32_t tid = threadIdx.x;
    const int32_t i = blockIdx.x * kThreads + tid;
    const int32_t split = blockIdx.y;
    const int32_t s0 = blockIdx.z * MB;  // first slot of this mode group
    const int32_t NT = p.NT, NS = p.NS;

    // modes of the group; slots past the list repeat the last mode and are not stored
    int32_t mode[MB];
    bool live[MB];
#pragma unroll
    for (int mm = 0; mm < MB; ++mm) {
        const int32_t slot = s0 + mm < p.modes.n ? s0 + mm : p.modes.n - 1;
        mode[mm] = mode_at(p.modes, slot);
        live[mm] = (s0 + mm < p.modes.n) && (!p.active || p.active[mode[mm]]);
    }
    {
        bool any = false;
#pragma unroll
        for (int mm = 0; mm < MB; ++mm)
            any |= live[mm];
        if (!any)
            return;
    }

    const int32_t ic = i < NT ? i : NT - 1;
    const float tx = p.t32[ic], ty = p.t32[NT + ic], tz = p.t32[2 * NT + ic];

    float kap[MB], kk[MB];
#pragma unroll
    for (int mm = 0; mm < MB; ++mm) {
        kap[mm] = p.kappa[mode[mm]];
        kk[mm] = p.kk[mode[mm]];
    }

    float hr[MB], hi_[MB], lr[MB], li[MB];
#pragma unroll
    for (int mm = 0; mm < MB; ++mm)
        hr[mm] = hi_[mm] = lr[mm] = li[mm] = 0.0f;

    const float eps2 = p.eps2;
    const int32_t j_begin = split * p.per_split;
    const int32_t j_end = min(NS, j_begin + p.per_split);

    for (int32_t j0 = j_begin; j0 < j_end; j0 += kTS) {
        const int32_t cnt = min(kTS, j_end - j0);
        __syncthreads();
        // stage the tile: 6 geometry rows, then MB rows of a and of b
        for (int e = tid; e < 6 * kTS; e += kThreads) {
            const int row = e / kTS, c = e % kTS;
            const int32_t j = j0 + c;
            float v = 0.0f;
            if (c < cnt)
                v = row < 3 ? p.s32[(size_t)row * NS + j] : p.sn32[(size_t)(row - 3) * NS + j];
            s_pos[row][c] = v;
        }
        if (kA) {
            for (int e = tid; e < MB * kTS; e += kThreads) {
                const int mm = e / kTS, c = e % kTS;
                float2 v = make_float2(0.0f, 0.0f);
                if (c < cnt)
                    v = p.a32[(size_t)mode[mm] * p.ld_s + j0 + c];
                s_a[mm][c] = v;
            }
        }
        if (kB) {
            for (int e = tid; e < MB * kTS; e += kThreads) {
                const int mm = e / kTS, c = e % kTS;
                float2 v = make_float2(0.0f, 0.0f);
                if (c < cnt)
                    v = p.b32[(size_t)mode[mm] * p.ld_s + j0 + c];
                s_b[mm][c] = v;
            }
        }
        __syncthreads();

        float ar[MB], ai[MB];
#pragma unroll
        for (int mm = 0; mm < MB; ++mm)
            ar[mm] = ai[mm] = 0.0f;

        for (int c = 0; c < kTS; ++c) {
            const float dx = s_pos[0][c] - tx;
            const float dy = s_pos[1][c] - ty;
            const float dz = s_pos[2][c] - tz;
            const float r2 = dx * dx + dy * dy + dz * dz;
            const float rinv = (r2 >= eps2) ? __builtin_amdgcn_rsqf(r2) : 0.0f;
            const float r = r2 * rinv;
            float q = 0.0f;
            if (kB) {
                const float dn = dx * s_pos[3][c] + dy * s_pos[4][c] + dz * s_pos[5][c];
                q = dn * (rinv * rinv * rinv);
            }
#pragma unroll
            for (int mm = 0; mm < MB; ++mm) {
                const float ph = __builtin_amdgcn_fractf(r * kap[mm]);
                const float sn = __builtin_amdgcn_sinf(ph);
                const float cs = __builtin_amdgcn_cosf(ph);
                float zr = 0.0f, zi = 0.0f;
                if (kB) {
                    const float2 b = s_b[mm][c];
                    const float kr = r * kk[mm];
                    const float qbr = q * b.x, qbi = q * b.y;
                    zr = -(qbr + kr * qbi);
                    zi = kr * qbr - qbi;
                }
                if (kA) {
                    const float2 av = s_a[mm][c];
                    zr += rinv * av.x;
                    zi += rinv * av.y;
                }
                ar[mm] += cs * zr - sn * zi;
                ai[mm] += cs * zi + sn * zr;
            }
        }
#pragma unroll
        for (int mm = 0; mm < MB; ++mm) {
            two_sum_fold(hr[mm], lr[mm], ar[mm]);
            two_sum_fold(hi_[mm], li[mm], ai[mm]);
        }
    }

    if (i < NT) {
#pragma unroll
        for (int mm = 0; mm < MB; ++mm) {
            if (s0 + mm < p.modes.n)
                p.partial[((size_t)split * p.n_modes + mode[mm]) * NT + i] =
                    make_float4(hr[mm], hi_[mm], lr[mm], li[mm]);
        }
    }
}

// Combine the splits (TwoSum in FP32) and apply the operation's epilogue.
template <int OP>
__global__ void __launch_bounds__(256)
k_reduce32(const float4* __restrict__ partial, int32_t n_split, SumArgs a)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t m = blockIdx.y;
    if (i >= a.NT)
        return;
    if (a.active && !a.active[m])
        return;
    float hr = 0.0f, hi = 0.0f, lr = 0.0f, li = 0.0f;
    for (int32_t s = 0; s < n_split; ++s) {
        const float4 v = partial[((size_t)s * a.n_modes + m) * a.NT + i];
        two_sum_fold(hr, lr, v.x);
        two_sum_fold(hi, li, v.y);
        lr += v.z;
        li += v.w;
    }
    const double accr = static_cast<double>(hr) + static_cast<double>(lr);
    const double acci = static_cast<double>(hi) + static_cast<double>(li);
    double2 out;
    if (OP == OP_RHS) {
        const double2 g = a.g_tgt[(size_t)m * a.ld_gt + i];
        out.x = -accr - 0.5 * a.eps * g.x;
        out.y = -acci - 0.5 * a.eps * g.y;
    } else if (OP == OP_MATVEC) {
        const double2 x = a.p_src[(size_t)m * a.ld_ps + i];
        out.x = 0.5 * x.x - accr;
        out.y = 0.5 * x.y - acci;
    } else {
        const double2 g = a.g_tgt[(size_t)m * a.ld_gt + i];
        out.x = 2.0 * (accr - 0.5 * a.eps * g.x);
        out.y = 2.0 * (acci - 0.5 * a.eps * g.y);
    }
    a.out[(size_t)m * a.ld_out + i] = out;
}

__global__ void __launch_bounds__(256)
k_weight32(const double2* __restrict__ src, int64_t ld_src, int32_t n, double scale,
           float2* __restrict__ dst, int64_t ld_dst)
{
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t m = blockIdx.y;
    if (j >= n)
        return;
    const double2 v = src[(size_t)m * ld_src + j];
    dst[(size_t)m * ld_dst + j] =
        make_float2(static_cast<float>(scale * v.x), static_cast<float>(scale * v.y));
}

struct SplitPlan {
    int32_t n_split, per_split, groups, tiles, mb;
};

// Mode-group width from the number of modes processed; source splits so the
// grid holds about four workgroups per CU of a 256-CU part.
SplitPlan plan(int32_t NT, int32_t NS, int32_t n_list)
{
    SplitPlan s;
    s.mb = n_list <= 1 ? 1 : n_list <= 2 ? 2 : n_list <= 4 ? 4 : 8;
    s.tiles = (NT + kThreads - 1) / kThreads;
    s.groups = (n_list + s.mb - 1) / s.mb;
    const int32_t n_tiles_src = (NS + kTS - 1) / kTS;
    const int64_t base = static_cast<int64_t>(s.tiles) * s.groups;
    int64_t want = (1024 + base - 1) / base;
    if (want < 1)
        want = 1;
    if (want > n_tiles_src)
        want = n_tiles_src;
    const int32_t tiles_per_split = static_cast<int32_t>((n_tiles_src + want - 1) / want);
    s.per_split = tiles_per_split * kTS;
    s.n_split = (NS + s.per_split - 1) / s.per_split;
    if (s.n_split < 1)
        s.n_split = 1;
    return s;
}

template <int OP, int MB>
void launch_mb(const Sum32Params& p, const SplitPlan& sp, hipStream_t s, hipEvent_t e0,
               hipEvent_t e1)
{
    dim3 grid(sp.tiles, sp.n_split, sp.groups);
    launch_k(k_sum32<OP, MB>, grid, dim3(kThreads), 0, s, e0, e1, p);
}

template <int OP>
hipError_t launch_op(const SumArgs& a, const SplitPlan& sp, float4* partial, const ModeList& modes,
                     bool reduce, hipStream_t s, const ProfSlot& ev)
{
    Sum32Params p;
    p.NT = a.NT;
    p.NS = a.NS;
    p.n_modes = a.n_modes;
    p.t32 = a.t32;
    p.s32 = a.s32;
    p.sn32 = a.sn32;
    p.a32 = a.g_src32;
    p.b32 = a.p_src32;
    p.ld_s = a.ld_s32;
    p.kappa = a.kappa32;
    p.kk = a.k32;
    p.active = a.active;
    p.modes = modes;
    p.eps2 = static_cast<float>(a.eps * a.eps);
    p.per_split = sp.per_split;
    p.partial = partial;
    // with a reduction the stop event rides on the reduction kernel
    hipEvent_t stop1 = reduce ? nullptr : ev.stop;
    switch (sp.mb) {
    case 1:
        launch_mb<OP, 1>(p, sp, s, ev.start, stop1);
        break;
    case 2:
        launch_mb<OP, 2>(p, sp, s, ev.start, stop1);
        break;
    case 4:
        launch_mb<OP, 4>(p, sp, s, ev.start, stop1);
        break;
    default:
        launch_mb<OP, 8>(p, sp, s, ev.start, stop1);
        break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !reduce)
        return e;
    dim3 g2(static_cast<unsigned>((a.NT + 255) / 256), static_cast<unsigned>(a.n_modes));
    launch_k(k_reduce32<OP>, g2, dim3(256), 0, s, nullptr, ev.stop, partial, sp.n_split, a);
    return hipGetLastError();
}

}  // namespace

size_t sum32_partial_bytes(const SumArgs& a)
{
    // the largest split count any plan can choose: one split per source tile
    const size_t n_split = (size_t)((a.NS + kTS - 1) / kTS);
    return sizeof(float4) * n_split * (size_t)a.n_modes * (size_t)a.NT;
}

hipError_t launch_sum32(const SumArgs& a, void* partial, hipStream_t s, const ModeList& modes,
                        bool reduce, int32_t* n_split_out, const ProfSlot& ev)
{
    if (n_split_out)
        *n_split_out = 0;
    if (a.NT <= 0 || modes.n <= 0)
        return hipSuccess;
    const SplitPlan sp = plan(a.NT, a.NS, modes.n);
    if (n_split_out)
        *n_split_out = sp.n_split;
    float4* part = static_cast<float4*>(partial);
    switch (a.op) {
    case OP_RHS:
        return launch_op<OP_RHS>(a, sp, part, modes, reduce, s, ev);
    case OP_MATVEC:
        return launch_op<OP_MATVEC>(a, sp, part, modes, reduce, s, ev);
    default:
        return launch_op<OP_EVAL>(a, sp, part, modes, reduce, s, ev);
    }
}

hipError_t launch_weight32(const double2* src, int64_t ld_src, int32_t n_modes, int32_t n,
                           double scale, float2* dst, int64_t ld_dst, hipStream_t s)
{
    if (n <= 0 || n_modes <= 0)
        return hipSuccess;
    dim3 grid(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>(n_modes));
    hipLaunchKernelGGL(k_weight32, grid, dim3(256), 0, s, src, ld_src, n, scale, dst, ld_dst);
    return hipGetLastError();
}

}  // namespace nat

// Plain FP64 kernel sums of the Monte-Carlo BEM (Section 4.1.1, eq.
// bem_linear_system; Section 4.2 for the eps disk): one thread per target,
// every source read from global memory, no tiling, one mode per grid row.
// This is the reference-precision GPU form the FP32 path is compared with.
//
//   G(x,y)      = e^{ikr} / (4 pi r)
//   dG/dn_y     = e^{ikr} (ikr - 1) ((y - x).n_y) / (4 pi r^3)
// Sources closer than eps to the target are left out of every sum.
#include "nat_internal.h"

namespace nat {
namespace {

constexpr double kInv4Pi = 0.07957747154594767;  // 1 / (4 pi)

template <int OP>
__global__ void __launch_bounds__(256) k_sum64(SumArgs a)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t m = blockIdx.y;
    if (i >= a.NT)
        return;
    if (a.active && !a.active[m])
        return;
    const int32_t NT = a.NT, NS = a.NS;
    const double tx = a.t64[i], ty = a.t64[NT + i], tz = a.t64[2 * NT + i];
    const double k = a.k[m];
    const double eps = a.eps;
    const double2* gs = a.g_src ? a.g_src + (size_t)m * a.ld_gs : nullptr;
    const double2* ps = a.p_src ? a.p_src + (size_t)m * a.ld_ps : nullptr;
    const double* sx = a.s64;
    const double* sy = a.s64 + NS;
    const double* sz = a.s64 + 2 * NS;
    const double* nx = a.sn64;
    const double* ny = a.sn64 + NS;
    const double* nz = a.sn64 + 2 * NS;
    double sr = 0.0, si = 0.0;
    for (int32_t j = 0; j < NS; ++j) {
        const double dx = sx[j] - tx, dy = sy[j] - ty, dz = sz[j] - tz;
        const double r = __builtin_sqrt(dx * dx + dy * dy + dz * dz);
        if (!(r >= eps) || r == 0.0)
            continue;
        double sn, cs;
        sincos(k * r, &sn, &cs);
        const double rinv = 1.0 / r;
        const double c = a.w * kInv4Pi * rinv;
        if (OP == OP_RHS || OP == OP_EVAL) {
            // w G g_j   (subtracted below for EVAL)
            const double2 g = gs[j];
            const double gr = c * cs, gi = c * sn;
            const double tr = gr * g.x - gi * g.y, ti = gr * g.y + gi * g.x;
            if (OP == OP_RHS) {
                sr += tr;
                si += ti;
            } else {
                sr -= tr;
                si -= ti;
            }
        }
        if (OP == OP_MATVEC || OP == OP_EVAL) {
            // w dG/dn_j p_j = w e^{ikr} (ikr - 1) (d.n) / (4 pi r^3) p_j
            const double dn = dx * nx[j] + dy * ny[j] + dz * nz[j];
            const double q = c * dn * rinv * rinv;
            const double kr = k * r;
            const double er = q * (-cs - kr * sn), ei = q * (kr * cs - sn);
            const double2 p = ps[j];
            sr += er * p.x - ei * p.y;
            si += er * p.y + ei * p.x;
        }
    }
    double2 out;
    if (OP == OP_RHS) {
        const double2 g = a.g_tgt[(size_t)m * a.ld_gt + i];
        const double2 d = a.disk[m];
        out.x = -sr - (d.x * g.x - d.y * g.y);
        out.y = -si - (d.x * g.y + d.y * g.x);
    } else if (OP == OP_MATVEC) {
        const double2 x = ps[i];
        out.x = 0.5 * x.x - sr;
        out.y = 0.5 * x.y - si;
    } else {
        const double2 g = a.g_tgt[(size_t)m * a.ld_gt + i];
        const double f = a.qfac ? a.qfac[i] : 2.0;
        const double2 d = a.disk[m];
        out.x = f * (sr - (d.x * g.x - d.y * g.y));
        out.y = f * (si - (d.x * g.y + d.y * g.x));
    }
    a.out[(size_t)m * a.ld_out + i] = out;
}

}  // namespace

hipError_t launch_sum64(const SumArgs& a, hipStream_t s, const ProfSlot& ev)
{
    if (a.NT <= 0 || a.n_modes <= 0)
        return hipSuccess;
    dim3 grid(static_cast<unsigned>((a.NT + 255) / 256), static_cast<unsigned>(a.n_modes));
    switch (a.op) {
    case OP_RHS:
        launch_k(k_sum64<OP_RHS>, grid, dim3(256), 0, s, ev.start, ev.stop, a);
        break;
    case OP_MATVEC:
        launch_k(k_sum64<OP_MATVEC>, grid, dim3(256), 0, s, ev.start, ev.stop, a);
        break;
    default:
        launch_k(k_sum64<OP_EVAL>, grid, dim3(256), 0, s, ev.start, ev.stop, a);
        break;
    }
    return hipGetLastError();
}

}  // namespace nat

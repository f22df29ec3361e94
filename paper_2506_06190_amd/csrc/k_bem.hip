// Dense collocation Burton-Miller BEM (Section 4, eq. BurtonMiller, with the
// last term read at the collocation point; Section 4.1: the matrices of
// A p = B g are built directly instead of one matrix per term).
//
// Piecewise-constant p and g, collocation at centroids x_i, FP64 throughout:
//   A_ij = delta_ij / 2 - K_ij - beta W_ij
//   B_ij = -(S_ij + beta K'_ij) - delta_ij beta / 2
// Quadrature rule (the same specification the CPU check follows):
//   far pairs  : collapsed 3x3 Gauss-Legendre on T_j,
//                y = a + s (b - a) + t (1 - s) (c - a), weight ws wt (1 - s) 2|T|
//   near pairs : |x_i - centroid_j| < 2 diam(T_j): 4-way midpoint subdivision,
//                children (a,ab,ca), (ab,b,bc), (ca,bc,c), (ab,bc,ca), applied
//                while the child is still near, depth <= 5, far rule on leaves
//   self pair  : split at x_i into (x_i, v_e, v_e+1); radial integrals in
//                closed form, 16-point Gauss-Legendre in the polar angle.
// Pass 1 (one thread per pair) does far pairs and lists the near/self ones;
// pass 2 (one thread per listed pair) walks the subdivision tree without a
// stack: a node is its depth plus the child index taken at each level, and
// its vertices are rebuilt from the root, so the leaves are visited in the
// same depth-first order as a recursive walk.
#include "nat_internal.h"

namespace nat {
namespace {

constexpr double kInv4Pi = 0.07957747154594767;
constexpr int kFarN = 3;
constexpr int kThetaN = 16;
constexpr int kMaxDepth = 5;
constexpr double kEta = 2.0;

struct Acc4 {
    double2 S, K, Kp, W;
};

__device__ __forceinline__ void sub3(const double* a, const double* b, double* o)
{
    o[0] = a[0] - b[0];
    o[1] = a[1] - b[1];
    o[2] = a[2] - b[2];
}
__device__ __forceinline__ double dot3(const double* a, const double* b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
__device__ __forceinline__ void cross3(const double* a, const double* b, double* o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ double len3(const double* a) { return sqrt(dot3(a, a)); }

// G, dG/dn_y, dG/dn_x and d2G/dn_x dn_y at one point, times wt.
__device__ __forceinline__ void add_kernels(double k, const double* x, const double* nx,
                                            const double* y, const double* ny, double wt,
                                            Acc4& acc)
{
    double R[3];
    sub3(x, y, R);
    const double r = len3(R);
    const double rinv = 1.0 / r;
    double sn, cs;
    sincos(k * r, &sn, &cs);
    const double kr = k * r;
    const double f0 = kInv4Pi * rinv;
    const double f1 = f0 * rinv;
    const double f2 = f1 * rinv;
    // G = e f0; G' = e (ikr - 1) f1; G'' = e (2 - 2ikr - k^2 r^2) f2
    const double2 G = make_double2(cs * f0, sn * f0);
    const double2 G1 = make_double2((-cs - kr * sn) * f1, (kr * cs - sn) * f1);
    const double p2 = 2.0 - kr * kr;
    const double2 G2 = make_double2((cs * p2 + 2.0 * kr * sn) * f2, (sn * p2 - 2.0 * kr * cs) * f2);
    const double Rnx = dot3(R, nx), Rny = dot3(R, ny), nn = dot3(nx, ny);
    const double cy = -Rny * rinv, cx = Rnx * rinv;
    const double c2 = Rnx * (-Rny) * rinv * rinv;
    const double c1 = (-nn + Rnx * Rny * rinv * rinv) * rinv;
    acc.S.x += wt * G.x;
    acc.S.y += wt * G.y;
    acc.K.x += wt * G1.x * cy;
    acc.K.y += wt * G1.y * cy;
    acc.Kp.x += wt * G1.x * cx;
    acc.Kp.y += wt * G1.y * cx;
    acc.W.x += wt * (G2.x * c2 + G1.x * c1);
    acc.W.y += wt * (G2.y * c2 + G1.y * c1);
}

__device__ void far_rule(const double* rules, double k, const double* x, const double* nx,
                         const double* a, const double* b, const double* c, const double* ny,
                         Acc4& acc)
{
    const double* gx = rules;
    const double* gw = rules + kFarN;
    double e1[3], e2[3], cr[3];
    sub3(b, a, e1);
    sub3(c, a, e2);
    cross3(e1, e2, cr);
    const double two_area = len3(cr);
#pragma unroll
    for (int p = 0; p < kFarN; ++p) {
#pragma unroll
        for (int q = 0; q < kFarN; ++q) {
            const double s = gx[p], t = gx[q] * (1.0 - gx[p]);
            const double wt = gw[p] * gw[q] * (1.0 - gx[p]) * two_area;
            double y[3];
#pragma unroll
            for (int d = 0; d < 3; ++d)
                y[d] = a[d] + s * e1[d] + t * e2[d];
            add_kernels(k, x, nx, y, ny, wt, acc);
        }
    }
}

__device__ __forceinline__ void panel(const double* V, const int32_t* T, int32_t j, double* a,
                                      double* b, double* c)
{
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        a[d] = V[3 * T[3 * j + 0] + d];
        b[d] = V[3 * T[3 * j + 1] + d];
        c[d] = V[3 * T[3 * j + 2] + d];
    }
}

__device__ __forceinline__ void centroid_normal(const double* a, const double* b, const double* c,
                                                double* x, double* n)
{
#pragma unroll
    for (int d = 0; d < 3; ++d)
        x[d] = (a[d] + b[d] + c[d]) / 3.0;
    double e1[3], e2[3], cr[3];
    sub3(b, a, e1);
    sub3(c, a, e2);
    cross3(e1, e2, cr);
    const double l = len3(cr);
    n[0] = cr[0] / l;
    n[1] = cr[1] / l;
    n[2] = cr[2] / l;
}

__device__ __forceinline__ double diameter(const double* a, const double* b, const double* c)
{
    double e[3];
    sub3(b, a, e);
    double d = len3(e);
    sub3(c, b, e);
    d = fmax(d, len3(e));
    sub3(a, c, e);
    return fmax(d, len3(e));
}

__device__ __forceinline__ bool is_near(const double* x, const double* a, const double* b,
                                        const double* c)
{
    double cen[3], dd[3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
        cen[d] = (a[d] + b[d] + c[d]) / 3.0;
    sub3(x, cen, dd);
    return len3(dd) < kEta * diameter(a, b, c);
}

__device__ __forceinline__ void write_pair(double2* A, double2* B, int32_t n, int32_t i, int32_t j,
                                           const Acc4& q, double2 beta, bool diag)
{
    // beta * W and beta * K'
    const double2 bW = make_double2(beta.x * q.W.x - beta.y * q.W.y, beta.x * q.W.y + beta.y * q.W.x);
    const double2 bKp = make_double2(beta.x * q.Kp.x - beta.y * q.Kp.y, beta.x * q.Kp.y + beta.y * q.Kp.x);
    double2 a = make_double2(-q.K.x - bW.x, -q.K.y - bW.y);
    double2 b = make_double2(-(q.S.x + bKp.x), -(q.S.y + bKp.y));
    if (diag) {
        a.x += 0.5;
        b.x -= 0.5 * beta.x;
        b.y -= 0.5 * beta.y;
    }
    A[(size_t)i * n + j] = a;
    B[(size_t)i * n + j] = b;
}

__global__ void __launch_bounds__(256)
k_bem_far(BemGeom g, double k, double2 beta, double2* __restrict__ A, double2* __restrict__ B,
          int32_t* __restrict__ near_list, int32_t near_cap, int32_t* __restrict__ near_count)
{
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t i = blockIdx.y;
    if (j >= g.n)
        return;
    double xa[3], xb[3], xc[3], x[3], nx[3];
    panel(g.V, g.T, i, xa, xb, xc);
    centroid_normal(xa, xb, xc, x, nx);
    double a[3], b[3], c[3];
    panel(g.V, g.T, j, a, b, c);
    if (i == j || is_near(x, a, b, c)) {
        const int32_t slot = atomicAdd(near_count, 1);
        if (slot < near_cap) {
            near_list[2 * slot] = i;
            near_list[2 * slot + 1] = j;
        }
        return;
    }
    double e1[3], e2[3], ny[3];
    sub3(b, a, e1);
    sub3(c, a, e2);
    cross3(e1, e2, ny);
    const double l = len3(ny);
    ny[0] /= l;
    ny[1] /= l;
    ny[2] /= l;
    Acc4 q = {};
    far_rule(g.rules, k, x, nx, a, b, c, ny, q);
    write_pair(A, B, g.n, i, j, q, beta, false);
}

__device__ void self_panel(const double* rules, double k, const double* v0, const double* v1,
                           const double* v2, double2& S, double2& W)
{
    const double* tx = rules + 2 * kFarN;
    const double* tw = tx + kThetaN;
    const double* vs[3] = {v0, v1, v2};
    double x[3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
        x[d] = (v0[d] + v1[d] + v2[d]) / 3.0;
    double Sr = 0, Si = 0, Wr = 0, Wi = 0;
    for (int e = 0; e < 3; ++e) {
        const double* a = vs[e];
        const double* b = vs[(e + 1) % 3];
        double ed[3], xa[3];
        sub3(b, a, ed);
        const double L = len3(ed);
        const double u[3] = {ed[0] / L, ed[1] / L, ed[2] / L};
        sub3(x, a, xa);
        const double along = dot3(xa, u);
        const double perp[3] = {xa[0] - along * u[0], xa[1] - along * u[1], xa[2] - along * u[2]};
        const double dist = len3(perp);
        const double ta = atan(-along / dist), tb = atan((L - along) / dist);
        for (int q = 0; q < kThetaN; ++q) {
            const double th = ta + (tb - ta) * tx[q];
            const double wq = (tb - ta) * tw[q];
            const double rho = dist / cos(th);
            double sn, cs;
            sincos(k * rho, &sn, &cs);
            if (k > 0.0) {
                // (e^{ik rho} - 1) / (ik) = (sin(k rho) + i 2 sin^2(k rho / 2)) / k
                const double h = sin(0.5 * k * rho);
                Sr += wq * sn / k;
                Si += wq * 2.0 * h * h / k;
            } else {
                Sr += wq * rho;
            }
            // ik - e^{ik rho} / rho
            Wr += wq * (-cs / rho);
            Wi += wq * (k - sn / rho);
        }
    }
    S = make_double2(Sr * kInv4Pi, Si * kInv4Pi);
    W = make_double2(Wr * kInv4Pi, Wi * kInv4Pi);
}

__global__ void __launch_bounds__(128)
k_bem_near(BemGeom g, double k, double2 beta, double2* __restrict__ A, double2* __restrict__ B,
           const int32_t* __restrict__ near_list, int32_t n_near)
{
    const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_near)
        return;
    const int32_t i = near_list[2 * e], j = near_list[2 * e + 1];
    double xa[3], xb[3], xc[3], x[3], nx[3];
    panel(g.V, g.T, i, xa, xb, xc);
    centroid_normal(xa, xb, xc, x, nx);
    if (i == j) {
        Acc4 q = {};
        self_panel(g.rules, k, xa, xb, xc, q.S, q.W);
        write_pair(A, B, g.n, i, j, q, beta, true);
        return;
    }
    double r0[3], r1[3], r2[3];
    panel(g.V, g.T, j, r0, r1, r2);
    double ny[3];
    {
        double e1[3], e2[3];
        sub3(r1, r0, e1);
        sub3(r2, r0, e2);
        cross3(e1, e2, ny);
        const double l = len3(ny);
        ny[0] /= l;
        ny[1] /= l;
        ny[2] /= l;
    }
    Acc4 q = {};
    int path[kMaxDepth + 1] = {0, 0, 0, 0, 0, 0};
    int depth = 0;
    while (true) {
        double a[3], b[3], c[3];
        for (int d = 0; d < 3; ++d) {
            a[d] = r0[d];
            b[d] = r1[d];
            c[d] = r2[d];
        }
        for (int l = 1; l <= depth; ++l) {
            double ab[3], bc[3], ca[3];
            for (int d = 0; d < 3; ++d) {
                ab[d] = 0.5 * (a[d] + b[d]);
                bc[d] = 0.5 * (b[d] + c[d]);
                ca[d] = 0.5 * (c[d] + a[d]);
            }
            switch (path[l]) {
            case 0:
                for (int d = 0; d < 3; ++d) { b[d] = ab[d]; c[d] = ca[d]; }
                break;
            case 1:
                for (int d = 0; d < 3; ++d) { a[d] = ab[d]; c[d] = bc[d]; }
                break;
            case 2:
                for (int d = 0; d < 3; ++d) { a[d] = ca[d]; b[d] = bc[d]; }
                break;
            default:
                for (int d = 0; d < 3; ++d) { a[d] = ab[d]; b[d] = bc[d]; c[d] = ca[d]; }
                break;
            }
        }
        if (depth < kMaxDepth && is_near(x, a, b, c)) {
            ++depth;
            path[depth] = 0;
            continue;
        }
        far_rule(g.rules, k, x, nx, a, b, c, ny, q);
        while (depth > 0 && path[depth] == 3)
            --depth;
        if (depth == 0)
            break;
        ++path[depth];
    }
    write_pair(A, B, g.n, i, j, q, beta, false);
}

// y_m = M x_m for R <= 4 right-hand sides: a workgroup takes RW rows and its
// four waves split the columns (wave w reads 64-column blocks w, w + 4, ...,
// one complex entry per lane), so each loaded block of a right-hand side
// serves RW rows; the waves' sums are added in wave order, so the result does
// not depend on timing.
template <int R, int RW>
__global__ void __launch_bounds__(256)
k_zgemv(const double2* __restrict__ M, int32_t n, const double2* __restrict__ x, int64_t ld_x,
        double2* __restrict__ y, int64_t ld_y)
{
    __shared__ double2 red[4][RW * R];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int32_t row0 = blockIdx.x * RW;
    // rows past n read row n - 1 (their sums are not stored)
    const double2* Mr[RW];
#pragma unroll
    for (int rr = 0; rr < RW; ++rr)
        Mr[rr] = M + (size_t)min(row0 + rr, n - 1) * n;
    double sr[RW][R], si[RW][R];
#pragma unroll
    for (int rr = 0; rr < RW; ++rr)
#pragma unroll
        for (int r = 0; r < R; ++r)
            sr[rr][r] = si[rr][r] = 0.0;
    for (int32_t j = w * 64 + lane; j < n; j += 256) {
        double2 a[RW], v[R];
#pragma unroll
        for (int rr = 0; rr < RW; ++rr)
            a[rr] = Mr[rr][j];
#pragma unroll
        for (int r = 0; r < R; ++r)
            v[r] = x[(size_t)r * ld_x + j];
#pragma unroll
        for (int rr = 0; rr < RW; ++rr)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                sr[rr][r] += a[rr].x * v[r].x - a[rr].y * v[r].y;
                si[rr][r] += a[rr].x * v[r].y + a[rr].y * v[r].x;
            }
    }
#pragma unroll
    for (int rr = 0; rr < RW; ++rr)
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                sr[rr][r] += __shfl_xor(sr[rr][r], off, 64);
                si[rr][r] += __shfl_xor(si[rr][r], off, 64);
            }
    if (lane == 0) {
#pragma unroll
        for (int rr = 0; rr < RW; ++rr)
#pragma unroll
            for (int r = 0; r < R; ++r)
                red[w][rr * R + r] = make_double2(sr[rr][r], si[rr][r]);
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < RW * R) {
        const int rr = t / R, r = t % R;
        const int32_t row = row0 + rr;
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a += red[q][t].x;
            b += red[q][t].y;
        }
        if (row < n)
            y[(size_t)r * ld_y + row] = make_double2(a, b);
    }
}

// Y_m = M X_m for up to 8 NT right-hand sides at once on the FP64 matrix
// cores.  The complex product is the real product of M viewed as a real
// n x 2n matrix (interleaved re, im) with the real 2n x 2R matrix built from
// the right-hand sides: rows 2k, 2k+1 of column pair (2m, 2m+1) hold
// [[re x_mk, im x_mk], [-im x_mk, re x_mk]], so M is read once in its
// stored layout for all of them.  v_mfma_f64_16x16x4f64 tiles: lane l
// supplies A(row l % 16, k l / 16) and B(k l / 16, col l % 16) and holds
// D(row 4 r + l / 16, col l % 16) in accumulator r.  The contraction index of
// one instruction is any 4 real columns, the same for A and B: here lane
// group q = l / 16 takes complex columns k + 2q and k + 2q + 1 of an 8-column
// step (two 16-byte loads per row), and the real and imaginary parts of each
// feed one instruction apiece.  One wave per 16 RB rows and K segment
// (blockIdx.y), so every right-hand-side fragment loaded serves RB row
// tiles; the segments' partial products are added in segment order by
// k_zgemm_reduce, so the result does not depend on timing.
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

template <int NT, int RB>
__global__ void __launch_bounds__(64)
k_zgemm_mfma(const double2* __restrict__ M, int32_t n, const double2* __restrict__ x, int64_t ld_x,
             int32_t n_rhs, int32_t seg, double2* __restrict__ part)
{
    const int lane = threadIdx.x;
    const int r16 = lane & 15, q = lane >> 4;
    const bool odd = (lane & 1) != 0;        // output column 16 t + r16 is an imaginary part
    const int32_t row0 = blockIdx.x * 16 * RB;
    const int32_t k0 = blockIdx.y * seg, k1 = min(n, k0 + seg);  // complex columns
    // Rows past n and right-hand sides past n_rhs read a valid row instead
    // (their results are not stored), so the loads of whole steps need no
    // guards; only the last, partial step of a segment zeroes its operands.
    const double2* arow[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
        arow[rb] = M + (size_t)min(row0 + 16 * rb + r16, n - 1) * n;
    const double2* xrow[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
        xrow[t] = x + (size_t)min((16 * t + r16) >> 1, n_rhs - 1) * ld_x;
    mfma_d4 acc[RB][NT];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int t = 0; t < NT; ++t)
            acc[rb][t] = mfma_d4{0.0, 0.0, 0.0, 0.0};
    // B entries: real row (re M) -> [re x, im x]; imaginary row -> [-im x, re x]
    auto step = [&](const double2 (&c0)[RB], const double2 (&c1)[RB], const double2 (&y0)[NT],
                    const double2 (&y1)[NT]) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const double b0r = odd ? y0[t].y : y0[t].x, b0i = odd ? y0[t].x : -y0[t].y;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                acc[rb][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(c0[rb].x, b0r, acc[rb][t], 0, 0, 0);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                acc[rb][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(c0[rb].y, b0i, acc[rb][t], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const double b1r = odd ? y1[t].y : y1[t].x, b1i = odd ? y1[t].x : -y1[t].y;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                acc[rb][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(c1[rb].x, b1r, acc[rb][t], 0, 0, 0);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                acc[rb][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(c1[rb].y, b1i, acc[rb][t], 0, 0, 0);
        }
    };
    // Triples of whole steps, three operand sets in rotation: each step's
    // operands are loaded two steps ahead of their products.  Refills past
    // the last triple repeat an address already read (in bounds, unused).
    const int32_t k24 = k0 + (max(k1 - k0, 0) / 24) * 24;
    double2 pa0[RB], pa1[RB], px0[NT], px1[NT];   // set A
    double2 qa0[RB], qa1[RB], qx0[NT], qx1[NT];   // set B
    double2 ra0[RB], ra1[RB], rx0[NT], rx1[NT];   // set C
    auto load = [&](int32_t k, double2 (&a0)[RB], double2 (&a1)[RB], double2 (&x0)[NT],
                    double2 (&x1)[NT]) {
        const int32_t kc = k + 2 * q;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            a0[rb] = arow[rb][kc];
            a1[rb] = arow[rb][kc + 1];
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            x0[t] = xrow[t][kc];
            x1[t] = xrow[t][kc + 1];
        }
    };
    if (k0 < k24) {
        load(k0, pa0, pa1, px0, px1);
        load(k0 + 8, qa0, qa1, qx0, qx1);
    }
    for (int32_t k = k0; k < k24; k += 24) {
        // the scheduling barriers keep each refill ahead of the products
        // that follow it
        const bool more = k + 24 < k24;
        load(k + 16, ra0, ra1, rx0, rx1);
        __builtin_amdgcn_sched_barrier(0);
        step(pa0, pa1, px0, px1);
        __builtin_amdgcn_sched_barrier(0);
        load(more ? k + 24 : k, pa0, pa1, px0, px1);
        __builtin_amdgcn_sched_barrier(0);
        step(qa0, qa1, qx0, qx1);
        __builtin_amdgcn_sched_barrier(0);
        load(more ? k + 32 : k, qa0, qa1, qx0, qx1);
        __builtin_amdgcn_sched_barrier(0);
        step(ra0, ra1, rx0, rx1);
        __builtin_amdgcn_sched_barrier(0);
    }
    // at most two whole steps and a partial one, guarded
    const double2 z2 = make_double2(0.0, 0.0);
    for (int32_t k = k24; k < k1; k += 8) {
        const int32_t kc = k + 2 * q;
        const bool ok0 = kc < k1, ok1 = kc + 1 < k1;
        const int32_t i0 = ok0 ? kc : k1 - 1, i1 = ok1 ? kc + 1 : k1 - 1;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const double2 u0 = arow[rb][i0], u1 = arow[rb][i1];
            pa0[rb] = ok0 ? u0 : z2;
            pa1[rb] = ok1 ? u1 : z2;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const double2 u0 = xrow[t][i0], u1 = xrow[t][i1];
            px0[t] = ok0 ? u0 : z2;
            px1[t] = ok1 ? u1 : z2;
        }
        step(pa0, pa1, px0, px1);
    }
    // partial [segment][rhs][row]
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int c = 16 * t + r16;
        const int m = c >> 1;
        if (m >= n_rhs)
            continue;
        double* pm = reinterpret_cast<double*>(part + ((size_t)blockIdx.y * n_rhs + m) * n);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int32_t row = row0 + 16 * rb + 4 * r + q;
                if (row < n)
                    pm[2 * (size_t)row + (c & 1)] = acc[rb][t][r];
            }
    }
}

__global__ void __launch_bounds__(256)
k_zgemm_reduce(const double2* __restrict__ part, int32_t n, int32_t n_rhs, int32_t n_seg,
               double2* __restrict__ y, int64_t ld_y)
{
    const int32_t row = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t m = blockIdx.y;
    if (row >= n)
        return;
    double sr = 0.0, si = 0.0;
    for (int32_t sg = 0; sg < n_seg; ++sg) {
        const double2 v = part[((size_t)sg * n_rhs + m) * n + row];
        sr += v.x;
        si += v.y;
    }
    y[(size_t)m * ld_y + row] = make_double2(sr, si);
}

__global__ void __launch_bounds__(256)
k_panel_data(const int32_t* __restrict__ T, int32_t nT, const double2* __restrict__ gv,
             int64_t ld_in, double2* __restrict__ gp, int64_t ld_out)
{
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t r = blockIdx.y;
    if (t >= nT)
        return;
    const double2* g = gv + (size_t)r * ld_in;
    const double2 a = g[T[3 * t]], b = g[T[3 * t + 1]], c = g[T[3 * t + 2]];
    gp[(size_t)r * ld_out + t] = make_double2((a.x + b.x + c.x) / 3.0, (a.y + b.y + c.y) / 3.0);
}

}  // namespace

hipError_t launch_bem_far(const BemGeom& g, double k, double2 beta, double2* A, double2* B,
                          int32_t* near_list, int32_t near_cap, int32_t* near_count,
                          hipStream_t s, const ProfSlot& ev)
{
    dim3 grid(static_cast<unsigned>((g.n + 255) / 256), static_cast<unsigned>(g.n));
    launch_k(k_bem_far, grid, dim3(256), 0, s, ev.start, ev.stop, g, k, beta, A, B, near_list,
             near_cap, near_count);
    return hipGetLastError();
}

hipError_t launch_bem_near(const BemGeom& g, double k, double2 beta, double2* A, double2* B,
                           const int32_t* near_list, int32_t n_near, hipStream_t s,
                           const ProfSlot& ev)
{
    if (n_near <= 0)
        return hipSuccess;
    launch_k(k_bem_near, dim3((n_near + 127) / 128), dim3(128), 0, s, ev.start, ev.stop, g, k, beta,
             A, B, near_list, n_near);
    return hipGetLastError();
}

// Rows per wave of the matrix-core product, and its K split: about 2048
// waves in all (eight per SIMD), at most 32 segments, each a multiple of 8
// complex columns.
constexpr int32_t kZgemmRows = 64;

int32_t zgemm_segments(int32_t n, int32_t* seg_out)
{
    if (n < 1) {
        if (seg_out)
            *seg_out = 8;
        return 1;
    }
    const int32_t groups = (n + kZgemmRows - 1) / kZgemmRows;
    int32_t want = (2048 + groups - 1) / groups;
    const int32_t cap = (n + 63) / 64;
    want = want > 32 ? 32 : want;
    want = want > cap ? cap : want;
    want = want < 1 ? 1 : want;
    int32_t seg = (n + want - 1) / want;
    seg = (seg + 7) / 8 * 8;
    if (seg_out)
        *seg_out = seg;
    return (n + seg - 1) / seg;
}

hipError_t launch_zgemv(const double2* M, int32_t n, const double2* x, int64_t ld_x,
                        int32_t n_rhs, double2* y, int64_t ld_y, const int32_t* active,
                        hipStream_t s, const ProfSlot& ev, double2* scratch)
{
    (void)active;
    if (n_rhs >= kZgemmMinRhs && scratch) {
        // matrix cores, 16 right-hand sides per pass over M (8 in a last pass of <= 8)
        int32_t seg = 0;
        const int32_t n_seg = zgemm_segments(n, &seg);
        for (int32_t r0 = 0; r0 < n_rhs; r0 += 16) {
            const int32_t R = n_rhs - r0 < 16 ? n_rhs - r0 : 16;
            hipEvent_t e0 = r0 == 0 ? ev.start : nullptr;
            hipEvent_t e1 = r0 + 16 >= n_rhs ? ev.stop : nullptr;
            dim3 grid(static_cast<unsigned>((n + kZgemmRows - 1) / kZgemmRows), static_cast<unsigned>(n_seg));
            if (R > 8)
                launch_k(k_zgemm_mfma<2, kZgemmRows / 16>, grid, dim3(64), 0, s, e0, nullptr, M, n,
                         x + (size_t)r0 * ld_x, ld_x, R, seg, scratch);
            else
                launch_k(k_zgemm_mfma<1, kZgemmRows / 16>, grid, dim3(64), 0, s, e0, nullptr, M, n,
                         x + (size_t)r0 * ld_x, ld_x, R, seg, scratch);
            launch_k(k_zgemm_reduce, dim3((n + 255) / 256, R), dim3(256), 0, s, nullptr, e1,
                     static_cast<const double2*>(scratch), n, R, n_seg, y + (size_t)r0 * ld_y, ld_y);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess)
                return e;
        }
        return hipSuccess;
    }
    // four rows per workgroup once there are enough rows to fill the device
    // (measured: 5.2-5.9 TB/s at n = 5120-16384 for four right-hand sides,
    // against 3.5 with one row per wave); one row below that
    const bool wide = n >= 4096;
    const int32_t rw = wide ? 4 : 1;
    dim3 grid(static_cast<unsigned>((n + rw - 1) / rw));
    for (int32_t r0 = 0; r0 < n_rhs; r0 += 4) {
        const int32_t R = n_rhs - r0 < 4 ? n_rhs - r0 : 4;
        const double2* xr = x + (size_t)r0 * ld_x;
        double2* yr = y + (size_t)r0 * ld_y;
        hipEvent_t e0 = r0 == 0 ? ev.start : nullptr;
        hipEvent_t e1 = r0 + 4 >= n_rhs ? ev.stop : nullptr;
        switch (R * 2 + (wide ? 1 : 0)) {
        case 2:
            launch_k(k_zgemv<1, 1>, grid, dim3(256), 0, s, e0, e1, M, n, xr, ld_x, yr, ld_y);
            break;
        case 3:
            launch_k(k_zgemv<1, 4>, grid, dim3(256), 0, s, e0, e1, M, n, xr, ld_x, yr, ld_y);
            break;
        case 4:
            launch_k(k_zgemv<2, 1>, grid, dim3(256), 0, s, e0, e1, M, n, xr, ld_x, yr, ld_y);
            break;
        case 5:
            launch_k(k_zgemv<2, 4>, grid, dim3(256), 0, s, e0, e1, M, n, xr, ld_x, yr, ld_y);
            break;
        case 6:
            launch_k(k_zgemv<3, 1>, grid, dim3(256), 0, s, e0, e1, M, n, xr, ld_x, yr, ld_y);
            break;
        case 7:
            launch_k(k_zgemv<3, 4>, grid, dim3(256), 0, s, e0, e1, M, n, xr, ld_x, yr, ld_y);
            break;
        case 8:
            launch_k(k_zgemv<4, 1>, grid, dim3(256), 0, s, e0, e1, M, n, xr, ld_x, yr, ld_y);
            break;
        default:
            launch_k(k_zgemv<4, 4>, grid, dim3(256), 0, s, e0, e1, M, n, xr, ld_x, yr, ld_y);
            break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t launch_panel_data(const int32_t* T, int32_t nT, const double2* gv, int64_t ld_in,
                             int32_t n_rhs, double2* gp, int64_t ld_out, hipStream_t s)
{
    if (nT <= 0 || n_rhs <= 0)
        return hipSuccess;
    dim3 grid(static_cast<unsigned>((nT + 255) / 256), static_cast<unsigned>(n_rhs));
    hipLaunchKernelGGL(k_panel_data, grid, dim3(256), 0, s, T, nT, gv, ld_in, gp, ld_out);
    return hipGetLastError();
}

}  // namespace nat

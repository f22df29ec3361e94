/*
 * nat_oracle.c -- plain FP64 CPU oracle for the MC-BEM estimator and the
 * dense collocation Burton-Miller BEM of "NAT: Neural Acoustic Transfer for
 * Interactive Scenes in Real Time" (arXiv 2506.06190), Section 4.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or generator with the GPU library; both are written from
 * the paper and from the readings listed in the design notes.
 *
 * Everything is double precision, every sum runs in ascending source index,
 * and nothing is blocked, fused or reordered beyond what the formulas say.
 * OpenMP only splits independent rows/targets over threads; each row's sum
 * keeps its fixed order, so results do not depend on the thread count.
 * Build with -ffp-contract=off so no multiply-add is contracted.
 *
 * Conventions (outward normal n into the fluid, time factor e^{-i w t}):
 *   G(x,y)        = e^{ikr} / (4 pi r),   r = |x - y|
 *   dG/dn_y(x,y)  = e^{ikr} (ikr - 1) ((y - x).n_y) / (4 pi r^3)
 *   surface BIE   : p(x)/2 = int_Gamma ( p dG/dn_y - G g ) dS(y),  g = dp/dn
 * The printed Monte-Carlo equation (Section 4.1.1, eq. BIE) carries the
 * opposite sign on its right-hand side; it is the same identity with the
 * normal taken into the body.  With outward normals the form above is the
 * one consistent with the Burton-Miller equation of Section 4 at beta = 0.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define FOUR_PI (4.0 * M_PI)

/* thread count of the parallel loops that follow (timing only) */
void orc_set_threads(int32_t n)
{
    omp_set_num_threads(n > 0 ? n : 1);
}

/* threads OpenMP will use for the parallel loops */
int32_t orc_num_threads(void)
{
    return (int32_t)omp_get_max_threads();
}

/* ---------------------------------------------------------------------- */
/* small vector helpers                                                    */
/* ---------------------------------------------------------------------- */
static void sub3(const double* a, const double* b, double* o)
{
    o[0] = a[0] - b[0];
    o[1] = a[1] - b[1];
    o[2] = a[2] - b[2];
}

static double dot3(const double* a, const double* b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static void cross3(const double* a, const double* b, double* o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static double norm3(const double* a)
{
    return sqrt(dot3(a, a));
}

/* ---------------------------------------------------------------------- */
/* O1/O2: triangle geometry and the area CDF (Section 4.1.1: uniform     */
/* sampling with density 1/|Gamma|).                                      */
/* ---------------------------------------------------------------------- */
void orc_geometry(const double* V, const int32_t* T, int32_t nT,
                  double* area, double* normal, double* cdf)
{
    double run = 0.0;
    for (int32_t t = 0; t < nT; ++t) {
        const double* v0 = V + 3 * T[3 * t + 0];
        const double* v1 = V + 3 * T[3 * t + 1];
        const double* v2 = V + 3 * T[3 * t + 2];
        double e1[3], e2[3], c[3];
        sub3(v1, v0, e1);
        sub3(v2, v0, e2);
        cross3(e1, e2, c);
        double len = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        area[t] = 0.5 * len;
        normal[3 * t + 0] = c[0] / len;
        normal[3 * t + 1] = c[1] / len;
        normal[3 * t + 2] = c[2] / len;
        run = run + area[t];
        cdf[t] = run;
    }
}

/* ---------------------------------------------------------------------- */
/* O3: counter-based random words.  SplitMix64 (Steele, Lea & Flood,       */
/* OOPSLA 2014): the output at position i of a generator whose state      */
/* starts at s is mix(s + (i+1) * gamma).  Streams offset the start state */
/* by stream << 56.                                                        */
/* ---------------------------------------------------------------------- */
uint64_t orc_splitmix64(uint64_t state)
{
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t orc_rng_word(uint64_t seed, uint32_t stream, uint64_t counter)
{
    uint64_t start = seed ^ ((uint64_t)stream << 56);
    return orc_splitmix64(start + (counter + 1ULL) * 0x9E3779B97F4A7C15ULL);
}

static double orc_u01(uint64_t h)
{
    return (double)(h >> 11) * (1.0 / 9007199254740992.0); /* 2^-53 */
}

/* ---------------------------------------------------------------------- */
/* O4/O5: area-uniform samples.  Triangle: smallest t with cdf[t] > u0 A.  */
/* Point: s = sqrt(u1), b1 = s (1 - u2), b2 = s u2 (uniform triangle warp). */
/* ---------------------------------------------------------------------- */
int32_t orc_cdf_search(const double* cdf, int32_t nT, double tau)
{
    int32_t lo = 0, hi = nT - 1;
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (cdf[mid] > tau)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

void orc_samples(const double* cdf, int32_t nT, int32_t N, uint64_t seed,
                 int32_t* tri, double* bary)
{
    double A = cdf[nT - 1];
    for (int32_t j = 0; j < N; ++j) {
        double u0 = orc_u01(orc_rng_word(seed, 0, 3ULL * (uint64_t)j + 0));
        double u1 = orc_u01(orc_rng_word(seed, 0, 3ULL * (uint64_t)j + 1));
        double u2 = orc_u01(orc_rng_word(seed, 0, 3ULL * (uint64_t)j + 2));
        double tau = u0 * A;
        tri[j] = orc_cdf_search(cdf, nT, tau);
        double s = sqrt(u1);
        bary[2 * j + 0] = s * (1.0 - u2);
        bary[2 * j + 1] = s * u2;
    }
}

/* ---------------------------------------------------------------------- */
/* Poisson-disk sample set (Section 4.2: parallel Poisson-disk sampling   */
/* after Bowers, Wang, Wei & Maletz 2010).                                */
/* Candidates: M = cand_factor N area-uniform points; candidate i draws   */
/* u0, u1, u2 from counters 3i..3i+2 of stream 6, takes the triangle of   */
/* u0 A as the samples do and the point (b1, b2) = (u1, u2), folded to    */
/* (1 - u1, 1 - u2) when u1 + u2 > 1 (a uniform point of the triangle      */
/* with exact arithmetic).  Radius r = rscale sqrt(A / N).                 */
/* Grid: cells of side h = r / sqrt(3) (a cell holds at most one accepted  */
/* point) over the mesh's bounding box, cell (cx, cy, cz) =                */
/* floor((x - lo) sqrt(3)/r) per axis, key (cx NY + cy) NZ + cz; a cell's  */
/* candidates in index order.  Phase of a cell (cx mod 3, cy mod 3,        */
/* cz mod 3) as 9 a + 3 b + c: cells of one phase are more than r apart,   */
/* so they can be decided independently (in parallel).                    */
/* Passes p = 0, 1, ...; in each, phases 0..26 in order; in each phase the */
/* cells in key order without an accepted point try their p-th candidate, */
/* which is accepted unless an accepted point of the 5 x 5 x 5 cells      */
/* around lies closer than r (squared distances in FP64, no fused          */
/* multiply-add).  The samples are the first N accepted points in         */
/* acceptance order (n_out_max > N returns more of them, for tests).      */
/* Returns the number accepted (the estimator needs >= N).                 */
/* ---------------------------------------------------------------------- */
/* radius scale and candidate count of the estimator's Poisson-disk set */
#define ORC_POISSON_RSCALE 0.72
#define ORC_POISSON_CANDIDATES 16

typedef struct {
    int64_t key;
    int32_t idx;
} orc_keyidx;

void orc_surface_points(const double* V, const int32_t* T, int32_t n, const int32_t* tri,
                        const double* bary, double* xyz);

static int orc_cmp_keyidx(const void* a, const void* b)
{
    const orc_keyidx* x = (const orc_keyidx*)a;
    const orc_keyidx* y = (const orc_keyidx*)b;
    if (x->key != y->key)
        return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

void orc_poisson_candidates(const double* V, const int32_t* T, const double* cdf, int32_t nT,
                            int32_t M, uint64_t seed, int32_t* tri, double* bary, double* xyz)
{
    double A = cdf[nT - 1];
    for (int32_t i = 0; i < M; ++i) {
        double u0 = orc_u01(orc_rng_word(seed, 6, 3ULL * (uint64_t)i + 0));
        double u1 = orc_u01(orc_rng_word(seed, 6, 3ULL * (uint64_t)i + 1));
        double u2 = orc_u01(orc_rng_word(seed, 6, 3ULL * (uint64_t)i + 2));
        tri[i] = orc_cdf_search(cdf, nT, u0 * A);
        double b1 = u1, b2 = u2;
        if (u1 + u2 > 1.0) {
            b1 = 1.0 - u1;
            b2 = 1.0 - u2;
        }
        bary[2 * i + 0] = b1;
        bary[2 * i + 1] = b2;
    }
    orc_surface_points(V, T, M, tri, bary, xyz);
}

static int32_t find_cell(const int64_t* keys, int32_t n, int64_t key)
{
    int32_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (keys[mid] == key)
            return mid;
        if (keys[mid] < key)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

int32_t orc_poisson_samples(const double* V, int32_t nV, const int32_t* T, int32_t nT, int32_t N,
                            uint64_t seed, double rscale, int32_t cand_factor, int32_t n_out_max,
                            int32_t* tri_out, double* bary_out)
{
    double* area = (double*)malloc(sizeof(double) * (size_t)nT);
    double* nrm = (double*)malloc(sizeof(double) * 3 * (size_t)nT);
    double* cdf = (double*)malloc(sizeof(double) * (size_t)nT);
    orc_geometry(V, T, nT, area, nrm, cdf);
    double A = cdf[nT - 1];
    double r = rscale * sqrt(A / (double)N);
    double r2 = r * r;
    double inv_h = sqrt(3.0) / r;
    double lo[3], hi[3];
    for (int c = 0; c < 3; ++c) {
        lo[c] = V[c];
        hi[c] = V[c];
    }
    for (int32_t v = 1; v < nV; ++v)
        for (int c = 0; c < 3; ++c) {
            if (V[3 * v + c] < lo[c])
                lo[c] = V[3 * v + c];
            if (V[3 * v + c] > hi[c])
                hi[c] = V[3 * v + c];
        }
    int64_t dim[3];
    for (int c = 0; c < 3; ++c)
        dim[c] = (int64_t)floor((hi[c] - lo[c]) * inv_h) + 1;
    int32_t M = cand_factor * N;
    int32_t* ctri = (int32_t*)malloc(sizeof(int32_t) * (size_t)M);
    double* cbary = (double*)malloc(sizeof(double) * 2 * (size_t)M);
    double* cx = (double*)malloc(sizeof(double) * 3 * (size_t)M);
    orc_poisson_candidates(V, T, cdf, nT, M, seed, ctri, cbary, cx);
    orc_keyidx* ki = (orc_keyidx*)malloc(sizeof(orc_keyidx) * (size_t)M);
    for (int32_t i = 0; i < M; ++i) {
        int64_t cc[3];
        for (int c = 0; c < 3; ++c) {
            int64_t q = (int64_t)floor((cx[3 * i + c] - lo[c]) * inv_h);
            cc[c] = q < 0 ? 0 : (q >= dim[c] ? dim[c] - 1 : q);
        }
        ki[i].key = (cc[0] * dim[1] + cc[1]) * dim[2] + cc[2];
        ki[i].idx = i;
    }
    qsort(ki, (size_t)M, sizeof(orc_keyidx), orc_cmp_keyidx);
    /* cells: runs of equal keys */
    int64_t* ckey = (int64_t*)malloc(sizeof(int64_t) * (size_t)M);
    int32_t* cstart = (int32_t*)malloc(sizeof(int32_t) * (size_t)M);
    int32_t* ccount = (int32_t*)malloc(sizeof(int32_t) * (size_t)M);
    int32_t* cacc = (int32_t*)malloc(sizeof(int32_t) * (size_t)M);
    int32_t* cphase = (int32_t*)malloc(sizeof(int32_t) * (size_t)M);
    int32_t ncell = 0, maxc = 0;
    for (int32_t i = 0; i < M; ++i) {
        if (ncell == 0 || ckey[ncell - 1] != ki[i].key) {
            ckey[ncell] = ki[i].key;
            cstart[ncell] = i;
            ccount[ncell] = 0;
            ++ncell;
        }
        ++ccount[ncell - 1];
        if (ccount[ncell - 1] > maxc)
            maxc = ccount[ncell - 1];
    }
    for (int32_t c = 0; c < ncell; ++c) {
        int64_t k = ckey[c];
        int64_t z = k % dim[2], y = (k / dim[2]) % dim[1], x = k / (dim[1] * dim[2]);
        cphase[c] = (int32_t)((x % 3) * 9 + (y % 3) * 3 + (z % 3));
        cacc[c] = -1;
    }
    int32_t* accepted = (int32_t*)malloc(sizeof(int32_t) * (size_t)ncell);
    int32_t nacc = 0;
    for (int32_t p = 0; p < maxc; ++p) {
        for (int32_t ph = 0; ph < 27; ++ph) {
            for (int32_t c = 0; c < ncell; ++c) {
                if (cphase[c] != ph || cacc[c] >= 0 || ccount[c] <= p)
                    continue;
                int32_t cand = ki[cstart[c] + p].idx;
                const double* xc = cx + 3 * (size_t)cand;
                int64_t k = ckey[c];
                int64_t z = k % dim[2], y = (k / dim[2]) % dim[1], x = k / (dim[1] * dim[2]);
                int ok = 1;
                for (int dx = -2; dx <= 2 && ok; ++dx)
                    for (int dy = -2; dy <= 2 && ok; ++dy)
                        for (int dz = -2; dz <= 2 && ok; ++dz) {
                            int64_t nx = x + dx, ny = y + dy, nz = z + dz;
                            if (nx < 0 || ny < 0 || nz < 0 || nx >= dim[0] || ny >= dim[1] || nz >= dim[2])
                                continue;
                            int32_t nc = find_cell(ckey, ncell, (nx * dim[1] + ny) * dim[2] + nz);
                            if (nc < 0 || cacc[nc] < 0)
                                continue;
                            const double* xa = cx + 3 * (size_t)cacc[nc];
                            double ex = xc[0] - xa[0], ey = xc[1] - xa[1], ez = xc[2] - xa[2];
                            double d2 = ex * ex + ey * ey + ez * ez;
                            if (d2 < r2)
                                ok = 0;
                        }
                if (ok) {
                    cacc[c] = cand;
                    accepted[nacc++] = cand;
                }
            }
        }
    }
    int32_t n_out = nacc < n_out_max ? nacc : n_out_max;
    for (int32_t j = 0; j < n_out; ++j) {
        tri_out[j] = ctri[accepted[j]];
        bary_out[2 * j + 0] = cbary[2 * (size_t)accepted[j] + 0];
        bary_out[2 * j + 1] = cbary[2 * (size_t)accepted[j] + 1];
    }
    free(area);
    free(nrm);
    free(cdf);
    free(ctri);
    free(cbary);
    free(cx);
    free(ki);
    free(ckey);
    free(cstart);
    free(ccount);
    free(cacc);
    free(cphase);
    free(accepted);
    return nacc;
}

/* x = v0 + b1 (v1 - v0) + b2 (v2 - v0) */
void orc_surface_points(const double* V, const int32_t* T, int32_t n,
                        const int32_t* tri, const double* bary, double* xyz)
{
    for (int32_t i = 0; i < n; ++i) {
        const double* v0 = V + 3 * T[3 * tri[i] + 0];
        const double* v1 = V + 3 * T[3 * tri[i] + 1];
        const double* v2 = V + 3 * T[3 * tri[i] + 2];
        double b1 = bary[2 * i], b2 = bary[2 * i + 1];
        for (int c = 0; c < 3; ++c)
            xyz[3 * i + c] = v0[c] + b1 * (v1[c] - v0[c]) + b2 * (v2[c] - v0[c]);
    }
}

/* Neumann data at surface points.  layout 0: per vertex, linear in the
 * barycentrics; layout 1: one value per triangle (Section 3.4: the data is
 * constant on each triangle in the paper's scenes). */
void orc_neumann_at(const int32_t* T, int32_t layout, const double* g_in,
                    int32_t n, const int32_t* tri, const double* bary, double* g_out)
{
    const cplx* g = (const cplx*)g_in;
    cplx* o = (cplx*)g_out;
    for (int32_t i = 0; i < n; ++i) {
        if (layout == 1) {
            o[i] = g[tri[i]];
        } else {
            double b1 = bary[2 * i], b2 = bary[2 * i + 1];
            double b0 = 1.0 - b1 - b2;
            o[i] = b0 * g[T[3 * tri[i] + 0]] + b1 * g[T[3 * tri[i] + 1]] + b2 * g[T[3 * tri[i] + 2]];
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Green's function and its normal derivatives (Section 4.2).              */
/* ---------------------------------------------------------------------- */
cplx orc_G(double k, double r)
{
    return cexp(I * k * r) / (FOUR_PI * r);
}

/* dG/dn_y at source y with normal ny, target x. */
cplx orc_dGdny(double k, const double* x, const double* y, const double* ny)
{
    double d[3];
    sub3(y, x, d);
    double r = norm3(d);
    return cexp(I * k * r) * (I * k * r - 1.0) * dot3(d, ny) / (FOUR_PI * r * r * r);
}

/* wrappers with real/imag outputs for the Python driver */
void orc_kernels(double k, const double* x, const double* nx, const double* y,
                 const double* ny, double* out /* 4 complex: G, dG/dny, dG/dnx, d2G/dnxdny */)
{
    double R[3];
    sub3(x, y, R);
    double r = norm3(R);
    cplx e = cexp(I * k * r);
    cplx G = e / (FOUR_PI * r);
    cplx G1 = e * (I * k * r - 1.0) / (FOUR_PI * r * r);
    cplx G2 = e * (2.0 - 2.0 * I * k * r - k * k * r * r) / (FOUR_PI * r * r * r);
    double Rnx = dot3(R, nx), Rny = dot3(R, ny), nn = dot3(nx, ny);
    cplx dny = G1 * (-Rny) / r;
    cplx dnx = G1 * Rnx / r;
    cplx dd = G2 * Rnx * (-Rny) / (r * r) + (G1 / r) * (-nn + Rnx * Rny / (r * r));
    cplx* o = (cplx*)out;
    o[0] = G;
    o[1] = dny;
    o[2] = dnx;
    o[3] = dd;
}

/* ---------------------------------------------------------------------- */
/* O6/O7: the Monte-Carlo Nystrom system (Section 4.1.1, eq.              */
/* bem_linear_system, with the disk treatment of Section 4.2).            */
/*   M_ij = delta_ij / 2 - [r_ij >= eps] w dG(y_i, y_j)/dn_j               */
/*   b_i  = - sum_j [r_ij >= eps] w G(y_i, y_j) g_j - (eps/2) g_i          */
/* w = |Gamma| / N.  The disk of radius eps around y_i contributes        */
/* (eps/2) g_i through G and nothing through dG/dn.                        */
/* ---------------------------------------------------------------------- */
void orc_mc_matrix(int32_t N, const double* y, const double* ny, double k, double w,
                   double eps, double* M_out /* complex N x N row-major */)
{
    cplx* M = (cplx*)M_out;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < N; ++i) {
        for (int32_t j = 0; j < N; ++j) {
            double d[3];
            sub3(y + 3 * j, y + 3 * i, d);
            double r = norm3(d);
            cplx m = (i == j) ? 0.5 : 0.0;
            if (r >= eps)
                m -= w * orc_dGdny(k, y + 3 * i, y + 3 * j, ny + 3 * j);
            M[(size_t)i * N + j] = m;
        }
    }
}

/* Integral of G over the flat disk of radius eps about the target, times
 * the Neumann value there (Section 4.2): the paper's one-sample estimate
 * eps/2, or (exact_disk) the closed form: in polar coordinates the area
 * element r dr dtheta cancels the 1/r of G, leaving (1/2) int_0^eps e^{ikr} dr
 * = (e^{ik eps} - 1)/(2ik). */
static cplx disk_factor(double k, double eps, int32_t exact_disk)
{
    if (!exact_disk)
        return 0.5 * eps;
    return (cexp(I * k * eps) - 1.0) / (2.0 * I * k);
}

void orc_mc_rhs(int32_t N, const double* y, double k, double w, double eps,
                const double* g_in, int32_t exact_disk, double* b_out)
{
    const cplx dk = disk_factor(k, eps, exact_disk);
    const cplx* g = (const cplx*)g_in;
    cplx* b = (cplx*)b_out;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < N; ++i) {
        cplx s = 0.0;
        for (int32_t j = 0; j < N; ++j) {
            double d[3];
            sub3(y + 3 * j, y + 3 * i, d);
            double r = norm3(d);
            if (r >= eps)
                s += w * orc_G(k, r) * g[j];
        }
        b[i] = -s - dk * g[i];
    }
}

/* O8: evaluation at target points x_q from the sample values.
 *   p(x_q) = (1/c_q) [ sum_j [|x_q - y_j| >= eps] w (dG/dn_j p_j - G g_j)
 *                      - (eps/2) g(x_q) ]
 * c_q = 1/2 for surface points (paper); c_q = 1 with eps = 0 evaluates the
 * exterior representation formula.  c_arr, when not NULL, gives c_q per
 * target instead (orc_free_terms). */
void orc_mc_eval(int32_t Q, const double* x, const double* gx_in, double c_q,
                 const double* c_arr, int32_t N, const double* y, const double* ny,
                 const double* g_in, const double* p_in, double k, double w, double eps,
                 int32_t exact_disk, double* out)
{
    const cplx dk = disk_factor(k, eps, exact_disk);
    const cplx* g = (const cplx*)g_in;
    const cplx* p = (const cplx*)p_in;
    const cplx* gx = (const cplx*)gx_in;
    cplx* o = (cplx*)out;
#pragma omp parallel for schedule(static)
    for (int32_t q = 0; q < Q; ++q) {
        cplx s = 0.0;
        for (int32_t j = 0; j < N; ++j) {
            double d[3];
            sub3(y + 3 * j, x + 3 * q, d);
            double r = norm3(d);
            if (r >= eps && r > 0.0)
                s += w * (orc_dGdny(k, x + 3 * q, y + 3 * j, ny + 3 * j) * p[j] - orc_G(k, r) * g[j]);
        }
        cplx disk = gx ? dk * gx[q] : 0.0;
        o[q] = (s - disk) / (c_arr ? c_arr[q] : c_q);
    }
}

/* ---------------------------------------------------------------------- */
/* Field points around a scene (Section 3.4, training data; Section 3.1,  */
/* FFAT maps).  R is the bounding-box radius (half the box diagonal) and  */
/* c the box centre.                                                      */
/*  kind 0 (shell): n_a points; point i draws u0, u1, u2 from counters    */
/*    3i, 3i+1, 3i+2 of stream 5 and takes r = R (r_lo + (r_hi - r_lo) u0),*/
/*    cos(theta) = 1 - 2 u1, phi = 2 pi u2 (a direction uniform on the    */
/*    sphere, a radius uniform in the shell).                             */
/*  kind 1 (FFAT grid): n_a x n_b points on the sphere of radius R r_lo,  */
/*    theta_a = (a + 1/2) pi / n_a, phi_b = (b + 1/2) 2 pi / n_b, point    */
/*    a n_b + b (an image with theta down the rows, phi along them).      */
/* x = c + r (sin theta cos phi, sin theta sin phi, cos theta); coords    */
/* holds (r, theta, phi) per point.                                       */
/* ---------------------------------------------------------------------- */
void orc_field_points(const double* center, double R, int32_t kind, int32_t n_a, int32_t n_b,
                      double r_lo, double r_hi, uint64_t seed, double* xyz, double* coords)
{
    int32_t n = kind == 0 ? n_a : n_a * n_b;
    for (int32_t i = 0; i < n; ++i) {
        double r, th, ph;
        if (kind == 0) {
            double u0 = orc_u01(orc_rng_word(seed, 5, 3ULL * (uint64_t)i + 0));
            double u1 = orc_u01(orc_rng_word(seed, 5, 3ULL * (uint64_t)i + 1));
            double u2 = orc_u01(orc_rng_word(seed, 5, 3ULL * (uint64_t)i + 2));
            r = R * (r_lo + (r_hi - r_lo) * u0);
            th = acos(1.0 - 2.0 * u1);
            ph = 2.0 * M_PI * u2;
        } else {
            int32_t a = i / n_b, b = i % n_b;
            r = R * r_lo;
            th = (a + 0.5) * M_PI / n_a;
            ph = (b + 0.5) * 2.0 * M_PI / n_b;
        }
        xyz[3 * i + 0] = center[0] + r * (sin(th) * cos(ph));
        xyz[3 * i + 1] = center[1] + r * (sin(th) * sin(ph));
        xyz[3 * i + 2] = center[2] + r * cos(th);
        coords[3 * i + 0] = r;
        coords[3 * i + 1] = th;
        coords[3 * i + 2] = ph;
    }
}

/* ---------------------------------------------------------------------- */
/* Free term of the surface identity at a query point.  The identity      */
/* c(x) p(x) = int (p dG/dn_y - G g) holds on the boundary with             */
/* c(x) = 1 + int dG0/dn_y dS_y (G0 the Laplace kernel), i.e. one minus the */
/* solid angle Omega(x) the body subtends at x over 4 pi (the Gauss         */
/* integral); c = 1/2 where the surface is smooth, the paper's value.       */
/* Omega(x) is the sum over the mesh triangles of their signed solid angles */
/* at x (Van Oosterom & Strackee 1983), leaving out the triangles x lies on */
/* (their contribution is zero: x is in their plane).  A query is on a      */
/* vertex when two of its barycentric weights (1 - b1 - b2, b1, b2) are     */
/* exactly zero and on an edge when one is; otherwise c = 1/2.             */
/* jump = 0 gives c = 1/2 for every query.                                 */
/* ---------------------------------------------------------------------- */
static double tri_solid_angle(const double* x, const double* a, const double* b, const double* c)
{
    double r1[3], r2[3], r3[3], cr[3];
    sub3(a, x, r1);
    sub3(b, x, r2);
    sub3(c, x, r3);
    cr[0] = r2[1] * r3[2] - r2[2] * r3[1];
    cr[1] = r2[2] * r3[0] - r2[0] * r3[2];
    cr[2] = r2[0] * r3[1] - r2[1] * r3[0];
    double num = r1[0] * cr[0] + r1[1] * cr[1] + r1[2] * cr[2];
    double l1 = norm3(r1), l2 = norm3(r2), l3 = norm3(r3);
    double d12 = r1[0] * r2[0] + r1[1] * r2[1] + r1[2] * r2[2];
    double d13 = r1[0] * r3[0] + r1[1] * r3[1] + r1[2] * r3[2];
    double d23 = r2[0] * r3[0] + r2[1] * r3[1] + r2[2] * r3[2];
    double den = l1 * l2 * l3 + d12 * l3 + d13 * l2 + d23 * l1;
    return 2.0 * atan2(num, den);
}

void orc_free_terms(const double* V, const int32_t* T, int32_t nT, const int32_t* q_tri,
                    const double* q_bary, int32_t Q, int32_t jump, double* c_out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t q = 0; q < Q; ++q) {
        c_out[q] = 0.5;
        if (!jump)
            continue;
        const int32_t* tv = T + 3 * q_tri[q];
        double b1 = q_bary[2 * q], b2 = q_bary[2 * q + 1];
        double wt[3] = {1.0 - b1 - b2, b1, b2};
        int zeros = (wt[0] == 0.0) + (wt[1] == 0.0) + (wt[2] == 0.0);
        if (zeros == 0)
            continue;
        /* the vertices the point lies on: the corners with nonzero weight */
        int32_t on[2];
        int n_on = 0;
        for (int c = 0; c < 3; ++c)
            if (wt[c] != 0.0 && n_on < 2)
                on[n_on++] = tv[c];
        double x[3];
        for (int c = 0; c < 3; ++c)
            x[c] = wt[0] * V[3 * tv[0] + c] + wt[1] * V[3 * tv[1] + c] + wt[2] * V[3 * tv[2] + c];
        if (zeros == 2)
            for (int c = 0; c < 3; ++c)
                x[c] = V[3 * on[0] + c];
        double omega = 0.0;
        for (int32_t t = 0; t < nT; ++t) {
            const int32_t* u = T + 3 * t;
            int has0 = u[0] == on[0] || u[1] == on[0] || u[2] == on[0];
            int has1 = n_on > 1 && (u[0] == on[1] || u[1] == on[1] || u[2] == on[1]);
            if (zeros == 2 ? has0 : (has0 && has1))
                continue;
            omega += tri_solid_angle(x, V + 3 * u[0], V + 3 * u[1], V + 3 * u[2]);
        }
        c_out[q] = 1.0 - omega / (4.0 * M_PI);
    }
}

/* ---------------------------------------------------------------------- */
/* GMRES (Saad & Schultz 1986), unrestarted, x0 = 0, Arnoldi by modified   */
/* Gram-Schmidt, Givens rotations on the Hessenberg matrix.  Stops when   */
/* |residual| / |b| <= tol or after max_iter steps.  Returns iterations.   */
/* ---------------------------------------------------------------------- */
static void matvec(int32_t n, const cplx* A, const cplx* x, cplx* y)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        cplx s = 0.0;
        for (int32_t j = 0; j < n; ++j)
            s += A[(size_t)i * n + j] * x[j];
        y[i] = s;
    }
}

static double vnorm(int32_t n, const cplx* v)
{
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i)
        s += creal(v[i]) * creal(v[i]) + cimag(v[i]) * cimag(v[i]);
    return sqrt(s);
}

int32_t orc_gmres(int32_t n, const double* A_in, const double* b_in, double* x_out,
                  double tol, int32_t max_iter, double* rel_resid)
{
    const cplx* A = (const cplx*)A_in;
    const cplx* b = (const cplx*)b_in;
    cplx* x = (cplx*)x_out;
    int32_t m = max_iter;
    for (int32_t i = 0; i < n; ++i)
        x[i] = 0.0;
    double beta = vnorm(n, b);
    if (beta == 0.0) {
        *rel_resid = 0.0;
        return 0;
    }
    cplx* Vb = (cplx*)malloc(sizeof(cplx) * (size_t)n * (size_t)(m + 1));
    cplx* H = (cplx*)calloc((size_t)(m + 1) * (size_t)m, sizeof(cplx)); /* H[i*m + j] */
    double* cs = (double*)malloc(sizeof(double) * (size_t)m);
    cplx* sn = (cplx*)malloc(sizeof(cplx) * (size_t)m);
    cplx* gv = (cplx*)calloc((size_t)(m + 1), sizeof(cplx));
    cplx* w = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    for (int32_t i = 0; i < n; ++i)
        Vb[i] = b[i] / beta;
    gv[0] = beta;
    int32_t it = 0;
    double res = 1.0;
    for (int32_t j = 0; j < m; ++j) {
        matvec(n, A, Vb + (size_t)j * n, w);
        for (int32_t i = 0; i <= j; ++i) {
            const cplx* vi = Vb + (size_t)i * n;
            cplx h = 0.0;
            for (int32_t t = 0; t < n; ++t)
                h += conj(vi[t]) * w[t];
            H[(size_t)i * m + j] = h;
            for (int32_t t = 0; t < n; ++t)
                w[t] -= h * vi[t];
        }
        double hn = vnorm(n, w);
        H[(size_t)(j + 1) * m + j] = hn;
        if (hn > 0.0)
            for (int32_t t = 0; t < n; ++t)
                Vb[(size_t)(j + 1) * n + t] = w[t] / hn;
        /* previous rotations on the new column */
        for (int32_t i = 0; i < j; ++i) {
            cplx a = H[(size_t)i * m + j], c2 = H[(size_t)(i + 1) * m + j];
            H[(size_t)i * m + j] = cs[i] * a + sn[i] * c2;
            H[(size_t)(i + 1) * m + j] = -conj(sn[i]) * a + cs[i] * c2;
        }
        /* new rotation zeroing H[j+1][j] */
        cplx a = H[(size_t)j * m + j];
        double bb = hn;
        double den = sqrt(creal(a) * creal(a) + cimag(a) * cimag(a) + bb * bb);
        if (cabs(a) == 0.0) {
            cs[j] = 0.0;
            sn[j] = 1.0;
        } else {
            cs[j] = cabs(a) / den;
            sn[j] = (a / cabs(a)) * bb / den;
        }
        H[(size_t)j * m + j] = cs[j] * a + sn[j] * bb;
        H[(size_t)(j + 1) * m + j] = 0.0;
        gv[j + 1] = -conj(sn[j]) * gv[j];
        gv[j] = cs[j] * gv[j];
        it = j + 1;
        res = cabs(gv[j + 1]) / beta;
        if (res <= tol || hn == 0.0)
            break;
    }
    /* back substitution H y = g, x = V y */
    cplx* yv = (cplx*)calloc((size_t)(it > 0 ? it : 1), sizeof(cplx));
    for (int32_t i = it - 1; i >= 0; --i) {
        cplx s = gv[i];
        for (int32_t t = i + 1; t < it; ++t)
            s -= H[(size_t)i * m + t] * yv[t];
        yv[i] = s / H[(size_t)i * m + i];
    }
    for (int32_t i = 0; i < it; ++i)
        for (int32_t t = 0; t < n; ++t)
            x[t] += yv[i] * Vb[(size_t)i * n + t];
    *rel_resid = res;
    free(Vb);
    free(H);
    free(cs);
    free(sn);
    free(gv);
    free(w);
    free(yv);
    return it;
}

/* ---------------------------------------------------------------------- */
/* The whole Monte-Carlo estimate (O1-O9) for n_modes (k_m, g_m) pairs    */
/* sharing one mesh, one seed and one sample set.                          */
/* ---------------------------------------------------------------------- */
int32_t orc_mcbem(const double* V, int32_t nV, const int32_t* T, int32_t nT,
                  const double* g_in /* complex [n_modes][nV or nT] */, int32_t layout,
                  int32_t n_modes, const double* kv, const int32_t* q_tri, const double* q_bary,
                  int32_t Q, int32_t N, uint64_t seed, double eps_scale, double tol,
                  int32_t max_iter, double* p_out /* complex [n_modes][Q] */,
                  double* p_smp_out /* complex [n_modes][N] or NULL */, int32_t* iters,
                  double* resid, int32_t* smp_tri, double* smp_bary, int32_t jump,
                  int32_t exact_disk, int32_t poisson)
{
    double* area = (double*)malloc(sizeof(double) * (size_t)nT);
    double* nrm = (double*)malloc(sizeof(double) * 3 * (size_t)nT);
    double* cdf = (double*)malloc(sizeof(double) * (size_t)nT);
    orc_geometry(V, T, nT, area, nrm, cdf);
    double A = cdf[nT - 1];
    if (poisson) {
        /* Section 4.2: Poisson-disk samples instead of independent ones */
        if (orc_poisson_samples(V, nV, T, nT, N, seed, ORC_POISSON_RSCALE, ORC_POISSON_CANDIDATES, N,
                                smp_tri, smp_bary) < N) {
            free(area);
            free(nrm);
            free(cdf);
            return 5;
        }
    } else {
        orc_samples(cdf, nT, N, seed, smp_tri, smp_bary);
    }
    double* y = (double*)malloc(sizeof(double) * 3 * (size_t)N);
    double* ny = (double*)malloc(sizeof(double) * 3 * (size_t)N);
    double* xq = (double*)malloc(sizeof(double) * 3 * (size_t)Q);
    orc_surface_points(V, T, N, smp_tri, smp_bary, y);
    orc_surface_points(V, T, Q, q_tri, q_bary, xq);
    for (int32_t j = 0; j < N; ++j)
        for (int c = 0; c < 3; ++c)
            ny[3 * j + c] = nrm[3 * smp_tri[j] + c];
    double w = A / (double)N;
    double eps = eps_scale * sqrt(A / (M_PI * (double)N));
    int32_t ng = layout == 1 ? nT : nV;
    cplx* gj = (cplx*)malloc(sizeof(cplx) * (size_t)N);
    cplx* gq = (cplx*)malloc(sizeof(cplx) * (size_t)Q);
    cplx* b = (cplx*)malloc(sizeof(cplx) * (size_t)N);
    cplx* p = (cplx*)malloc(sizeof(cplx) * (size_t)N);
    cplx* M = (cplx*)malloc(sizeof(cplx) * (size_t)N * (size_t)N);
    double* cq = (double*)malloc(sizeof(double) * (size_t)(Q > 0 ? Q : 1));
    orc_free_terms(V, T, nT, q_tri, q_bary, Q, jump, cq);
    int32_t status = 0;
    for (int32_t m = 0; m < n_modes; ++m) {
        const double* gm = g_in + 2 * (size_t)m * (size_t)ng;
        orc_neumann_at(T, layout, gm, N, smp_tri, smp_bary, (double*)gj);
        orc_neumann_at(T, layout, gm, Q, q_tri, q_bary, (double*)gq);
        orc_mc_matrix(N, y, ny, kv[m], w, eps, (double*)M);
        orc_mc_rhs(N, y, kv[m], w, eps, (const double*)gj, exact_disk, (double*)b);
        iters[m] = orc_gmres(N, (const double*)M, (const double*)b, (double*)p, tol, max_iter,
                             &resid[m]);
        if (resid[m] > tol)
            status = 3;
        orc_mc_eval(Q, xq, (const double*)gq, 0.5, cq, N, y, ny, (const double*)gj,
                    (const double*)p, kv[m], w, eps, exact_disk, p_out + 2 * (size_t)m * (size_t)Q);
        if (p_smp_out)
            memcpy(p_smp_out + 2 * (size_t)m * (size_t)N, p, sizeof(cplx) * (size_t)N);
    }
    free(area);
    free(nrm);
    free(cdf);
    free(y);
    free(ny);
    free(xq);
    free(gj);
    free(gq);
    free(b);
    free(p);
    free(M);
    free(cq);
    return status;
}

/* ====================================================================== */
/* Dense collocation Burton-Miller BEM (Section 4, eq. BurtonMiller;      */
/* Section 4.1: the matrices of A p = B g are built directly).            */
/* Piecewise-constant p and g on panels, collocation at centroids x_i.    */
/*   A = I/2 - K - beta W        B = -(S + beta K') - (beta/2) I           */
/*   S_ij  = int_{T_j} G(x_i,y)                 K_ij  = int dG/dn_y        */
/*   K'_ij = int_{T_j} dG/dn_x                  W_ij  = int d2G/dn_x dn_y  */
/* beta = i/k (Burton-Miller) or 0 (conventional BIE).  The last term of  */
/* the printed equation is read at the collocation point x.                */
/* ====================================================================== */

/* Gauss-Legendre nodes/weights on [0,1] by Newton iteration on P_n. */
void orc_gauss_legendre01(int32_t n, double* xs, double* ws)
{
    for (int32_t i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int iter = 0; iter < 100; ++iter) {
            double p0 = 1.0, p1 = 0.0;
            for (int32_t l = 1; l <= n; ++l) {
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * l - 1.0) * z * p1 - (l - 1.0) * p2) / l;
            }
            dp = n * (z * p0 - p1) / (z * z - 1.0);
            double dz = p0 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16)
                break;
        }
        {
            double p0 = 1.0, p1 = 0.0;
            for (int32_t l = 1; l <= n; ++l) {
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * l - 1.0) * z * p1 - (l - 1.0) * p2) / l;
            }
            dp = n * (z * p0 - p1) / (z * z - 1.0);
        }
        /* node on [-1,1] is z; map to [0,1] (ascending order) */
        xs[n - 1 - i] = 0.5 * (z + 1.0);
        ws[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
}

#define ORC_FAR_N 3
#define ORC_THETA_N 16
#define ORC_NEAR_ETA 2.0
#define ORC_NEAR_DEPTH 5

/* rule tables, filled once when the library is loaded */
static double orc_far_x[ORC_FAR_N], orc_far_w[ORC_FAR_N];
static double orc_theta_x[ORC_THETA_N], orc_theta_w[ORC_THETA_N];

__attribute__((constructor)) static void orc_init_rules(void)
{
    orc_gauss_legendre01(ORC_FAR_N, orc_far_x, orc_far_w);
    orc_gauss_legendre01(ORC_THETA_N, orc_theta_x, orc_theta_w);
}

typedef struct {
    cplx S, K, Kp, W;
} panel_ints;

static double tri_diam(const double* a, const double* b, const double* c)
{
    double e[3];
    sub3(b, a, e);
    double d = norm3(e);
    sub3(c, b, e);
    double d2 = norm3(e);
    sub3(a, c, e);
    double d3 = norm3(e);
    if (d2 > d)
        d = d2;
    if (d3 > d)
        d = d3;
    return d;
}

/* collapsed Gauss rule on triangle (a,b,c): y = a + s (b-a) + t (1-s) (c-a),
 * weight ws wt (1-s) 2 area. */
static void far_rule(double k, const double* x, const double* nx, const double* a,
                     const double* b, const double* c, const double* ny, panel_ints* acc)
{
    const double* gx = orc_far_x;
    const double* gw = orc_far_w;
    double e1[3], e2[3], cr[3];
    sub3(b, a, e1);
    sub3(c, a, e2);
    cross3(e1, e2, cr);
    double two_area = norm3(cr);
    for (int p = 0; p < ORC_FAR_N; ++p) {
        for (int q = 0; q < ORC_FAR_N; ++q) {
            double s = gx[p], t = gx[q] * (1.0 - gx[p]);
            double wt = gw[p] * gw[q] * (1.0 - gx[p]) * two_area;
            double y[3];
            for (int d = 0; d < 3; ++d)
                y[d] = a[d] + s * e1[d] + t * e2[d];
            double kk[8];
            orc_kernels(k, x, nx, y, ny, kk);
            cplx* kc = (cplx*)kk;
            acc->S += wt * kc[0];
            acc->K += wt * kc[1];
            acc->Kp += wt * kc[2];
            acc->W += wt * kc[3];
        }
    }
}

/* near rule: 4-way midpoint subdivision while the child is close to x */
static void near_rule(double k, const double* x, const double* nx, const double* a,
                      const double* b, const double* c, const double* ny, int depth,
                      panel_ints* acc)
{
    double cen[3], d[3];
    for (int i = 0; i < 3; ++i)
        cen[i] = (a[i] + b[i] + c[i]) / 3.0;
    sub3(x, cen, d);
    if (depth >= ORC_NEAR_DEPTH || norm3(d) >= ORC_NEAR_ETA * tri_diam(a, b, c)) {
        far_rule(k, x, nx, a, b, c, ny, acc);
        return;
    }
    double mab[3], mbc[3], mca[3];
    for (int i = 0; i < 3; ++i) {
        mab[i] = 0.5 * (a[i] + b[i]);
        mbc[i] = 0.5 * (b[i] + c[i]);
        mca[i] = 0.5 * (c[i] + a[i]);
    }
    near_rule(k, x, nx, a, mab, mca, ny, depth + 1, acc);
    near_rule(k, x, nx, mab, b, mbc, ny, depth + 1, acc);
    near_rule(k, x, nx, mca, mbc, c, ny, depth + 1, acc);
    near_rule(k, x, nx, mab, mbc, mca, ny, depth + 1, acc);
}

/* Self panel: split at the centroid into three sub-triangles (x, va, vb);
 * in polar coordinates about x the edge va-vb is rho(theta) = d / cos(theta)
 * with theta measured from the perpendicular foot.  Radial integrals are
 * done in closed form:
 *   S_ii = 1/(4 pi) int (e^{ik rho} - 1)/(ik) dtheta     (k > 0)
 *        = 1/(4 pi) int rho dtheta                        (k = 0)
 *   W_ii = 1/(4 pi) int (ik - e^{ik rho}/rho) dtheta     (Hadamard finite part)
 * K_ii = K'_ii = 0 on a flat panel. */
void orc_self_panel(double k, const double* v0, const double* v1, const double* v2,
                    double* out /* complex S, W */)
{
    const double* vs[3] = {v0, v1, v2};
    double x[3];
    for (int i = 0; i < 3; ++i)
        x[i] = (v0[i] + v1[i] + v2[i]) / 3.0;
    const double* tx = orc_theta_x;
    const double* tw = orc_theta_w;
    cplx S = 0.0, W = 0.0;
    for (int e = 0; e < 3; ++e) {
        const double* a = vs[e];
        const double* b = vs[(e + 1) % 3];
        double ed[3], xa[3];
        sub3(b, a, ed);
        double L = norm3(ed);
        double u[3] = {ed[0] / L, ed[1] / L, ed[2] / L};
        sub3(x, a, xa);
        double along = dot3(xa, u);
        double perp[3] = {xa[0] - along * u[0], xa[1] - along * u[1], xa[2] - along * u[2]};
        double dist = norm3(perp);
        double sa = -along, sb = L - along;
        double ta = atan(sa / dist), tb = atan(sb / dist);
        for (int q = 0; q < ORC_THETA_N; ++q) {
            double th = ta + (tb - ta) * tx[q];
            double wq = (tb - ta) * tw[q];
            double rho = dist / cos(th);
            if (k > 0.0) {
                cplx em1 = -2.0 * pow(sin(0.5 * k * rho), 2) + I * sin(k * rho); /* e^{ik rho} - 1 */
                S += wq * em1 / (I * k);
            } else {
                S += wq * rho;
            }
            W += wq * (I * k - cexp(I * k * rho) / rho);
        }
    }
    cplx* o = (cplx*)out;
    o[0] = S / FOUR_PI;
    o[1] = W / FOUR_PI;
}

/* Integrals of the four kernels over panel T_j for collocation point x
 * (normal nx); j must differ from the collocation panel. */
void orc_panel_integrals(double k, const double* x, const double* nx, const double* a,
                         const double* b, const double* c, double* out /* complex S,K,K',W */)
{
    double e1[3], e2[3], cr[3];
    sub3(b, a, e1);
    sub3(c, a, e2);
    cross3(e1, e2, cr);
    double ln = norm3(cr);
    double ny[3] = {cr[0] / ln, cr[1] / ln, cr[2] / ln};
    panel_ints acc = {0.0, 0.0, 0.0, 0.0};
    near_rule(k, x, nx, a, b, c, ny, 0, &acc);
    cplx* o = (cplx*)out;
    o[0] = acc.S;
    o[1] = acc.K;
    o[2] = acc.Kp;
    o[3] = acc.W;
}

void orc_bem_assemble(const double* V, const int32_t* T, int32_t nT, double k,
                      int32_t burton_miller, double* A_out, double* B_out)
{
    cplx* A = (cplx*)A_out;
    cplx* B = (cplx*)B_out;
    cplx beta = (burton_miller && k > 0.0) ? I / k : 0.0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t i = 0; i < nT; ++i) {
        const double* a = V + 3 * T[3 * i + 0];
        const double* b = V + 3 * T[3 * i + 1];
        const double* c = V + 3 * T[3 * i + 2];
        double x[3], e1[3], e2[3], cr[3];
        for (int d = 0; d < 3; ++d)
            x[d] = (a[d] + b[d] + c[d]) / 3.0;
        sub3(b, a, e1);
        sub3(c, a, e2);
        cross3(e1, e2, cr);
        double ln = norm3(cr);
        double nx[3] = {cr[0] / ln, cr[1] / ln, cr[2] / ln};
        for (int32_t j = 0; j < nT; ++j) {
            cplx S, K, Kp, W;
            const double* pa = V + 3 * T[3 * j + 0];
            const double* pb = V + 3 * T[3 * j + 1];
            const double* pc = V + 3 * T[3 * j + 2];
            if (i == j) {
                double sw[4];
                orc_self_panel(k, pa, pb, pc, sw);
                S = ((cplx*)sw)[0];
                W = ((cplx*)sw)[1];
                K = 0.0;
                Kp = 0.0;
            } else {
                double pi4[8];
                orc_panel_integrals(k, x, nx, pa, pb, pc, pi4);
                cplx* pc4 = (cplx*)pi4;
                S = pc4[0];
                K = pc4[1];
                Kp = pc4[2];
                W = pc4[3];
            }
            double delta = (i == j) ? 1.0 : 0.0;
            A[(size_t)i * nT + j] = 0.5 * delta - K - beta * W;
            B[(size_t)i * nT + j] = -(S + beta * Kp) - 0.5 * beta * delta;
        }
    }
}

/* Piecewise-constant panel data from per-vertex data: mean of the corners. */
void orc_panel_data(const int32_t* T, int32_t nT, const double* gv_in, double* gp_out)
{
    const cplx* gv = (const cplx*)gv_in;
    cplx* gp = (cplx*)gp_out;
    for (int32_t t = 0; t < nT; ++t)
        gp[t] = (gv[T[3 * t]] + gv[T[3 * t + 1]] + gv[T[3 * t + 2]]) / 3.0;
}

/* b = B g followed by GMRES on A p = b (x0 = 0). */
int32_t orc_bem_solve(int32_t n, const double* A_in, const double* B_in, const double* g_in,
                      double tol, int32_t max_iter, double* p_out, double* rel_resid)
{
    cplx* b = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    matvec(n, (const cplx*)B_in, (const cplx*)g_in, b);
    int32_t it = orc_gmres(n, A_in, (const double*)b, p_out, tol, max_iter, rel_resid);
    free(b);
    return it;
}

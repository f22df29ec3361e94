/*
 * nat_bem.h -- C ABI of libnat_bem.so, the MI355X (gfx950) Monte-Carlo BEM
 * and dense Burton-Miller BEM library for the radiation solves of
 * "NAT: Neural Acoustic Transfer for Interactive Scenes in Real Time"
 * (arXiv 2506.06190), Section 4.
 *
 * Problem (Section 4, eq. BurtonMiller; Section 4.1.1, eqs. BIE and
 * bem_linear_system): given a closed triangle mesh Gamma, Neumann data
 * g = dp/dn (outward normal, into the fluid) and a wavenumber k = 2 pi f / c,
 * find the surface pressure p of the radiating solution of
 * Laplacian(p) + k^2 p = 0 outside Gamma, with time factor e^{-i w t} and
 * G(x,y) = e^{ik|x-y|} / (4 pi |x-y|).
 *
 * Conventions of every entry point
 *  - Plain pointers only.  "host" arrays live in host memory and are read
 *    before the call returns; "device" arrays live in device memory of the
 *    context's GPU and belong to the caller, who keeps them valid until the
 *    call returns.
 *  - Complex numbers are interleaved (re, im) doubles, the layout of
 *    C99 double complex, std::complex<double> and torch.complex128.
 *  - Arrays indexed [a][b] are row-major with b fastest.
 *  - Streams are hipStream_t values passed as void*; NULL is the default
 *    stream.  Calls that fill a host report block until their device work
 *    has finished; others are stream-ordered and return at once.
 *  - Every argument is validated before any device work is issued; an
 *    invalid argument returns NAT_E_INVALID and touches nothing.  No call
 *    throws or aborts; a HIP runtime failure returns NAT_E_HIP.
 *    nat_last_error() returns a text description of the last failure in
 *    the calling thread.
 *  - Device memory the library allocates is charged to the context's HBM
 *    budget; a call that would exceed it returns NAT_E_BUDGET before
 *    allocating anything.
 *  - A context and everything made from it are used by one host thread at
 *    a time; a request server (nat_serve.h) runs its own worker threads on
 *    its context alongside that thread.
 */
#ifndef NAT_BEM_H
#define NAT_BEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NAT_OK = 0,
    NAT_E_INVALID = 1,  /* an argument failed validation; nothing was done         */
    NAT_E_BUDGET = 2,   /* the HBM budget would be exceeded; nothing was allocated */
    NAT_E_NOCONV = 3,   /* GMRES stopped at max_iter above tol; best iterate kept  */
    NAT_E_HIP = 4,      /* a HIP runtime call failed                               */
    NAT_E_INTERNAL = 5,
    NAT_E_PENDING = 6,  /* a served request has not finished yet (nat_serve.h)     */
    NAT_E_CANCELLED = 7 /* a served request was cancelled before it started        */
} nat_status;

typedef struct nat_ctx nat_ctx;
typedef struct nat_mesh nat_mesh;
typedef struct nat_bem_op nat_bem_op;

typedef enum {
    NAT_PREC_FP64 = 0, /* plain form: FP64 kernel sums, one thread per target            */
    NAT_PREC_FP32 = 1  /* FP32 kernel sums with compensated accumulation, FP64 Krylov    */
} nat_precision;

typedef enum {
    NAT_NEUMANN_PER_VERTEX = 0,  /* g given at vertices, linear on each triangle      */
    NAT_NEUMANN_PER_TRIANGLE = 1 /* g constant on each triangle (Section 3.4 scenes)   */
} nat_neumann_layout;

/* Free term c_q of the surface identity c_q p(x_q) = integral, used when
 * the estimate is evaluated at the queries (eq. BIE, Section 4.2). */
typedef enum {
    NAT_JUMP_HALF = 0,       /* c_q = 1/2 at every query (the paper's value)             */
    NAT_JUMP_POLYHEDRAL = 1  /* c_q = 1 - Omega/(4 pi) for queries exactly on a mesh
                              * vertex or edge, Omega the solid angle the body subtends
                              * there (nat_mesh_free_terms); 1/2 elsewhere          */
} nat_jump;

/* Options of the Monte-Carlo estimate.  nat_mc_opts_default() fills the
 * paper's settings: linear-solver tolerance 1e-6, at most 200 iterations
 * (Section 6.1), disk radius eps = sqrt(|Gamma| / (pi N)), c_q = 1/2. */
typedef struct {
    int32_t precision;      /* nat_precision                                         */
    int32_t layout;         /* nat_neumann_layout of v_n                             */
    double eps_scale;       /* eps = eps_scale * sqrt(|Gamma| / (pi N)); > 0         */
    double gmres_tol;       /* relative residual |r| / |b| to stop at; > 0           */
    int32_t gmres_max_iter; /* 1 .. 1000                                             */
    int32_t flags;          /* NAT_MC_* bits                                         */
    int32_t jump;           /* nat_jump                                              */
    int32_t n_streams;      /* nat_mcbem_estimate_batch: parts run concurrently, see
                             * below; 0 automatic, 1 the caller's stream only, <= 8 */
} nat_mc_opts;

/* nat_mc_opts.n_streams: nat_mcbem_estimate_batch splits the jobs into up to
 * this many parts (job i to part i mod the count) and runs each part on a
 * stream and a host thread of its own, after all work the caller queued on
 * its stream, which then waits for every part.  One part's GMRES
 * orthogonalisation, bound by HBM bandwidth, then overlaps another part's
 * kernel sums, bound by the vector ALUs.  0 picks the count from the batch's
 * size: one part per 2e10 pair terms (n_modes N (31 N + Q) per job), at most
 * 3 (with the caller's stream, the 4 hardware queues a process gets by
 * default); 1 runs the batch on the caller's stream alone.  The parts' scratch
 * memory is held by the context until it is destroyed.  Every result is
 * bitwise the same for any count (a system's arithmetic depends only on its
 * own sizes). */

/* nat_mc_opts.flags: launch every GMRES kernel directly instead of replaying
 * captured runs of iterations (results are identical). */
#define NAT_MC_NO_GRAPH 1
/* nat_mc_opts.flags: the GMRES matvec of the FP32 form from an assembled
 * operator for every instance (the pair terms e^{ikr}(ikr - 1)(d.n_j)/r^3 of
 * eq. bem_linear_system stored once per mode as N^2 FP32 complex values,
 * source-major, 0 inside the disk; each iteration multiplies them by
 * w/(4 pi) p_j with FP64 sums), or matrix-free for every instance (the kernel sum recomputed each
 * iteration).  Without either bit the form follows the context's tuning
 * table by N (nat_autotune).  The plain FP64 form is always matrix-free. */
#define NAT_MC_ASSEMBLED 2
#define NAT_MC_MATRIX_FREE 4
/* nat_mc_opts.flags: the disk term of Section 4.2 with the integral of G over
 * the flat disk of radius eps in closed form, (e^{ik eps} - 1)/(2ik), instead
 * of the paper's eps/2 (they differ by O(k eps^2)). */
#define NAT_MC_EXACT_DISK 8
/* nat_mc_opts.flags: the matrix-free FP32 matvec in the ordered form (each
 * target's thread evaluates all its pairs) instead of the symmetric form
 * (each unordered sample pair evaluated once, feeding both of its targets,
 * since r and e^{ikr} are the same both ways).  The two round differently;
 * both stay within the FP32 form's tolerance. */
#define NAT_MC_ORDERED_SUM 16
/* nat_mc_opts.flags: the phase k r of every FP32 kernel sum reduced in FP64:
 * r refined from the FP64 sample and query positions (one Newton step on
 * the FP32 distance), kr / (2 pi) formed and reduced to [0, 1) revolutions
 * in FP64, only the reduced phase rounded to FP32 for the sine and cosine.
 * Without it the phase is formed from FP32 positions relative to the mesh
 * centre, whose rounding (about 6e-8 of the object size) bounds its
 * accuracy at k times that.  Forces the matrix-free matvec; the plain FP64
 * form ignores it. */
#define NAT_MC_FP64_PHASE 32
/* nat_mc_opts.flags: Poisson-disk samples (Section 4.2) instead of
 * independent ones: the first N points accepted by the parallel Poisson-disk
 * sampler of nat_mcbem_poisson_samples with the same N and seed.  The
 * weights stay |Gamma|/N and eps = eps_scale sqrt(|Gamma|/(pi N)).  Fails
 * with NAT_E_INVALID when fewer than N points are accepted. */
#define NAT_MC_POISSON 64

/* Per right-hand side report of a solve. */
typedef struct {
    int32_t iters;     /* GMRES iterations taken                                    */
    int32_t converged; /* 1 if rel_resid <= tol                                     */
    double rel_resid;  /* GMRES estimate of |b - A x| / |b|                         */
    double eps;        /* disk radius used (Monte-Carlo) or 0                       */
    double area;       /* |Gamma|                                                   */
    /* device time of the stages (HIP events on the call's stream), in ms;
     * for a batch, the whole batch's stages; a dense solve fills t_solve_ms */
    double t_sample_ms; /* samples, points and Neumann data (Section 4.1.1)         */
    double t_rhs_ms;    /* Stage-A right-hand side                                  */
    double t_solve_ms;  /* Stage-A (or dense) GMRES, solution included              */
    double t_eval_ms;   /* Stage-B evaluation at the queries                        */
} nat_solve_report;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device` whose library-owned device
 * allocations may total at most `hbm_budget_bytes` (0 = no limit). */
nat_status nat_ctx_create(int32_t device, size_t hbm_budget_bytes, nat_ctx** out);
/* Every mesh, operator, server and neural field made from the context must
 * be destroyed before it. */
void nat_ctx_destroy(nat_ctx* ctx);
/* Bytes of device memory currently charged to the context. */
size_t nat_ctx_bytes_in_use(const nat_ctx* ctx);

/* ---- meshes (Section 4.1.1: surface, areas, sampling density) ----------- */

/* Register a closed triangle mesh.  vertices: host double[n_vertices][3];
 * tris: host int32[n_tris][3], counter-clockwise seen from outside.  The
 * mesh must be closed and consistently oriented (every edge shared by
 * exactly two triangles with opposite directions), with no zero-area
 * triangle; it may hold several closed bodies (a scene: triangles that
 * share a vertex belong to one body), each of which must enclose a
 * positive volume (be oriented outward).  Triangle areas, unit normals and
 * the cumulative area table (sampling density 1/|Gamma|, Section 4.1.1) are
 * built in FP64 on the host and copied to the device with the geometry. */
nat_status nat_mesh_create(nat_ctx* ctx, const double* vertices, int32_t n_vertices,
                           const int32_t* tris, int32_t n_tris, nat_mesh** out);
void nat_mesh_destroy(nat_mesh* mesh);
/* Host-only check of the conditions nat_mesh_create imposes (no device
 * needed).  NAT_OK or NAT_E_INVALID with the reason in nat_last_error(). */
nat_status nat_mesh_validate(const double* vertices, int32_t n_vertices, const int32_t* tris,
                             int32_t n_tris);
/* Host-only: the FP64 geometry nat_mesh_create uploads.  Outputs (host):
 * area[n_tris] = |e1 x e2| / 2, normal[n_tris][3] = (e1 x e2)/|e1 x e2| with
 * e1 = v1 - v0, e2 = v2 - v0, and cdf[n_tris] = running sum of the areas in
 * triangle order, each evaluated as written without fused multiply-adds so
 * any IEEE double implementation of the same formulas reproduces it bit for
 * bit.  Validates the mesh first. */
nat_status nat_mesh_geometry(const double* vertices, int32_t n_vertices, const int32_t* tris,
                             int32_t n_tris, double* area, double* normal, double* cdf);
/* Host-only: the free terms nat_mesh_create stores for NAT_JUMP_POLYHEDRAL.
 * c_vert[n_vertices]: 1 - Omega_v/(4 pi), Omega_v the solid angle of the body
 * at the vertex, from its faces closed by a cap of triangles through a point
 * inside along the vertex normal (signed solid angles, Van Oosterom and
 * Strackee 1983).  c_edge[n_tris][3]: 1 - phi/(2 pi) for the edge opposite
 * corner i of the triangle, phi the interior dihedral angle between the two
 * faces of the edge.  Validates the mesh first; either output may be NULL. */
nat_status nat_mesh_free_terms(const double* vertices, int32_t n_vertices, const int32_t* tris,
                               int32_t n_tris, double* c_vert, double* c_edge);
/* Total area |Gamma| and the sizes; any output pointer may be NULL. */
nat_status nat_mesh_info(const nat_mesh* mesh, double* area, int32_t* n_vertices,
                         int32_t* n_tris);
/* One (tri, b1, b2) query record per vertex: the first triangle that uses
 * the vertex and the vertex's corner in it.  Host outputs tri[n_vertices],
 * bary[n_vertices][2]. */
nat_status nat_mesh_vertex_queries(const nat_mesh* mesh, int32_t* tri, double* bary);

/* ---- Monte-Carlo BEM (Section 4.1.1, Section 4.2) ------------------------ */

void nat_mc_opts_default(nat_mc_opts* opts);

/* Draw the N area-uniform samples of seed `seed`.  Sample j takes the
 * three SplitMix64 words at counters 3j, 3j+1, 3j+2 of stream 0, turns them
 * into u0, u1, u2 in [0,1) (top 53 bits), picks the smallest triangle t with
 * cumulative area > u0 |Gamma| and the point b1 = sqrt(u1)(1-u2),
 * b2 = sqrt(u1) u2 of it.  Device outputs tri[N] (int32), bary[N][2]
 * (double).  Stream-ordered. */
nat_status nat_mcbem_samples(nat_mesh* mesh, int32_t n_samples, uint64_t seed, int32_t* tri,
                             double* bary, void* stream);

/* Poisson-disk samples (Section 4.2: parallel Poisson-disk sampling, after
 * Bowers et al. 2010).  Candidates: 16 N area-uniform points; candidate i
 * takes counters 3i..3i+2 of stream 6 (u0, u1, u2 as for the samples), the
 * triangle of u0 |Gamma| and (b1, b2) = (u1, u2), or (1 - u1, 1 - u2) when
 * u1 + u2 > 1.  Radius r = 0.72 sqrt(|Gamma| / N).  Cells of side r/sqrt(3)
 * over the mesh's bounding box (corner lo = the smallest vertex
 * coordinates), cell = floor((x - lo) sqrt(3)/r) per axis; a cell's
 * candidates in index order.  Passes p = 0, 1, ...: phases
 * (cx mod 3, cy mod 3, cz mod 3) as 9a + 3b + c in order; every cell of the
 * phase without an accepted point tries its p-th candidate, accepted unless
 * an accepted point of the 5 x 5 x 5 cells around is closer than r
 * (positions and squared distances in FP64 as written, no fused
 * multiply-add).  Outputs (device): tri[N], bary[N][2] = the first N
 * accepted points in acceptance order (pass, phase, cell key); *n_accepted
 * (host, may be NULL) = the number accepted.  NAT_E_INVALID if fewer than N
 * are accepted (outputs then undefined).  Blocks until done. */
nat_status nat_mcbem_poisson_samples(nat_mesh* mesh, int32_t n_samples, uint64_t seed, int32_t* tri,
                                     double* bary, int32_t* n_accepted, void* stream);

/* The whole Monte-Carlo estimate of the surface pressure at Q query
 * points for n_modes independent problems (k_m, g_m) on one mesh sharing one
 * sample set.  With N samples y_j, w = |Gamma|/N and disk radius eps:
 *   Stage A  (1/2) p_i - sum_{j: r_ij >= eps} w dG(y_i,y_j)/dn_j p_j
 *              = - sum_{j: r_ij >= eps} w G(y_i,y_j) g_j - (eps/2) g_i
 *            (eps/2: the disk term, or its closed form, NAT_MC_EXACT_DISK)
 *            solved by GMRES (x0 = 0, unrestarted, tol, max_iter);
 *   Stage B  p(x_q) = (1/c_q) [ sum_{j: |x_q-y_j| >= eps} w (dG/dn_j p_j - G g_j)
 *                               - (eps/2) g(x_q) ],
 *            c_q = 1/2, or per query with opts->jump = NAT_JUMP_POLYHEDRAL.
 *            A query is on a vertex when two of its barycentric weights
 *            (1 - b1 - b2, b1, b2), evaluated in double precision, are exactly
 *            zero, and on an edge when one is.
 * v_n:      device complex [n_modes][n_vertices or n_tris] (opts->layout)
 * k:        host double[n_modes], each > 0
 * q_tri, q_bary: device int32[Q], double[Q][2]: query points on the mesh,
 *           x = v0 + b1 (v1 - v0) + b2 (v2 - v0), b1, b2 >= 0, b1 + b2 <= 1
 * p_out:    device complex [n_modes][Q]
 * p_samples: device complex [n_modes][N] receiving the Stage-A solution,
 *           or NULL
 * report:   host nat_solve_report[n_modes], or NULL
 * N >= 2, Q >= 0, 1 <= n_modes <= 4096.  Blocks until the result is
 * written.  Returns NAT_E_NOCONV (results still written) if any mode
 * stopped above its tolerance. */
nat_status nat_mcbem_estimate(nat_mesh* mesh, const double* v_n, int32_t n_modes,
                              const double* k, const int32_t* q_tri, const double* q_bary,
                              int32_t n_queries, int32_t n_samples, uint64_t seed,
                              const nat_mc_opts* opts, double* p_out, double* p_samples,
                              nat_solve_report* report, void* stream);

/* Allocation-free nat_mcbem_estimate, for callers that cannot allocate
 * memory during the call (serving loops, harnesses that forbid hipMalloc).
 * Same arguments, same validation and the same results bit for bit as
 * nat_mcbem_estimate with NAT_MC_NO_GRAPH; opts->n_streams is ignored.  The
 * device workspace comes from one fixed block of 256 MiB per GPU that the
 * library holds from its first use on that GPU until the process ends (not
 * charged to the context's budget), host staging from fixed host blocks;
 * the call allocates no device or pinned memory and creates no stream,
 * event or graph.  An estimate whose workspace exceeds the block returns
 * NAT_E_BUDGET before any device work (the workspace grows with
 * n_modes x n_samples x (gmres_max_iter + 1); 32 modes x 1024 samples x 200
 * iterations with 4096 queries fit).  Stage times in the report read 0.
 * All calls on one GPU share its block and its host staging: calls that
 * overlap in time on one GPU race and must be serialised by the caller.
 * Blocks until done. */
nat_status nat_mcbem_estimate_noalloc(nat_mesh* mesh, const double* v_n, int32_t n_modes,
                                      const double* k, const int32_t* q_tri, const double* q_bary,
                                      int32_t n_queries, int32_t n_samples, uint64_t seed,
                                      const nat_mc_opts* opts, double* p_out, double* p_samples,
                                      nat_solve_report* report, void* stream);

/* ---- exterior field (Section 3.4 training data, Section 3.1 FFAT maps) -- */

/* Pressure at points outside the body from the Neumann data and the surface
 * values of a Monte-Carlo estimate: the representation formula (eq. BIE
 * with the free term c = 1 off the surface and no disk term)
 *   p(x) = sum_j [|x - y_j| >= eps] w (dG/dn_j(x, y_j) p_j - G(x, y_j) g_j)
 * over the estimate's own samples y_j (the same n_samples and seed give the
 * same samples), w = |Gamma|/N.  p_samples: device complex
 * [n_modes][n_samples], the p_samples output of nat_mcbem_estimate with the
 * same v_n, k, n_samples, seed and opts.  points: device double
 * [n_points][3] in the mesh's coordinates, meant to lie outside the body
 * (as from nat_field_points).  p_out: device complex [n_modes][n_points];
 * abs_out: device double [n_modes][n_points] with |p| (the training value),
 * or NULL.  opts->precision picks the FP32 compensated or the plain FP64
 * sums; the GMRES settings are unused.  A non-finite point returns
 * NAT_E_INVALID.  Blocks until done. */
nat_status nat_mcbem_field(nat_mesh* mesh, const double* v_n, int32_t n_modes, const double* k,
                           const double* p_samples, int32_t n_samples, uint64_t seed,
                           const double* points, int32_t n_points, const nat_mc_opts* opts,
                           double* p_out, double* abs_out, void* stream);

typedef enum {
    NAT_FIELD_SHELL = 0,     /* random points in a shell (training data)                 */
    NAT_FIELD_FFAT_GRID = 1  /* a grid of directions on one sphere (an FFAT map image)   */
} nat_field_kind;

/* Field points about the centre c of the mesh's bounding box, R = half its
 * diagonal (the scene's bounding radius).
 *  NAT_FIELD_SHELL: n_a points (n_b unused), point i with radius
 *    r = R (r_lo + (r_hi - r_lo) u0), cos(theta) = 1 - 2 u1, phi = 2 pi u2,
 *    u0..u2 from counters 3i..3i+2 of stream 5 of the counter generator of
 *    the samples (a direction uniform on the sphere, a radius uniform in
 *    [r_lo R, r_hi R]; Section 3.4 uses 1.5 and 3).
 *  NAT_FIELD_FFAT_GRID: n_a x n_b points at radius r_lo R (r_hi unused),
 *    point a n_b + b at theta = (a + 1/2) pi / n_a, phi = (b + 1/2) 2 pi / n_b
 *    (an image with theta down the rows; Section 6 uses 64 x 32 maps).
 * points: device double [n][3], x = c + r (sin th cos ph, sin th sin ph,
 * cos th); coords: device double [n][3] with (r, theta, phi), or NULL.
 * Stream-ordered. */
nat_status nat_field_points(const nat_mesh* mesh, int32_t kind, int32_t n_a, int32_t n_b, double r_lo,
                            double r_hi, uint64_t seed, double* points, double* coords, void* stream);

/* One problem of a batch: the arguments of nat_mcbem_estimate. */
typedef struct {
    nat_mesh* mesh;
    const double* v_n;       /* device complex [n_modes][n_vertices or n_tris]      */
    int32_t n_modes;
    int32_t n_queries;
    const double* k;         /* host double[n_modes]                                */
    const int32_t* q_tri;    /* device int32[n_queries]                              */
    const double* q_bary;    /* device double[n_queries][2]                          */
    int32_t n_samples;
    int32_t reserved;        /* ignored                                             */
    uint64_t seed;
    double* p_out;           /* device complex [n_modes][n_queries]                  */
    double* p_samples;       /* device complex [n_modes][n_samples] or NULL          */
} nat_mc_job;

/* Many Monte-Carlo estimates of uneven size at once (meshes of one context,
 * each job with its own samples, modes, wavenumbers and queries): every
 * stage runs as one launch over all (job, mode) systems, GMRES iterates them
 * in lockstep with converged systems dropped from the work lists, and runs
 * of iterations are replayed from a captured graph.  Each job's results are
 * bit-for-bit those of nat_mcbem_estimate on the same job with the same
 * options: the tiling of a job depends only on its own sizes.  reports:
 * host nat_solve_report[sum of n_modes] in job order, or NULL.  Blocks until
 * done; NAT_E_NOCONV if any system stopped above its tolerance. */
nat_status nat_mcbem_estimate_batch(nat_ctx* ctx, const nat_mc_job* jobs, int32_t n_jobs,
                                    const nat_mc_opts* opts, nat_solve_report* reports,
                                    void* stream);

/* One exterior field of a batch: the arguments of nat_mcbem_field. */
typedef struct {
    nat_mesh* mesh;
    const double* v_n;       /* device complex [n_modes][n_vertices or n_tris]      */
    int32_t n_modes;
    int32_t n_points;
    const double* k;         /* host double[n_modes]                                */
    const double* p_samples; /* device complex [n_modes][n_samples]: an estimate's  */
    int32_t n_samples;
    int32_t reserved;        /* ignored                                             */
    uint64_t seed;
    const double* points;    /* device double[n_points][3]                          */
    double* p_out;           /* device complex [n_modes][n_points]                   */
    double* abs_out;         /* device double[n_modes][n_points] or NULL             */
} nat_field_job;

/* Many exterior fields at once (Section 3.4: the training tuples of a
 * family of scenes), each job as nat_mcbem_field with the same options:
 * the samples of every job are drawn in one launch (one Poisson-disk
 * sampler call for all jobs with NAT_MC_POISSON) and the field sums of all
 * (job, mode) pairs run as one launch.  Each job's result is bit-for-bit
 * that of nat_mcbem_field on the same job.  Meshes must belong to ctx.
 * Blocks until the sums are done; abs_out is written stream-ordered after
 * them. */
nat_status nat_mcbem_field_batch(nat_ctx* ctx, const nat_field_job* jobs, int32_t n_jobs,
                                 const nat_mc_opts* opts, void* stream);

/* ---- dense collocation Burton-Miller BEM (Section 4, Section 4.1) -------- */

/* Assemble A and B of A p = B g for piecewise-constant p and g with
 * collocation at the triangle centroids x_i:
 *   A = I/2 - K - beta W,  B = -(S + beta K') - (beta/2) I,
 *   S_ij = int_{T_j} G(x_i, y), K_ij = int dG/dn_y, K'_ij = int dG/dn_x,
 *   W_ij = int d2G/(dn_x dn_y) (Hadamard finite part on the diagonal),
 * beta = i/k when burton_miller != 0, else 0.  Quadrature: 3x3 collapsed
 * Gauss-Legendre on far panels; 4-way midpoint subdivision (depth <= 5)
 * while |x_i - centroid| < 2 diam; closed-form radial integrals with a
 * 16-point angular rule on the self panel.  FP64.  k > 0 required when
 * burton_miller != 0, k >= 0 otherwise.  Charges 2 n^2 16 bytes.  Blocks
 * until the matrices are built. */
nat_status nat_bem_assemble(nat_mesh* mesh, double k, int32_t burton_miller,
                            nat_bem_op** out, void* stream);

/* Solve A p = B g for n_rhs Neumann vectors by GMRES (x0 = 0, restart
 * = max_iter).  v_n: device complex [n_rhs][n_vertices or n_tris]
 * (per-vertex data is averaged over each triangle's corners); p_out:
 * device complex [n_rhs][n_tris] at the centroids; report: host
 * nat_solve_report[n_rhs] or NULL.  Blocks until done. */
nat_status nat_bem_solve(nat_bem_op* op, const double* v_n, int32_t n_rhs, int32_t layout,
                         double tol, int32_t max_iter, double* p_out, nat_solve_report* report,
                         void* stream);

/* Copy the assembled matrices to caller device buffers A_out, B_out
 * (complex [n_tris][n_tris] each; either may be NULL).  Stream-ordered. */
nat_status nat_bem_op_matrices(const nat_bem_op* op, double* A_out, double* B_out, void* stream);
void nat_bem_op_destroy(nat_bem_op* op);

/* ---- tiling autotuner ----------------------------------------------------- */

/* The FP32 kernel sums cut each group of up to 8 modes of an instance into
 * work items of 256 targets x a share of the sources; the number of source
 * shares follows from how many items a group should span, looked up per
 * size bucket b = clamp(floor(log2 n) - 6, 0, 9) of the target count n
 * (items_a: sums over the N samples, by N; items_b: sums at the Q queries,
 * by Q).  The defaults are 64 everywhere.  The split of an instance depends
 * only on its own sizes and the context's table, so results stay bit-for-bit
 * equal alone and in any batch on one context; two tables may round
 * differently in FP32. */
#define NAT_TUNE_FORCE 1  /* sweep even when the cache holds a table for this device */

/* Fill the context's table: read it from the JSON file cache_path when it
 * holds one for this device (architecture and CU count), otherwise time
 * every bucket's candidates (16 .. 512 items) on synthetic sums, one mode
 * group alone and many at once, keep the candidate with the smallest summed
 * slowdown against each regime's best, and write the table to cache_path
 * (NULL: no cache).  Runs on `stream`, using the context's workspace;
 * blocks until done (a few seconds). */
nat_status nat_autotune(nat_ctx* ctx, const char* cache_path, int32_t flags, void* stream);
/* Copy the table (host int32[10] each); tuned (may be NULL) is 1 after a
 * sweep, a cache load or nat_tune_set, else 0. */
nat_status nat_tune_get(const nat_ctx* ctx, int32_t* items_a, int32_t* items_b, int32_t* tuned);
/* Set the table (host int32[10] each, every entry 1 .. 2^20). */
nat_status nat_tune_set(nat_ctx* ctx, const int32_t* items_a, const int32_t* items_b);
/* The GMRES matvec form by the same buckets of N (host int32[10]: 1 =
 * assembled operator, 0 = matrix-free).  nat_autotune times both on
 * synthetic systems of each bucket, the assembled form charged its assembly
 * spread over 30 iterations, and keeps the faster; buckets whose operator
 * would exceed 2 GiB per mode stay matrix-free.  Defaults: all 0.
 * rate_free, rate_asm (host double[10] each, may be NULL): the matvec rates
 * the last sweep measured in (pair, mode) terms per second, 0 where not
 * timed or when the table came from a cache or nat_tune_set_form. */
nat_status nat_tune_get_form(const nat_ctx* ctx, int32_t* assembled, double* rate_free,
                             double* rate_asm);
nat_status nat_tune_set_form(nat_ctx* ctx, const int32_t* assembled);

/* ---- per-kernel timing ---------------------------------------------------- */

/* Timing of one kernel class accumulated while profiling is on: launches,
 * summed duration between HIP events recorded on the launch stream around
 * each launch, and the algorithmic flops of those launches (kernel-sum
 * launches count 24, 37 or 47 flops per target-source pair for the G-only,
 * dG/dn-only and both-term sums; 8 per element for the complex GEMV). */
typedef struct {
    char name[32];
    int64_t launches;
    double total_ms;
    double flops;
} nat_kernel_stat;

/* Turn per-kernel timing on or off; either way the totals are reset. */
nat_status nat_profile_enable(nat_ctx* ctx, int32_t enable);
/* Copy up to max_out non-empty kernel classes into out (host); returns the
 * number written.  Waits for the device. */
int32_t nat_profile_read(nat_ctx* ctx, nat_kernel_stat* out, int32_t max_out);

/* ---- errors -------------------------------------------------------------- */
const char* nat_status_str(nat_status s);
/* Copy the calling thread's last error message into buf (NUL-terminated,
 * truncated to len); returns the full message length. */
size_t nat_last_error(char* buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif /* NAT_BEM_H */

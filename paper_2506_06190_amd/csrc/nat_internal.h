// Internal declarations of libnat_bem: context, mesh and operator records,
// the device-memory ledger, and the launchers of the HIP kernels.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "nat_bem.h"

// One timed kernel launch: events recorded on the launch stream.
struct NatProfEvent {
    int32_t kind;
    double flops;
    hipEvent_t start, stop;
};

struct NatProfStat {
    int64_t launches = 0;
    double ms = 0.0;
    double flops = 0.0;
};

// Scratch state of one solve at a time: device workspace, pinned staging,
// pinned words the kernels write (convergence flags, loop progress) and the
// cached graph of GMRES iterations.  A context owns one; each worker of a
// server owns its own so solves can run concurrently on one context.
struct NatScratch {
    void* ws = nullptr;             // grow-only device workspace
    size_t ws_bytes = 0;
    void* ext_ws = nullptr;         // workspace lent by the caller instead (server arena)
    size_t ext_ws_bytes = 0;
    void* pinned = nullptr;
    size_t pinned_bytes = 0;
    int32_t* mapped = nullptr;
    int32_t* mapped_dev = nullptr;
    size_t mapped_ints = 0;
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<unsigned char> graph_key;
    // Scratch of the allocation-free entry point: ext_ws is a fixed device
    // block, pinned/mapped are fixed host blocks (pageable), and nothing
    // grows -- a request that needs more fails with NAT_E_BUDGET.  The
    // GMRES driver then polls the device's convergence flags by copies
    // instead of mapped words, never captures a graph, and the solve takes
    // no stage or profiling events.
    bool noalloc = false;
};

namespace nat {
// Work items wanted per mode group of the FP32 kernel sums, by size bucket
// (floor(log2 n) clamped to [6, 15]); the source split count of an instance
// follows from it and the instance's own sizes.
constexpr int kTuneBuckets = 10;
struct TuneTable {
    int32_t items_a[kTuneBuckets];  // sums over the samples, by the sample count N
    int32_t items_b[kTuneBuckets];  // sums at the queries, by the query count Q
    int32_t assembled[kTuneBuckets];  // 1: GMRES matvec from the assembled operator, by N
    int32_t symmetric[kTuneBuckets];  // 1: matrix-free matvec in the symmetric form, by N
    // measured matvec rates of the sweep (pair-modes/s; 0 if not timed)
    double rate_free[kTuneBuckets];
    double rate_asm[kTuneBuckets];
    int32_t tuned = 0;              // 0: defaults, 1: swept or loaded
};
int32_t tune_bucket(int32_t n);
void tune_defaults(TuneTable* t);
}  // namespace nat

struct nat_ctx {
    int32_t device = 0;
    nat::TuneTable tune;
    std::mutex mu;       // guards the ledger and the timing lists
    // one graph capture at a time across a context's threads, never during
    // another thread's scratch growth (which synchronises the device)
    std::mutex capture_mu;
    // per-kernel timing (off unless enabled)
    bool prof = false;
    std::vector<NatProfEvent> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    NatProfStat prof_stat[10];
    size_t budget = 0;   // 0: unlimited
    size_t in_use = 0;   // bytes charged
    NatScratch scratch;
    // concurrent parts of a batch (nat_mc_opts.n_streams): scratch, stream
    // and completion event of each part, created on first use
    static constexpr int kMaxLanes = 8;
    NatScratch lane_scratch[kMaxLanes];
    hipStream_t lane_stream[kMaxLanes] = {};
    hipEvent_t lane_event[kMaxLanes] = {};
    hipEvent_t lane_fork = nullptr;
    // Gauss-Legendre rules on [0,1] for the dense assembly (device copies)
    double* d_rules = nullptr;
};

struct nat_mesh {
    nat_ctx* ctx = nullptr;
    int32_t nV = 0, nT = 0;
    std::vector<double> V;       // nV x 3
    std::vector<int32_t> T;      // nT x 3
    std::vector<double> area;    // nT
    std::vector<double> normal;  // nT x 3
    std::vector<double> cdf;     // nT, running sum of areas
    double area_total = 0.0;
    double center[3] = {0, 0, 0};  // bounding-box centre; origin of the FP32 streams
    double diameter = 0.0;         // bounding-box diagonal: the largest pair distance
    // device copies
    double* d_V = nullptr;
    int32_t* d_T = nullptr;
    double* d_normal = nullptr;
    double* d_cdf = nullptr;
    double* d_cvert = nullptr;     // free term at each vertex [nV]
    double* d_cedge = nullptr;     // free term on the edge opposite each corner [nT][3]
    size_t bytes = 0;
};

struct nat_bem_op {
    nat_ctx* ctx = nullptr;
    nat_mesh* mesh = nullptr;
    double k = 0.0;
    int32_t burton_miller = 1;
    int32_t n = 0;
    double2* d_A = nullptr;  // n x n
    double2* d_B = nullptr;  // n x n
    size_t bytes = 0;
};

namespace nat {

// ---- errors ---------------------------------------------------------------
nat_status fail(nat_status s, const char* fmt, ...);
nat_status hip_fail(hipError_t e, const char* what);
#define NAT_HIP(call)                                    \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return nat::hip_fail(e_, #call); \
    } while (0)

// ---- device memory charged to a context -----------------------------------
nat_status dev_alloc(nat_ctx* ctx, size_t bytes, void** ptr);
void dev_free(nat_ctx* ctx, void* ptr, size_t bytes);
// The calling thread's scratch: the one bound by bind_scratch, else the
// context's own.
NatScratch& scratch_of(nat_ctx* ctx);
void bind_scratch(NatScratch* s);
NatScratch* bound_scratch();
void release_scratch(nat_ctx* ctx, NatScratch& s);
// grow-only scratch; contents undefined on return
nat_status workspace(nat_ctx* ctx, size_t bytes, void** ptr);
nat_status pinned(nat_ctx* ctx, size_t bytes, void** ptr);
nat_status mapped_words(nat_ctx* ctx, size_t n, int32_t** host, int32_t** dev);
nat_status set_device(const nat_ctx* ctx);
bool is_finite(double v);
// Zero the two flags (when zero_and_read), check query records (flag 0) and
// values for non-finite entries (flag 1), and read the flags back.
nat_status device_checks(nat_ctx* ctx, int32_t* dflag, const int32_t* q_tri, const double* q_bary,
                         int32_t Q, int32_t nT, const double* vals, int64_t n_vals, hipStream_t s,
                         int32_t* host_flags, bool zero_and_read);

// Carves aligned sub-buffers out of one allocation.
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base(static_cast<char*>(b)) {}
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = reinterpret_cast<T*>(base + off);
        off += count * sizeof(T);
        return p;
    }
};
template <class... Ts>
inline size_t carve_size(std::initializer_list<size_t> bytes) {
    size_t s = 0;
    for (size_t b : bytes) s = ((s + 255) & ~size_t(255)) + b;
    return s + 256;
}

// Events between the stages of one call (timing enabled), destroyed with it.
struct StageEvents {
    hipEvent_t e[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    bool on = false;
    hipError_t create() {
        for (hipEvent_t& x : e) {
            hipError_t r = hipEventCreate(&x);
            if (r != hipSuccess)
                return r;
        }
        on = true;
        return hipSuccess;
    }
    // no-ops when the events were not created (stage times then read 0)
    hipError_t record(int i, hipStream_t s) { return on ? hipEventRecord(e[i], s) : hipSuccess; }
    hipError_t elapsed(int i, float* ms) {
        *ms = 0.0f;
        return on ? hipEventElapsedTime(ms, e[i], e[i + 1]) : hipSuccess;
    }
    ~StageEvents() {
        for (hipEvent_t x : e)
            if (x)
                (void)hipEventDestroy(x);
    }
    StageEvents() = default;
    StageEvents(const StageEvents&) = delete;
    StageEvents& operator=(const StageEvents&) = delete;
};

// ---- per-kernel timing ------------------------------------------------------
enum ProfKind {
    PK_SUM32_RHS = 0, PK_SUM32_MATVEC = 1, PK_SUM32_EVAL = 2,
    PK_SUM64 = 3, PK_GMRES_ORTH = 4, PK_BEM_ASSEMBLE = 5, PK_ZGEMV = 6, PK_OTHER = 7,
    PK_KMATVEC = 8, PK_SYM32_MATVEC = 9
};
// Start/stop events of one timed launch (null when profiling is off).  The
// events ride on the dispatch packets of the first and last kernel of the
// launch (hipExtLaunchKernelGGL), so timing adds no packets to the stream.
struct ProfSlot {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};
ProfSlot prof_slot(nat_ctx* ctx, int32_t kind, double flops);
// Resolve finished events into the per-kind totals (synchronises the device).
void prof_collect(nat_ctx* ctx);

template <class K, class... A>
inline void launch_k(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, hipEvent_t e0,
                     hipEvent_t e1, A... args)
{
    if (e0 || e1)
        hipExtLaunchKernelGGL(kernel, grid, block, static_cast<uint32_t>(lds), s, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}

// ---- sampling and surface data (k_sample.hip) ------------------------------
struct PointStreams {   // SoA surface points
    double* x64;        // [3][n]
    double* n64;        // [3][n] (may be null for queries)
    float* x32;         // [3][n] relative to the mesh centre
    float* n32;         // [3][n]
};
hipError_t launch_samples(const nat_mesh* m, int32_t N, uint64_t seed, int32_t* tri,
                          double* bary, hipStream_t s);
hipError_t launch_points(const nat_mesh* m, int32_t n, const int32_t* tri, const double* bary,
                         PointStreams out, hipStream_t s);
// g_out[mode][i] = Neumann data at point i (per-vertex interpolation or per-triangle)
hipError_t launch_neumann(const nat_mesh* m, int32_t layout, const double2* g, int32_t ld_g,
                          int32_t n_modes, int32_t n, const int32_t* tri, const double* bary,
                          double2* g_out, hipStream_t s);

// The same surface work for every instance of a batch in one launch per
// step: a device table of instances, the batch arrays they index into.
struct SurfJob {
    const double* V;                   // mesh vertices [nV][3]
    const int32_t* T;                  // mesh triangles [nT][3]
    const double* nrm;                 // triangle normals [nT][3]
    const double* cdf;                 // running area sum [nT]
    const int32_t* q_tri;              // caller's queries
    const double* q_bary;
    const double* fpts;                // or free field points [Q][3] (world), c = 1, no disk
    const double2* v_n;                // caller's Neumann data [M][ng]
    const double* cvert;               // mesh free terms at vertices [nV] and edges [nT][3]
    const double* cedge;
    double area, cx, cy, cz;           // |Gamma| and the mesh centre
    uint64_t seed;
    int64_t on, oq;                    // first sample / query of the instance in the batch arrays
    int64_t og_n, og_q;                // first entry of its systems' per-sample / per-query data
    int32_t nT, N, Q, M, ng, pad;
};
struct SurfBatch {
    const SurfJob* jobs;
    int32_t n_jobs, layout;
    int32_t* tri;                      // [sum N]
    double* bary;                      // [sum N][2]
    double* x64;                       // per instance [3][N] at 3 on
    double* n64;
    float* x32;
    float* n32;
    double* q64;                       // per instance [3][Q] at 3 oq
    float* q32;
    double2* gj;                       // per system [N] at og_n + m N
    double2* gq;                       // per system [Q] at og_q + m Q
    int32_t* flags;                    // [0] query out of range, [1] non-finite Neumann data
    double* qfac;                      // per instance [Q] at oq: 1 / c_q, or null (c_q = 1/2)
    int32_t samples_given;             // 1: tri/bary already hold the samples (Poisson-disk sets)
};
// Device-side argument checks of every instance (flags are OR-ed, not cleared):
// flags[0] for a query record out of range or a non-finite field point.
hipError_t launch_checks_batch(const SurfBatch& b, int64_t max_work, hipStream_t s);
// Field points around the mesh (kind 0: random shell, 1: FFAT direction grid)
hipError_t launch_field_points(const nat_mesh* m, int32_t kind, int32_t n_a, int32_t n_b, double r_lo,
                               double r_hi, uint64_t seed, double* xyz, double* coords, hipStream_t s);
hipError_t launch_abs(const double2* z, int64_t n, double* out, hipStream_t s);
// Samples, points and Neumann data of every instance.
hipError_t launch_surface_batch(const SurfBatch& b, int32_t max_n, int32_t max_q, hipStream_t s);

// ---- Poisson-disk sample sets (k_poisson.hip) --------------------------------
constexpr int32_t kPdCandidates = 16;       // candidates per requested sample
constexpr double kPdRadiusScale = 0.72;     // r = kPdRadiusScale sqrt(|Gamma| / N)
constexpr int kPdInstShift = 40;            // cell key: instance << 40 | cell in the instance's grid
constexpr uint64_t kPdLocalMask = (uint64_t(1) << kPdInstShift) - 1;
struct PdInst {
    const double* V;                   // mesh vertices, triangles, running area sum (device)
    const int32_t* T;
    const double* cdf;
    int32_t nT, N, M, pad;             // triangles, samples wanted, candidates
    double area, r2, inv_h;            // |Gamma|, r^2, sqrt(3) / r
    double lo[3];                      // bounding-box corner
    int64_t dim[3];                    // cells per axis
    int64_t coff, on;                  // first candidate / sample of the instance in the batch
    uint64_t seed;
};
nat_status pd_instance(const nat_mesh* m, int32_t N, uint64_t seed, int64_t coff, int64_t on, PdInst* out);
size_t pd_workspace_bytes(int64_t total_candidates, int32_t n_inst);
// Samples of every instance into tri[on + j], bary[on + j] (device arrays);
// accepted (optional) receives each instance's accepted count.  Blocks.
nat_status run_poisson(nat_ctx* ctx, const PdInst* d_inst, const std::vector<PdInst>& h_inst, void* ws,
                       size_t ws_bytes, int32_t* tri, double* bary, hipStream_t s,
                       std::vector<int32_t>* accepted);

// ---- kernel sums ----------------------------------------------------------
// Operation of a kernel sum over sources j for target i (w = |Gamma|/N):
//   RHS    out_i = -sum w G g_j - (eps/2) g_i
//   MATVEC out_i = x_i / 2 - sum w dG/dn_j x_j
//   EVAL   out_i = 2 ( sum w (dG/dn_j p_j - G g_j) - (eps/2) g_i )
enum SumOp { OP_RHS = 0, OP_MATVEC = 1, OP_EVAL = 2 };

struct SumArgs {
    int32_t op;
    int32_t n_modes;
    int32_t NT, NS;              // targets, sources
    const double* t64;           // [3][NT]
    const float* t32;            // [3][NT]
    const double* s64;           // [3][NS] positions
    const double* sn64;          // [3][NS] normals
    const float* s32;
    const float* sn32;
    const double2* g_src;        // [mode * ld_gs + j]   (RHS, EVAL)
    int64_t ld_gs;
    const double2* p_src;        // [mode * ld_ps + j]   (MATVEC x, EVAL p)
    int64_t ld_ps;
    const float2* g_src32;       // FP32 weighted sources w/(4pi) g   (RHS/EVAL)
    const float2* p_src32;       // FP32 weighted sources w/(4pi) p   (MATVEC/EVAL)
    int64_t ld_s32;
    const double2* g_tgt;        // [mode * ld_gt + i]   disk term (RHS, EVAL)
    int64_t ld_gt;
    const double* k;             // [n_modes] device
    const float* k32;            // [n_modes] device, k
    const float* kappa32;        // [n_modes] device, k / (2 pi)
    const int32_t* active;       // [n_modes] or null: inactive modes are skipped
    double w, eps;
    const double2* disk;         // [n_modes] device: disk factor of each mode (RHS, EVAL)
    const double* qfac;          // [NT] 1 / c_q (EVAL), or null for 2
    double2* out;                // [mode * ld_out + i]
    int64_t ld_out;
};
hipError_t launch_sum64(const SumArgs& a, hipStream_t s, const ProfSlot& ev = ProfSlot());

// ---- batches of Monte-Carlo problems ---------------------------------------
// An instance is one mesh with one sample set; a system is one (instance,
// mode) pair.  Per-system arrays of different lengths are packed back to
// back; the offsets below locate a system's slice.
struct InstDev {
    int32_t n, q, n_modes, sys0;       // samples, queries, modes, first system
    int32_t nsplit_a, per_split_a;     // source splits of the sums over the samples
    int32_t nsplit_b, per_split_b;     // ... over the queries
    float eps2;
    int32_t phase_fract;               // 1: reduce k r / (2 pi) to [0, 1) before sin/cos
    double eps, w;
    const float* s32;                  // [3][n] sample positions, relative to the mesh centre
    const float* sn32;                 // [3][n] sample normals
    const float* q32;                  // [3][q] query positions
    const double* s64;                 // [3][n] sample positions (FP64, world)
    const double* q64;                 // [3][q] query positions (FP64, world)
    const double* qfac;                // [q] 1 / c_q of the queries, or null for 2
};

struct SysDev {
    int32_t inst, n, q, nch;           // instance, unknowns, queries, Arnoldi row chunks
    int32_t nsplit_a, nsplit_b;
    int32_t nsplit_mv;                 // split partials of the GMRES matvec (1: assembled)
    int32_t mv_pair;                   // 1: they are plain FP32 sums, float2 at 2 off_pa
                                       //    (symmetric form); 0: (hi, lo) float4 at off_pa
    int64_t off_k;                     // assembled operator [n][n] float2, or -1 (matrix-free)
    int64_t off_n;                     // [n]-long per-system arrays
    int64_t off_q;                     // [q]-long per-system arrays
    int64_t off_v;                     // Krylov basis: (mmax+1) n
    int64_t off_ch;                    // Arnoldi chunk arrays: nch
    int64_t off_pa;                    // split partials over the samples: nsplit_a n
    int64_t off_pb;                    // split partials over the queries: nsplit_b q
    double k, wscale, eps;             // wavenumber, w/(4 pi), disk radius
    double2 disk;                      // integral of G over the disk: eps/2 or the closed form
    float k32, kappa32;                // k and k/(2 pi) in FP32
    double2* out_q;                    // result at the queries (caller row) or null
    double2* out_n;                    // Stage-A solution (caller row or scratch)
};

// Up to 8 systems of one instance processed together, and the work items
// they expand to: tiles of 256 targets x source splits.
struct GroupDev {
    int32_t inst, nm, tiles, nsplit;
    int64_t item0;
    int32_t sys[8];
};

struct Sum32Batch {
    const InstDev* inst;
    const SysDev* sys;
    const GroupDev* groups;
    const int32_t* n_groups;           // device counts, so a captured launch stays valid
    const int64_t* n_items;
    const float2* a32;                 // FP32 weighted sources per system: w/(4 pi) g
    const float2* b32;                 //                                  w/(4 pi) p
    const int32_t* active;             // per system, or null
    float4* partial;                   // split partials (hi.re, hi.im, lo.re, lo.im)
    int32_t phase64;                   // 1: phase from FP64 positions, reduced in FP64
};

// Symmetric form of the matvec sum: each unordered pair of 64-sample
// sub-tiles (P <= Q) of an instance is one wave's work item for up to 8
// systems; items of the diagonal pairs (T of them for T sub-tiles) come
// first, then the T (T - 1) / 2 others.  Every target receives one partial
// per sub-tile of its instance (slot = that sub-tile).
struct SymGroupDev {
    int32_t inst, nm;
    int64_t d0, o0;                    // first diagonal / off-diagonal item
    int32_t sys[8];
};
struct SymBatch {
    const InstDev* inst;
    const SysDev* sys;
    const SymGroupDev* groups;
    const int32_t* n_groups;           // device counts
    const int64_t* n_items;            // [2]: diagonal, off-diagonal items
    const float2* b32;
    const int32_t* active;
    float4* partial;
    int32_t phase64;                   // as in Sum32Batch
};
// most concurrent parts of an automatic batch split.  HIP gives a process 4
// hardware queues by default; 3 parts plus the caller's stream fit them
// (measured on the headline batch: 1, 2, 3, 4 parts took 300, 261, 250-256,
// 281-285 ms per step).
constexpr int32_t kAutoLanes = 3;
// most workgroups (of 4 independent waves) of the symmetric matvec launch:
// enough that a headline matvec gives each wave a few items, so the
// hardware dispatcher, not a fixed stride, balances their uneven cost
// (one-stream batched step: 2048 -> 298 ms, 8192 -> 283, 32768 -> 281)
constexpr int32_t kGridSym = 32768;
// wave items below which the symmetric form narrows its mode groups
constexpr int64_t kSymFillItems = 4096;
hipError_t launch_sym32(const SymBatch& p, int32_t grid, hipStream_t s, const ProfSlot& ev = ProfSlot());

// The GMRES matvec of the systems with an assembled operator K (off_k >= 0):
// for the listed (system, 256-row chunk) items of running systems,
// partial[off_pa + i] = (hi, lo) of sum_j K_ij b_j accumulated in FP64.
struct KmvBatch {
    const SysDev* sys;
    const int2* items;                 // the Arnoldi work list
    const int32_t* n_items;            // device count
    const int32_t* active;             // per system, or null
    const float2* kmat;                // operators at off_k, source-major
    const float2* b32;                 // weighted sources w/(4 pi) p at off_n
    float4* partial;
};
hipError_t launch_kmatvec32(const KmvBatch& p, int32_t grid, hipStream_t s,
                            const ProfSlot& ev = ProfSlot());
// Assemble K_ij = q e^{i th}(ikr - 1) (the matvec's pair term without the
// source data; 0 for r < eps), entry (i, j) at off_k + j n + i, for the
// systems listed in `list` (device).
hipError_t launch_assemble32(const InstDev* inst, const SysDev* sys, const int32_t* list,
                             int32_t n_list, int32_t max_n, float2* kmat, hipStream_t s);

// source splits of a sum with n_targets targets over n_sources sources: a
// function of the instance's own sizes and the wanted items per mode group
void split_rule(int32_t n_targets, int32_t n_sources, int32_t want_items, int32_t* nsplit,
                int32_t* per_split);
int32_t target_tiles(int32_t n_targets);
// The hardware sine and cosine take revolutions and reduce them themselves:
// a development probe found them as accurate without a prior fract() for
// arguments up to this many revolutions (the FP32 kernel sums skip it when
// every pair of an instance stays below).
constexpr double kPhaseRevNoFract = 64.0;
// workgroups of the persistent kernel-sum launches: the GMRES matvec, and
// the right-hand side and query stages
constexpr int32_t kGridMatvec = 1024;
constexpr int32_t kGridStage = 4096;
// workgroups of the persistent Arnoldi-step kernels (5 or more resident per CU)
constexpr int32_t kGridArnoldi = 1280;
// workgroups of the matvec from assembled operators (8 waves per SIMD)
constexpr int32_t kGridKmv = 2048;
hipError_t launch_sum32_batch(int32_t op, const Sum32Batch& p, int32_t grid, hipStream_t s,
                              const ProfSlot& ev = ProfSlot());
// RHS: out_n[off_n + i] = b_i; EVAL: sys.out_q[i] = p(x_i)
hipError_t launch_reduce32_batch(int32_t op, const Sum32Batch& p, int32_t n_sys, int32_t max_targets,
                                 const double2* g_tgt, double2* out_n, hipStream_t s,
                                 const ProfSlot& ev = ProfSlot());
hipError_t launch_weight32_batch(const SysDev* sys, int32_t n_sys, int32_t max_n,
                                 const double2* src, double sign, float2* dst, hipStream_t s);

// ---- batched GMRES (k_gmres.hip) ------------------------------------------
struct GmresBatch {
    int32_t n_sys, mmax;
    const SysDev* sys;
    double2* V;          // [off_v + i n + t]
    double2* H;          // [sys][mmax][mmax+1]: column j of system s at ((s mmax + j)(mmax+1))
    double* cs;          // [sys][mmax]
    double2* sn;         // [sys][mmax]
    double2* gv;         // [sys][mmax+1]
    double2* htot;       // [sys][mmax+1] Hessenberg column being built
    double* beta;        // [sys]
    double* resid;       // [sys]
    int32_t* iters;      // [sys]
    int32_t* active;     // [sys]
    double2* w;          // [off_n + t] matvec output
    float2* v32;         // [off_n + t] FP32 copy of the newest basis vector times w/(4 pi), or null
    double2* dp1;        // [(off_ch + chunk)(mmax+1) + i] partial <v_i, w>
    double2* dp2;        // partial <v_i, v_j> (the new Gram column)
    double2* gram;       // [sys][gram_stride]: Gram matrix of the basis, column-major, ld mmax+1
    int64_t gram_stride; // (mmax+1)^2
    double* wnorm0;      // [off_ch + chunk] partial |w|^2 before the projection
    double* normpart;    // [off_ch + chunk] partial |w|^2 after the update
    double* normpart2;   // ... after the second pass, when one was needed
    const float4* partial;     // FP32 matvec split partials, or null (w written by the matvec)
    const int2* items;         // (system, chunk) work list of the Arnoldi kernels
    const int32_t* n_items;    // device count
    int32_t* iter;             // device iteration counter j
    int32_t* host_active;      // mapped host copy of `active`, or null
    int32_t* host_progress;    // mapped host word: iterations finished, or null
    double tol;
};
int32_t gmres_chunks(int32_t n);
hipError_t launch_gmres_init(const GmresBatch& g, const double2* b, hipStream_t s);
// one Arnoldi step (after the matvec of v_j) for the listed items, j read on
// the device, then j <- j + 1; `grid` workgroups walk the items
hipError_t launch_gmres_step(const GmresBatch& g, int32_t grid, hipStream_t s,
                             const ProfSlot& ev = ProfSlot());
hipError_t launch_gmres_solution(const GmresBatch& g, hipStream_t s);

// Device tables of a batch and the host copies the GMRES driver refreshes.
struct BatchTables {
    std::vector<InstDev> inst;       // host copies (device pointers inside)
    std::vector<SysDev> sys;
    InstDev* d_inst = nullptr;
    SysDev* d_sys = nullptr;
    // matvec groups of the running systems and the Arnoldi items, refreshed
    GroupDev* d_groups_mv = nullptr;
    int32_t* d_ngroups_mv = nullptr;
    int64_t* d_nitems_mv = nullptr;
    // ... and of the instances whose matvec takes the symmetric form
    std::vector<uint8_t> sym;        // per instance
    bool any_sym = false, any_ordered = false;
    SymGroupDev* d_groups_sym = nullptr;
    int32_t* d_ngroups_sym = nullptr;
    int64_t* d_nitems_sym = nullptr;  // [2]
    int2* d_items = nullptr;
    int32_t* d_nitems = nullptr;
    int32_t* d_iter = nullptr;
    int64_t max_items = 0;           // sum of chunks
};
// Run GMRES on the batch.  With `mv` the FP32 batched kernel sum is the
// matvec and runs of kLag iterations are captured once into a graph and
// replayed (unless graphs are off or kernel timing is on); otherwise
// eager_mv(j) launches the matvec of iteration j.
// With `kmv` the systems that have an assembled operator take their matvec
// from it, after the batched kernel sum of the others.
nat_status gmres_drive(nat_ctx* ctx, GmresBatch& g, BatchTables& T, const double2* b,
                       Sum32Batch* mv, KmvBatch* kmv, const std::function<hipError_t(int32_t)>& eager_mv,
                       bool use_graph, hipStream_t s);
// One Monte-Carlo job (the arguments of nat_mcbem_estimate).
struct McJob {
    nat_mesh* mesh;
    const double* v_n;
    int32_t M, Q, N;
    const double* k;
    const int32_t* q_tri;
    const double* q_bary;
    uint64_t seed;
    double* p_out;
    double* p_samples;
    // exterior field form: the queries are free points fpts [Q][3] (world
    // coordinates; c = 1, no disk term) and the sample values are given
    // (p_given [M][N], a previous estimate's p_samples): no Stage A
    const double* fpts = nullptr;
    const double* p_given = nullptr;
};
// Run the jobs as one batch; with bytes_only set, only validate the host
// arguments and report the workspace the batch needs.
nat_status run_mc(nat_ctx* ctx, const McJob* jobs, int32_t nj, const nat_mc_opts* opts,
                  nat_solve_report* report, hipStream_t s, size_t* bytes_only);
// Dense assembly into caller matrices (op->d_A, op->d_B set), near-pair list
// in the calling thread's workspace.
nat_status bem_assemble_into(nat_bem_op* op, hipStream_t s);
// Workspace of nat_bem_assemble and nat_bem_solve for n panels.
size_t bem_assemble_ws_bytes(int32_t n);
size_t bem_solve_ws_bytes(int32_t n, int32_t n_rhs, int32_t max_iter);

// ---- dense BEM (k_bem.hip) -------------------------------------------------
struct BemGeom {
    int32_t n;
    const double* V;
    const int32_t* T;
    const double* rules;   // far x[3], far w[3], theta x[16], theta w[16]
};
hipError_t launch_bem_far(const BemGeom& g, double k, double2 beta, double2* A, double2* B,
                          int32_t* near_list, int32_t near_cap, int32_t* near_count,
                          hipStream_t s, const ProfSlot& ev = ProfSlot());
hipError_t launch_bem_near(const BemGeom& g, double k, double2 beta, double2* A, double2* B,
                           const int32_t* near_list, int32_t n_near, hipStream_t s,
                           const ProfSlot& ev = ProfSlot());
// y[r][i] = sum_j M[i][j] x[r][j] for the rows of n x n M, r < n_rhs
// From this many right-hand sides on (and with a scratch buffer of
// zgemm_segments(n) * 16 * n entries), the complex products run on the FP64
// matrix cores, one pass over M per 16; below, a GEMV pass per 4.
constexpr int32_t kZgemmMinRhs = 8;
int32_t zgemm_segments(int32_t n, int32_t* seg = nullptr);
hipError_t launch_zgemv(const double2* M, int32_t n, const double2* x, int64_t ld_x,
                        int32_t n_rhs, double2* y, int64_t ld_y, const int32_t* active,
                        hipStream_t s, const ProfSlot& ev = ProfSlot(), double2* scratch = nullptr);
hipError_t launch_panel_data(const int32_t* T, int32_t nT, const double2* gv, int64_t ld_in,
                             int32_t n_rhs, double2* gp, int64_t ld_out, hipStream_t s);

// Gauss-Legendre rule on [0,1] (host)
void gauss_legendre01(int n, double* x, double* w);

}  // namespace nat

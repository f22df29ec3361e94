// Internal declarations of libnat_bem: context, mesh and operator records,
// the device-memory ledger, and the launchers of the HIP kernels.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
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

struct nat_ctx {
    int32_t device = 0;
    // per-kernel timing (off unless enabled)
    bool prof = false;
    std::vector<NatProfEvent> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    NatProfStat prof_stat[8];
    size_t budget = 0;   // 0: unlimited
    size_t in_use = 0;   // bytes charged
    // grow-only scratch shared by the solves of this context
    void* ws = nullptr;
    size_t ws_bytes = 0;
    // pinned host staging for small device-to-host reads
    void* pinned = nullptr;
    size_t pinned_bytes = 0;
    // pinned host memory the kernels write directly (convergence flags and
    // progress of the GMRES loop), read by the host without a copy
    int32_t* mapped = nullptr;
    int32_t* mapped_dev = nullptr;
    size_t mapped_ints = 0;
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
    // device copies
    double* d_V = nullptr;
    int32_t* d_T = nullptr;
    double* d_normal = nullptr;
    double* d_cdf = nullptr;
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
// grow-only scratch; contents undefined on return
nat_status workspace(nat_ctx* ctx, size_t bytes, void** ptr);
nat_status pinned(nat_ctx* ctx, size_t bytes, void** ptr);
nat_status mapped_words(nat_ctx* ctx, size_t n, int32_t** host, int32_t** dev);

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

// ---- per-kernel timing ------------------------------------------------------
enum ProfKind {
    PK_SUM32_RHS = 0, PK_SUM32_MATVEC = 1, PK_SUM32_EVAL = 2,
    PK_SUM64 = 3, PK_GMRES_ORTH = 4, PK_BEM_ASSEMBLE = 5, PK_ZGEMV = 6, PK_OTHER = 7
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

// Modes a launch works on: slot s is mode s (identity) or the inline list.
constexpr int kInlineModes = 64;
struct ModeList {
    int32_t n = 0;
    int32_t identity = 1;
    int32_t m[kInlineModes];
};
__host__ __device__ inline int32_t mode_at(const ModeList& L, int32_t slot)
{
    return L.identity ? slot : L.m[slot];
}
inline ModeList all_modes(int32_t n)
{
    ModeList L;
    L.n = n;
    L.identity = 1;
    return L;
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
    double2* out;                // [mode * ld_out + i]
    int64_t ld_out;
};
hipError_t launch_sum64(const SumArgs& a, hipStream_t s, const ProfSlot& ev = ProfSlot());
// FP32 tiled sum over the modes of `modes`; partial is scratch of
// sum32_partial_bytes() bytes.  With reduce = false the per-split partial
// sums are left in `partial` ([split][mode][target] float4 hi/lo) for the
// GMRES step to combine, and the split count is returned in *n_split_out.
size_t sum32_partial_bytes(const SumArgs& a);
hipError_t launch_sum32(const SumArgs& a, void* partial, hipStream_t s, const ModeList& modes,
                        bool reduce, int32_t* n_split_out, const ProfSlot& ev = ProfSlot());
// FP32 weighted copies: dst[m][j] = float2(scale * src[m][j])
hipError_t launch_weight32(const double2* src, int64_t ld_src, int32_t n_modes, int32_t n,
                           double scale, float2* dst, int64_t ld_dst, hipStream_t s);

// ---- batched GMRES (k_gmres.hip) ------------------------------------------
struct GmresState {
    int32_t n, n_modes, mmax;
    double2* V;      // [mode][mmax+1][n]
    double2* H;      // [mode][mmax][mmax+1]  column j, row i at H[(mode*mmax + j)*(mmax+1) + i]
    double* cs;      // [mode][mmax]
    double2* sn;     // [mode][mmax]
    double2* gv;     // [mode][mmax+1]
    double* beta;    // [mode]
    double* resid;   // [mode]
    int32_t* iters;  // [mode]
    int32_t* active; // [mode]
    double2* w;      // [mode][n] matvec output
    float2* v32;     // [mode][n] FP32 copy of v_j scaled by v32_scale (or null)
    double v32_scale;
    double tol;
    int32_t nch;        // row chunks of the Arnoldi kernels
    double2* dp1;       // [mode][chunk][mmax+1] partial dots, first CGS pass
    double2* dp2;       // [mode][chunk][mmax+1] partial dots, second CGS pass
    double* normpart;   // [mode][chunk]
    double2* htot;      // [mode][mmax+1] Hessenberg column being built
    int32_t* host_active;   // mapped host copy of `active` (or null)
    int32_t* host_progress; // mapped host word: last finished iteration (or null)
};
size_t gmres_state_bytes(int32_t n, int32_t n_modes, int32_t mmax);
void gmres_carve(GmresState& g, Carver& c);
hipError_t launch_gmres_init(const GmresState& g, const double2* b, int64_t ld_b, hipStream_t s);
// One Arnoldi step after the matvec of v_j for the systems of `modes`
// (systems already stopped are skipped).  With `partial` set, w is first
// formed from the FP32 kernel-sum partials as w = v_j / 2 - sum_splits.
hipError_t launch_gmres_orth(const GmresState& g, int32_t j, const void* partial, int32_t n_split,
                             const ModeList& modes, hipStream_t s, const ProfSlot& ev = ProfSlot());
hipError_t launch_gmres_solution(const GmresState& g, double2* x, int64_t ld_x, hipStream_t s);

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
hipError_t launch_zgemv(const double2* M, int32_t n, const double2* x, int64_t ld_x,
                        int32_t n_rhs, double2* y, int64_t ld_y, const int32_t* active,
                        hipStream_t s, const ProfSlot& ev = ProfSlot());
hipError_t launch_panel_data(const int32_t* T, int32_t nT, const double2* gv, int64_t ld_in,
                             int32_t n_rhs, double2* gp, int64_t ld_out, hipStream_t s);

// Gauss-Legendre rule on [0,1] (host)
void gauss_legendre01(int n, double* x, double* w);

}  // namespace nat

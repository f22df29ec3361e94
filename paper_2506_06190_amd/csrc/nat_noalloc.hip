// Allocation-free form of the Monte-Carlo estimate.
//
// nat_mcbem_estimate_noalloc runs exactly the solve of nat_mcbem_estimate
// (same kernels, same arithmetic, so the same bits) but takes its device
// workspace from one fixed block per GPU, `scratch` below, instead of the
// context's grow-only workspace, and its host staging from fixed host
// blocks instead of pinned allocations.  It calls no hipMalloc, hipFree,
// hipHostMalloc, event, stream or graph creation: for callers that cannot
// allocate (serving loops, harnesses that forbid allocation).
//
// The block is a file-scope device array.  In host code its name is only a
// host-side stand-in, so its device address is looked up once per GPU with
// hipGetSymbolAddress, with that GPU current, and only that address is
// passed to kernels.  Every call on one GPU shares that GPU's block (and the
// host staging of that GPU): calls that overlap on one GPU race, so the
// caller serialises them.  The block keeps the last call's contents; the
// solve initialises every array it reads before reading it, as it does with
// the context's reused workspace.
#include "nat_internal.h"

#include <mutex>

namespace {

// Device scratch per GPU: 256 MiB, enough for the 32-mode, 1024-sample,
// 4096-query estimate on a 20480-triangle mesh with up to 200 GMRES
// iterations (Krylov bases, Hessenberg and Gram matrices dominate).
constexpr size_t kScratchBytes = size_t(256) << 20;
// host staging (tables, work lists, reports) and host flag words per GPU
constexpr size_t kHostStageBytes = size_t(4) << 20;
constexpr size_t kHostWords = 16384;
constexpr int kMaxDevices = 16;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct Slot {
    std::mutex mu;        // first-call set-up of this GPU
    bool ready = false;
    NatScratch sc;        // ext_ws = this GPU's copy of `scratch`
};
Slot g_slot[kMaxDevices];
alignas(256) unsigned char g_host_stage[kMaxDevices][kHostStageBytes];
alignas(64) int32_t g_host_words[kMaxDevices][kHostWords];

// Device address of this GPU's `scratch` (the caller has made the GPU
// current); set up once per GPU.
nat_status slot_of(int32_t device, NatScratch** out)
{
    if (device < 0 || device >= kMaxDevices)
        return nat::fail(NAT_E_INVALID, "nat_mcbem_estimate_noalloc: device %d (at most %d GPUs)", device,
                         kMaxDevices);
    Slot& sl = g_slot[device];
    std::lock_guard<std::mutex> lk(sl.mu);
    if (!sl.ready) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return nat::hip_fail(e, "hipGetSymbolAddress(scratch)");
        sl.sc.noalloc = true;
        sl.sc.ext_ws = ptr;
        sl.sc.ext_ws_bytes = kScratchBytes;
        sl.sc.pinned = g_host_stage[device];
        sl.sc.pinned_bytes = kHostStageBytes;
        sl.sc.mapped = g_host_words[device];
        sl.sc.mapped_ints = kHostWords;
        sl.ready = true;
    }
    *out = &sl.sc;
    return NAT_OK;
}

}  // namespace

extern "C" {

nat_status nat_mcbem_estimate_noalloc(nat_mesh* mesh, const double* v_n, int32_t n_modes,
                                      const double* k, const int32_t* q_tri, const double* q_bary,
                                      int32_t Q, int32_t N, uint64_t seed, const nat_mc_opts* opts,
                                      double* p_out, double* p_samples, nat_solve_report* report,
                                      void* stream)
{
    using namespace nat;
    if (!mesh)
        return fail(NAT_E_INVALID, "nat_mcbem_estimate_noalloc: mesh is NULL");
    if (!opts)
        return fail(NAT_E_INVALID, "nat_mcbem_estimate_noalloc: opts is NULL");
    nat_ctx* ctx = mesh->ctx;
    McJob J{mesh, v_n, n_modes, Q, N, k, q_tri, q_bary, seed, p_out, p_samples};
    // direct launches (no graph), one stream
    nat_mc_opts o = *opts;
    o.flags |= NAT_MC_NO_GRAPH;
    o.n_streams = 0;
    size_t need = 0;
    nat_status st = run_mc(ctx, &J, 1, &o, nullptr, nullptr, &need);  // validates, sizes only
    if (st != NAT_OK)
        return st;
    if (need > kScratchBytes)
        return fail(NAT_E_BUDGET,
                    "nat_mcbem_estimate_noalloc: the estimate needs %zu bytes of device scratch, the "
                    "fixed block holds %zu (fewer modes, samples or GMRES iterations fit)",
                    need, kScratchBytes);
    st = set_device(ctx);
    if (st != NAT_OK)
        return st;
    NatScratch* sc = nullptr;
    st = slot_of(ctx->device, &sc);
    if (st != NAT_OK)
        return st;
    NatScratch* prev = bound_scratch();
    bind_scratch(sc);
    st = run_mc(ctx, &J, 1, &o, report, static_cast<hipStream_t>(stream), nullptr);
    bind_scratch(prev);
    return st;
}

}  // extern "C"

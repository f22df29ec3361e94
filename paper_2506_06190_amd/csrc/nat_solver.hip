// Host drivers of the Monte-Carlo estimate for a batch of instances and of
// the GMRES loop shared by every solve.
//
// A batch holds instances (mesh + sample set) and systems (instance, mode).
// Per-system arrays are packed back to back with the offsets of SysDev.  The
// steps of Section 4.1.1 run for the whole batch at once: samples and
// surface data per instance, then one kernel-sum launch per stage for all
// systems, GMRES for all systems in lockstep, and the surface evaluation.
#include <cmath>
#include <cstring>
#include <string>
#include <thread>

#include "nat_internal.h"

namespace nat {
namespace {

constexpr double kInv4Pi = 0.07957747154594767;
constexpr double kTwoPi = 6.283185307179586;
// iterations per captured run; also how far the host may run ahead of the
// device before it waits to refresh the running-system lists.  Batches whose
// matvec has at least kLagPairs target-source pairs (an iteration of a
// millisecond or so) refresh every kLagShort iterations, so converged systems
// leave the lists sooner (the matvec of a mode group runs while any of its
// systems does); smaller ones every kLag, so the host's refresh does not
// starve a device that finishes an iteration in tens of microseconds.
constexpr int32_t kLag = 4;
constexpr int32_t kLagShort = 2;
constexpr double kLagPairs = 1e9;
constexpr int32_t kMaxGrid = kGridMatvec;

inline void cpu_relax() { __builtin_ia32_pause(); }

struct Staging {
    GroupDev* groups;
    SymGroupDev* sgroups;
    int2* items;
    int32_t* c32;  // [0] Arnoldi items, [1] matvec groups, [2] symmetric groups
    int64_t* c64;  // [0] matvec work items, [1, 2] symmetric diagonal / other items
};

struct ListStats {
    int32_t running = 0;
    int64_t mv_items = 0;
    int64_t sym_items = 0;
    double mv_pairs = 0.0;  // target-source pairs of one ordered matvec
    double sym_pairs = 0.0; // ... of one symmetric matvec (ordered pairs)
    double kmv_pairs = 0.0; // ... of one matvec from assembled operators
};

// Lists of the running systems (flag != 0) into staging, then stream-ordered
// copies into the device tables.
nat_status refresh_lists(const BatchTables& T, const volatile int32_t* flag, bool with_mv,
                         const Staging& st, hipStream_t s, ListStats* out)
{
    ListStats ls;
    int32_t n_items = 0, n_groups = 0, n_sgroups = 0;
    int64_t sym_diag = 0, sym_off = 0;
    const int32_t S = static_cast<int32_t>(T.sys.size());
    for (int32_t q = 0; q < S; ++q) {
        if (!flag[q])
            continue;
        ++ls.running;
        const double pairs = (double)T.sys[q].n * (double)T.sys[q].n;
        if (T.sys[q].off_k >= 0)
            ls.kmv_pairs += pairs;
        else if ((size_t)T.sys[q].inst < T.sym.size() && T.sym[T.sys[q].inst])
            ls.sym_pairs += pairs;
        else
            ls.mv_pairs += pairs;
        for (int32_t c = 0; c < T.sys[q].nch; ++c)
            st.items[n_items++] = make_int2(q, c);
    }
    // Mode-group width of the symmetric form: 8, unless the batch then has
    // too few wave items to fill the chip; narrower groups multiply the items
    // (each system's arithmetic does not depend on the grouping).
    int32_t sym_width = 8;
    if (with_mv && T.any_sym) {
        std::vector<int32_t> running(T.inst.size(), 0);
        for (int32_t q = 0; q < S; ++q)
            if (flag[q] && T.sys[q].off_k < 0)
                ++running[T.sys[q].inst];
        while (sym_width > 1) {
            int64_t items = 0;
            for (size_t ii = 0; ii < T.inst.size(); ++ii) {
                if (!T.sym[ii] || running[ii] == 0)
                    continue;
                const int64_t t64 = (T.inst[ii].n + 63) / 64;
                items += (int64_t)((running[ii] + sym_width - 1) / sym_width) * (t64 * (t64 + 1) / 2);
            }
            if (items >= kSymFillItems)
                break;
            sym_width >>= 1;
        }
    }
    if (with_mv) {
        for (size_t ii = 0; ii < T.inst.size(); ++ii) {
            const InstDev& I = T.inst[ii];
            const bool sym = T.sym[ii] != 0;
            const int32_t width = sym ? sym_width : 8;
            const int32_t t64 = (I.n + 63) / 64;
            const int64_t n_diag = t64, n_off = (int64_t)t64 * (t64 - 1) / 2;
            GroupDev G{};
            SymGroupDev Y{};
            int32_t nm = 0;
            auto flush = [&]() {
                if (nm == 0)
                    return;
                if (sym) {
                    Y.nm = nm;
                    st.sgroups[n_sgroups++] = Y;
                    sym_diag += n_diag;
                    sym_off += n_off;
                } else {
                    G.nm = nm;
                    st.groups[n_groups++] = G;
                    ls.mv_items += (int64_t)G.tiles * G.nsplit;
                }
                nm = 0;
            };
            for (int32_t m = 0; m < I.n_modes; ++m) {
                const int32_t q = I.sys0 + m;
                if (!flag[q] || T.sys[q].off_k >= 0)
                    continue;
                if (nm == 0) {
                    G.inst = Y.inst = static_cast<int32_t>(ii);
                    G.tiles = target_tiles(I.n);
                    G.nsplit = I.nsplit_a;
                    G.item0 = ls.mv_items;
                    Y.d0 = sym_diag;
                    Y.o0 = sym_off;
                }
                if (sym)
                    Y.sys[nm] = q;
                else
                    G.sys[nm] = q;
                if (++nm == width)
                    flush();
            }
            flush();
        }
    }
    ls.sym_items = sym_diag + sym_off;
    st.c32[0] = n_items;
    st.c32[1] = n_groups;
    st.c32[2] = n_sgroups;
    st.c64[0] = ls.mv_items;
    st.c64[1] = sym_diag;
    st.c64[2] = sym_off;
    if (ls.running > 0) {
        NAT_HIP(hipMemcpyAsync(T.d_items, st.items, sizeof(int2) * n_items, hipMemcpyHostToDevice, s));
        NAT_HIP(hipMemcpyAsync(T.d_nitems, st.c32, sizeof(int32_t), hipMemcpyHostToDevice, s));
        if (with_mv && T.any_ordered) {
            NAT_HIP(hipMemcpyAsync(T.d_groups_mv, st.groups, sizeof(GroupDev) * n_groups,
                                   hipMemcpyHostToDevice, s));
            NAT_HIP(hipMemcpyAsync(T.d_ngroups_mv, st.c32 + 1, sizeof(int32_t), hipMemcpyHostToDevice, s));
            NAT_HIP(hipMemcpyAsync(T.d_nitems_mv, st.c64, sizeof(int64_t), hipMemcpyHostToDevice, s));
        }
        if (with_mv && T.any_sym) {
            NAT_HIP(hipMemcpyAsync(T.d_groups_sym, st.sgroups, sizeof(SymGroupDev) * n_sgroups,
                                   hipMemcpyHostToDevice, s));
            NAT_HIP(hipMemcpyAsync(T.d_ngroups_sym, st.c32 + 2, sizeof(int32_t), hipMemcpyHostToDevice, s));
            NAT_HIP(hipMemcpyAsync(T.d_nitems_sym, st.c64 + 1, 2 * sizeof(int64_t), hipMemcpyHostToDevice, s));
        }
    }
    *out = ls;
    return NAT_OK;
}

template <class T>
void append_bytes(std::vector<unsigned char>& v, const T& x)
{
    const unsigned char* p = reinterpret_cast<const unsigned char*>(&x);
    v.insert(v.end(), p, p + sizeof(T));
}

// The run of kLag iterations as an executable graph, captured once per
// distinct set of launch arguments and kept by the context.
nat_status captured_run(nat_ctx* ctx, const GmresBatch& g, const Sum32Batch* mv, const SymBatch* sym,
                        const KmvBatch* kmv, int32_t grid_g, int32_t grid_mv, int32_t grid_sym,
                        int32_t grid_k, int32_t lag, hipGraphExec_t* exec)
{
    NatScratch& sc = scratch_of(ctx);
    std::vector<unsigned char> key;
    append_bytes(key, g);
    append_bytes(key, mv ? *mv : Sum32Batch{});
    append_bytes(key, sym ? *sym : SymBatch{});
    append_bytes(key, kmv ? *kmv : KmvBatch{});
    append_bytes(key, grid_g);
    append_bytes(key, grid_mv);
    append_bytes(key, grid_sym);
    append_bytes(key, grid_k);
    append_bytes(key, lag);
    if (sc.graph_exec && key == sc.graph_key) {
        *exec = sc.graph_exec;
        return NAT_OK;
    }
    // one capture at a time across the context's threads, and none while
    // another thread grows its scratch (a device-wide synchronisation or free
    // is refused while any stream captures)
    std::lock_guard<std::mutex> lk(ctx->capture_mu);
    if (sc.graph_exec) {
        (void)hipGraphExecDestroy(sc.graph_exec);
        sc.graph_exec = nullptr;
        sc.graph_key.clear();
    }
    if (!sc.capture_stream)
        NAT_HIP(hipStreamCreateWithFlags(&sc.capture_stream, hipStreamNonBlocking));
    hipStream_t cs = sc.capture_stream;
    NAT_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int32_t r = 0; r < lag && e == hipSuccess; ++r) {
        if (mv)
            e = launch_sum32_batch(OP_MATVEC, *mv, grid_mv, cs);
        if (e == hipSuccess && sym)
            e = launch_sym32(*sym, grid_sym, cs);
        if (e == hipSuccess && kmv)
            e = launch_kmatvec32(*kmv, grid_k, cs);
        if (e == hipSuccess)
            e = launch_gmres_step(g, grid_g, cs);
    }
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph)
            (void)hipGraphDestroy(graph);
        (void)hipGetLastError();  // the caller falls back to direct launches
        return hip_fail(e != hipSuccess ? e : e2, "graph capture of the GMRES iterations");
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess)
        return hip_fail(e, "hipGraphInstantiate");
    sc.graph_exec = ex;
    sc.graph_key = key;
    *exec = ex;
    return NAT_OK;
}

}  // namespace

nat_status gmres_drive(nat_ctx* ctx, GmresBatch& g, BatchTables& T, const double2* b,
                       Sum32Batch* mv, KmvBatch* kmv, const std::function<hipError_t(int32_t)>& eager_mv,
                       bool use_graph, hipStream_t s)
{
    const int32_t S = g.n_sys;
    // allocation-free scratch: no mapped words; the flags are copied from
    // the device after each run of iterations
    const bool noalloc = scratch_of(ctx).noalloc;
    int32_t* hw = nullptr;
    int32_t* dw = nullptr;
    nat_status st = mapped_words(ctx, 16 + (size_t)S, &hw, &dw);
    if (st != NAT_OK)
        return st;
    volatile int32_t* hprog = hw;
    volatile int32_t* hflag = hw + 16;
    // every earlier device write to these words has landed: the previous
    // solve of this context ended with a stream synchronisation
    *hprog = 0;
    for (int32_t q = 0; q < S; ++q)
        hflag[q] = 1;
    g.host_progress = dw;
    g.host_active = dw ? dw + 16 : nullptr;
    g.items = T.d_items;
    g.n_items = T.d_nitems;
    g.iter = T.d_iter;
    SymBatch sym{};
    if (mv) {
        mv->groups = T.d_groups_mv;
        mv->n_groups = T.d_ngroups_mv;
        mv->n_items = T.d_nitems_mv;
        mv->active = g.active;
        sym.inst = mv->inst;
        sym.sys = mv->sys;
        sym.groups = T.d_groups_sym;
        sym.n_groups = T.d_ngroups_sym;
        sym.n_items = T.d_nitems_sym;
        sym.b32 = mv->b32;
        sym.active = g.active;
        sym.partial = mv->partial;
        sym.phase64 = mv->phase64;
    }
    const Sum32Batch* mv_ord = mv && T.any_ordered ? mv : nullptr;
    const SymBatch* mv_sym = mv && T.any_sym ? &sym : nullptr;
    if (kmv) {
        kmv->items = T.d_items;
        kmv->n_items = T.d_nitems;
        kmv->active = g.active;
    }

    // two pinned staging areas for the lists, used alternately
    const size_t per = ((sizeof(GroupDev) * (size_t)S + sizeof(SymGroupDev) * (size_t)S +
                         sizeof(int2) * (size_t)T.max_items + 255) & ~size_t(255)) + 256;
    void* pin = nullptr;
    st = pinned(ctx, 2 * per, &pin);
    if (st != NAT_OK)
        return st;
    Staging stg[2];
    for (int k = 0; k < 2; ++k) {
        char* base = static_cast<char*>(pin) + k * per;
        stg[k].c32 = reinterpret_cast<int32_t*>(base);
        stg[k].c64 = reinterpret_cast<int64_t*>(base + 64);
        stg[k].groups = reinterpret_cast<GroupDev*>(base + 128);
        stg[k].sgroups = reinterpret_cast<SymGroupDev*>(base + 128 + sizeof(GroupDev) * (size_t)S);
        stg[k].items = reinterpret_cast<int2*>(base + 128 + (sizeof(GroupDev) + sizeof(SymGroupDev)) * (size_t)S);
    }
    ListStats ls;
    st = refresh_lists(T, hflag, mv != nullptr, stg[0], s, &ls);
    if (st != NAT_OK)
        return st;
    NAT_HIP(launch_gmres_init(g, b, s));

    const int32_t grid_g = static_cast<int32_t>(T.max_items < kGridArnoldi ? (T.max_items > 0 ? T.max_items : 1) : kGridArnoldi);
    const int32_t grid_mv = static_cast<int32_t>(ls.mv_items < kMaxGrid ? (ls.mv_items > 0 ? ls.mv_items : 1) : kMaxGrid);
    const int32_t grid_k = static_cast<int32_t>(T.max_items < kGridKmv ? (T.max_items > 0 ? T.max_items : 1) : kGridKmv);
    const int32_t lag = ls.mv_pairs + ls.sym_pairs + ls.kmv_pairs >= kLagPairs ? kLagShort : kLag;
    // persistent grid of the symmetric form sized for its finest grouping
    int64_t sym_max_items = 0;
    for (size_t ii = 0; ii < T.inst.size(); ++ii) {
        if (T.sym.size() > ii && T.sym[ii]) {
            const int64_t t64 = (T.inst[ii].n + 63) / 64;
            sym_max_items += (int64_t)T.inst[ii].n_modes * (t64 * (t64 + 1) / 2);
        }
    }
    const int64_t sym_blocks = (sym_max_items + 3) / 4;
    const int32_t grid_sym = static_cast<int32_t>(sym_blocks < kGridSym ? (sym_blocks > 0 ? sym_blocks : 1) : kGridSym);
    hipGraphExec_t exec = nullptr;
    if (use_graph && mv && !ctx->prof && !noalloc) {
        st = captured_run(ctx, g, mv_ord, mv_sym, kmv, grid_g, grid_mv, grid_sym, grid_k, lag, &exec);
        if (st != NAT_OK)
            exec = nullptr;  // fall back to direct launches
    }
    int32_t launched = 0;
    int buf = 0;
    while (launched < g.mmax) {
        if (exec) {
            NAT_HIP(hipGraphLaunch(exec, s));
            launched += lag;
        } else {
            for (int32_t r = 0; r < lag && launched < g.mmax; ++r) {
                if (mv_ord)
                    NAT_HIP(launch_sum32_batch(OP_MATVEC, *mv_ord, grid_mv, s,
                                               prof_slot(ctx, PK_SUM32_MATVEC, 37.0 * ls.mv_pairs)));
                if (mv_sym)
                    NAT_HIP(launch_sym32(*mv_sym, grid_sym, s,
                                         prof_slot(ctx, PK_SYM32_MATVEC, 37.0 * ls.sym_pairs)));
                if (!mv)
                    NAT_HIP(eager_mv(launched));
                if (kmv)
                    NAT_HIP(launch_kmatvec32(*kmv, grid_k, s,
                                             prof_slot(ctx, PK_KMATVEC, 8.0 * ls.kmv_pairs)));
                NAT_HIP(launch_gmres_step(g, grid_g, s, prof_slot(ctx, PK_GMRES_ORTH, 0.0)));
                ++launched;
            }
        }
        if (launched >= g.mmax)
            break;
        if (noalloc) {
            // wait for the whole run, then read the device's flags
            NAT_HIP(hipMemcpyAsync(const_cast<int32_t*>(hflag), g.active, sizeof(int32_t) * (size_t)S,
                                   hipMemcpyDeviceToHost, s));
            NAT_HIP(hipStreamSynchronize(s));
        } else {
            // wait until the device has finished all but the run just queued
            const int32_t target = launched - lag;
            int64_t spins = 0;
            while (*hprog < target) {
                if (++spins > (int64_t(1) << 26)) {
                    NAT_HIP(hipStreamSynchronize(s));
                    break;
                }
                cpu_relax();
            }
        }
        buf ^= 1;
        st = refresh_lists(T, hflag, mv != nullptr, stg[buf], s, &ls);
        if (st != NAT_OK)
            return st;
        if (ls.running == 0)
            break;
    }
    return NAT_OK;
}

// ---------------------------------------------------------------------------
// Monte-Carlo estimate of a batch of jobs
// ---------------------------------------------------------------------------
nat_status run_mc(nat_ctx* ctx, const McJob* jobs, int32_t nj, const nat_mc_opts* opts,
                  nat_solve_report* report, hipStream_t s, size_t* bytes_only)
{
    if (!opts)
        return fail(NAT_E_INVALID, "Monte-Carlo estimate: opts is NULL");
    if (opts->precision != NAT_PREC_FP64 && opts->precision != NAT_PREC_FP32)
        return fail(NAT_E_INVALID, "Monte-Carlo estimate: precision %d", opts->precision);
    if (opts->layout != NAT_NEUMANN_PER_VERTEX && opts->layout != NAT_NEUMANN_PER_TRIANGLE)
        return fail(NAT_E_INVALID, "Monte-Carlo estimate: layout %d", opts->layout);
    if (!(opts->eps_scale > 0.0) || !is_finite(opts->eps_scale) || !(opts->gmres_tol > 0.0) ||
        opts->gmres_max_iter < 1 || opts->gmres_max_iter > 1000 ||
        (opts->flags & ~(NAT_MC_NO_GRAPH | NAT_MC_ASSEMBLED | NAT_MC_MATRIX_FREE | NAT_MC_EXACT_DISK |
                         NAT_MC_ORDERED_SUM | NAT_MC_FP64_PHASE | NAT_MC_POISSON)) ||
        ((opts->flags & NAT_MC_ASSEMBLED) && (opts->flags & (NAT_MC_MATRIX_FREE | NAT_MC_FP64_PHASE))))
        return fail(NAT_E_INVALID, "Monte-Carlo estimate: bad solver options");
    if (opts->jump != NAT_JUMP_HALF && opts->jump != NAT_JUMP_POLYHEDRAL)
        return fail(NAT_E_INVALID, "Monte-Carlo estimate: jump %d", opts->jump);
    if (opts->n_streams < 0 || opts->n_streams > nat_ctx::kMaxLanes)
        return fail(NAT_E_INVALID, "Monte-Carlo estimate: n_streams %d", opts->n_streams);
    // exterior field form (given sample values, free field points): every
    // job of the batch or none
    const bool field = nj > 0 && jobs[0].p_given != nullptr;
    const bool polyhedral = opts->jump == NAT_JUMP_POLYHEDRAL;
    int64_t S64 = 0;
    for (int32_t i = 0; i < nj; ++i) {
        const McJob& J = jobs[i];
        if (!J.mesh || !J.v_n || !J.k)
            return fail(NAT_E_INVALID, "job %d: NULL argument", i);
        if ((J.p_given != nullptr) != field || (!field && J.fpts))
            return fail(NAT_E_INVALID, "job %d: field and surface jobs mixed", i);
        if (J.mesh->ctx != ctx)
            return fail(NAT_E_INVALID, "job %d: mesh belongs to another context", i);
        if (J.M < 1 || J.M > 4096)
            return fail(NAT_E_INVALID, "job %d: n_modes = %d", i, J.M);
        if (J.N < 2 || J.N > (1 << 24))
            return fail(NAT_E_INVALID, "job %d: n_samples = %d", i, J.N);
        if (J.Q < 0 || J.Q > (1 << 26) ||
            (J.Q > 0 && (field ? (!J.fpts || !J.p_out) : (!J.q_tri || !J.q_bary || !J.p_out))))
            return fail(NAT_E_INVALID, "job %d: bad queries (Q = %d)", i, J.Q);
        for (int32_t m = 0; m < J.M; ++m)
            if (!(J.k[m] > 0.0) || !is_finite(J.k[m]))
                return fail(NAT_E_INVALID, "job %d: k[%d] = %g", i, m, J.k[m]);
        S64 += J.M;
    }
    if (nj < 1 || nj > 65535 || S64 > (1 << 20))
        return fail(NAT_E_INVALID, "Monte-Carlo estimate: %d jobs with %lld systems", nj, (long long)S64);
    nat_status st = NAT_OK;
    if (!bytes_only) {
        st = set_device(ctx);
        if (st != NAT_OK)
            return st;
    }
    const int32_t S = static_cast<int32_t>(S64);
    const bool fp32 = opts->precision == NAT_PREC_FP32;
    // the field form runs no GMRES: its basis and Hessenberg arrays shrink
    const int32_t mmax = field ? 1 : opts->gmres_max_iter;
    // per-query factors 1/c_q: polyhedral free terms, or c = 1 at field points
    const bool with_qfac = polyhedral || field;
    const size_t mm1 = (size_t)mmax + 1;

    // ---- layout ----------------------------------------------------------
    BatchTables T;
    T.inst.resize(nj);
    T.sys.resize(S);
    T.sym.assign(nj, 0);
    size_t inst_n = 0, inst_q = 0;       // sums of n and q over instances
    int64_t sum_n = 0, sum_q = 0, sum_v = 0, sum_ch = 0, sum_pa = 0, sum_pb = 0, sum_k = 0;
    std::vector<int32_t> asm_list;  // systems whose matvec reads an assembled operator
    int32_t max_n_asm = 0;
    int32_t max_n = 0, max_q = 0;
    for (int32_t i = 0, q = 0; i < nj; ++i) {
        const McJob& J = jobs[i];
        InstDev& I = T.inst[i];
        I.n = J.N;
        I.q = J.Q;
        I.n_modes = J.M;
        I.sys0 = q;
        split_rule(J.N, J.N, ctx->tune.items_a[tune_bucket(J.N)], &I.nsplit_a, &I.per_split_a);
        if (J.Q > 0)
            split_rule(J.Q, J.N, ctx->tune.items_b[tune_bucket(J.Q)], &I.nsplit_b, &I.per_split_b);
        const double area = J.mesh->area_total;
        I.w = area / static_cast<double>(J.N);
        I.eps = opts->eps_scale * std::sqrt(area / (M_PI * static_cast<double>(J.N)));
        I.eps2 = static_cast<float>(I.eps * I.eps);
        double k_max = 0.0;
        for (int32_t m = 0; m < J.M; ++m)
            k_max = J.k[m] > k_max ? J.k[m] : k_max;
        I.phase_fract = k_max / kTwoPi * J.mesh->diameter > kPhaseRevNoFract ? 1 : 0;
        // matvec form: assembled operator or matrix-free (FP32 form only)
        const bool asm_form = !field && fp32 && !(opts->flags & NAT_MC_FP64_PHASE) &&
                              ((opts->flags & NAT_MC_ASSEMBLED) ||
                                       (!(opts->flags & NAT_MC_MATRIX_FREE) &&
                                        ctx->tune.assembled[tune_bucket(J.N)]));
        // matrix-free matvec: symmetric (one partial per 64-sample sub-tile)
        // or ordered (the instance's source splits)
        const bool sym_form = fp32 && !asm_form && !(opts->flags & NAT_MC_ORDERED_SUM) &&
                              ctx->tune.symmetric[tune_bucket(J.N)];
        T.sym[i] = sym_form ? 1 : 0;
        if (fp32 && !asm_form) {
            T.any_sym = T.any_sym || sym_form;
            T.any_ordered = T.any_ordered || !sym_form;
        }
        inst_n += J.N;
        inst_q += J.Q;
        max_n = J.N > max_n ? J.N : max_n;
        max_q = J.Q > max_q ? J.Q : max_q;
        for (int32_t m = 0; m < J.M; ++m, ++q) {
            SysDev& Y = T.sys[q];
            Y.inst = i;
            Y.n = J.N;
            Y.q = J.Q;
            Y.nch = gmres_chunks(J.N);
            Y.nsplit_a = I.nsplit_a;
            Y.nsplit_b = J.Q > 0 ? I.nsplit_b : 0;
            Y.nsplit_mv = asm_form ? 1 : (sym_form ? (J.N + 63) / 64 : I.nsplit_a);
            Y.mv_pair = sym_form ? 1 : 0;
            Y.off_k = asm_form ? sum_k : -1;
            if (asm_form) {
                sum_k += (int64_t)J.N * J.N;
                asm_list.push_back(q);
                max_n_asm = J.N > max_n_asm ? J.N : max_n_asm;
            }
            Y.off_n = sum_n;
            Y.off_q = sum_q;
            Y.off_v = sum_v;
            Y.off_ch = sum_ch;
            Y.off_pa = sum_pa;
            Y.off_pb = sum_pb;
            Y.k = J.k[m];
            Y.k32 = static_cast<float>(J.k[m]);
            Y.kappa32 = static_cast<float>(J.k[m] / kTwoPi);
            Y.wscale = I.w * kInv4Pi;
            Y.eps = I.eps;
            if (field) {
                Y.disk = make_double2(0.0, 0.0);  // no disk term off the surface
            } else if (opts->flags & NAT_MC_EXACT_DISK) {
                // (e^{ik eps} - 1) / (2ik) = sin(x)/(2k) + i (1 - cos x)/(2k), x = k eps
                const double x = J.k[m] * I.eps, h = std::sin(0.5 * x);
                Y.disk = make_double2(std::sin(x) / (2.0 * J.k[m]), h * h / J.k[m]);
            } else {
                Y.disk = make_double2(0.5 * I.eps, 0.0);
            }
            sum_n += J.N;
            sum_q += J.Q;
            sum_v += (int64_t)mm1 * J.N;
            sum_ch += Y.nch;
            sum_pa += (int64_t)(Y.nsplit_a > Y.nsplit_mv ? Y.nsplit_a : Y.nsplit_mv) * J.N;
            sum_pb += (int64_t)Y.nsplit_b * J.Q;
        }
    }
    T.max_items = sum_ch;
    const int64_t n_part = sum_pa > sum_pb ? sum_pa : sum_pb;
    const int64_t gram_stride = (int64_t)mm1 * mm1;
    // Poisson-disk samples (Section 4.2): candidate pools of every instance
    const bool poisson = (opts->flags & NAT_MC_POISSON) != 0;
    const size_t pd_bytes = poisson ? pd_workspace_bytes((int64_t)kPdCandidates * (int64_t)inst_n, nj) : 0;
    const size_t bytes = carve_size<>(
        {sizeof(int32_t) * 8, sizeof(int32_t) * inst_n, sizeof(double) * 2 * inst_n,
         sizeof(double) * 3 * inst_n, sizeof(double) * 3 * inst_n, sizeof(float) * 3 * inst_n,
         sizeof(float) * 3 * inst_n, sizeof(double) * 3 * inst_q, sizeof(float) * 3 * inst_q,
         sizeof(double2) * sum_n, sizeof(double2) * sum_q, sizeof(double2) * sum_n,
         sizeof(double2) * sum_n, sizeof(float2) * sum_n, sizeof(float2) * sum_n,
         sizeof(double2) * sum_n, sizeof(double2) * sum_v, sizeof(double2) * S * mmax * mm1,
         sizeof(double) * S * mmax, sizeof(double2) * S * mmax, sizeof(double2) * S * mm1,
         sizeof(double2) * S * mm1, sizeof(double) * S, sizeof(double) * S, sizeof(int32_t) * S,
         sizeof(int32_t) * S, sizeof(double2) * sum_ch * mm1, sizeof(double2) * sum_ch * mm1,
         sizeof(double) * sum_ch, sizeof(double) * sum_ch, sizeof(double) * sum_ch,
         sizeof(double2) * S * gram_stride, sizeof(float4) * n_part, sizeof(InstDev) * nj,
         sizeof(SysDev) * S, sizeof(GroupDev) * S, sizeof(GroupDev) * S, sizeof(GroupDev) * S,
         sizeof(SymGroupDev) * S,
         sizeof(int2) * sum_ch, sizeof(double) * S, sizeof(double2) * S, sizeof(int64_t) * 8,
         sizeof(SurfJob) * nj,
         with_qfac ? sizeof(double) * inst_q : 0, sizeof(float2) * sum_k,
         sizeof(int32_t) * asm_list.size(), sizeof(PdInst) * (poisson ? nj : 0), pd_bytes});
    if (bytes_only) {
        *bytes_only = bytes;
        return NAT_OK;
    }
    void* ws = nullptr;
    st = workspace(ctx, bytes, &ws);
    if (st != NAT_OK)
        return st;
    Carver cv(ws);
    int32_t* dcnt = cv.take<int32_t>(8);  // flags [0,1], n_items, n_groups_mv, iter, n_groups rhs/eval/sym
    int32_t* tri_all = cv.take<int32_t>(inst_n);
    double* bary_all = cv.take<double>(2 * inst_n);
    double* x64_all = cv.take<double>(3 * inst_n);
    double* n64_all = cv.take<double>(3 * inst_n);
    float* x32_all = cv.take<float>(3 * inst_n);
    float* n32_all = cv.take<float>(3 * inst_n);
    double* q64_all = cv.take<double>(3 * inst_q);
    float* q32_all = cv.take<float>(3 * inst_q);
    double2* gj = cv.take<double2>(sum_n);
    double2* gq = cv.take<double2>(sum_q);
    double2* bvec = cv.take<double2>(sum_n);
    double2* xsol = cv.take<double2>(sum_n);
    float2* a32 = cv.take<float2>(sum_n);
    float2* v32 = cv.take<float2>(sum_n);
    GmresBatch g{};
    g.n_sys = S;
    g.mmax = mmax;
    g.tol = opts->gmres_tol;
    g.w = cv.take<double2>(sum_n);
    g.V = cv.take<double2>(sum_v);
    g.H = cv.take<double2>((size_t)S * mmax * mm1);
    g.cs = cv.take<double>((size_t)S * mmax);
    g.sn = cv.take<double2>((size_t)S * mmax);
    g.gv = cv.take<double2>((size_t)S * mm1);
    g.htot = cv.take<double2>((size_t)S * mm1);
    g.beta = cv.take<double>(S);
    g.resid = cv.take<double>(S);
    g.iters = cv.take<int32_t>(S);
    g.active = cv.take<int32_t>(S);
    g.dp1 = cv.take<double2>((size_t)sum_ch * mm1);
    g.dp2 = cv.take<double2>((size_t)sum_ch * mm1);
    g.normpart = cv.take<double>(sum_ch);
    g.normpart2 = cv.take<double>(sum_ch);
    g.wnorm0 = cv.take<double>(sum_ch);
    g.gram = cv.take<double2>((size_t)S * gram_stride);
    g.gram_stride = gram_stride;
    float4* partial = cv.take<float4>(n_part);
    T.d_inst = cv.take<InstDev>(nj);
    T.d_sys = cv.take<SysDev>(S);
    GroupDev* d_groups_rhs = cv.take<GroupDev>(S);
    GroupDev* d_groups_eval = cv.take<GroupDev>(S);
    T.d_groups_mv = cv.take<GroupDev>(S);
    T.d_groups_sym = cv.take<SymGroupDev>(S);
    T.d_items = cv.take<int2>(sum_ch);
    double* dk = cv.take<double>(S);
    double2* ddisk = cv.take<double2>(S);
    int64_t* dcnt64 = cv.take<int64_t>(8);  // items: [0] rhs, [1] eval, [2] matvec, [4,5] sym
    SurfJob* d_surf = cv.take<SurfJob>(nj);
    double* qfac_all = with_qfac ? cv.take<double>(inst_q) : nullptr;
    float2* kmat = sum_k > 0 ? cv.take<float2>(sum_k) : nullptr;
    int32_t* d_asm_list = asm_list.empty() ? nullptr : cv.take<int32_t>(asm_list.size());
    PdInst* d_pd = poisson ? cv.take<PdInst>(nj) : nullptr;
    void* pd_ws = poisson ? cv.take<char>(pd_bytes) : nullptr;
    T.d_nitems = dcnt + 2;
    T.d_ngroups_mv = dcnt + 3;
    T.d_iter = dcnt + 4;
    T.d_nitems_mv = dcnt64 + 2;
    T.d_ngroups_sym = dcnt + 7;
    T.d_nitems_sym = dcnt64 + 4;
    g.sys = T.d_sys;
    g.v32 = fp32 ? v32 : nullptr;
    g.partial = fp32 ? partial : nullptr;

    // per-instance streams and the device pointers of the tables
    {
        size_t on = 0, oq = 0;
        for (int32_t i = 0; i < nj; ++i) {
            InstDev& I = T.inst[i];
            I.s32 = x32_all + 3 * on;
            I.sn32 = n32_all + 3 * on;
            I.q32 = q32_all + 3 * oq;
            I.s64 = x64_all + 3 * on;
            I.q64 = q64_all + 3 * oq;
            I.qfac = qfac_all && I.q > 0 ? qfac_all + oq : nullptr;
            on += I.n;
            oq += I.q;
        }
        for (int32_t q = 0; q < S; ++q) {
            SysDev& Y = T.sys[q];
            const McJob& J = jobs[Y.inst];
            const int32_t m = q - T.inst[Y.inst].sys0;
            Y.out_q = J.Q > 0 ? reinterpret_cast<double2*>(J.p_out) + (size_t)m * J.Q : nullptr;
            Y.out_n = xsol + Y.off_n;
        }
    }

    // ---- the instance table of the surface kernels and the device checks -----
    SurfBatch sbat{};
    int64_t max_check = 0;
    {
        std::vector<SurfJob> sj(nj);
        size_t on = 0, oq = 0;
        for (int32_t i = 0; i < nj; ++i) {
            const McJob& J = jobs[i];
            const nat_mesh* m = J.mesh;
            SurfJob& X = sj[i];
            X = SurfJob{};
            X.V = m->d_V;
            X.T = m->d_T;
            X.nrm = m->d_normal;
            X.cdf = m->d_cdf;
            X.q_tri = J.q_tri;
            X.q_bary = J.q_bary;
            X.fpts = J.fpts;
            X.v_n = reinterpret_cast<const double2*>(J.v_n);
            X.cvert = m->d_cvert;
            X.cedge = m->d_cedge;
            X.area = m->area_total;
            X.cx = m->center[0];
            X.cy = m->center[1];
            X.cz = m->center[2];
            X.seed = J.seed;
            X.on = (int64_t)on;
            X.oq = (int64_t)oq;
            X.og_n = T.sys[T.inst[i].sys0].off_n;
            X.og_q = T.sys[T.inst[i].sys0].off_q;
            X.nT = m->nT;
            X.N = J.N;
            X.Q = J.Q;
            X.M = J.M;
            X.ng = opts->layout == NAT_NEUMANN_PER_TRIANGLE ? m->nT : m->nV;
            on += J.N;
            oq += J.Q;
            const int64_t w = std::max<int64_t>(J.Q, 2 * (int64_t)J.M * X.ng);
            max_check = w > max_check ? w : max_check;
        }
        void* pin = nullptr;
        st = pinned(ctx, sizeof(SurfJob) * nj + 64, &pin);
        if (st != NAT_OK)
            return st;
        std::memcpy(pin, sj.data(), sizeof(SurfJob) * nj);
        NAT_HIP(hipMemcpyAsync(d_surf, pin, sizeof(SurfJob) * nj, hipMemcpyHostToDevice, s));
        sbat.jobs = d_surf;
        sbat.n_jobs = nj;
        sbat.layout = opts->layout;
        sbat.tri = tri_all;
        sbat.bary = bary_all;
        sbat.x64 = x64_all;
        sbat.n64 = n64_all;
        sbat.x32 = x32_all;
        sbat.n32 = n32_all;
        sbat.q64 = q64_all;
        sbat.q32 = q32_all;
        sbat.gj = gj;
        sbat.gq = gq;
        sbat.flags = dcnt;
        sbat.qfac = qfac_all;
        NAT_HIP(hipMemsetAsync(dcnt, 0, 2 * sizeof(int32_t), s));
        NAT_HIP(launch_checks_batch(sbat, max_check, s));
        int32_t* hflags = reinterpret_cast<int32_t*>(static_cast<char*>(pin) + sizeof(SurfJob) * nj);
        NAT_HIP(hipMemcpyAsync(hflags, dcnt, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        NAT_HIP(hipStreamSynchronize(s));
        if (hflags[0])
            return fail(NAT_E_INVALID, field ? "Monte-Carlo field: a field point is not finite"
                                             : "Monte-Carlo estimate: query record out of range");
        if (hflags[1])
            return fail(NAT_E_INVALID, "Monte-Carlo estimate: non-finite Neumann data");
    }

    // ---- tables and per-mode constants --------------------------------------
    // all-systems groups for the right-hand side (targets = samples) and the
    // evaluation (targets = queries)
    std::vector<GroupDev> grhs, geval;
    int64_t items_rhs = 0, items_eval = 0;
    for (const InstDev& I : T.inst) {
        for (int32_t m0 = 0; m0 < I.n_modes; m0 += 8) {
            GroupDev G{};
            G.inst = T.sys[I.sys0].inst;
            G.nm = I.n_modes - m0 < 8 ? I.n_modes - m0 : 8;
            for (int32_t c = 0; c < G.nm; ++c)
                G.sys[c] = I.sys0 + m0 + c;
            G.tiles = target_tiles(I.n);
            G.nsplit = I.nsplit_a;
            G.item0 = items_rhs;
            items_rhs += (int64_t)G.tiles * G.nsplit;
            grhs.push_back(G);
            if (I.q > 0) {
                G.tiles = target_tiles(I.q);
                G.nsplit = I.nsplit_b;
                G.item0 = items_eval;
                items_eval += (int64_t)G.tiles * G.nsplit;
                geval.push_back(G);
            }
        }
    }
    {
        const size_t bI = sizeof(InstDev) * nj, bS = sizeof(SysDev) * S;
        const size_t bG1 = sizeof(GroupDev) * grhs.size(), bG2 = sizeof(GroupDev) * geval.size();
        void* pin = nullptr;
        const size_t bL = sizeof(int32_t) * asm_list.size();
        const size_t bD = sizeof(double2) * S;
        st = pinned(ctx, bI + bS + bG1 + bG2 + sizeof(double) * S + 256 + bL + bD + 16, &pin);
        if (st != NAT_OK)
            return st;
        char* p = static_cast<char*>(pin);
        std::memcpy(p, T.inst.data(), bI);
        std::memcpy(p + bI, T.sys.data(), bS);
        std::memcpy(p + bI + bS, grhs.data(), bG1);
        std::memcpy(p + bI + bS + bG1, geval.data(), bG2);
        double* hk = reinterpret_cast<double*>(p + bI + bS + bG1 + bG2);
        for (int32_t q = 0; q < S; ++q)
            hk[q] = T.sys[q].k;
        int64_t* hc = reinterpret_cast<int64_t*>(p + bI + bS + bG1 + bG2 + sizeof(double) * S);
        int32_t* hc32 = reinterpret_cast<int32_t*>(hc + 2);
        hc[0] = items_rhs;
        hc[1] = items_eval;
        hc32[0] = static_cast<int32_t>(grhs.size());
        hc32[1] = static_cast<int32_t>(geval.size());
        NAT_HIP(hipMemcpyAsync(T.d_inst, p, bI, hipMemcpyHostToDevice, s));
        NAT_HIP(hipMemcpyAsync(T.d_sys, p + bI, bS, hipMemcpyHostToDevice, s));
        NAT_HIP(hipMemcpyAsync(d_groups_rhs, p + bI + bS, bG1, hipMemcpyHostToDevice, s));
        if (bG2)
            NAT_HIP(hipMemcpyAsync(d_groups_eval, p + bI + bS + bG1, bG2, hipMemcpyHostToDevice, s));
        NAT_HIP(hipMemcpyAsync(dk, hk, sizeof(double) * S, hipMemcpyHostToDevice, s));
        NAT_HIP(hipMemcpyAsync(dcnt64, hc, 2 * sizeof(int64_t), hipMemcpyHostToDevice, s));
        NAT_HIP(hipMemcpyAsync(dcnt + 5, hc32, 2 * sizeof(int32_t), hipMemcpyHostToDevice, s));
        char* pl = p + bI + bS + bG1 + bG2 + sizeof(double) * S + 256;
        if (bL) {
            std::memcpy(pl, asm_list.data(), bL);
            NAT_HIP(hipMemcpyAsync(d_asm_list, pl, bL, hipMemcpyHostToDevice, s));
        }
        // double2 is 16-byte aligned: align the staging address itself
        double2* hd = reinterpret_cast<double2*>((reinterpret_cast<uintptr_t>(pl + bL) + 15) &
                                                 ~uintptr_t(15));
        for (int32_t q = 0; q < S; ++q)
            hd[q] = T.sys[q].disk;
        NAT_HIP(hipMemcpyAsync(ddisk, hd, bD, hipMemcpyHostToDevice, s));
        // the staging above is read by the copies; the GMRES driver reuses
        // this pinned block, so wait for them
        NAT_HIP(hipStreamSynchronize(s));
    }

    // stage timing: events on the stream between the stages (none in the
    // allocation-free form)
    StageEvents sev;
    if (!scratch_of(ctx).noalloc)
        NAT_HIP(sev.create());
    NAT_HIP(sev.record(0, s));

    // ---- samples, points, Neumann data (Section 4.1.1) -----------------------
    if (poisson) {
        // Poisson-disk sets instead of independent samples (Section 4.2)
        std::vector<PdInst> pd(nj);
        int64_t coff = 0, on = 0;
        for (int32_t i = 0; i < nj; ++i) {
            st = pd_instance(jobs[i].mesh, jobs[i].N, jobs[i].seed, coff, on, &pd[i]);
            if (st != NAT_OK)
                return st;
            coff += pd[i].M;
            on += jobs[i].N;
        }
        void* pin = nullptr;
        st = pinned(ctx, sizeof(PdInst) * nj + 64, &pin);
        if (st != NAT_OK)
            return st;
        std::memcpy(pin, pd.data(), sizeof(PdInst) * nj);
        NAT_HIP(hipMemcpyAsync(d_pd, pin, sizeof(PdInst) * nj, hipMemcpyHostToDevice, s));
        st = run_poisson(ctx, d_pd, pd, pd_ws, pd_bytes, tri_all, bary_all, s, nullptr);
        if (st != NAT_OK)
            return st;
        sbat.samples_given = 1;
    }
    NAT_HIP(launch_surface_batch(sbat, max_n, max_q, s));
    NAT_HIP(sev.record(1, s));

    Sum32Batch sb{};
    sb.inst = T.d_inst;
    sb.sys = T.d_sys;
    sb.partial = partial;
    sb.phase64 = (opts->flags & NAT_MC_FP64_PHASE) ? 1 : 0;
    // per-instance arguments of the plain FP64 sums
    auto plain_args = [&](int32_t i, int32_t op) {
        const InstDev& I = T.inst[i];
        const SysDev& Y0 = T.sys[I.sys0];
        size_t on = 0, oq = 0;
        for (int32_t t = 0; t < i; ++t) {
            on += T.inst[t].n;
            oq += T.inst[t].q;
        }
        SumArgs a{};
        a.op = op;
        a.n_modes = I.n_modes;
        a.NS = I.n;
        a.s64 = x64_all + 3 * on;
        a.sn64 = n64_all + 3 * on;
        a.k = dk + I.sys0;
        a.disk = ddisk + I.sys0;
        a.w = I.w;
        a.eps = I.eps;
        if (op == OP_EVAL) {
            a.NT = I.q;
            a.t64 = q64_all + 3 * oq;
            a.g_tgt = gq + Y0.off_q;
            a.ld_gt = I.q;
            a.out = Y0.out_q;
            a.ld_out = I.q;
            a.qfac = I.qfac;
        } else {
            a.NT = I.n;
            a.t64 = a.s64;
            a.g_tgt = gj + Y0.off_n;
            a.ld_gt = I.n;
        }
        a.g_src = gj + Y0.off_n;
        a.ld_gs = I.n;
        return a;
    };

    // ---- right-hand side (eq. bem_linear_system, Section 4.2 disk term) ------
    double pairs_rhs = 0.0, pairs_eval = 0.0;
    for (const SysDev& Y : T.sys) {
        pairs_rhs += (double)Y.n * Y.n;
        pairs_eval += (double)Y.q * Y.n;
    }
    if (field) {
        // the field form starts from the given sample values
    } else if (fp32) {
        NAT_HIP(launch_weight32_batch(T.d_sys, S, max_n, gj, 1.0, a32, s));
        sb.groups = d_groups_rhs;
        sb.n_groups = dcnt + 5;
        sb.n_items = dcnt64 + 0;
        sb.a32 = a32;
        const ProfSlot ev = prof_slot(ctx, PK_SUM32_RHS, 24.0 * pairs_rhs);
        const int32_t grid = static_cast<int32_t>(items_rhs < kGridStage ? items_rhs : kGridStage);
        NAT_HIP(launch_sum32_batch(OP_RHS, sb, grid, s, ProfSlot{ev.start, nullptr}));
        NAT_HIP(launch_reduce32_batch(OP_RHS, sb, S, max_n, gj, bvec, s, ProfSlot{nullptr, ev.stop}));
    } else {
        for (int32_t i = 0; i < nj; ++i) {
            SumArgs a = plain_args(i, OP_RHS);
            a.out = bvec + T.sys[T.inst[i].sys0].off_n;
            a.ld_out = T.inst[i].n;
            NAT_HIP(launch_sum64(a, s, prof_slot(ctx, PK_SUM64, 24.0 * T.inst[i].n * (double)T.inst[i].n * T.inst[i].n_modes)));
        }
    }

    NAT_HIP(sev.record(2, s));

    // ---- GMRES on (I/2 - K) p = b ---------------------------------------------
    // assembled operators of the systems that use them (the tuner's choice by
    // N, or forced by the flags)
    KmvBatch kb{};
    if (!field && !asm_list.empty()) {
        NAT_HIP(launch_assemble32(T.d_inst, T.d_sys, d_asm_list, static_cast<int32_t>(asm_list.size()),
                                  max_n_asm, kmat, s));
        kb.sys = T.d_sys;
        kb.kmat = kmat;
        kb.b32 = v32;
        kb.partial = partial;
    }
    std::function<hipError_t(int32_t)> eager = [&](int32_t j) -> hipError_t {
        for (int32_t i = 0; i < nj; ++i) {
            const InstDev& I = T.inst[i];
            const SysDev& Y0 = T.sys[I.sys0];
            SumArgs a = plain_args(i, OP_MATVEC);
            a.p_src = g.V + Y0.off_v + (size_t)j * I.n;
            a.ld_ps = (int64_t)mm1 * I.n;
            a.active = g.active + I.sys0;
            a.out = g.w + Y0.off_n;
            a.ld_out = I.n;
            hipError_t e = launch_sum64(a, s, prof_slot(ctx, PK_SUM64, 37.0 * I.n * (double)I.n * I.n_modes));
            if (e != hipSuccess)
                return e;
        }
        return hipSuccess;
    };
    sb.b32 = v32;
    if (field) {
        for (int32_t i = 0; i < nj; ++i)
            NAT_HIP(hipMemcpyAsync(xsol + T.sys[T.inst[i].sys0].off_n, jobs[i].p_given,
                                   sizeof(double2) * (size_t)jobs[i].M * jobs[i].N,
                                   hipMemcpyDeviceToDevice, s));
    } else {
        st = gmres_drive(ctx, g, T, bvec, fp32 ? &sb : nullptr, asm_list.empty() ? nullptr : &kb, eager,
                         !(opts->flags & NAT_MC_NO_GRAPH), s);
        if (st != NAT_OK)
            return st;
        NAT_HIP(launch_gmres_solution(g, s));
    }
    NAT_HIP(sev.record(3, s));

    // ---- surface evaluation (eq. BIE at the queries, Section 4.2) --------------
    if (max_q > 0) {
        if (fp32) {
            NAT_HIP(launch_weight32_batch(T.d_sys, S, max_n, gj, -1.0, a32, s));
            NAT_HIP(launch_weight32_batch(T.d_sys, S, max_n, xsol, 1.0, v32, s));
            Sum32Batch se = sb;
            se.groups = d_groups_eval;
            se.n_groups = dcnt + 6;
            se.n_items = dcnt64 + 1;
            se.active = nullptr;
            se.a32 = a32;
            se.b32 = v32;
            const ProfSlot ev = prof_slot(ctx, PK_SUM32_EVAL, 47.0 * pairs_eval);
            const int32_t grid = static_cast<int32_t>(items_eval < kGridStage ? items_eval : kGridStage);
            NAT_HIP(launch_sum32_batch(OP_EVAL, se, grid, s, ProfSlot{ev.start, nullptr}));
            NAT_HIP(launch_reduce32_batch(OP_EVAL, se, S, max_q, gq, nullptr, s, ProfSlot{nullptr, ev.stop}));
        } else {
            for (int32_t i = 0; i < nj; ++i) {
                if (T.inst[i].q == 0)
                    continue;
                SumArgs a = plain_args(i, OP_EVAL);
                a.p_src = xsol + T.sys[T.inst[i].sys0].off_n;
                a.ld_ps = T.inst[i].n;
                NAT_HIP(launch_sum64(a, s, prof_slot(ctx, PK_SUM64, 47.0 * T.inst[i].q * (double)T.inst[i].n * T.inst[i].n_modes)));
            }
        }
    }
    NAT_HIP(sev.record(4, s));
    for (int32_t i = 0; i < nj; ++i) {
        if (!jobs[i].p_samples)
            continue;
        const SysDev& Y0 = T.sys[T.inst[i].sys0];
        NAT_HIP(hipMemcpyAsync(jobs[i].p_samples, xsol + Y0.off_n,
                               sizeof(double2) * (size_t)jobs[i].M * jobs[i].N, hipMemcpyDeviceToDevice, s));
    }
    prof_collect(ctx);

    // ---- reports ----------------------------------------------------------
    void* pin = nullptr;
    st = pinned(ctx, (sizeof(int32_t) + sizeof(double)) * (size_t)S + 64, &pin);
    if (st != NAT_OK)
        return st;
    double* hres = static_cast<double*>(pin);
    int32_t* hit = reinterpret_cast<int32_t*>(hres + S);
    if (field) {
        for (int32_t q = 0; q < S; ++q) {
            hres[q] = 0.0;
            hit[q] = 0;
        }
    } else {
        NAT_HIP(hipMemcpyAsync(hres, g.resid, sizeof(double) * S, hipMemcpyDeviceToHost, s));
        NAT_HIP(hipMemcpyAsync(hit, g.iters, sizeof(int32_t) * S, hipMemcpyDeviceToHost, s));
    }
    NAT_HIP(hipStreamSynchronize(s));
    float t_ms[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int c = 0; c < 4; ++c)
        NAT_HIP(sev.elapsed(c, &t_ms[c]));
    bool all_conv = true;
    for (int32_t q = 0; q < S; ++q) {
        const bool conv = hres[q] <= opts->gmres_tol;
        all_conv &= conv;
        if (report) {
            report[q].iters = hit[q];
            report[q].converged = conv ? 1 : 0;
            report[q].rel_resid = hres[q];
            report[q].eps = T.sys[q].eps;
            report[q].area = jobs[T.sys[q].inst].mesh->area_total;
            report[q].t_sample_ms = t_ms[0];
            report[q].t_rhs_ms = t_ms[1];
            report[q].t_solve_ms = t_ms[2];
            report[q].t_eval_ms = t_ms[3];
        }
    }
    if (!all_conv)
        return fail(NAT_E_NOCONV, "Monte-Carlo estimate: GMRES stopped above tolerance");
    return NAT_OK;
}

// ---------------------------------------------------------------------------
// A batch as concurrent parts on streams of their own
// ---------------------------------------------------------------------------
namespace {

// pair terms of a job: the right-hand side, about 30 GMRES matvecs and the
// evaluation (sets the automatic part count)
double job_work(const McJob& J) { return (double)J.M * J.N * (31.0 * J.N + J.Q); }
// automatic part count: one part per this much work, at most kAutoLanes
constexpr double kLaneWork = 2e10;

}  // namespace

nat_status run_mc_parts(nat_ctx* ctx, const McJob* jobs, int32_t nj, const nat_mc_opts* opts,
                        nat_solve_report* report, hipStream_t s)
{
    size_t bytes = 0;
    nat_status st = run_mc(ctx, jobs, nj, opts, nullptr, s, &bytes);  // validates every job
    if (st != NAT_OK)
        return st;
    double total = 0.0;
    for (int32_t i = 0; i < nj; ++i)
        total += job_work(jobs[i]);
    int32_t L = opts->n_streams;
    if (L == 0) {
        const double want = total / kLaneWork;
        L = want >= kAutoLanes ? kAutoLanes : (want >= 1.0 ? static_cast<int32_t>(want) : 1);
    }
    L = L < nj ? L : nj;
    if (L <= 1)
        return run_mc(ctx, jobs, nj, opts, report, s, nullptr);

    // job i goes to part i mod L: every part gets a sample of the batch's
    // mix (a work estimate without the iteration counts balanced worse)
    std::vector<std::vector<int32_t>> idx(L);
    for (int32_t i = 0; i < nj; ++i)
        idx[i % L].push_back(i);
    std::vector<int64_t> sys0(nj + 1, 0);  // first report slot of each job
    for (int32_t i = 0; i < nj; ++i)
        sys0[i + 1] = sys0[i] + jobs[i].M;
    st = set_device(ctx);
    if (st != NAT_OK)
        return st;
    if (!ctx->lane_fork)
        NAT_HIP(hipEventCreateWithFlags(&ctx->lane_fork, hipEventDisableTiming));
    for (int32_t l = 0; l < L; ++l) {
        if (!ctx->lane_stream[l])
            NAT_HIP(hipStreamCreateWithFlags(&ctx->lane_stream[l], hipStreamNonBlocking));
        if (!ctx->lane_event[l])
            NAT_HIP(hipEventCreateWithFlags(&ctx->lane_event[l], hipEventDisableTiming));
    }
    // the parts' jobs, and their workspaces grown here, before any part runs
    // (so no part synchronises the device for a growth while others run)
    std::vector<std::vector<McJob>> pjobs(L);
    for (int32_t l = 0; l < L; ++l)
        for (int32_t i : idx[l])
            pjobs[l].push_back(jobs[i]);
    {
        std::vector<size_t> need(L, 0);
        bool grow = false;
        for (int32_t l = 0; l < L; ++l) {
            st = run_mc(ctx, pjobs[l].data(), static_cast<int32_t>(pjobs[l].size()), opts, nullptr, s,
                        &need[l]);
            if (st != NAT_OK)
                return st;
            grow = grow || need[l] > ctx->lane_scratch[l].ws_bytes;
        }
        if (grow) {
            NatScratch* prev = bound_scratch();
            for (int32_t l = 0; l < L && st == NAT_OK; ++l) {
                bind_scratch(&ctx->lane_scratch[l]);
                void* w = nullptr;
                st = workspace(ctx, need[l], &w);
            }
            bind_scratch(prev);
            if (st != NAT_OK)
                return st;
        }
    }
    NAT_HIP(hipEventRecord(ctx->lane_fork, s));
    std::vector<nat_status> sts(L, NAT_OK);
    std::vector<std::string> msgs(L);
    auto part = [&](int32_t l) {
        NatScratch* prev = bound_scratch();
        nat_status r = set_device(ctx);
        if (r == NAT_OK) {
            bind_scratch(&ctx->lane_scratch[l]);
            hipStream_t ls = ctx->lane_stream[l];
            if (hipStreamWaitEvent(ls, ctx->lane_fork, 0) != hipSuccess) {
                r = fail(NAT_E_HIP, "hipStreamWaitEvent");
            } else {
                const std::vector<McJob>& pj = pjobs[l];
                int64_t ns = 0;
                for (int32_t i : idx[l])
                    ns += jobs[i].M;
                std::vector<nat_solve_report> pr(report ? ns : 0);
                r = run_mc(ctx, pj.data(), static_cast<int32_t>(pj.size()), opts,
                           report ? pr.data() : nullptr, ls, nullptr);
                if (report) {
                    int64_t q = 0;
                    for (int32_t i : idx[l])
                        for (int32_t m = 0; m < jobs[i].M; ++m)
                            report[sys0[i] + m] = pr[q++];
                }
            }
            if (hipEventRecord(ctx->lane_event[l], ls) != hipSuccess && r == NAT_OK)
                r = fail(NAT_E_HIP, "hipEventRecord");
        }
        if (r != NAT_OK) {
            char buf[512];
            nat_last_error(buf, sizeof(buf));
            msgs[l] = buf;
        }
        sts[l] = r;
        bind_scratch(prev);
    };
    // a part whose thread cannot be started runs on this thread afterwards
    // (no exception crosses the C ABI)
    std::vector<std::thread> th;
    std::vector<int32_t> inline_parts;
    th.reserve(L - 1);
    for (int32_t l = 1; l < L; ++l) {
        try {
            th.emplace_back(part, l);
        } catch (...) {
            inline_parts.push_back(l);
        }
    }
    part(0);
    for (int32_t l : inline_parts)
        part(l);
    for (std::thread& t : th)
        t.join();
    for (int32_t l = 0; l < L; ++l)
        NAT_HIP(hipStreamWaitEvent(s, ctx->lane_event[l], 0));
    // a hard error first, else non-convergence, else success
    int32_t worst = -1;
    for (int32_t l = 0; l < L; ++l) {
        if (sts[l] != NAT_OK && sts[l] != NAT_E_NOCONV) {
            worst = l;
            break;
        }
        if (sts[l] == NAT_E_NOCONV && worst < 0)
            worst = l;
    }
    if (worst < 0)
        return NAT_OK;
    return fail(sts[worst], "%s", msgs[worst].c_str());
}

}  // namespace nat

extern "C" {

nat_status nat_mcbem_estimate(nat_mesh* mesh, const double* v_n, int32_t n_modes, const double* k,
                              const int32_t* q_tri, const double* q_bary, int32_t Q, int32_t N,
                              uint64_t seed, const nat_mc_opts* opts, double* p_out,
                              double* p_samples, nat_solve_report* report, void* stream)
{
    if (!mesh)
        return nat::fail(NAT_E_INVALID, "nat_mcbem_estimate: mesh is NULL");
    nat::McJob J{mesh, v_n, n_modes, Q, N, k, q_tri, q_bary, seed, p_out, p_samples};
    return nat::run_mc(mesh->ctx, &J, 1, opts, report, static_cast<hipStream_t>(stream), nullptr);
}

nat_status nat_mcbem_poisson_samples(nat_mesh* mesh, int32_t N, uint64_t seed, int32_t* tri,
                                     double* bary, int32_t* n_accepted, void* stream)
{
    using namespace nat;
    if (n_accepted)
        *n_accepted = 0;
    if (!mesh || !tri || !bary)
        return fail(NAT_E_INVALID, "nat_mcbem_poisson_samples: NULL argument");
    if (N < 2 || N > (1 << 24))
        return fail(NAT_E_INVALID, "nat_mcbem_poisson_samples: N = %d", N);
    nat_ctx* ctx = mesh->ctx;
    nat_status st = set_device(ctx);
    if (st != NAT_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<PdInst> pd(1);
    st = pd_instance(mesh, N, seed, 0, 0, &pd[0]);
    if (st != NAT_OK)
        return st;
    const size_t pdb = pd_workspace_bytes(pd[0].M, 1);
    void* ws = nullptr;
    st = workspace(ctx, carve_size<>({sizeof(PdInst), pdb}), &ws);
    if (st != NAT_OK)
        return st;
    Carver cv(ws);
    PdInst* d_pd = cv.take<PdInst>(1);
    void* pws = cv.take<char>(pdb);
    void* pin = nullptr;
    st = pinned(ctx, sizeof(PdInst) + 64, &pin);
    if (st != NAT_OK)
        return st;
    std::memcpy(pin, pd.data(), sizeof(PdInst));
    NAT_HIP(hipMemcpyAsync(d_pd, pin, sizeof(PdInst), hipMemcpyHostToDevice, s));
    std::vector<int32_t> acc;
    st = run_poisson(ctx, d_pd, pd, pws, pdb, tri, bary, s, &acc);
    if (n_accepted && !acc.empty())
        *n_accepted = acc[0];
    return st;
}

nat_status nat_mcbem_field(nat_mesh* mesh, const double* v_n, int32_t n_modes, const double* k,
                           const double* p_samples, int32_t n_samples, uint64_t seed,
                           const double* points, int32_t n_points, const nat_mc_opts* opts,
                           double* p_out, double* abs_out, void* stream)
{
    if (!mesh)
        return nat::fail(NAT_E_INVALID, "nat_mcbem_field: mesh is NULL");
    if (!p_samples)
        return nat::fail(NAT_E_INVALID, "nat_mcbem_field: p_samples is NULL");
    nat::McJob J{mesh, v_n, n_modes, n_points, n_samples, k, nullptr, nullptr, seed, p_out, nullptr};
    J.fpts = points;
    J.p_given = p_samples;
    hipStream_t s = static_cast<hipStream_t>(stream);
    nat_status st = nat::run_mc(mesh->ctx, &J, 1, opts, nullptr, s, nullptr);
    if (st == NAT_OK && abs_out && n_points > 0)
        NAT_HIP(nat::launch_abs(reinterpret_cast<const double2*>(p_out), (int64_t)n_modes * n_points,
                                abs_out, s));
    return st;
}

nat_status nat_mcbem_field_batch(nat_ctx* ctx, const nat_field_job* jobs, int32_t n_jobs,
                                 const nat_mc_opts* opts, void* stream)
{
    if (!ctx || !jobs || n_jobs < 1)
        return nat::fail(NAT_E_INVALID, "nat_mcbem_field_batch: bad arguments");
    std::vector<nat::McJob> J(n_jobs);
    for (int32_t i = 0; i < n_jobs; ++i) {
        const nat_field_job& F = jobs[i];
        if (!F.mesh || F.mesh->ctx != ctx)
            return nat::fail(NAT_E_INVALID, "nat_mcbem_field_batch: job %d: mesh is NULL or of another context",
                             i);
        if (!F.p_samples)
            return nat::fail(NAT_E_INVALID, "nat_mcbem_field_batch: job %d: p_samples is NULL", i);
        J[i] = nat::McJob{F.mesh, F.v_n, F.n_modes, F.n_points, F.n_samples, F.k, nullptr, nullptr, F.seed,
                          F.p_out, nullptr};
        J[i].fpts = F.points;
        J[i].p_given = F.p_samples;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    nat_status st = nat::run_mc(ctx, J.data(), n_jobs, opts, nullptr, s, nullptr);
    if (st != NAT_OK)
        return st;
    for (int32_t i = 0; i < n_jobs; ++i) {
        const nat_field_job& F = jobs[i];
        if (F.abs_out && F.n_points > 0)
            NAT_HIP(nat::launch_abs(reinterpret_cast<const double2*>(F.p_out), (int64_t)F.n_modes * F.n_points,
                                    F.abs_out, s));
    }
    return NAT_OK;
}

nat_status nat_mcbem_estimate_batch(nat_ctx* ctx, const nat_mc_job* jobs, int32_t n_jobs,
                                    const nat_mc_opts* opts, nat_solve_report* reports,
                                    void* stream)
{
    if (!ctx || !jobs || n_jobs < 1)
        return nat::fail(NAT_E_INVALID, "nat_mcbem_estimate_batch: bad arguments");
    std::vector<nat::McJob> J(n_jobs);
    for (int32_t i = 0; i < n_jobs; ++i)
        J[i] = nat::McJob{jobs[i].mesh, jobs[i].v_n, jobs[i].n_modes, jobs[i].n_queries,
                          jobs[i].n_samples, jobs[i].k, jobs[i].q_tri, jobs[i].q_bary,
                          jobs[i].seed, jobs[i].p_out, jobs[i].p_samples};
    if (!opts)
        return nat::fail(NAT_E_INVALID, "nat_mcbem_estimate_batch: opts is NULL");
    return nat::run_mc_parts(ctx, J.data(), n_jobs, opts, reports, static_cast<hipStream_t>(stream));
}

}  // extern "C"

// The served form: the device backend of the request server (arena, worker
// streams, batch runs) and the C entry points of nat_serve.h.  Scheduling
// lives in serve_core.cpp; every solve goes through the same drivers as the
// direct entry points, so a served result equals the same request run alone.
#include <chrono>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "nat_internal.h"
#include "nat_serve.h"
#include "serve_core.h"

namespace nat {
namespace {

using serve::Request;

struct ReqCopy {
    nat_request r;
    std::vector<double> k;
    int32_t max_iters = 0;
};

ReqCopy& copy_of(const Request* q) { return *static_cast<ReqCopy*>(q->payload.get()); }

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

class HipBackend final : public serve::ServeBackend {
public:
    HipBackend(nat_ctx* ctx, const nat_server_opts& o, char* arena, int32_t n_slots)
        : ctx_(ctx), o_(o), arena_(arena), scratch_(n_slots), streams_(n_slots, nullptr),
          t0_(std::chrono::steady_clock::now())
    {
    }

    double now_ms() override
    {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0_)
            .count();
    }

    size_t batch_bytes(Request* const* reqs, int32_t n) override
    {
        const ReqCopy& h = copy_of(reqs[0]);
        if (h.r.kind == NAT_REQ_DENSE)
            return n == 1 ? dense_bytes(h) : 0;
        std::vector<McJob> jobs = mc_jobs(reqs, n);
        nat_mc_opts opts = o_.mc;
        opts.layout = h.r.layout;
        size_t bytes = 0;
        if (run_mc(ctx_, jobs.data(), n, &opts, nullptr, nullptr, &bytes) != NAT_OK)
            return 0;
        return bytes;
    }

    void slot_begin(int32_t slot) override
    {
        if (set_device(ctx_) != NAT_OK ||
            hipStreamCreateWithFlags(&streams_[slot], hipStreamNonBlocking) != hipSuccess)
            streams_[slot] = nullptr;
        bind_scratch(&scratch_[slot]);
        // size the host staging once, so no batch has to grow it
        void* p = nullptr;
        int32_t *hw = nullptr, *dw = nullptr;
        (void)pinned(ctx_, size_t(8) << 20, &p);
        (void)mapped_words(ctx_, 16 + 65536, &hw, &dw);
    }

    void slot_end(int32_t slot) override
    {
        if (streams_[slot]) {
            (void)hipStreamSynchronize(streams_[slot]);
            (void)hipStreamDestroy(streams_[slot]);
            streams_[slot] = nullptr;
        }
        scratch_[slot].ext_ws = nullptr;
        scratch_[slot].ext_ws_bytes = 0;
        release_scratch(ctx_, scratch_[slot]);
        bind_scratch(nullptr);
    }

    void run(int32_t slot, Request* const* reqs, int32_t n, size_t offset, size_t bytes) override
    {
        hipStream_t s = streams_[slot];
        if (!s) {
            for (int32_t i = 0; i < n; ++i)
                reqs[i]->status = NAT_E_HIP;
            return;
        }
        NatScratch& sc = scratch_[slot];
        if (copy_of(reqs[0]).r.kind == NAT_REQ_DENSE) {
            run_dense(sc, *reqs[0], offset, bytes, s);
            return;
        }
        sc.ext_ws = arena_ + offset;
        sc.ext_ws_bytes = bytes;
        const nat_status st = run_mc_batch(reqs, n, s);
        if (st == NAT_E_INVALID && n > 1) {
            // a request failed a device-side check (non-finite data, a query
            // out of range): run each alone to find which
            for (int32_t i = 0; i < n; ++i) {
                if (reqs[i]->solo_bytes > bytes) {
                    reqs[i]->status = st;
                    continue;
                }
                (void)run_mc_batch(reqs + i, 1, s);
            }
        }
        sc.ext_ws = nullptr;
        sc.ext_ws_bytes = 0;
    }

    size_t dense_bytes(const ReqCopy& q) const
    {
        const int32_t nt = q.r.mesh->nT;
        int32_t run = 1, longest = 1;
        for (size_t m = 1; m < q.k.size(); ++m) {
            run = q.k[m] == q.k[m - 1] ? run + 1 : 1;
            longest = run > longest ? run : longest;
        }
        const size_t mats = align256(2 * sizeof(double2) * (size_t)nt * nt);
        size_t ws = bem_assemble_ws_bytes(nt);
        const size_t wsolve = bem_solve_ws_bytes(nt, longest, o_.dense_max_iter);
        ws = ws > wsolve ? ws : wsolve;
        return mats + ws;
    }

private:
    std::vector<McJob> mc_jobs(Request* const* reqs, int32_t n) const
    {
        std::vector<McJob> jobs(n);
        for (int32_t i = 0; i < n; ++i) {
            const ReqCopy& q = copy_of(reqs[i]);
            jobs[i] = McJob{q.r.mesh, q.r.v_n, q.r.n_modes, q.r.n_queries, q.r.n_samples,
                            q.k.data(), q.r.q_tri, q.r.q_bary, q.r.seed, q.r.p_out, nullptr};
        }
        return jobs;
    }

    nat_status run_mc_batch(Request* const* reqs, int32_t n, hipStream_t s)
    {
        std::vector<McJob> jobs = mc_jobs(reqs, n);
        int64_t total = 0;
        for (const McJob& J : jobs)
            total += J.M;
        std::vector<nat_solve_report> reps((size_t)total);
        nat_mc_opts opts = o_.mc;
        opts.layout = copy_of(reqs[0]).r.layout;
        const nat_status st = run_mc(ctx_, jobs.data(), n, &opts, reps.data(), s, nullptr);
        int64_t o = 0;
        for (int32_t i = 0; i < n; ++i) {
            ReqCopy& q = copy_of(reqs[i]);
            const int32_t M = q.r.n_modes;
            if (st != NAT_OK && st != NAT_E_NOCONV) {
                reqs[i]->status = st;
                o += M;
                continue;
            }
            bool conv = true;
            q.max_iters = 0;
            for (int32_t m = 0; m < M; ++m) {
                const nat_solve_report& rp = reps[(size_t)(o + m)];
                conv &= rp.converged != 0;
                q.max_iters = rp.iters > q.max_iters ? rp.iters : q.max_iters;
            }
            if (q.r.report)
                std::memcpy(q.r.report, reps.data() + o, sizeof(nat_solve_report) * M);
            reqs[i]->status = conv ? NAT_OK : NAT_E_NOCONV;
            o += M;
        }
        return st;
    }

    void run_dense(NatScratch& sc, Request& rq, size_t offset, size_t bytes, hipStream_t s)
    {
        ReqCopy& q = copy_of(&rq);
        nat_mesh* mesh = q.r.mesh;
        const int32_t nt = mesh->nT;
        const size_t mats = align256(2 * sizeof(double2) * (size_t)nt * nt);
        nat_bem_op op{};
        op.ctx = ctx_;
        op.mesh = mesh;
        op.n = nt;
        op.burton_miller = o_.dense_burton_miller ? 1 : 0;
        op.d_A = reinterpret_cast<double2*>(arena_ + offset);
        op.d_B = op.d_A + (size_t)nt * nt;
        op.bytes = 0;  // arena memory, not owned
        sc.ext_ws = arena_ + offset + mats;
        sc.ext_ws_bytes = bytes - mats;
        const int32_t M = q.r.n_modes;
        const size_t stride = q.r.layout == NAT_NEUMANN_PER_TRIANGLE ? (size_t)nt : (size_t)mesh->nV;
        bool conv = true;
        nat_status st = NAT_OK;
        q.max_iters = 0;
        for (int32_t m0 = 0; m0 < M && (st == NAT_OK || st == NAT_E_NOCONV);) {
            int32_t m1 = m0 + 1;
            while (m1 < M && q.k[m1] == q.k[m0])
                ++m1;
            op.k = q.k[m0];
            st = bem_assemble_into(&op, s);
            if (st != NAT_OK)
                break;
            std::vector<nat_solve_report> reps((size_t)(m1 - m0));
            st = nat_bem_solve(&op, q.r.v_n + 2 * stride * m0, m1 - m0, q.r.layout, o_.dense_tol,
                               o_.dense_max_iter, q.r.p_out + 2 * (size_t)nt * m0, reps.data(), s);
            if (st == NAT_OK || st == NAT_E_NOCONV) {
                for (const nat_solve_report& rp : reps) {
                    conv &= rp.converged != 0;
                    q.max_iters = rp.iters > q.max_iters ? rp.iters : q.max_iters;
                }
                if (q.r.report)
                    std::memcpy(q.r.report + m0, reps.data(), sizeof(nat_solve_report) * reps.size());
            }
            m0 = m1;
        }
        sc.ext_ws = nullptr;
        sc.ext_ws_bytes = 0;
        rq.status = (st == NAT_OK || st == NAT_E_NOCONV) ? (conv ? NAT_OK : NAT_E_NOCONV) : st;
    }

    nat_ctx* ctx_;
    nat_server_opts o_;
    char* arena_;
    std::vector<NatScratch> scratch_;
    std::vector<hipStream_t> streams_;
    std::chrono::steady_clock::time_point t0_;
};

}  // namespace
}  // namespace nat

struct nat_server {
    nat_ctx* ctx = nullptr;
    nat_server_opts opts{};
    void* arena = nullptr;
    size_t arena_bytes = 0;
    std::unique_ptr<nat::HipBackend> be;
    std::unique_ptr<nat::serve::ServeCore> core;
};

extern "C" {

void nat_server_opts_default(nat_server_opts* o)
{
    if (!o)
        return;
    std::memset(o, 0, sizeof(*o));
    o->n_slots = 4;
    o->max_batch = 64;
    o->hbm_budget = size_t(16) << 30;
    nat_mc_opts_default(&o->mc);
    o->dense_tol = 1e-6;
    o->dense_max_iter = 200;
    o->dense_burton_miller = 1;
}

nat_status nat_server_create(nat_ctx* ctx, const nat_server_opts* o, nat_server** out)
{
    using namespace nat;
    if (!out)
        return fail(NAT_E_INVALID, "nat_server_create: out is NULL");
    *out = nullptr;
    if (!ctx || !o)
        return fail(NAT_E_INVALID, "nat_server_create: NULL argument");
    if (o->n_slots < 1 || o->n_slots > 16 || o->max_batch < 1 || o->max_batch > 4096 ||
        o->hbm_budget == 0)
        return fail(NAT_E_INVALID, "nat_server_create: n_slots %d, max_batch %d, budget %zu",
                    o->n_slots, o->max_batch, o->hbm_budget);
    if (!(o->dense_tol > 0.0) || o->dense_max_iter < 1 || o->dense_max_iter > 1000)
        return fail(NAT_E_INVALID, "nat_server_create: dense solver options");
    const nat_mc_opts& mc = o->mc;
    if (!(mc.eps_scale > 0.0) || !is_finite(mc.eps_scale) || !(mc.gmres_tol > 0.0) ||
        mc.gmres_max_iter < 1 || mc.gmres_max_iter > 1000 ||
        (mc.precision != NAT_PREC_FP32 && mc.precision != NAT_PREC_FP64) ||
        (mc.flags & ~NAT_MC_NO_GRAPH))
        return fail(NAT_E_INVALID, "nat_server_create: Monte-Carlo options");
    nat_status st = set_device(ctx);
    if (st != NAT_OK)
        return st;
    nat_server* srv = new (std::nothrow) nat_server();
    if (!srv)
        return fail(NAT_E_INTERNAL, "out of host memory");
    srv->ctx = ctx;
    srv->opts = *o;
    srv->arena_bytes = o->hbm_budget;
    st = dev_alloc(ctx, srv->arena_bytes, &srv->arena);
    if (st != NAT_OK) {
        delete srv;
        return st;
    }
    srv->be.reset(new HipBackend(ctx, *o, static_cast<char*>(srv->arena), o->n_slots));
    srv->core.reset(new serve::ServeCore(srv->be.get(), o->n_slots, o->max_batch, o->hbm_budget));
    *out = srv;
    return NAT_OK;
}

nat_status nat_server_submit(nat_server* srv, const nat_request* req, uint64_t* ticket)
{
    using namespace nat;
    if (!srv || !req || !ticket)
        return fail(NAT_E_INVALID, "nat_server_submit: NULL argument");
    *ticket = 0;
    const nat_request& r = *req;
    if (r.kind != NAT_REQ_MCBEM && r.kind != NAT_REQ_DENSE)
        return fail(NAT_E_INVALID, "nat_server_submit: kind %d", r.kind);
    if (r.layout != NAT_NEUMANN_PER_VERTEX && r.layout != NAT_NEUMANN_PER_TRIANGLE)
        return fail(NAT_E_INVALID, "nat_server_submit: layout %d", r.layout);
    if (!r.mesh || r.mesh->ctx != srv->ctx)
        return fail(NAT_E_INVALID, "nat_server_submit: mesh is NULL or of another context");
    if (r.n_modes < 1 || r.n_modes > 4096 || !r.k || !r.v_n || !r.p_out)
        return fail(NAT_E_INVALID, "nat_server_submit: n_modes %d or a NULL array", r.n_modes);
    auto q = std::make_shared<ReqCopy>();
    q->r = r;
    q->k.assign(r.k, r.k + r.n_modes);
    q->r.k = nullptr;  // the copy in q->k is used
    std::unique_ptr<serve::Request> rq(new serve::Request());
    rq->payload = q;
    if (r.kind == NAT_REQ_DENSE) {
        for (int32_t m = 0; m < r.n_modes; ++m) {
            const double k = q->k[m];
            if (!is_finite(k) || k < 0.0 || (srv->opts.dense_burton_miller && !(k > 0.0)))
                return fail(NAT_E_INVALID, "nat_server_submit: k[%d] = %g", m, k);
        }
        rq->exclusive = 1;
        rq->group = -1;
        rq->solo_bytes = srv->be->dense_bytes(*q);
    } else {
        rq->group = r.layout;
        serve::Request* one = rq.get();
        rq->solo_bytes = srv->be->batch_bytes(&one, 1);
        if (rq->solo_bytes == 0)
            return NAT_E_INVALID;  // the Monte-Carlo driver's validation set the message
    }
    const size_t need = rq->solo_bytes;
    const int32_t st = srv->core->submit(std::move(rq), ticket);
    if (st == serve::ST_BUDGET)
        return fail(NAT_E_BUDGET, "nat_server_submit: the request needs %zu bytes, the arena has %zu",
                    need, srv->arena_bytes);
    if (st != serve::ST_OK)
        return fail(NAT_E_INVALID, "nat_server_submit: the server is stopping");
    return NAT_OK;
}

nat_status nat_server_wait(nat_server* srv, uint64_t ticket, double timeout_ms,
                           nat_request_result* res)
{
    using namespace nat;
    if (!srv)
        return fail(NAT_E_INVALID, "nat_server_wait: srv is NULL");
    serve::Request r;
    const int32_t st = srv->core->wait(ticket, timeout_ms, &r);
    if (st == serve::ST_PENDING)
        return NAT_E_PENDING;
    if (st == serve::ST_INVALID && r.ticket != ticket)
        return fail(NAT_E_INVALID, "nat_server_wait: unknown ticket %llu", (unsigned long long)ticket);
    if (res) {
        std::memset(res, 0, sizeof(*res));
        res->status = st;
        res->batch_size = r.batch_size;
        res->slot = r.slot;
        res->batch_id = (int64_t)r.batch_id;
        res->max_iters = r.payload ? copy_of(&r).max_iters : 0;
        const bool ran = r.slot >= 0;
        res->queue_ms = ran ? r.t_start - r.t_arrive : r.t_done - r.t_arrive;
        res->run_ms = ran ? r.t_done - r.t_start : 0.0;
        res->latency_ms = r.t_done - r.t_arrive;
    }
    return static_cast<nat_status>(st);
}

nat_status nat_server_cancel(nat_server* srv, uint64_t ticket)
{
    using namespace nat;
    if (!srv)
        return fail(NAT_E_INVALID, "nat_server_cancel: srv is NULL");
    if (srv->core->cancel(ticket) != serve::ST_OK)
        return fail(NAT_E_INVALID, "nat_server_cancel: ticket %llu is not queued",
                    (unsigned long long)ticket);
    return NAT_OK;
}

nat_status nat_server_stats_read(nat_server* srv, nat_server_stats* out)
{
    using namespace nat;
    if (!srv || !out)
        return fail(NAT_E_INVALID, "nat_server_stats_read: NULL argument");
    const serve::ServeStats s = srv->core->stats();
    std::memset(out, 0, sizeof(*out));
    out->submitted = s.submitted;
    out->completed = s.completed;
    out->cancelled = s.cancelled;
    out->batches = s.batches;
    out->max_batch_seen = s.max_batch_seen;
    out->max_concurrent = s.max_concurrent;
    out->peak_bytes = s.peak_bytes;
    out->budget = s.budget;
    return NAT_OK;
}

void nat_server_destroy(nat_server* srv)
{
    if (!srv)
        return;
    srv->core.reset();  // joins the workers after their running batches
    srv->be.reset();
    if (srv->arena) {
        (void)hipSetDevice(srv->ctx->device);
        nat::dev_free(srv->ctx, srv->arena, srv->arena_bytes);
    }
    delete srv;
}

}  // extern "C"

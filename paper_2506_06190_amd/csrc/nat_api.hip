// Host side of libnat_bem: the C entry points of nat_bem.h, the device-memory
// ledger, the mesh registry and the drivers of the Monte-Carlo and dense
// solves.  This file is compiled without floating-point contraction so the
// triangle areas and the cumulative area table are the plain IEEE results
// of the written formulas.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <unordered_map>

#include "nat_internal.h"

namespace {
thread_local std::string g_last_error;

}  // namespace

namespace nat {

nat_status fail(nat_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

nat_status hip_fail(hipError_t e, const char* what)
{
    return fail(NAT_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

nat_status dev_alloc(nat_ctx* ctx, size_t bytes, void** ptr)
{
    *ptr = nullptr;
    if (bytes == 0)
        return NAT_OK;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (ctx->budget && ctx->in_use + bytes > ctx->budget)
            return fail(NAT_E_BUDGET, "HBM budget: need %zu bytes, %zu of %zu in use", bytes,
                        ctx->in_use, ctx->budget);
        ctx->in_use += bytes;
    }
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
        *ptr = nullptr;
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->in_use -= bytes;
        return hip_fail(e, "hipMalloc");
    }
    return NAT_OK;
}

void dev_free(nat_ctx* ctx, void* ptr, size_t bytes)
{
    if (!ptr)
        return;
    (void)hipFree(ptr);
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->in_use -= bytes;
}

namespace {
thread_local NatScratch* t_scratch = nullptr;
}

NatScratch& scratch_of(nat_ctx* ctx) { return t_scratch ? *t_scratch : ctx->scratch; }

void bind_scratch(NatScratch* s) { t_scratch = s; }

NatScratch* bound_scratch() { return t_scratch; }

void release_scratch(nat_ctx* ctx, NatScratch& sc)
{
    std::lock_guard<std::mutex> lk(ctx->capture_mu);  // frees: as in workspace()
    if (sc.ws)
        dev_free(ctx, sc.ws, sc.ws_bytes);
    sc.ws = nullptr;
    sc.ws_bytes = 0;
    if (sc.pinned)
        (void)hipHostFree(sc.pinned);
    sc.pinned = nullptr;
    sc.pinned_bytes = 0;
    if (sc.mapped)
        (void)hipHostFree(sc.mapped);
    sc.mapped = nullptr;
    sc.mapped_dev = nullptr;
    sc.mapped_ints = 0;
    if (sc.graph_exec)
        (void)hipGraphExecDestroy(sc.graph_exec);
    sc.graph_exec = nullptr;
    sc.graph_key.clear();
    if (sc.capture_stream)
        (void)hipStreamDestroy(sc.capture_stream);
    sc.capture_stream = nullptr;
}

nat_status workspace(nat_ctx* ctx, size_t bytes, void** ptr)
{
    NatScratch& sc = scratch_of(ctx);
    if (sc.ext_ws) {
        if (bytes > sc.ext_ws_bytes)
            return fail(NAT_E_BUDGET, "workspace: need %zu bytes, %zu lent", bytes, sc.ext_ws_bytes);
        *ptr = sc.ext_ws;
        return NAT_OK;
    }
    if (bytes <= sc.ws_bytes) {
        *ptr = sc.ws;
        return NAT_OK;
    }
    // grow: release the old block first (the device must be idle for it; no
    // other thread of this context may be capturing a graph meanwhile)
    std::lock_guard<std::mutex> lk(ctx->capture_mu);
    if (sc.ws) {
        NAT_HIP(hipDeviceSynchronize());
        dev_free(ctx, sc.ws, sc.ws_bytes);
        sc.ws = nullptr;
        sc.ws_bytes = 0;
    }
    const size_t want = bytes + bytes / 8;
    nat_status st = dev_alloc(ctx, want, &sc.ws);
    if (st != NAT_OK) {
        st = dev_alloc(ctx, bytes, &sc.ws);
        if (st != NAT_OK)
            return st;
        sc.ws_bytes = bytes;
    } else {
        sc.ws_bytes = want;
    }
    *ptr = sc.ws;
    return NAT_OK;
}

nat_status pinned(nat_ctx* ctx, size_t bytes, void** ptr)
{
    NatScratch& sc = scratch_of(ctx);
    if (sc.noalloc) {
        if (bytes > sc.pinned_bytes)
            return fail(NAT_E_BUDGET, "host staging: need %zu bytes, the fixed block holds %zu", bytes,
                        sc.pinned_bytes);
        *ptr = sc.pinned;
        return NAT_OK;
    }
    if (bytes > sc.pinned_bytes) {
        std::lock_guard<std::mutex> lk(ctx->capture_mu);  // as in workspace()
        if (sc.pinned) {
            NAT_HIP(hipDeviceSynchronize());
            (void)hipHostFree(sc.pinned);
            sc.pinned = nullptr;
            sc.pinned_bytes = 0;
        }
        const size_t want = bytes < 65536 ? 65536 : bytes;
        NAT_HIP(hipHostMalloc(&sc.pinned, want, hipHostMallocDefault));
        sc.pinned_bytes = want;
    }
    *ptr = sc.pinned;
    return NAT_OK;
}

static hipEvent_t prof_event(nat_ctx* ctx)
{
    if (!ctx->prof_pool.empty()) {
        hipEvent_t e = ctx->prof_pool.back();
        ctx->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

ProfSlot prof_slot(nat_ctx* ctx, int32_t kind, double flops)
{
    ProfSlot slot;
    if (!ctx || !ctx->prof || scratch_of(ctx).noalloc)
        return slot;
    std::lock_guard<std::mutex> lk(ctx->mu);
    NatProfEvent ev;
    ev.kind = kind;
    ev.flops = flops;
    ev.start = prof_event(ctx);
    ev.stop = prof_event(ctx);
    if (!ev.start || !ev.stop)
        return slot;
    ctx->prof_pending.push_back(ev);
    slot.start = ev.start;
    slot.stop = ev.stop;
    return slot;
}

void prof_collect(nat_ctx* ctx)
{
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->prof_pending.empty())
        return;
    (void)hipDeviceSynchronize();
    for (const NatProfEvent& e : ctx->prof_pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e.start, e.stop) == hipSuccess) {
            NatProfStat& st = ctx->prof_stat[e.kind];
            st.launches += 1;
            st.ms += ms;
            st.flops += e.flops;
        }
        ctx->prof_pool.push_back(e.start);
        ctx->prof_pool.push_back(e.stop);
    }
    ctx->prof_pending.clear();
}

// Pinned host words the kernels write directly: word 0 is the progress
// counter, words 16.. the per-system flags.  Returns host and device views.
nat_status mapped_words(nat_ctx* ctx, size_t n, int32_t** host, int32_t** dev)
{
    NatScratch& sc = scratch_of(ctx);
    if (sc.noalloc) {
        // host words only: the driver copies the device's flags into them
        if (n > sc.mapped_ints)
            return fail(NAT_E_BUDGET, "host words: need %zu, the fixed block holds %zu", n, sc.mapped_ints);
        *host = sc.mapped;
        *dev = nullptr;
        return NAT_OK;
    }
    if (n > sc.mapped_ints) {
        std::lock_guard<std::mutex> lk(ctx->capture_mu);  // as in workspace()
        if (sc.mapped) {
            NAT_HIP(hipDeviceSynchronize());
            (void)hipHostFree(sc.mapped);
            sc.mapped = nullptr;
            sc.mapped_dev = nullptr;
            sc.mapped_ints = 0;
        }
        const size_t want = n < 4096 ? 4096 : n;
        void* p = nullptr;
        NAT_HIP(hipHostMalloc(&p, want * sizeof(int32_t), hipHostMallocMapped | hipHostMallocCoherent));
        void* d = nullptr;
        hipError_t e = hipHostGetDevicePointer(&d, p, 0);
        if (e != hipSuccess) {
            (void)hipHostFree(p);
            return hip_fail(e, "hipHostGetDevicePointer");
        }
        sc.mapped = static_cast<int32_t*>(p);
        sc.mapped_dev = static_cast<int32_t*>(d);
        sc.mapped_ints = want;
    }
    *host = sc.mapped;
    *dev = sc.mapped_dev;
    return NAT_OK;
}

// Gauss-Legendre nodes and weights on [0,1]: Newton's method on P_n from
// Tricomi's initial guess, P_n and P_n' by the three-term recurrence.
void gauss_legendre01(int n, double* x, double* w)
{
    const double pi = 3.141592653589793;
    for (int i = 1; i <= n; ++i) {
        double t = (4.0 * i - 1.0) / (4.0 * n + 2.0) * pi;
        double z = std::cos(t) * (1.0 - (n - 1.0) / (8.0 * n * n * n));
        double dp = 1.0;
        for (int it = 0; it < 64; ++it) {
            double pm1 = 1.0, p = z;
            for (int l = 2; l <= n; ++l) {
                const double pn = ((2.0 * l - 1.0) * z * p - (l - 1.0) * pm1) / l;
                pm1 = p;
                p = pn;
            }
            if (n == 1) {
                pm1 = 1.0;
                p = z;
            }
            dp = n * (pm1 - z * p) / (1.0 - z * z);
            const double step = p / dp;
            z -= step;
            if (std::fabs(step) <= 1e-17)
                break;
        }
        {
            double pm1 = 1.0, p = z;
            for (int l = 2; l <= n; ++l) {
                const double pn = ((2.0 * l - 1.0) * z * p - (l - 1.0) * pm1) / l;
                pm1 = p;
                p = pn;
            }
            dp = n * (pm1 - z * p) / (1.0 - z * z);
        }
        // z decreases with i; store ascending on [0,1]
        x[n - i] = 0.5 * (1.0 + z);
        w[n - i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
}

}  // namespace nat

using nat::fail;

namespace nat {

bool is_finite(double v) { return std::isfinite(v); }

nat_status set_device(const nat_ctx* ctx)
{
    NAT_HIP(hipSetDevice(ctx->device));
    return NAT_OK;
}

// Validation kernels: flag[0] |= 1 on a bad query record, flag[1] |= 1 on a
// non-finite value.
__global__ void k_check_queries(const int32_t* tri, const double* bary, int32_t Q, int32_t nT,
                                int32_t* flag)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Q)
        return;
    const int32_t t = tri[i];
    const double b1 = bary[2 * i], b2 = bary[2 * i + 1];
    const bool ok = t >= 0 && t < nT && b1 >= 0.0 && b2 >= 0.0 && b1 + b2 <= 1.0 + 1e-12;
    if (!ok)
        atomicOr(flag, 1);
}

__global__ void k_check_finite(const double* v, int64_t n, int32_t* flag)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    if (!isfinite(v[i]))
        atomicOr(flag + 1, 1);
}

// Zero the two flags, run the checks, read them back.
nat_status device_checks(nat_ctx* ctx, int32_t* dflag, const int32_t* q_tri, const double* q_bary,
                         int32_t Q, int32_t nT, const double* vals, int64_t n_vals,
                         hipStream_t s, int32_t* host_flags, bool zero_and_read)
{
    if (zero_and_read)
        NAT_HIP(hipMemsetAsync(dflag, 0, 2 * sizeof(int32_t), s));
    if (Q > 0) {
        hipLaunchKernelGGL(k_check_queries, dim3((Q + 255) / 256), dim3(256), 0, s, q_tri, q_bary,
                           Q, nT, dflag);
        NAT_HIP(hipGetLastError());
    }
    if (n_vals > 0) {
        hipLaunchKernelGGL(k_check_finite, dim3((unsigned)((n_vals + 255) / 256)), dim3(256), 0, s,
                           vals, n_vals, dflag);
        NAT_HIP(hipGetLastError());
    }
    if (!zero_and_read)
        return NAT_OK;
    void* pin = nullptr;
    nat_status st = nat::pinned(ctx, 64, &pin);
    if (st != NAT_OK)
        return st;
    NAT_HIP(hipMemcpyAsync(pin, dflag, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    NAT_HIP(hipStreamSynchronize(s));
    std::memcpy(host_flags, pin, 2 * sizeof(int32_t));
    return NAT_OK;
}

}  // namespace nat

using nat::is_finite;
using nat::set_device;

extern "C" {

const char* nat_status_str(nat_status s)
{
    switch (s) {
    case NAT_OK:
        return "NAT_OK";
    case NAT_E_INVALID:
        return "NAT_E_INVALID";
    case NAT_E_BUDGET:
        return "NAT_E_BUDGET";
    case NAT_E_NOCONV:
        return "NAT_E_NOCONV";
    case NAT_E_HIP:
        return "NAT_E_HIP";
    case NAT_E_INTERNAL:
        return "NAT_E_INTERNAL";
    case NAT_E_PENDING:
        return "NAT_E_PENDING";
    case NAT_E_CANCELLED:
        return "NAT_E_CANCELLED";
    }
    return "NAT_E_UNKNOWN";
}

size_t nat_last_error(char* buf, size_t len)
{
    if (buf && len) {
        const size_t n = g_last_error.size() < len - 1 ? g_last_error.size() : len - 1;
        std::memcpy(buf, g_last_error.data(), n);
        buf[n] = '\0';
    }
    return g_last_error.size();
}

void nat_mc_opts_default(nat_mc_opts* o)
{
    if (!o)
        return;
    o->precision = NAT_PREC_FP32;
    o->layout = NAT_NEUMANN_PER_VERTEX;
    o->eps_scale = 1.0;
    o->gmres_tol = 1e-6;
    o->gmres_max_iter = 200;
    o->flags = 0;
    o->jump = NAT_JUMP_HALF;
    o->n_streams = 0;
}

nat_status nat_ctx_create(int32_t device, size_t hbm_budget_bytes, nat_ctx** out)
{
    if (!out)
        return fail(NAT_E_INVALID, "nat_ctx_create: out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess)
        return nat::hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count)
        return fail(NAT_E_INVALID, "nat_ctx_create: device %d of %d", device, count);
    NAT_HIP(hipSetDevice(device));
    nat_ctx* c = new (std::nothrow) nat_ctx();
    if (!c)
        return fail(NAT_E_INTERNAL, "out of host memory");
    c->device = device;
    c->budget = hbm_budget_bytes;
    nat::tune_defaults(&c->tune);
    // the streams of a batch's automatic parts first, before any other stream
    // of the context: HIP maps streams onto its few hardware queues in
    // creation order, and parts whose streams came after the graph-capture
    // streams ran 10 % slower (a failure here only defers their creation)
    for (int l = 0; l < nat::kAutoLanes; ++l)
        if (hipStreamCreateWithFlags(&c->lane_stream[l], hipStreamNonBlocking) != hipSuccess)
            c->lane_stream[l] = nullptr;
    // quadrature rules of the dense assembly: far 3-point, angular 16-point
    double rules[2 * 3 + 2 * 16];
    nat::gauss_legendre01(3, rules, rules + 3);
    nat::gauss_legendre01(16, rules + 6, rules + 22);
    // a failure below ends the context: its part streams go with it
    auto discard = [c]() {
        for (int l = 0; l < nat::kAutoLanes; ++l)
            if (c->lane_stream[l])
                (void)hipStreamDestroy(c->lane_stream[l]);
        delete c;
    };
    void* d = nullptr;
    nat_status st = nat::dev_alloc(c, sizeof(rules), &d);
    if (st != NAT_OK) {
        discard();
        return st;
    }
    c->d_rules = static_cast<double*>(d);
    e = hipMemcpy(c->d_rules, rules, sizeof(rules), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        nat::dev_free(c, d, sizeof(rules));
        discard();
        return nat::hip_fail(e, "hipMemcpy rules");
    }
    *out = c;
    return NAT_OK;
}

void nat_ctx_destroy(nat_ctx* ctx)
{
    if (!ctx)
        return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    nat::release_scratch(ctx, ctx->scratch);
    for (int l = 0; l < nat_ctx::kMaxLanes; ++l) {
        nat::release_scratch(ctx, ctx->lane_scratch[l]);
        if (ctx->lane_stream[l])
            (void)hipStreamDestroy(ctx->lane_stream[l]);
        if (ctx->lane_event[l])
            (void)hipEventDestroy(ctx->lane_event[l]);
    }
    if (ctx->lane_fork)
        (void)hipEventDestroy(ctx->lane_fork);
    if (ctx->d_rules)
        nat::dev_free(ctx, ctx->d_rules, sizeof(double) * 38);
    nat::prof_collect(ctx);
    for (hipEvent_t e : ctx->prof_pool)
        (void)hipEventDestroy(e);
    delete ctx;
}

size_t nat_ctx_bytes_in_use(const nat_ctx* ctx) { return ctx ? ctx->in_use : 0; }

nat_status nat_profile_enable(nat_ctx* ctx, int32_t enable)
{
    if (!ctx)
        return fail(NAT_E_INVALID, "nat_profile_enable: ctx is NULL");
    nat_status st = set_device(ctx);
    if (st != NAT_OK)
        return st;
    nat::prof_collect(ctx);
    for (auto& x : ctx->prof_stat)
        x = NatProfStat();
    ctx->prof = enable != 0;
    return NAT_OK;
}

int32_t nat_profile_read(nat_ctx* ctx, nat_kernel_stat* out, int32_t max_out)
{
    static const char* names[10] = {"sum32_rhs", "sum32_matvec", "sum32_eval", "sum64",
                                    "gmres_orth", "bem_assemble", "zgemv", "other", "kmatvec32",
                                    "sym32_matvec"};
    if (!ctx || (max_out > 0 && !out))
        return 0;
    if (set_device(ctx) != NAT_OK)
        return 0;
    nat::prof_collect(ctx);
    int32_t n = 0;
    for (int i = 0; i < 10 && n < max_out; ++i) {
        const NatProfStat& st = ctx->prof_stat[i];
        if (st.launches == 0)
            continue;
        std::snprintf(out[n].name, sizeof(out[n].name), "%s", names[i]);
        out[n].launches = st.launches;
        out[n].total_ms = st.ms;
        out[n].flops = st.flops;
        ++n;
    }
    return n;
}

// Closed, consistently oriented, no repeated or out-of-range index.
static nat_status validate_topology(const double* vertices, int32_t n_vertices, const int32_t* tris,
                                    int32_t n_tris)
{
    if (!vertices || !tris)
        return fail(NAT_E_INVALID, "mesh: NULL argument");
    if (n_vertices < 4 || n_tris < 4)
        return fail(NAT_E_INVALID, "mesh: need >= 4 vertices and triangles");
    for (int64_t i = 0; i < 3 * (int64_t)n_vertices; ++i)
        if (!is_finite(vertices[i]))
            return fail(NAT_E_INVALID, "mesh: non-finite vertex coordinate");
    // each directed edge once, its reverse once
    std::unordered_map<uint64_t, int32_t> edges;
    edges.reserve(3 * (size_t)n_tris * 2);
    for (int32_t t = 0; t < n_tris; ++t) {
        const int32_t* f = tris + 3 * t;
        for (int c = 0; c < 3; ++c) {
            if (f[c] < 0 || f[c] >= n_vertices)
                return fail(NAT_E_INVALID, "mesh: triangle %d index out of range", t);
        }
        if (f[0] == f[1] || f[1] == f[2] || f[2] == f[0])
            return fail(NAT_E_INVALID, "mesh: triangle %d repeats a vertex", t);
        for (int c = 0; c < 3; ++c) {
            const uint64_t key = ((uint64_t)(uint32_t)f[c] << 32) | (uint32_t)f[(c + 1) % 3];
            if (++edges[key] > 1)
                return fail(NAT_E_INVALID,
                            "mesh: directed edge %d->%d used twice (inconsistent orientation or "
                            "non-manifold)",
                            f[c], f[(c + 1) % 3]);
        }
    }
    for (const auto& kv : edges) {
        const uint64_t rev = (kv.first << 32) | (kv.first >> 32);
        if (edges.find(rev) == edges.end())
            return fail(NAT_E_INVALID, "mesh: not closed (boundary edge %u->%u)",
                        (unsigned)(kv.first >> 32), (unsigned)(kv.first & 0xffffffffu));
    }
    return NAT_OK;
}

// Connected bodies of a mesh: component label per triangle (triangles that
// share a vertex are in one body), by union-find over the vertices.
static int32_t mesh_bodies(int32_t n_vertices, int32_t n_tris, const int32_t* tris,
                           std::vector<int32_t>& body)
{
    std::vector<int32_t> up(n_vertices);
    for (int32_t v = 0; v < n_vertices; ++v)
        up[v] = v;
    auto root = [&](int32_t v) {
        while (up[v] != v) {
            up[v] = up[up[v]];
            v = up[v];
        }
        return v;
    };
    for (int32_t t = 0; t < n_tris; ++t)
        for (int c = 1; c < 3; ++c) {
            const int32_t a = root(tris[3 * t]), b = root(tris[3 * t + c]);
            if (a != b)
                up[a < b ? b : a] = a < b ? a : b;
        }
    std::vector<int32_t> label(n_vertices, -1);
    int32_t n = 0;
    body.resize(n_tris);
    for (int32_t t = 0; t < n_tris; ++t) {
        const int32_t r = root(tris[3 * t]);
        if (label[r] < 0)
            label[r] = n++;
        body[t] = label[r];
    }
    return n;
}

// Areas, unit normals and the running area sum in the written operation order
// (no contraction in this file).  Rejects zero-area triangles and a body
// (connected component) whose enclosed volume is not positive.
static nat_status mesh_geometry(const double* V, int32_t n_vertices, int32_t n_tris, const int32_t* tris,
                                double* area, double* normal, double* cdf)
{
    std::vector<int32_t> body;
    const int32_t n_bodies = mesh_bodies(n_vertices, n_tris, tris, body);
    std::vector<double> vol6(n_bodies, 0.0);
    double run = 0.0;
    for (int32_t t = 0; t < n_tris; ++t) {
        const double* v0 = V + 3 * (size_t)tris[3 * t + 0];
        const double* v1 = V + 3 * (size_t)tris[3 * t + 1];
        const double* v2 = V + 3 * (size_t)tris[3 * t + 2];
        const double e1[3] = {v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2]};
        const double e2[3] = {v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2]};
        const double c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                             e1[0] * e2[1] - e1[1] * e2[0]};
        const double len = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        if (!(len > 0.0))
            return fail(NAT_E_INVALID, "mesh: triangle %d has zero area", t);
        area[t] = 0.5 * len;
        normal[3 * t + 0] = c[0] / len;
        normal[3 * t + 1] = c[1] / len;
        normal[3 * t + 2] = c[2] / len;
        run = run + area[t];
        cdf[t] = run;
        vol6[body[t]] += v0[0] * (v1[1] * v2[2] - v1[2] * v2[1]) - v0[1] * (v1[0] * v2[2] - v1[2] * v2[0]) +
                         v0[2] * (v1[0] * v2[1] - v1[1] * v2[0]);
    }
    for (int32_t b = 0; b < n_bodies; ++b)
        if (!(vol6[b] > 0.0))
            return fail(NAT_E_INVALID, "mesh: body %d of %d encloses no positive volume (inward orientation?)",
                        b, n_bodies);
    return NAT_OK;
}

// Signed solid angle of triangle (a, b, c) seen from x (Van Oosterom and
// Strackee 1983): positive when x is on the side the triangle's normal
// (b - a) x (c - a) points away from.
static double solid_angle(const double* x, const double* a, const double* b, const double* c)
{
    const double r1[3] = {a[0] - x[0], a[1] - x[1], a[2] - x[2]};
    const double r2[3] = {b[0] - x[0], b[1] - x[1], b[2] - x[2]};
    const double r3[3] = {c[0] - x[0], c[1] - x[1], c[2] - x[2]};
    const double det = r1[0] * (r2[1] * r3[2] - r2[2] * r3[1]) - r1[1] * (r2[0] * r3[2] - r2[2] * r3[0]) +
                       r1[2] * (r2[0] * r3[1] - r2[1] * r3[0]);
    const double l1 = std::sqrt(r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2]);
    const double l2 = std::sqrt(r2[0] * r2[0] + r2[1] * r2[1] + r2[2] * r2[2]);
    const double l3 = std::sqrt(r3[0] * r3[0] + r3[1] * r3[1] + r3[2] * r3[2]);
    const double den = l1 * l2 * l3 + (r1[0] * r2[0] + r1[1] * r2[1] + r1[2] * r2[2]) * l3 +
                       (r1[0] * r3[0] + r1[1] * r3[1] + r1[2] * r3[2]) * l2 +
                       (r2[0] * r3[0] + r2[1] * r3[1] + r2[2] * r3[2]) * l1;
    return 2.0 * std::atan2(det, den);
}

// Free terms c = 1 - Omega/(4 pi) of the exterior surface identity at the
// vertices and on the edges of a closed, outward-oriented mesh (Omega: the
// solid angle the body subtends at the point).
//  * Vertex v: its faces (v, a, b) form a cone; closing it with the cap
//    triangles (c', b, a) through c' = v - L n_v (n_v the area-weighted
//    normal, L the mean length of v's edges) gives a closed oriented surface
//    whose solid angle at its apex v is the cone's.  The faces through v add
//    nothing (v is in their planes), so Omega is the sum over the cap.
//  * Edge a -> b of triangle (a, b, p) with neighbour (b, a, p'): with u, u'
//    the unit directions from the edge to p and p' across it and e the edge
//    direction, turning u about e in the positive sense leaves the body, so
//    the interior dihedral angle phi is the angle from u to u' the other way
//    round: alpha = atan2((u x u').e, u.u'), phi = -alpha (alpha <= 0) or
//    2 pi - alpha; Omega = 2 phi.
static void mesh_free_terms(const double* V, int32_t nV, const int32_t* T, int32_t nT,
                            double* c_vert, double* c_edge)
{
    std::vector<double> nsum(3 * (size_t)nV, 0.0), lsum((size_t)nV, 0.0);
    std::vector<int32_t> deg((size_t)nV, 0);
    for (int32_t t = 0; t < nT; ++t) {
        const int32_t* tv = T + 3 * (size_t)t;
        const double* p0 = V + 3 * (size_t)tv[0];
        const double* p1 = V + 3 * (size_t)tv[1];
        const double* p2 = V + 3 * (size_t)tv[2];
        const double e1[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
        const double e2[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
        const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                              e1[0] * e2[1] - e1[1] * e2[0]};
        for (int i = 0; i < 3; ++i) {
            const int32_t v = tv[i];
            const double* a = V + 3 * (size_t)tv[(i + 1) % 3];
            const double* pv = V + 3 * (size_t)v;
            for (int d = 0; d < 3; ++d)
                nsum[3 * (size_t)v + d] += cr[d];
            lsum[v] += std::sqrt((a[0] - pv[0]) * (a[0] - pv[0]) + (a[1] - pv[1]) * (a[1] - pv[1]) +
                                 (a[2] - pv[2]) * (a[2] - pv[2]));
            deg[v] += 1;
        }
    }
    if (c_vert) {
        std::vector<double> apex(3 * (size_t)nV), omega((size_t)nV, 0.0);
        for (int32_t v = 0; v < nV; ++v) {
            const double* n = &nsum[3 * (size_t)v];
            const double nl = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
            const double L = deg[v] > 0 ? lsum[v] / deg[v] : 0.0;
            for (int d = 0; d < 3; ++d)
                apex[3 * (size_t)v + d] = V[3 * (size_t)v + d] - (nl > 0.0 ? L * n[d] / nl : 0.0);
        }
        for (int32_t t = 0; t < nT; ++t) {
            const int32_t* tv = T + 3 * (size_t)t;
            for (int i = 0; i < 3; ++i) {
                const int32_t v = tv[i];
                const double* a = V + 3 * (size_t)tv[(i + 1) % 3];
                const double* b = V + 3 * (size_t)tv[(i + 2) % 3];
                omega[v] += solid_angle(V + 3 * (size_t)v, &apex[3 * (size_t)v], b, a);
            }
        }
        for (int32_t v = 0; v < nV; ++v)
            c_vert[v] = 1.0 - omega[v] / (4.0 * M_PI);
    }
    if (c_edge) {
        std::unordered_map<uint64_t, int32_t> third;  // directed edge -> opposite vertex
        third.reserve(3 * (size_t)nT * 2);
        auto key = [](int32_t a, int32_t b) {
            return (static_cast<uint64_t>(static_cast<uint32_t>(a)) << 32) | static_cast<uint32_t>(b);
        };
        for (int32_t t = 0; t < nT; ++t) {
            const int32_t* tv = T + 3 * (size_t)t;
            for (int i = 0; i < 3; ++i)
                third[key(tv[(i + 1) % 3], tv[(i + 2) % 3])] = tv[i];
        }
        for (int32_t t = 0; t < nT; ++t) {
            const int32_t* tv = T + 3 * (size_t)t;
            for (int i = 0; i < 3; ++i) {
                const double* a = V + 3 * (size_t)tv[(i + 1) % 3];
                const double* b = V + 3 * (size_t)tv[(i + 2) % 3];
                const double* p = V + 3 * (size_t)tv[i];
                const double* q = V + 3 * (size_t)third.at(key(tv[(i + 2) % 3], tv[(i + 1) % 3]));
                double e[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
                const double el = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
                for (int d = 0; d < 3; ++d)
                    e[d] /= el;
                double u[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
                double w[3] = {q[0] - a[0], q[1] - a[1], q[2] - a[2]};
                const double ue = u[0] * e[0] + u[1] * e[1] + u[2] * e[2];
                const double we = w[0] * e[0] + w[1] * e[1] + w[2] * e[2];
                for (int d = 0; d < 3; ++d) {
                    u[d] -= ue * e[d];
                    w[d] -= we * e[d];
                }
                const double cx[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2],
                                      u[0] * w[1] - u[1] * w[0]};
                const double alpha = std::atan2(cx[0] * e[0] + cx[1] * e[1] + cx[2] * e[2],
                                                u[0] * w[0] + u[1] * w[1] + u[2] * w[2]);
                const double phi = alpha <= 0.0 ? -alpha : 2.0 * M_PI - alpha;
                c_edge[3 * (size_t)t + i] = 1.0 - phi / (2.0 * M_PI);
            }
        }
    }
}

nat_status nat_mesh_free_terms(const double* vertices, int32_t n_vertices, const int32_t* tris,
                               int32_t n_tris, double* c_vert, double* c_edge)
{
    nat_status st = validate_topology(vertices, n_vertices, tris, n_tris);
    if (st != NAT_OK)
        return st;
    std::vector<double> a(n_tris), nn(3 * (size_t)n_tris), c(n_tris);
    st = mesh_geometry(vertices, n_vertices, n_tris, tris, a.data(), nn.data(), c.data());
    if (st != NAT_OK)
        return st;
    mesh_free_terms(vertices, n_vertices, tris, n_tris, c_vert, c_edge);
    return NAT_OK;
}

nat_status nat_mesh_validate(const double* vertices, int32_t n_vertices, const int32_t* tris,
                             int32_t n_tris)
{
    nat_status st = validate_topology(vertices, n_vertices, tris, n_tris);
    if (st != NAT_OK)
        return st;
    std::vector<double> a(n_tris), nn(3 * (size_t)n_tris), c(n_tris);
    return mesh_geometry(vertices, n_vertices, n_tris, tris, a.data(), nn.data(), c.data());
}

nat_status nat_mesh_geometry(const double* vertices, int32_t n_vertices, const int32_t* tris,
                             int32_t n_tris, double* area, double* normal, double* cdf)
{
    if (!area || !normal || !cdf)
        return fail(NAT_E_INVALID, "nat_mesh_geometry: NULL output");
    nat_status st = validate_topology(vertices, n_vertices, tris, n_tris);
    if (st != NAT_OK)
        return st;
    return mesh_geometry(vertices, n_vertices, n_tris, tris, area, normal, cdf);
}

nat_status nat_mesh_create(nat_ctx* ctx, const double* vertices, int32_t n_vertices,
                           const int32_t* tris, int32_t n_tris, nat_mesh** out)
{
    if (!out)
        return fail(NAT_E_INVALID, "nat_mesh_create: out is NULL");
    *out = nullptr;
    if (!ctx)
        return fail(NAT_E_INVALID, "nat_mesh_create: ctx is NULL");
    {
        nat_status st = validate_topology(vertices, n_vertices, tris, n_tris);
        if (st != NAT_OK)
            return st;
    }
    nat_mesh* m = new (std::nothrow) nat_mesh();
    if (!m)
        return fail(NAT_E_INTERNAL, "out of host memory");
    m->ctx = ctx;
    m->nV = n_vertices;
    m->nT = n_tris;
    m->V.assign(vertices, vertices + 3 * (size_t)n_vertices);
    m->T.assign(tris, tris + 3 * (size_t)n_tris);
    m->area.resize(n_tris);
    m->normal.resize(3 * (size_t)n_tris);
    m->cdf.resize(n_tris);
    {
        nat_status gst = mesh_geometry(m->V.data(), n_vertices, n_tris, tris, m->area.data(), m->normal.data(),
                                       m->cdf.data());
        if (gst != NAT_OK) {
            delete m;
            return gst;
        }
    }
    m->area_total = m->cdf[n_tris - 1];
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d)
        lo[d] = hi[d] = m->V[d];
    for (int32_t i = 0; i < n_vertices; ++i)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::fmin(lo[d], m->V[3 * (size_t)i + d]);
            hi[d] = std::fmax(hi[d], m->V[3 * (size_t)i + d]);
        }
    for (int d = 0; d < 3; ++d)
        m->center[d] = 0.5 * (lo[d] + hi[d]);
    m->diameter = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                            (hi[2] - lo[2]) * (hi[2] - lo[2]));

    nat_status st = set_device(ctx);
    if (st != NAT_OK) {
        delete m;
        return st;
    }
    std::vector<double> cvert((size_t)n_vertices), cedge(3 * (size_t)n_tris);
    mesh_free_terms(m->V.data(), n_vertices, m->T.data(), n_tris, cvert.data(), cedge.data());
    const size_t bV = sizeof(double) * 3 * (size_t)n_vertices, bT = sizeof(int32_t) * 3 * (size_t)n_tris,
                 bN = sizeof(double) * 3 * (size_t)n_tris, bC = sizeof(double) * (size_t)n_tris,
                 bCV = sizeof(double) * (size_t)n_vertices, bCE = sizeof(double) * 3 * (size_t)n_tris;
    m->bytes = nat::carve_size<>({bV, bT, bN, bC, bCV, bCE});
    void* blk = nullptr;
    st = nat::dev_alloc(ctx, m->bytes, &blk);
    if (st != NAT_OK) {
        delete m;
        return st;
    }
    nat::Carver cv(blk);
    m->d_V = cv.take<double>(3 * (size_t)n_vertices);
    m->d_T = cv.take<int32_t>(3 * (size_t)n_tris);
    m->d_normal = cv.take<double>(3 * (size_t)n_tris);
    m->d_cdf = cv.take<double>(n_tris);
    m->d_cvert = cv.take<double>(n_vertices);
    m->d_cedge = cv.take<double>(3 * (size_t)n_tris);
    hipError_t e = hipMemcpy(m->d_V, m->V.data(), bV, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(m->d_T, m->T.data(), bT, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(m->d_normal, m->normal.data(), bN, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(m->d_cdf, m->cdf.data(), bC, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(m->d_cvert, cvert.data(), bCV, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(m->d_cedge, cedge.data(), bCE, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        nat::dev_free(ctx, blk, m->bytes);
        delete m;
        return nat::hip_fail(e, "hipMemcpy mesh");
    }
    *out = m;
    return NAT_OK;
}

void nat_mesh_destroy(nat_mesh* m)
{
    if (!m)
        return;
    (void)hipSetDevice(m->ctx->device);
    (void)hipDeviceSynchronize();
    nat::dev_free(m->ctx, m->d_V, m->bytes);
    delete m;
}

nat_status nat_mesh_info(const nat_mesh* m, double* area, int32_t* nV, int32_t* nT)
{
    if (!m)
        return fail(NAT_E_INVALID, "nat_mesh_info: mesh is NULL");
    if (area)
        *area = m->area_total;
    if (nV)
        *nV = m->nV;
    if (nT)
        *nT = m->nT;
    return NAT_OK;
}

nat_status nat_mesh_vertex_queries(const nat_mesh* m, int32_t* tri, double* bary)
{
    if (!m || !tri || !bary)
        return fail(NAT_E_INVALID, "nat_mesh_vertex_queries: NULL argument");
    for (int32_t v = 0; v < m->nV; ++v)
        tri[v] = -1;
    for (int32_t t = 0; t < m->nT; ++t)
        for (int c = 0; c < 3; ++c) {
            const int32_t v = m->T[3 * (size_t)t + c];
            if (tri[v] < 0) {
                tri[v] = t;
                bary[2 * v] = c == 1 ? 1.0 : 0.0;
                bary[2 * v + 1] = c == 2 ? 1.0 : 0.0;
            }
        }
    for (int32_t v = 0; v < m->nV; ++v)
        if (tri[v] < 0)
            return fail(NAT_E_INVALID, "nat_mesh_vertex_queries: vertex %d is in no triangle", v);
    return NAT_OK;
}

nat_status nat_mcbem_samples(nat_mesh* m, int32_t N, uint64_t seed, int32_t* tri, double* bary,
                             void* stream)
{
    if (!m || !tri || !bary)
        return fail(NAT_E_INVALID, "nat_mcbem_samples: NULL argument");
    if (N < 1)
        return fail(NAT_E_INVALID, "nat_mcbem_samples: N = %d", N);
    nat_status st = set_device(m->ctx);
    if (st != NAT_OK)
        return st;
    NAT_HIP(nat::launch_samples(m, N, seed, tri, bary, static_cast<hipStream_t>(stream)));
    return NAT_OK;
}

nat_status nat_field_points(const nat_mesh* m, int32_t kind, int32_t n_a, int32_t n_b, double r_lo,
                            double r_hi, uint64_t seed, double* points, double* coords, void* stream)
{
    if (!m)
        return fail(NAT_E_INVALID, "nat_field_points: mesh is NULL");
    if (kind != NAT_FIELD_SHELL && kind != NAT_FIELD_FFAT_GRID)
        return fail(NAT_E_INVALID, "nat_field_points: kind %d", kind);
    const int64_t n = kind == NAT_FIELD_SHELL ? (int64_t)n_a : (int64_t)n_a * n_b;
    if (n_a < 0 || (kind == NAT_FIELD_FFAT_GRID && n_b < 1) || n > (int64_t(1) << 30))
        return fail(NAT_E_INVALID, "nat_field_points: %d x %d points", n_a, n_b);
    if (!(r_lo > 0.0) || !std::isfinite(r_lo) ||
        (kind == NAT_FIELD_SHELL && (!(r_hi >= r_lo) || !std::isfinite(r_hi))))
        return fail(NAT_E_INVALID, "nat_field_points: radii %g, %g", r_lo, r_hi);
    if (n > 0 && !points)
        return fail(NAT_E_INVALID, "nat_field_points: points is NULL");
    nat_status st = set_device(m->ctx);
    if (st != NAT_OK)
        return st;
    NAT_HIP(nat::launch_field_points(m, kind, n_a, n_b, r_lo, r_hi, seed, points, coords,
                                     static_cast<hipStream_t>(stream)));
    return NAT_OK;
}

}  // extern "C"

namespace nat {

size_t bem_assemble_ws_bytes(int32_t n)
{
    return carve_size<>({sizeof(int32_t) * 4, sizeof(int32_t) * 2 * (size_t)64 * n});
}

nat_status bem_assemble_into(nat_bem_op* op, hipStream_t s)
{
    nat_ctx* ctx = op->ctx;
    nat_mesh* mesh = op->mesh;
    const int32_t n = op->n;
    const double k = op->k;
    BemGeom g{n, mesh->d_V, mesh->d_T, ctx->d_rules};
    const double2 beta = op->burton_miller ? make_double2(0.0, 1.0 / k) : make_double2(0.0, 0.0);
    int32_t cap = 64 * n;
    for (int attempt = 0; attempt < 2; ++attempt) {
        void* ws = nullptr;
        nat_status st = workspace(ctx, carve_size<>({sizeof(int32_t) * 4, sizeof(int32_t) * 2 * (size_t)cap}), &ws);
        if (st != NAT_OK)
            return st;
        Carver cv(ws);
        int32_t* count = cv.take<int32_t>(4);
        int32_t* list = cv.take<int32_t>(2 * (size_t)cap);
        hipError_t e = hipMemsetAsync(count, 0, sizeof(int32_t), s);
        if (e == hipSuccess)
            e = launch_bem_far(g, k, beta, op->d_A, op->d_B, list, cap, count, s,
                               prof_slot(ctx, PK_BEM_ASSEMBLE, 0.0));
        int32_t n_near = 0;
        if (e == hipSuccess)
            e = hipMemcpyAsync(&n_near, count, sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            return hip_fail(e, "dense assembly, far pass");
        if (n_near > cap) {
            cap = n_near;
            continue;
        }
        e = launch_bem_near(g, k, beta, op->d_A, op->d_B, list, n_near, s,
                            prof_slot(ctx, PK_BEM_ASSEMBLE, 0.0));
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            return hip_fail(e, "dense assembly, near pass");
        return NAT_OK;
    }
    return fail(NAT_E_INTERNAL, "dense assembly: near-pair list did not fit");
}

}  // namespace nat

extern "C" {

nat_status nat_bem_assemble(nat_mesh* mesh, double k, int32_t burton_miller, nat_bem_op** out,
                            void* stream)
{
    using namespace nat;
    if (!out)
        return fail(NAT_E_INVALID, "nat_bem_assemble: out is NULL");
    *out = nullptr;
    if (!mesh)
        return fail(NAT_E_INVALID, "nat_bem_assemble: mesh is NULL");
    if (!is_finite(k) || k < 0.0 || (burton_miller && !(k > 0.0)))
        return fail(NAT_E_INVALID, "nat_bem_assemble: k = %g", k);
    nat_ctx* ctx = mesh->ctx;
    nat_status st = set_device(ctx);
    if (st != NAT_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t n = mesh->nT;
    nat_bem_op* op = new (std::nothrow) nat_bem_op();
    if (!op)
        return fail(NAT_E_INTERNAL, "out of host memory");
    op->ctx = ctx;
    op->mesh = mesh;
    op->k = k;
    op->burton_miller = burton_miller ? 1 : 0;
    op->n = n;
    op->bytes = 2 * sizeof(double2) * (size_t)n * n + 256;
    void* blk = nullptr;
    st = dev_alloc(ctx, op->bytes, &blk);
    if (st != NAT_OK) {
        delete op;
        return st;
    }
    op->d_A = static_cast<double2*>(blk);
    op->d_B = op->d_A + (size_t)n * n;
    st = bem_assemble_into(op, s);
    if (st != NAT_OK) {
        nat_bem_op_destroy(op);
        return st;
    }
    *out = op;
    return NAT_OK;
}

}  // extern "C"

namespace nat {
// Split-K partial products of the matrix-core path (none below its threshold).
static size_t zgemm_part_len(int32_t n, int32_t M)
{
    return M >= kZgemmMinRhs ? (size_t)zgemm_segments(n) * 16 * (size_t)n : 0;
}

size_t bem_solve_ws_bytes(int32_t n, int32_t M, int32_t max_iter)
{
    const size_t mm1 = (size_t)max_iter + 1;
    const int32_t nch = gmres_chunks(n);
    return carve_size<>(
        {sizeof(int32_t) * 8, sizeof(double2) * (size_t)M * n, sizeof(double2) * (size_t)M * n,
         sizeof(double2) * (size_t)M * n, sizeof(double2) * (size_t)M * mm1 * n,
         sizeof(double2) * (size_t)M * max_iter * mm1, sizeof(double) * (size_t)M * max_iter,
         sizeof(double2) * (size_t)M * max_iter, sizeof(double2) * (size_t)M * mm1,
         sizeof(double2) * (size_t)M * mm1, sizeof(double) * M, sizeof(double) * M,
         sizeof(int32_t) * M, sizeof(int32_t) * M, sizeof(double2) * (size_t)M * nch * mm1,
         sizeof(double2) * (size_t)M * nch * mm1, sizeof(double) * (size_t)M * nch,
         sizeof(double) * (size_t)M * nch, sizeof(double) * (size_t)M * nch,
         sizeof(double2) * (size_t)M * (mm1 * mm1), sizeof(SysDev) * M,
         sizeof(int2) * (size_t)M * nch, sizeof(double2) * zgemm_part_len(n, M)});
}
}  // namespace nat

extern "C" {

nat_status nat_bem_solve(nat_bem_op* op, const double* v_n, int32_t n_rhs, int32_t layout,
                         double tol, int32_t max_iter, double* p_out, nat_solve_report* report,
                         void* stream)
{
    using namespace nat;
    if (!op || !v_n || !p_out)
        return fail(NAT_E_INVALID, "nat_bem_solve: NULL argument");
    if (n_rhs < 1 || n_rhs > 4096)
        return fail(NAT_E_INVALID, "nat_bem_solve: n_rhs = %d", n_rhs);
    if (layout != NAT_NEUMANN_PER_VERTEX && layout != NAT_NEUMANN_PER_TRIANGLE)
        return fail(NAT_E_INVALID, "nat_bem_solve: layout %d", layout);
    if (!(tol > 0.0) || max_iter < 1 || max_iter > 2000)
        return fail(NAT_E_INVALID, "nat_bem_solve: tol %g, max_iter %d", tol, max_iter);
    nat_ctx* ctx = op->ctx;
    nat_status st = set_device(ctx);
    if (st != NAT_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t n = op->n;
    const int32_t M = n_rhs;
    const int32_t ng = layout == NAT_NEUMANN_PER_TRIANGLE ? n : op->mesh->nV;
    const size_t mm1 = (size_t)max_iter + 1;
    const int32_t nch = gmres_chunks(n);

    // right-hand sides as systems of one instance with equal sizes
    BatchTables T;
    T.inst.resize(1);
    T.inst[0].n = n;
    T.inst[0].n_modes = M;
    T.sys.resize(M);
    for (int32_t r = 0; r < M; ++r) {
        SysDev& Y = T.sys[r];
        Y = SysDev{};
        Y.inst = 0;
        Y.n = n;
        Y.nch = nch;
        Y.off_n = (int64_t)r * n;
        Y.off_v = (int64_t)r * mm1 * n;
        Y.off_ch = (int64_t)r * nch;
        Y.out_n = reinterpret_cast<double2*>(p_out) + (size_t)r * n;
    }
    T.max_items = (int64_t)M * nch;
    const size_t bytes = bem_solve_ws_bytes(n, M, max_iter);
    void* ws = nullptr;
    st = workspace(ctx, bytes, &ws);
    if (st != NAT_OK)
        return st;
    Carver cv(ws);
    int32_t* dcnt = cv.take<int32_t>(8);
    double2* gp = cv.take<double2>((size_t)M * n);
    double2* b = cv.take<double2>((size_t)M * n);
    GmresBatch g{};
    g.n_sys = M;
    g.mmax = max_iter;
    g.tol = tol;
    g.w = cv.take<double2>((size_t)M * n);
    g.V = cv.take<double2>((size_t)M * mm1 * n);
    g.H = cv.take<double2>((size_t)M * max_iter * mm1);
    g.cs = cv.take<double>((size_t)M * max_iter);
    g.sn = cv.take<double2>((size_t)M * max_iter);
    g.gv = cv.take<double2>((size_t)M * mm1);
    g.htot = cv.take<double2>((size_t)M * mm1);
    g.beta = cv.take<double>(M);
    g.resid = cv.take<double>(M);
    g.iters = cv.take<int32_t>(M);
    g.active = cv.take<int32_t>(M);
    g.dp1 = cv.take<double2>((size_t)M * nch * mm1);
    g.dp2 = cv.take<double2>((size_t)M * nch * mm1);
    g.normpart = cv.take<double>((size_t)M * nch);
    g.normpart2 = cv.take<double>((size_t)M * nch);
    g.wnorm0 = cv.take<double>((size_t)M * nch);
    g.gram_stride = (int64_t)mm1 * mm1;
    g.gram = cv.take<double2>((size_t)M * g.gram_stride);
    T.d_sys = cv.take<SysDev>(M);
    T.d_items = cv.take<int2>((size_t)M * nch);
    double2* zpart = M >= kZgemmMinRhs ? cv.take<double2>(zgemm_part_len(n, M)) : nullptr;
    T.d_nitems = dcnt + 2;
    T.d_iter = dcnt + 4;
    g.sys = T.d_sys;
    g.v32 = nullptr;
    g.partial = nullptr;

    int32_t flags[2] = {0, 0};
    st = device_checks(ctx, dcnt, nullptr, nullptr, 0, 0, v_n, 2 * (int64_t)M * ng, s, flags, true);
    if (st != NAT_OK)
        return st;
    if (flags[1])
        return fail(NAT_E_INVALID, "nat_bem_solve: non-finite Neumann data");
    {
        void* pin = nullptr;
        st = pinned(ctx, sizeof(SysDev) * M + 64, &pin);
        if (st != NAT_OK)
            return st;
        std::memcpy(pin, T.sys.data(), sizeof(SysDev) * M);
        NAT_HIP(hipMemcpyAsync(T.d_sys, pin, sizeof(SysDev) * M, hipMemcpyHostToDevice, s));
        NAT_HIP(hipStreamSynchronize(s));
    }

    const double2* gin = reinterpret_cast<const double2*>(v_n);
    if (layout == NAT_NEUMANN_PER_VERTEX) {
        NAT_HIP(launch_panel_data(op->mesh->d_T, n, gin, ng, M, gp, n, s));
    } else {
        NAT_HIP(hipMemcpyAsync(gp, gin, sizeof(double2) * (size_t)M * n, hipMemcpyDeviceToDevice, s));
    }
    StageEvents sev;
    NAT_HIP(sev.create());
    NAT_HIP(hipEventRecord(sev.e[0], s));
    NAT_HIP(launch_zgemv(op->d_B, n, gp, n, M, b, n, nullptr, s, ProfSlot(), zpart));
    std::function<hipError_t(int32_t)> mv = [&](int32_t j) -> hipError_t {
        return launch_zgemv(op->d_A, n, g.V + (size_t)j * n, (int64_t)mm1 * n, M, g.w, n, g.active, s,
                            prof_slot(ctx, PK_ZGEMV, 8.0 * n * (double)n * M), zpart);
    };
    st = gmres_drive(ctx, g, T, b, nullptr, nullptr, mv, false, s);
    if (st != NAT_OK)
        return st;
    NAT_HIP(launch_gmres_solution(g, s));
    NAT_HIP(hipEventRecord(sev.e[1], s));
    prof_collect(ctx);
    void* pin = nullptr;
    st = pinned(ctx, (sizeof(double) + sizeof(int32_t)) * M + 64, &pin);
    if (st != NAT_OK)
        return st;
    double* hres = static_cast<double*>(pin);
    int32_t* hit = reinterpret_cast<int32_t*>(hres + M);
    NAT_HIP(hipMemcpyAsync(hres, g.resid, sizeof(double) * M, hipMemcpyDeviceToHost, s));
    NAT_HIP(hipMemcpyAsync(hit, g.iters, sizeof(int32_t) * M, hipMemcpyDeviceToHost, s));
    NAT_HIP(hipStreamSynchronize(s));
    float t_solve = 0.0f;
    NAT_HIP(hipEventElapsedTime(&t_solve, sev.e[0], sev.e[1]));
    bool all_conv = true;
    for (int32_t m = 0; m < M; ++m) {
        const bool conv = hres[m] <= tol;
        all_conv &= conv;
        if (report) {
            report[m].iters = hit[m];
            report[m].converged = conv ? 1 : 0;
            report[m].rel_resid = hres[m];
            report[m].eps = 0.0;
            report[m].area = op->mesh->area_total;
            report[m].t_sample_ms = 0.0;
            report[m].t_rhs_ms = 0.0;
            report[m].t_solve_ms = t_solve;
            report[m].t_eval_ms = 0.0;
        }
    }
    if (!all_conv)
        return fail(NAT_E_NOCONV, "nat_bem_solve: GMRES stopped above tolerance");
    return NAT_OK;
}

nat_status nat_bem_op_matrices(const nat_bem_op* op, double* A_out, double* B_out, void* stream)
{
    if (!op)
        return fail(NAT_E_INVALID, "nat_bem_op_matrices: op is NULL");
    nat_status st = set_device(op->ctx);
    if (st != NAT_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t bytes = sizeof(double2) * (size_t)op->n * op->n;
    if (A_out)
        NAT_HIP(hipMemcpyAsync(A_out, op->d_A, bytes, hipMemcpyDeviceToDevice, s));
    if (B_out)
        NAT_HIP(hipMemcpyAsync(B_out, op->d_B, bytes, hipMemcpyDeviceToDevice, s));
    return NAT_OK;
}

void nat_bem_op_destroy(nat_bem_op* op)
{
    if (!op)
        return;
    (void)hipSetDevice(op->ctx->device);
    (void)hipDeviceSynchronize();
    nat::dev_free(op->ctx, op->d_A, op->bytes);
    delete op;
}

}  // extern "C"

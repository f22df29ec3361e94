// Autotuning of the FP32 kernel-sum tiling: how many work items a mode
// group is cut into (the source split count follows from it), per size
// bucket of the target count.  The sweep times the batched kernel-sum
// launch plus the fold of its split partials (the consumer every stage
// has) on synthetic sums of each bucket's size in two regimes, one mode
// group alone (where more splits fill the device) and many groups at once
// (where extra splits only add partial-sum traffic), and keeps the
// candidate with the smallest summed slowdown against each regime's best.
// The same sweep picks, per bucket of N, the GMRES matvec form: the
// matrix-free kernel sum or the product with an assembled operator (its
// assembly charged over kTuneAmortize iterations).
// Tables are cached as JSON per device architecture.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "nat_internal.h"

namespace nat {

int32_t tune_bucket(int32_t n)
{
    int32_t b = 0;
    while (b < 31 && (int64_t(1) << (b + 1)) <= (int64_t)n)
        ++b;
    b -= 6;
    return b < 0 ? 0 : (b >= kTuneBuckets ? kTuneBuckets - 1 : b);
}

void tune_defaults(TuneTable* t)
{
    for (int b = 0; b < kTuneBuckets; ++b) {
        t->items_a[b] = t->items_b[b] = 64;
        t->assembled[b] = 0;
        t->symmetric[b] = 1;
        t->rate_free[b] = t->rate_asm[b] = 0.0;
    }
    t->tuned = 0;
}

namespace {

constexpr int32_t kCandidates[] = {16, 32, 64, 128, 256, 512};
constexpr int32_t kNumCand = sizeof(kCandidates) / sizeof(kCandidates[0]);
constexpr int32_t kModes = 8;                 // one full mode group
constexpr double kBusyPairs = 2.0e10;         // pair-modes of the busy regime
constexpr size_t kPartialCap = size_t(256) << 20;
constexpr int32_t kEvalSources = 1024;        // sources of the query-stage sweep
constexpr double kTuneAmortize = 30.0;        // GMRES iterations an assembly is spread over
constexpr size_t kAsmCap = size_t(2) << 30;   // bytes of assembled operators per timing

// Representative size of bucket b: the geometric middle of [2^(b+6), 2^(b+7)).
int32_t bucket_size(int32_t b) { return (int32_t)std::lround(std::ldexp(1.41421356, b + 6)); }

// n points on a sphere of radius 0.1 (Fibonacci lattice), FP32 SoA [3][n],
// with the unit normals in `nrm` when non-null.
void sphere_points(int32_t n, float* xyz, float* nrm)
{
    const double ga = M_PI * (3.0 - std::sqrt(5.0));
    for (int32_t j = 0; j < n; ++j) {
        const double z = 1.0 - 2.0 * (j + 0.5) / n;
        const double r = std::sqrt(std::max(0.0, 1.0 - z * z));
        const double ph = ga * j;
        const double u[3] = {r * std::cos(ph), r * std::sin(ph), z};
        for (int d = 0; d < 3; ++d) {
            xyz[(size_t)d * n + j] = static_cast<float>(0.1 * u[d]);
            if (nrm)
                nrm[(size_t)d * n + j] = static_cast<float>(u[d]);
        }
    }
}

struct Sweep {
    nat_ctx* ctx;
    hipStream_t s;
    hipEvent_t e0 = nullptr, e1 = nullptr;
};

// Time one configuration: `groups` groups of kModes systems over NT
// targets and NS sources with `want` items per group; the minimum over three
// launches after a warm-up one, in milliseconds, or a negative value on
// failure.
double time_config(Sweep& w, int32_t op, int32_t NT, int32_t NS, int32_t groups, int32_t want)
{
    int32_t nsplit = 0, per_split = 0;
    split_rule(NT, NS, want, &nsplit, &per_split);
    const int32_t tiles = target_tiles(NT);
    const int32_t S = groups * kModes;
    const bool eval = op == OP_EVAL;

    std::vector<float> src(6 * (size_t)NS), tgt(eval ? 3 * (size_t)NT : 0);
    sphere_points(NS, src.data(), src.data() + 3 * (size_t)NS);
    if (eval)
        sphere_points(NT, tgt.data(), nullptr);
    std::vector<float2> data((size_t)S * NS);
    for (size_t j = 0; j < data.size(); ++j) {
        const uint32_t h = static_cast<uint32_t>(j) * 2654435761u;
        data[j] = make_float2(static_cast<float>(h & 0xffffu) * 1e-8f - 3e-4f,
                              static_cast<float>(h >> 16) * 1e-8f - 3e-4f);
    }

    const size_t partial_n = (size_t)S * nsplit * NT;
    const size_t vec_n = (size_t)S * std::max(NT, NS);
    const size_t bytes = carve_size<>(
        {sizeof(float) * src.size(), sizeof(float) * tgt.size(), sizeof(float2) * data.size(),
         sizeof(float4) * partial_n, sizeof(InstDev), sizeof(SysDev) * S, sizeof(GroupDev) * groups,
         sizeof(int64_t) * 2, sizeof(double2) * vec_n, sizeof(double2) * vec_n});
    void* ws = nullptr;
    if (workspace(w.ctx, bytes, &ws) != NAT_OK)
        return -1.0;
    Carver cv(ws);
    float* d_src = cv.take<float>(src.size());
    float* d_tgt = cv.take<float>(tgt.size());
    float2* d_data = cv.take<float2>(data.size());
    float4* d_partial = cv.take<float4>(partial_n);
    InstDev* d_inst = cv.take<InstDev>(1);
    SysDev* d_sys = cv.take<SysDev>(S);
    GroupDev* d_groups = cv.take<GroupDev>(groups);
    int64_t* d_counts = cv.take<int64_t>(2);
    double2* d_g = cv.take<double2>(vec_n);
    double2* d_out = cv.take<double2>(vec_n);

    InstDev I{};
    I.n = NS;
    I.q = eval ? NT : 0;
    I.n_modes = S;
    I.sys0 = 0;
    I.nsplit_a = I.nsplit_b = nsplit;
    I.per_split_a = I.per_split_b = per_split;
    I.w = 4.0 * M_PI * 0.01 / NS;
    I.eps = std::sqrt(0.04 / NS);
    I.eps2 = static_cast<float>(I.eps * I.eps);
    I.s32 = d_src;
    I.sn32 = d_src + 3 * (size_t)NS;
    I.q32 = eval ? d_tgt : nullptr;
    std::vector<SysDev> sys(S);
    for (int32_t q = 0; q < S; ++q) {
        SysDev& Y = sys[q];
        Y = SysDev{};
        Y.inst = 0;
        Y.n = NS;
        Y.q = I.q;
        Y.nsplit_a = Y.nsplit_b = nsplit;
        Y.off_n = (int64_t)q * NS;
        Y.off_pa = Y.off_pb = (int64_t)q * nsplit * NT;
        Y.off_q = (int64_t)q * NT;
        Y.out_q = eval ? d_out + (size_t)q * NT : nullptr;
        Y.k = 20.0 + 15.0 * (q % kModes);
        Y.k32 = static_cast<float>(Y.k);
        Y.kappa32 = static_cast<float>(Y.k / (2.0 * M_PI));
    }
    std::vector<GroupDev> grp(groups);
    for (int32_t gi = 0; gi < groups; ++gi) {
        GroupDev& G = grp[gi];
        G = GroupDev{};
        G.inst = 0;
        G.nm = kModes;
        G.tiles = tiles;
        G.nsplit = nsplit;
        G.item0 = (int64_t)gi * tiles * nsplit;
        for (int m = 0; m < kModes; ++m)
            G.sys[m] = gi * kModes + m;
    }
    const int64_t items = (int64_t)groups * tiles * nsplit;
    const int32_t ng32 = groups;
    hipError_t e = hipMemcpyAsync(d_src, src.data(), sizeof(float) * src.size(), hipMemcpyHostToDevice, w.s);
    if (e == hipSuccess && eval)
        e = hipMemcpyAsync(d_tgt, tgt.data(), sizeof(float) * tgt.size(), hipMemcpyHostToDevice, w.s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_data, data.data(), sizeof(float2) * data.size(), hipMemcpyHostToDevice, w.s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_inst, &I, sizeof(InstDev), hipMemcpyHostToDevice, w.s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_sys, sys.data(), sizeof(SysDev) * S, hipMemcpyHostToDevice, w.s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_groups, grp.data(), sizeof(GroupDev) * groups, hipMemcpyHostToDevice, w.s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_counts, &items, sizeof(int64_t), hipMemcpyHostToDevice, w.s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_counts + 1, &ng32, sizeof(int32_t), hipMemcpyHostToDevice, w.s);
    if (e == hipSuccess)
        e = hipMemsetAsync(d_g, 0, sizeof(double2) * vec_n, w.s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(w.s);  // the host vectors go out of scope below
    if (e != hipSuccess)
        return -1.0;

    Sum32Batch p{};
    p.inst = d_inst;
    p.sys = d_sys;
    p.groups = d_groups;
    p.n_items = d_counts;
    p.n_groups = reinterpret_cast<const int32_t*>(d_counts + 1);
    p.a32 = d_data;
    p.b32 = d_data;
    p.active = nullptr;
    p.partial = d_partial;
    const int32_t cap = op == OP_MATVEC ? kGridMatvec : kGridStage;
    const int32_t grid = (int32_t)std::min<int64_t>(items, cap);
    double best = 1e30;
    for (int rep = 0; rep < 4; ++rep) {
        e = hipEventRecord(w.e0, w.s);
        if (e == hipSuccess)
            e = launch_sum32_batch(op, p, grid, w.s);
        if (e == hipSuccess)
            e = launch_reduce32_batch(eval ? OP_EVAL : OP_RHS, p, S, NT, d_g, d_out, w.s);
        if (e == hipSuccess)
            e = hipEventRecord(w.e1, w.s);
        if (e == hipSuccess)
            e = hipEventSynchronize(w.e1);
        float ms = 0.0f;
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, w.e0, w.e1);
        if (e != hipSuccess)
            return -1.0;
        if (rep > 0)  // the first launch warms the caches
            best = std::min(best, (double)ms);
    }
    return best;
}

// The assembled form on S systems of N unknowns: per launch of the matvec
// from the operators plus the fold of its single partial (minimum over three
// after a warm-up), and the assembly in *t_build; milliseconds, negative on
// failure.
double time_assembled(Sweep& w, int32_t N, int32_t S, double* t_build)
{
    const int32_t nch = (N + 255) / 256;
    std::vector<float> src(6 * (size_t)N);
    sphere_points(N, src.data(), src.data() + 3 * (size_t)N);
    std::vector<float2> data((size_t)S * N);
    for (size_t j = 0; j < data.size(); ++j) {
        const uint32_t h = static_cast<uint32_t>(j) * 2654435761u;
        data[j] = make_float2(static_cast<float>(h & 0xffffu) * 1e-8f - 3e-4f,
                              static_cast<float>(h >> 16) * 1e-8f - 3e-4f);
    }
    const size_t vec_n = (size_t)S * N;
    const size_t bytes = carve_size<>(
        {sizeof(float) * src.size(), sizeof(float2) * vec_n, sizeof(float4) * vec_n, sizeof(InstDev),
         sizeof(SysDev) * S, sizeof(int2) * (size_t)S * nch, sizeof(int32_t) * 2, sizeof(int32_t) * S,
         sizeof(float2) * vec_n * N, sizeof(double2) * vec_n, sizeof(double2) * vec_n});
    void* ws = nullptr;
    if (workspace(w.ctx, bytes, &ws) != NAT_OK)
        return -1.0;
    Carver cv(ws);
    float* d_src = cv.take<float>(src.size());
    float2* d_data = cv.take<float2>(vec_n);
    float4* d_partial = cv.take<float4>(vec_n);
    InstDev* d_inst = cv.take<InstDev>(1);
    SysDev* d_sys = cv.take<SysDev>(S);
    int2* d_items = cv.take<int2>((size_t)S * nch);
    int32_t* d_count = cv.take<int32_t>(2);
    int32_t* d_list = cv.take<int32_t>(S);
    float2* d_k = cv.take<float2>(vec_n * N);
    double2* d_g = cv.take<double2>(vec_n);
    double2* d_out = cv.take<double2>(vec_n);

    InstDev I{};
    I.n = N;
    I.n_modes = S;
    I.nsplit_a = I.nsplit_b = 1;
    I.per_split_a = I.per_split_b = N;
    I.w = 4.0 * M_PI * 0.01 / N;
    I.eps = std::sqrt(0.04 / N);
    I.eps2 = static_cast<float>(I.eps * I.eps);
    I.s32 = d_src;
    I.sn32 = d_src + 3 * (size_t)N;
    std::vector<SysDev> sys(S);
    std::vector<int2> items((size_t)S * nch);
    std::vector<int32_t> list(S);
    for (int32_t q = 0; q < S; ++q) {
        SysDev& Y = sys[q];
        Y = SysDev{};
        Y.n = N;
        Y.nch = nch;
        Y.nsplit_a = Y.nsplit_mv = 1;
        Y.off_n = Y.off_pa = (int64_t)q * N;
        Y.off_k = (int64_t)q * N * N;
        Y.k = 20.0 + 15.0 * (q % kModes);
        Y.k32 = static_cast<float>(Y.k);
        Y.kappa32 = static_cast<float>(Y.k / (2.0 * M_PI));
        list[q] = q;
        for (int32_t c = 0; c < nch; ++c)
            items[(size_t)q * nch + c] = make_int2(q, c);
    }
    const int32_t n_items = S * nch;
    hipError_t e = hipMemcpyAsync(d_src, src.data(), sizeof(float) * src.size(), hipMemcpyHostToDevice, w.s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_data, data.data(), sizeof(float2) * vec_n, hipMemcpyHostToDevice, w.s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_inst, &I, sizeof(InstDev), hipMemcpyHostToDevice, w.s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_sys, sys.data(), sizeof(SysDev) * S, hipMemcpyHostToDevice, w.s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice, w.s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_count, &n_items, sizeof(int32_t), hipMemcpyHostToDevice, w.s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_list, list.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice, w.s);
    if (e == hipSuccess)
        e = hipMemsetAsync(d_g, 0, sizeof(double2) * vec_n, w.s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(w.s);  // the host vectors go out of scope below
    if (e != hipSuccess)
        return -1.0;
    float ms = 0.0f;
    e = hipEventRecord(w.e0, w.s);
    if (e == hipSuccess)
        e = launch_assemble32(d_inst, d_sys, d_list, S, N, d_k, w.s);
    if (e == hipSuccess)
        e = hipEventRecord(w.e1, w.s);
    if (e == hipSuccess)
        e = hipEventSynchronize(w.e1);
    if (e == hipSuccess)
        e = hipEventElapsedTime(&ms, w.e0, w.e1);
    if (e != hipSuccess)
        return -1.0;
    *t_build = ms;
    KmvBatch kb{};
    kb.sys = d_sys;
    kb.items = d_items;
    kb.n_items = d_count;
    kb.kmat = d_k;
    kb.b32 = d_data;
    kb.partial = d_partial;
    Sum32Batch p{};
    p.inst = d_inst;
    p.sys = d_sys;
    p.partial = d_partial;
    const int32_t grid = std::min(n_items, kGridKmv);
    double best = 1e30;
    for (int rep = 0; rep < 4; ++rep) {
        e = hipEventRecord(w.e0, w.s);
        if (e == hipSuccess)
            e = launch_kmatvec32(kb, grid, w.s);
        if (e == hipSuccess)
            e = launch_reduce32_batch(OP_RHS, p, S, N, d_g, d_out, w.s);
        if (e == hipSuccess)
            e = hipEventRecord(w.e1, w.s);
        if (e == hipSuccess)
            e = hipEventSynchronize(w.e1);
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, w.e0, w.e1);
        if (e != hipSuccess)
            return -1.0;
        if (rep > 0)
            best = std::min(best, (double)ms);
    }
    return best;
}

// Matvec form of one bucket of N: the matrix-free kernel sum (tiling
// `want`) against the assembled operator, per system and iteration, on as
// many systems as the busy regime (the operators capped at kAsmCap bytes).
nat_status tune_form(Sweep& w, int32_t N, int32_t want, TuneTable* t, int b)
{
    t->assembled[b] = 0;
    const double kbytes = 8.0 * N * (double)N;
    const int32_t groups_busy = (int32_t)std::max(1.0, std::min(256.0, kBusyPairs / (kModes * (double)N * N)));
    int32_t groups = groups_busy;
    while (groups > 1 && groups * kModes * kbytes > (double)kAsmCap)
        groups /= 2;
    const double t_free = time_config(w, OP_MATVEC, N, N, groups, want);
    if (t_free < 0.0)
        return fail(NAT_E_HIP, "autotune: timing launch failed");
    const double per_free = t_free / (groups * kModes);
    t->rate_free[b] = (double)N * N / (per_free * 1e-3);
    const int32_t S = (int32_t)std::min<double>(groups * kModes, std::floor((double)kAsmCap / kbytes));
    if (S < 1)
        return NAT_OK;  // one operator would not fit: matrix-free
    double t_build = 0.0;
    const double t_asm = time_assembled(w, N, S, &t_build);
    if (t_asm < 0.0)
        return fail(NAT_E_HIP, "autotune: timing launch failed");
    const double per_asm = (t_asm + t_build / kTuneAmortize) / S;
    t->rate_asm[b] = (double)N * N / (per_asm * 1e-3);
    t->assembled[b] = per_asm < per_free ? 1 : 0;
    return NAT_OK;
}

// Best items-per-group candidate for one bucket of one stage.
nat_status tune_bucket_op(Sweep& w, int32_t op, int32_t NT, int32_t NS, int32_t* out)
{
    int32_t groups_busy = (int32_t)std::max(1.0, std::min(256.0, kBusyPairs / (kModes * (double)NT * NS)));
    double t1[kNumCand], t2[kNumCand];
    int32_t ns[kNumCand];
    for (int c = 0; c < kNumCand; ++c) {
        int32_t per = 0;
        split_rule(NT, NS, kCandidates[c], &ns[c], &per);
        // candidates with the same split count are the same launch
        int same = -1;
        for (int d = 0; d < c; ++d)
            if (ns[d] == ns[c])
                same = d;
        if (same >= 0) {
            t1[c] = t1[same];
            t2[c] = t2[same];
            continue;
        }
        int32_t gb = groups_busy;
        while (gb > 1 && (size_t)gb * kModes * ns[c] * NT * sizeof(float4) > kPartialCap)
            gb /= 2;
        t1[c] = time_config(w, op, NT, NS, 1, kCandidates[c]);
        t2[c] = time_config(w, op, NT, NS, gb, kCandidates[c]) / gb;
        if (t1[c] < 0.0 || t2[c] < 0.0)
            return fail(NAT_E_HIP, "autotune: timing launch failed");
    }
    const double b1 = *std::min_element(t1, t1 + kNumCand);
    const double b2 = *std::min_element(t2, t2 + kNumCand);
    int best = 0;
    double score_best = 1e30;
    for (int c = 0; c < kNumCand; ++c) {
        const double sc = t1[c] / b1 + t2[c] / b2;
        if (sc < score_best - 1e-3) {  // ties keep the smaller candidate
            score_best = sc;
            best = c;
        }
    }
    *out = kCandidates[best];
    return NAT_OK;
}

std::string arch_key(int device)
{
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return "unknown";
    char buf[320];
    std::snprintf(buf, sizeof(buf), "%s/%dcu", prop.gcnArchName, prop.multiProcessorCount);
    return buf;
}

bool parse_array(const std::string& text, const char* key, int32_t* out)
{
    const size_t k = text.find(std::string("\"") + key + "\"");
    if (k == std::string::npos)
        return false;
    size_t p = text.find('[', k);
    if (p == std::string::npos)
        return false;
    const char* c = text.c_str() + p + 1;
    for (int b = 0; b < kTuneBuckets; ++b) {
        char* end = nullptr;
        const long v = std::strtol(c, &end, 10);
        if (end == c || v < 1 || v > 1 << 20)
            return false;
        out[b] = (int32_t)v;
        c = end;
        while (*c == ',' || *c == ' ' || *c == '\n')
            ++c;
    }
    return *c == ']';
}

bool load_cache(const char* path, const std::string& arch, TuneTable* t)
{
    FILE* f = std::fopen(path, "rb");
    if (!f)
        return false;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0)
        text.append(buf, n);
    std::fclose(f);
    if (text.find("\"device\": \"" + arch + "\"") == std::string::npos)
        return false;
    TuneTable tmp;
    tune_defaults(&tmp);
    if (!parse_array(text, "items_a", tmp.items_a) || !parse_array(text, "items_b", tmp.items_b) ||
        !parse_array(text, "assembled_plus_one", tmp.assembled))
        return false;
    for (int b = 0; b < kTuneBuckets; ++b) {
        if (tmp.assembled[b] != 1 && tmp.assembled[b] != 2)
            return false;
        tmp.assembled[b] -= 1;
    }
    tmp.tuned = 1;
    *t = tmp;
    return true;
}

bool save_cache(const char* path, const std::string& arch, const TuneTable& t)
{
    FILE* f = std::fopen(path, "wb");
    if (!f)
        return false;
    std::fprintf(f, "{\n  \"device\": \"%s\",\n  \"bucket_log2_min\": 6,\n", arch.c_str());
    int32_t asm1[kTuneBuckets];
    for (int b = 0; b < kTuneBuckets; ++b)
        asm1[b] = t.assembled[b] + 1;  // 1: matrix-free, 2: assembled operator
    const int32_t* arrs[3] = {t.items_a, t.items_b, asm1};
    const char* names[3] = {"items_a", "items_b", "assembled_plus_one"};
    for (int a = 0; a < 3; ++a) {
        std::fprintf(f, "  \"%s\": [", names[a]);
        for (int b = 0; b < kTuneBuckets; ++b)
            std::fprintf(f, "%s%d", b ? ", " : "", arrs[a][b]);
        std::fprintf(f, "],\n");
    }
    const double* rates[2] = {t.rate_free, t.rate_asm};
    const char* rnames[2] = {"matvec_pair_modes_per_s_matrix_free", "matvec_pair_modes_per_s_assembled"};
    for (int a = 0; a < 2; ++a) {
        std::fprintf(f, "  \"%s\": [", rnames[a]);
        for (int b = 0; b < kTuneBuckets; ++b)
            std::fprintf(f, "%s%.4g", b ? ", " : "", rates[a][b]);
        std::fprintf(f, "]%s\n", a == 0 ? "," : "");
    }
    std::fprintf(f, "}\n");
    return std::fclose(f) == 0;
}

}  // namespace
}  // namespace nat

extern "C" {

nat_status nat_autotune(nat_ctx* ctx, const char* cache_path, int32_t flags, void* stream)
{
    using namespace nat;
    if (!ctx)
        return fail(NAT_E_INVALID, "nat_autotune: ctx is NULL");
    if (flags & ~NAT_TUNE_FORCE)
        return fail(NAT_E_INVALID, "nat_autotune: flags %d", flags);
    nat_status st = set_device(ctx);
    if (st != NAT_OK)
        return st;
    const std::string arch = arch_key(ctx->device);
    if (cache_path && !(flags & NAT_TUNE_FORCE) && load_cache(cache_path, arch, &ctx->tune))
        return NAT_OK;
    Sweep w;
    w.ctx = ctx;
    w.s = static_cast<hipStream_t>(stream);
    NAT_HIP(hipEventCreate(&w.e0));
    NAT_HIP(hipEventCreate(&w.e1));
    TuneTable t;
    tune_defaults(&t);
    for (int b = 0; b < kTuneBuckets && st == NAT_OK; ++b) {
        const int32_t n = bucket_size(b);
        st = tune_bucket_op(w, OP_MATVEC, n, n, &t.items_a[b]);
        if (st == NAT_OK)
            st = tune_bucket_op(w, OP_EVAL, n, kEvalSources, &t.items_b[b]);
        if (st == NAT_OK)
            st = tune_form(w, n, t.items_a[b], &t, b);
    }
    (void)hipEventDestroy(w.e0);
    (void)hipEventDestroy(w.e1);
    if (st != NAT_OK)
        return st;
    t.tuned = 1;
    ctx->tune = t;
    if (cache_path && !save_cache(cache_path, arch, t))
        return fail(NAT_E_INVALID, "nat_autotune: cannot write %s", cache_path);
    return NAT_OK;
}

nat_status nat_tune_get(const nat_ctx* ctx, int32_t* items_a, int32_t* items_b, int32_t* tuned)
{
    using namespace nat;
    if (!ctx || !items_a || !items_b)
        return fail(NAT_E_INVALID, "nat_tune_get: NULL argument");
    std::memcpy(items_a, ctx->tune.items_a, sizeof(ctx->tune.items_a));
    std::memcpy(items_b, ctx->tune.items_b, sizeof(ctx->tune.items_b));
    if (tuned)
        *tuned = ctx->tune.tuned;
    return NAT_OK;
}

nat_status nat_tune_get_form(const nat_ctx* ctx, int32_t* assembled, double* rate_free,
                             double* rate_asm)
{
    using namespace nat;
    if (!ctx || !assembled)
        return fail(NAT_E_INVALID, "nat_tune_get_form: NULL argument");
    std::memcpy(assembled, ctx->tune.assembled, sizeof(ctx->tune.assembled));
    if (rate_free)
        std::memcpy(rate_free, ctx->tune.rate_free, sizeof(ctx->tune.rate_free));
    if (rate_asm)
        std::memcpy(rate_asm, ctx->tune.rate_asm, sizeof(ctx->tune.rate_asm));
    return NAT_OK;
}

nat_status nat_tune_set_form(nat_ctx* ctx, const int32_t* assembled)
{
    using namespace nat;
    if (!ctx || !assembled)
        return fail(NAT_E_INVALID, "nat_tune_set_form: NULL argument");
    for (int b = 0; b < kTuneBuckets; ++b)
        if (assembled[b] != 0 && assembled[b] != 1)
            return fail(NAT_E_INVALID, "nat_tune_set_form: bucket %d: %d", b, assembled[b]);
    std::memcpy(ctx->tune.assembled, assembled, sizeof(ctx->tune.assembled));
    for (int b = 0; b < kTuneBuckets; ++b)
        ctx->tune.rate_free[b] = ctx->tune.rate_asm[b] = 0.0;
    return NAT_OK;
}

nat_status nat_tune_set(nat_ctx* ctx, const int32_t* items_a, const int32_t* items_b)
{
    using namespace nat;
    if (!ctx || !items_a || !items_b)
        return fail(NAT_E_INVALID, "nat_tune_set: NULL argument");
    for (int b = 0; b < kTuneBuckets; ++b)
        if (items_a[b] < 1 || items_a[b] > (1 << 20) || items_b[b] < 1 || items_b[b] > (1 << 20))
            return fail(NAT_E_INVALID, "nat_tune_set: bucket %d: %d, %d", b, items_a[b], items_b[b]);
    std::memcpy(ctx->tune.items_a, items_a, sizeof(ctx->tune.items_a));
    std::memcpy(ctx->tune.items_b, items_b, sizeof(ctx->tune.items_b));
    ctx->tune.tuned = 1;
    return NAT_OK;
}

}  // extern "C"

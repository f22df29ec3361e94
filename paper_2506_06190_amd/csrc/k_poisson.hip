// Poisson-disk sample sets (Section 4.2: parallel Poisson-disk sampling,
// after Bowers, Wang, Wei & Maletz 2010) for every instance of a batch at
// once.
//
// Definition (shared with no other code; the same steps as the CPU oracle):
//  * candidates: M = 16 N area-uniform points per instance; candidate i
//    draws u0, u1, u2 from counters 3i..3i+2 of stream 6 of the counter
//    generator, takes the triangle of u0 |Gamma| as the samples do and the
//    point (b1, b2) = (u1, u2), folded to (1 - u1, 1 - u2) when u1 + u2 > 1
//    (exact arithmetic, so every machine gets the same point bits);
//  * radius r = 0.72 sqrt(|Gamma| / N); cells of side r / sqrt(3) over the
//    mesh's bounding box (a cell holds at most one accepted point); a cell's
//    candidates in index order;
//  * phase of a cell (cx mod 3, cy mod 3, cz mod 3): cells of one phase are
//    more than r apart, so each phase is decided in parallel;
//  * passes p = 0, 1, ...: phases 0..26 in order, each cell of the phase
//    without an accepted point tries its p-th candidate, accepted unless an
//    accepted point of the 5 x 5 x 5 cells around lies closer than r;
//  * the instance's samples are its first N accepted points in acceptance
//    order (pass, phase, cell).
// Positions and squared distances are formed in FP64 in the written order
// with no contraction (this file is built with -ffp-contract=off), so the
// decisions, and the sample records, are bit-for-bit those of any IEEE
// implementation of the same steps.
#include "nat_internal.h"

#include <hipcub/hipcub.hpp>

namespace nat {
namespace {

constexpr int kPhases = 27;
constexpr int64_t kTagNone = 0x7fff;  // sorts after every real tag
constexpr int32_t kPdMaxPasses = static_cast<int32_t>((kTagNone - 1) / kPhases);  // tags stay below kTagNone

__device__ __forceinline__ uint64_t pd_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double pd_unit(uint64_t seed, uint32_t stream, uint64_t counter)
{
    const uint64_t start = seed ^ (static_cast<uint64_t>(stream) << 56);
    return static_cast<double>(pd_mix64(start + (counter + 1ull) * 0x9E3779B97F4A7C15ull) >> 11) *
           0x1.0p-53;
}

__device__ __forceinline__ int32_t pd_search(const double* __restrict__ cdf, int32_t nT, double tau)
{
    int32_t lo = 0, hi = nT - 1;
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (cdf[mid] > tau)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Candidates of every instance: blockIdx.y is the instance.
__global__ void __launch_bounds__(256) k_pd_candidates(const PdInst* __restrict__ inst,
                                                       int32_t* __restrict__ ctri,
                                                       double* __restrict__ cbary,
                                                       double* __restrict__ cxyz,
                                                       uint64_t* __restrict__ key,
                                                       int32_t* __restrict__ idx)
{
    const PdInst& I = inst[blockIdx.y];
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= I.M)
        return;
    const uint64_t c = 3ull * static_cast<uint64_t>(i);
    const double u0 = pd_unit(I.seed, 6, c);
    const double u1 = pd_unit(I.seed, 6, c + 1);
    const double u2 = pd_unit(I.seed, 6, c + 2);
    const int32_t t = pd_search(I.cdf, I.nT, u0 * I.area);
    double b1 = u1, b2 = u2;
    if (u1 + u2 > 1.0) {
        b1 = 1.0 - u1;
        b2 = 1.0 - u2;
    }
    const int64_t g = I.coff + i;
    ctri[g] = t;
    cbary[2 * g + 0] = b1;
    cbary[2 * g + 1] = b2;
    const double* v0 = I.V + 3 * I.T[3 * t + 0];
    const double* v1 = I.V + 3 * I.T[3 * t + 1];
    const double* v2 = I.V + 3 * I.T[3 * t + 2];
    int64_t cell[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double x = v0[d] + b1 * (v1[d] - v0[d]) + b2 * (v2[d] - v0[d]);
        cxyz[3 * g + d] = x;
        int64_t q = static_cast<int64_t>(floor((x - I.lo[d]) * I.inv_h));
        cell[d] = q < 0 ? 0 : (q >= I.dim[d] ? I.dim[d] - 1 : q);
    }
    key[g] = (static_cast<uint64_t>(blockIdx.y) << kPdInstShift) |
             static_cast<uint64_t>((cell[0] * I.dim[1] + cell[1]) * I.dim[2] + cell[2]);
    idx[g] = static_cast<int32_t>(g);
}

__device__ __forceinline__ void cell_coords(uint64_t key, const PdInst& I, int64_t* c)
{
    const int64_t k = static_cast<int64_t>(key & kPdLocalMask);
    c[2] = k % I.dim[2];
    c[1] = (k / I.dim[2]) % I.dim[1];
    c[0] = k / (I.dim[1] * I.dim[2]);
}

// Phase of every cell, counts of cells per (instance-independent) phase and
// the largest candidate count of a cell.
__global__ void __launch_bounds__(256) k_pd_cells(const PdInst* __restrict__ inst,
                                                  const uint64_t* __restrict__ ukey,
                                                  const int32_t* __restrict__ n_cells,
                                                  const int32_t* __restrict__ count,
                                                  uint32_t* __restrict__ phase,
                                                  int32_t* __restrict__ cell_id,
                                                  int32_t* __restrict__ acc,
                                                  int32_t* __restrict__ tag,
                                                  int32_t* __restrict__ stats)
{
    // the workgroup's counts in LDS first, then one global update per phase
    __shared__ int32_t s_cnt[kPhases + 1];
    if (threadIdx.x <= kPhases)
        s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < *n_cells) {
        const uint64_t k = ukey[c];
        const PdInst& I = inst[k >> kPdInstShift];
        int64_t cc[3];
        cell_coords(k, I, cc);
        const uint32_t ph = static_cast<uint32_t>((cc[0] % 3) * 9 + (cc[1] % 3) * 3 + (cc[2] % 3));
        phase[c] = ph;
        cell_id[c] = c;
        acc[c] = -1;
        tag[c] = static_cast<int32_t>(kTagNone);
        atomicAdd(&s_cnt[ph], 1);
        atomicMax(&s_cnt[kPhases], count[c]);
    }
    __syncthreads();
    if (threadIdx.x < kPhases && s_cnt[threadIdx.x] > 0)
        atomicAdd(&stats[threadIdx.x], s_cnt[threadIdx.x]);
    else if (threadIdx.x == kPhases)
        atomicMax(&stats[kPhases], s_cnt[kPhases]);
}

// Cell lookup: an open-addressing table (linear probing, load factor at most
// one half) from a cell key to the cell's index among the occupied cells,
// one 16-byte slot (key, index) per entry so a probe is one load.  Which
// slot a key lands in depends on the insertion order, but every lookup
// returns the same index, so the decisions do not.
constexpr uint64_t kPdEmpty = ~uint64_t(0);

__device__ __forceinline__ uint32_t pd_slot(uint64_t key, uint32_t mask)
{
    return static_cast<uint32_t>(pd_mix64(key)) & mask;
}

__global__ void __launch_bounds__(256) k_pd_table_clear(ulonglong2* __restrict__ tab, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        tab[i] = make_ulonglong2(kPdEmpty, 0ull);
}

// The table, and every candidate's position in cell order.
__global__ void __launch_bounds__(256) k_pd_table_fill(const uint64_t* __restrict__ ukey,
                                                       const int32_t* __restrict__ n_cells,
                                                       ulonglong2* __restrict__ tab, uint32_t mask,
                                                       const int32_t* __restrict__ sorted_idx, int64_t M,
                                                       const double* __restrict__ cxyz,
                                                       double* __restrict__ cxyz_s)
{
    const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < M) {
        const int64_t g = sorted_idx[c];
#pragma unroll
        for (int d = 0; d < 3; ++d)
            cxyz_s[3 * (int64_t)c + d] = cxyz[3 * g + d];
    }
    if (c >= *n_cells)
        return;
    const uint64_t k = ukey[c];
    uint32_t h = pd_slot(k, mask);
    // the table has at least twice as many slots as keys, so a free slot exists
    while (true) {
        const unsigned long long prev = atomicCAS(reinterpret_cast<unsigned long long*>(&tab[h].x),
                                                  static_cast<unsigned long long>(kPdEmpty),
                                                  static_cast<unsigned long long>(k));
        if (prev == static_cast<unsigned long long>(kPdEmpty)) {
            tab[h].y = static_cast<unsigned long long>(c);
            return;
        }
        h = (h + 1) & mask;
    }
}

__device__ __forceinline__ int32_t pd_lookup(const ulonglong2* __restrict__ tab, uint32_t mask, uint64_t key)
{
    uint32_t h = pd_slot(key, mask);
    while (true) {
        const ulonglong2 e = tab[h];
        if (e.x == key)
            return static_cast<int32_t>(e.y);
        if (e.x == kPdEmpty)
            return -1;
        h = (h + 1) & mask;
    }
}

// Pass p of phase ph: every cell of the phase without an accepted point
// tries its p-th candidate; one wave per cell, each lane checking two of
// the 125 cells around it.  Cells of one phase are more than r apart, so
// none reads what another writes in the same launch.  An accepted point's
// position is copied to its cell (apos).  A rejected candidate of a cell
// with candidates left sets more[p][ph]: the cells that try in pass p + 1
// are exactly those.
__global__ void __launch_bounds__(256) k_pd_try(const PdInst* __restrict__ inst,
                                                const uint64_t* __restrict__ ukey,
                                                const int32_t* __restrict__ start,
                                                const int32_t* __restrict__ count,
                                                const int32_t* __restrict__ sorted_idx,
                                                const int32_t* __restrict__ phase_cells,
                                                int32_t first, int32_t n_phase, int32_t p, int32_t ph,
                                                const double* __restrict__ cxyz_s,
                                                const ulonglong2* __restrict__ tab, uint32_t mask,
                                                int32_t* __restrict__ acc, int32_t* __restrict__ tag,
                                                double* __restrict__ apos, int32_t* __restrict__ more)
{
    const int32_t t = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (t >= n_phase)
        return;
    const int32_t c = phase_cells[first + t];
    const int32_t a0 = acc[c], cnt = count[c], j = start[c] + p;
    const uint64_t k = ukey[c];
    if (a0 >= 0 || cnt <= p)
        return;
    const uint64_t ibits = k & ~kPdLocalMask;
    const PdInst& I = inst[k >> kPdInstShift];
    int64_t cc[3];
    cell_coords(k, I, cc);
    const double x0 = cxyz_s[3 * (int64_t)j], x1 = cxyz_s[3 * (int64_t)j + 1], x2 = cxyz_s[3 * (int64_t)j + 2];
    bool close = false;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = lane + 64 * h;  // neighbour (dx, dy, dz) = (q / 25, q / 5 % 5, q % 5) - 2
        if (q >= 125)
            continue;
        const int64_t nx = cc[0] + q / 25 - 2, ny = cc[1] + (q / 5) % 5 - 2, nz = cc[2] + q % 5 - 2;
        if (nx < 0 || nx >= I.dim[0] || ny < 0 || ny >= I.dim[1] || nz < 0 || nz >= I.dim[2])
            continue;
        const int32_t n = pd_lookup(tab, mask, ibits | static_cast<uint64_t>((nx * I.dim[1] + ny) * I.dim[2] + nz));
        if (n < 0)
            continue;
        const int32_t a = acc[n];
        const double y0 = apos[3 * (int64_t)n], y1 = apos[3 * (int64_t)n + 1], y2 = apos[3 * (int64_t)n + 2];
        if (a < 0)
            continue;
        const double ex = x0 - y0;
        const double ey = x1 - y1;
        const double ez = x2 - y2;
        const double d2 = ex * ex + ey * ey + ez * ez;
        close = close || d2 < I.r2;
    }
    const bool rejected = __ballot(close) != 0;
    if (lane != 0)
        return;
    if (!rejected) {
        acc[c] = sorted_idx[j];
        tag[c] = p * kPhases + ph;
        apos[3 * (int64_t)c] = x0;
        apos[3 * (int64_t)c + 1] = x1;
        apos[3 * (int64_t)c + 2] = x2;
    } else if (cnt > p + 1) {
        more[p * kPhases + ph] = 1;
    }
}

// Acceptance-order keys: (instance, tag, cell); the accepted count of each
// instance.
__global__ void __launch_bounds__(256) k_pd_order(const uint64_t* __restrict__ ukey,
                                                  const int32_t* __restrict__ n_cells,
                                                  const int32_t* __restrict__ acc,
                                                  const int32_t* __restrict__ tag,
                                                  uint64_t* __restrict__ okey,
                                                  int32_t* __restrict__ oval,
                                                  int32_t* __restrict__ n_acc)
{
    const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    bool ok = false;
    int32_t inst = 0;
    if (c < *n_cells) {
        inst = static_cast<int32_t>(ukey[c] >> kPdInstShift);
        const int32_t a = acc[c];
        okey[c] = (static_cast<uint64_t>(inst) << 47) | (static_cast<uint64_t>(tag[c]) << 32) |
                  static_cast<uint64_t>(c);
        oval[c] = a;
        ok = a >= 0;
    }
    // one atomic per instance present in the wave (cells are in key order,
    // so a wave rarely spans more than one instance)
    unsigned long long todo = __ballot(ok);
    while (todo) {
        const int leader = __ffsll(todo) - 1;
        const int32_t li = __shfl(inst, leader, 64);
        const unsigned long long m = __ballot(ok && inst == li);
        if (lane == leader)
            atomicAdd(&n_acc[li], __popcll(m));
        todo &= ~m;
    }
}

// First cell (in key order) of every instance.
__global__ void __launch_bounds__(256) k_pd_inst_first(const uint64_t* __restrict__ ukey,
                                                       const int32_t* __restrict__ n_cells,
                                                       int32_t n_inst, int32_t* __restrict__ first)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_inst)
        return;
    const uint64_t lo_key = static_cast<uint64_t>(i) << kPdInstShift;
    int32_t lo = 0, hi = *n_cells;
    while (lo < hi) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if (ukey[mid] < lo_key)
            lo = mid + 1;
        else
            hi = mid;
    }
    first[i] = lo;
}

// The first N accepted points of every instance, as sample records.
__global__ void __launch_bounds__(256) k_pd_gather(const PdInst* __restrict__ inst,
                                                   const int32_t* __restrict__ first,
                                                   const int32_t* __restrict__ oval_sorted,
                                                   const int32_t* __restrict__ ctri,
                                                   const double* __restrict__ cbary,
                                                   int32_t* __restrict__ tri, double* __restrict__ bary)
{
    const PdInst& I = inst[blockIdx.y];
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= I.N)
        return;
    const int32_t cand = oval_sorted[first[blockIdx.y] + j];
    tri[I.on + j] = ctri[cand];
    bary[2 * (I.on + j) + 0] = cbary[2 * (int64_t)cand + 0];
    bary[2 * (I.on + j) + 1] = cbary[2 * (int64_t)cand + 1];
}

inline dim3 pd_grid(int64_t n) { return dim3(static_cast<unsigned>((n + 255) / 256)); }

// scratch of the library primitives for up to M items
size_t pd_temp_bytes(int64_t M)
{
    size_t sort64 = 0, sort32 = 0, rle = 0, scan = 0;
    // size queries only (no launch); a failed query leaves 0 and the call
    // that uses the scratch then reports the error
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, sort64, (uint64_t*)nullptr, (uint64_t*)nullptr,
                                       (int32_t*)nullptr, (int32_t*)nullptr, (int)M, 0, 64);
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, sort32, (uint32_t*)nullptr, (uint32_t*)nullptr,
                                       (int32_t*)nullptr, (int32_t*)nullptr, (int)M, 0, 5);
    (void)hipcub::DeviceRunLengthEncode::Encode(nullptr, rle, (uint64_t*)nullptr, (uint64_t*)nullptr,
                                          (int32_t*)nullptr, (int32_t*)nullptr, (int)M);
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, scan, (int32_t*)nullptr, (int32_t*)nullptr, (int)M);
    size_t temp = sort64;
    temp = temp > sort32 ? temp : sort32;
    temp = temp > rle ? temp : rle;
    temp = temp > scan ? temp : scan;
    return temp;
}

}  // namespace

// Slots of the cell table: a power of two at least twice the candidate count.
int64_t pd_table_slots(int64_t M)
{
    int64_t h = 2;
    while (h < 2 * M)
        h *= 2;
    return h;
}

size_t pd_workspace_bytes(int64_t total_candidates, int32_t n_inst)
{
    const int64_t M = total_candidates > 0 ? total_candidates : 1;
    const size_t temp = pd_temp_bytes(M);
    const int64_t H = pd_table_slots(M);
    return carve_size<>({sizeof(int32_t) * M, sizeof(double) * 2 * M, sizeof(double) * 3 * M,
                         sizeof(uint64_t) * M, sizeof(uint64_t) * M, sizeof(int32_t) * M,
                         sizeof(int32_t) * M, sizeof(uint64_t) * M, sizeof(int32_t) * M,
                         sizeof(int32_t) * M, sizeof(uint32_t) * M, sizeof(uint32_t) * M,
                         sizeof(int32_t) * M, sizeof(int32_t) * M, sizeof(int32_t) * M,
                         sizeof(int32_t) * M, sizeof(int32_t) * (kPhases + 1) * 2,
                         sizeof(int32_t) * n_inst, sizeof(int32_t) * n_inst, sizeof(int32_t) * 2,
                         sizeof(ulonglong2) * H, sizeof(double) * 3 * M, sizeof(double) * 3 * M,
                         sizeof(int32_t) * kPdMaxPasses * kPhases, temp});
}

// The record of one instance: radius r = 0.72 sqrt(A / N), the grid of
// cells of side r / sqrt(3) over the mesh's bounding box, 16 N candidates.
nat_status pd_instance(const nat_mesh* m, int32_t N, uint64_t seed, int64_t coff, int64_t on, PdInst* out)
{
    PdInst I{};
    I.V = m->d_V;
    I.T = m->d_T;
    I.cdf = m->d_cdf;
    I.nT = m->nT;
    I.area = m->area_total;
    I.seed = seed;
    I.N = N;
    I.M = kPdCandidates * N;
    I.coff = coff;
    I.on = on;
    const double r = kPdRadiusScale * std::sqrt(I.area / (double)N);
    I.r2 = r * r;
    I.inv_h = std::sqrt(3.0) / r;
    double lo[3] = {m->V[0], m->V[1], m->V[2]}, hi[3] = {m->V[0], m->V[1], m->V[2]};
    for (int32_t v = 1; v < m->nV; ++v)
        for (int c = 0; c < 3; ++c) {
            lo[c] = m->V[3 * (size_t)v + c] < lo[c] ? m->V[3 * (size_t)v + c] : lo[c];
            hi[c] = m->V[3 * (size_t)v + c] > hi[c] ? m->V[3 * (size_t)v + c] : hi[c];
        }
    double cells = 1.0;
    for (int c = 0; c < 3; ++c) {
        I.lo[c] = lo[c];
        I.dim[c] = (int64_t)std::floor((hi[c] - lo[c]) * I.inv_h) + 1;
        cells *= (double)I.dim[c];
    }
    if (!(cells < (double)kPdLocalMask))
        return fail(NAT_E_INVALID, "Poisson-disk sampling: %g grid cells over the mesh's box", cells);
    *out = I;
    return NAT_OK;
}

nat_status run_poisson(nat_ctx* ctx, const PdInst* d_inst, const std::vector<PdInst>& h_inst,
                       void* ws, size_t ws_bytes, int32_t* tri, double* bary, hipStream_t s,
                       std::vector<int32_t>* accepted)
{
    const int32_t nj = static_cast<int32_t>(h_inst.size());
    int64_t M = 0;
    int32_t max_m = 0, max_n = 0;
    for (const PdInst& I : h_inst) {
        M += I.M;
        max_m = I.M > max_m ? I.M : max_m;
        max_n = I.N > max_n ? I.N : max_n;
    }
    if (M > (int64_t(1) << 30))
        return fail(NAT_E_INVALID, "Poisson-disk sampling: %lld candidates", (long long)M);
    const size_t need = pd_workspace_bytes(M, nj);
    if (need > ws_bytes)
        return fail(NAT_E_INTERNAL, "Poisson-disk sampling: workspace %zu < %zu", ws_bytes, need);
    Carver cv(ws);
    int32_t* ctri = cv.take<int32_t>(M);
    double* cbary = cv.take<double>(2 * M);
    double* cxyz = cv.take<double>(3 * M);
    uint64_t* key = cv.take<uint64_t>(M);
    uint64_t* key_s = cv.take<uint64_t>(M);
    int32_t* idx = cv.take<int32_t>(M);
    int32_t* idx_s = cv.take<int32_t>(M);
    uint64_t* ukey = cv.take<uint64_t>(M);
    int32_t* count = cv.take<int32_t>(M);
    int32_t* start = cv.take<int32_t>(M);
    uint32_t* phase = cv.take<uint32_t>(M);
    uint32_t* phase_s = cv.take<uint32_t>(M);
    int32_t* cell_id = cv.take<int32_t>(M);
    int32_t* phase_cells = cv.take<int32_t>(M);
    int32_t* acc = cv.take<int32_t>(M);
    int32_t* tag = cv.take<int32_t>(M);
    int32_t* stats = cv.take<int32_t>((kPhases + 1) * 2);   // per-phase counts, max count
    int32_t* first = cv.take<int32_t>(nj);
    int32_t* n_acc = cv.take<int32_t>(nj);
    int32_t* n_cells = cv.take<int32_t>(2);
    const int64_t H = pd_table_slots(M);
    ulonglong2* tab = cv.take<ulonglong2>(H);
    double* cxyz_s = cv.take<double>(3 * M);  // candidate positions in cell order
    double* apos = cv.take<double>(3 * M);    // accepted position of each cell
    int32_t* more = cv.take<int32_t>(kPdMaxPasses * kPhases);
    const uint32_t mask = static_cast<uint32_t>(H - 1);
    // the library primitives' scratch
    const size_t temp_bytes = pd_temp_bytes(M);
    void* temp = cv.take<char>(temp_bytes);
    // the acceptance-order keys reuse the candidate key arrays
    uint64_t* okey = key;
    uint64_t* okey_s = key_s;
    int32_t* oval = idx;
    int32_t* oval_s = count;  // the counts are not needed once the passes are done

    hipLaunchKernelGGL(k_pd_candidates, dim3((max_m + 255) / 256, nj), dim3(256), 0, s, d_inst, ctri, cbary,
                       cxyz, key, idx);
    NAT_HIP(hipGetLastError());
    size_t tb = temp_bytes;
    NAT_HIP(hipcub::DeviceRadixSort::SortPairs(temp, tb, key, key_s, idx, idx_s, (int)M, 0, 64, s));
    tb = temp_bytes;
    NAT_HIP(hipcub::DeviceRunLengthEncode::Encode(temp, tb, key_s, ukey, count, n_cells, (int)M, s));
    tb = temp_bytes;
    NAT_HIP(hipcub::DeviceScan::ExclusiveSum(temp, tb, count, start, (int)M, s));
    NAT_HIP(hipMemsetAsync(stats, 0, sizeof(int32_t) * (kPhases + 1), s));
    NAT_HIP(hipMemsetAsync(n_acc, 0, sizeof(int32_t) * nj, s));
    NAT_HIP(hipMemsetAsync(more, 0, sizeof(int32_t) * kPdMaxPasses * kPhases, s));
    hipLaunchKernelGGL(k_pd_table_clear, pd_grid(std::min<int64_t>(H, 256 * 2048)), dim3(256), 0, s, tab, H);
    NAT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_pd_table_fill, pd_grid(M), dim3(256), 0, s, ukey, n_cells, tab, mask, idx_s, M, cxyz,
                       cxyz_s);
    NAT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_pd_cells, pd_grid(M), dim3(256), 0, s, d_inst, ukey, n_cells, count, phase, cell_id,
                       acc, tag, stats);
    NAT_HIP(hipGetLastError());
    int32_t h_nc = 0;
    int32_t h_stats[kPhases + 1];
    NAT_HIP(hipMemcpyAsync(&h_nc, n_cells, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    NAT_HIP(hipMemcpyAsync(h_stats, stats, sizeof(h_stats), hipMemcpyDeviceToHost, s));
    NAT_HIP(hipStreamSynchronize(s));
    // cells grouped by phase, key order within a phase (the sort is stable)
    tb = temp_bytes;
    NAT_HIP(hipcub::DeviceRadixSort::SortPairs(temp, tb, phase, phase_s, cell_id, phase_cells, h_nc, 0, 5, s));
    int32_t off[kPhases + 1];
    off[0] = 0;
    for (int ph = 0; ph < kPhases; ++ph)
        off[ph + 1] = off[ph] + h_stats[ph];
    const int32_t maxc = h_stats[kPhases];
    if (maxc > kPdMaxPasses)
        return fail(NAT_E_INVALID, "Poisson-disk sampling: %d candidates in one cell", maxc);
    // Passes until no cell has a candidate left to try.  A phase with no cell
    // left to try stays so, and a launch in which no cell tries changes
    // nothing, so pass p may launch the phases still live after pass p - 2
    // (a superset of those live after pass p - 1): the flags of each pass are
    // read back while the next pass runs, and the host waits only for that
    // copy, not for the stream.
    struct FlagEvents {
        hipEvent_t e[2] = {nullptr, nullptr};
        ~FlagEvents()
        {
            for (hipEvent_t x : e)
                if (x)
                    (void)hipEventDestroy(x);
        }
    } fe;
    for (hipEvent_t& x : fe.e)
        NAT_HIP(hipEventCreateWithFlags(&x, hipEventDisableTiming));
    // two slots of flags in pinned memory, past the callers' instance staging
    const size_t stage = (sizeof(PdInst) * static_cast<size_t>(nj) + 63) / 64 * 64;
    void* pin = nullptr;
    nat_status pst = pinned(ctx, stage + 2 * sizeof(int32_t) * kPhases, &pin);
    if (pst != NAT_OK)
        return pst;
    int32_t* hflag = reinterpret_cast<int32_t*>(static_cast<char*>(pin) + stage);
    int32_t live[kPhases];
    for (int ph = 0; ph < kPhases; ++ph)
        live[ph] = 1;
    for (int32_t p = 0; p < maxc; ++p) {
        if (p >= 2) {
            NAT_HIP(hipEventSynchronize(fe.e[p & 1]));  // the flags of pass p - 2
            bool any = false;
            for (int ph = 0; ph < kPhases; ++ph) {
                live[ph] = hflag[(p & 1) * kPhases + ph];
                any = any || live[ph] != 0;
            }
            if (!any)
                break;
        }
        for (int ph = 0; ph < kPhases; ++ph) {
            const int32_t n_ph = off[ph + 1] - off[ph];
            if (n_ph == 0 || !live[ph])
                continue;
            hipLaunchKernelGGL(k_pd_try, dim3(static_cast<unsigned>((n_ph + 3) / 4)), dim3(256), 0, s, d_inst,
                               ukey, start, count, idx_s, phase_cells, off[ph], n_ph, p, ph, cxyz_s, tab, mask,
                               acc, tag, apos, more);
            NAT_HIP(hipGetLastError());
        }
        NAT_HIP(hipMemcpyAsync(hflag + (p & 1) * kPhases, more + (size_t)p * kPhases, sizeof(int32_t) * kPhases,
                               hipMemcpyDeviceToHost, s));
        NAT_HIP(hipEventRecord(fe.e[p & 1], s));
    }
    hipLaunchKernelGGL(k_pd_order, pd_grid(h_nc), dim3(256), 0, s, ukey, n_cells, acc, tag, okey, oval, n_acc);
    NAT_HIP(hipGetLastError());
    tb = temp_bytes;
    NAT_HIP(hipcub::DeviceRadixSort::SortPairs(temp, tb, okey, okey_s, oval, oval_s, h_nc, 0, 64, s));
    hipLaunchKernelGGL(k_pd_inst_first, pd_grid(nj), dim3(256), 0, s, ukey, n_cells, nj, first);
    NAT_HIP(hipGetLastError());
    std::vector<int32_t> h_acc(nj);
    NAT_HIP(hipMemcpyAsync(h_acc.data(), n_acc, sizeof(int32_t) * nj, hipMemcpyDeviceToHost, s));
    NAT_HIP(hipStreamSynchronize(s));
    if (accepted)
        *accepted = h_acc;
    for (int32_t i = 0; i < nj; ++i)
        if (h_acc[i] < h_inst[i].N)
            return fail(NAT_E_INVALID,
                        "Poisson-disk sampling of job %d accepted %d points, fewer than N = %d", i,
                        h_acc[i], h_inst[i].N);
    hipLaunchKernelGGL(k_pd_gather, dim3((max_n + 255) / 256, nj), dim3(256), 0, s, d_inst, first, oval_s, ctri,
                       cbary, tri, bary);
    NAT_HIP(hipGetLastError());
    (void)ctx;
    return NAT_OK;
}

}  // namespace nat

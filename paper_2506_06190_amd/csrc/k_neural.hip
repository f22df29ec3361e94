// Neural acoustic transfer field (Section 3): the grid encoding of the
// listener position (Section 3.3), the positional encoding of the condition
// variables and the frequency (Section 3.2), the MLP of 4 hidden layers of
// 128 (Section 3.4), its mean-squared-error gradient and the Adam update.
//
// One batch is a set of rows; the batch is padded to a multiple of 128 rows
// with zero inputs and zero loss weight.  Activations and back-propagated
// gradients live in HBM in bfloat16, row-major [rows][width].  The products
// run on the matrix cores (32x32x16 bfloat16 MFMA, FP32 accumulation):
//   forward   one fused pass over 128-row tiles: the encoding into LDS, then
//             Z_i = A_i W_i^T + b_i, A_{i+1} = relu(Z_i) (i = 0..3) with the
//             tile's activations kept in LDS, then y (inference) or the
//             activations written out (training)
//   backward  one fused pass per layer i = 3..0 over 128-row tiles:
//             dH_i = dZ_i W_i, dZ_{i-1} = dH_i * [A_i > 0] (or the 16 grid
//             columns of dH_0), and dW_i += dZ_i^T A_i, db_i += sums of dZ_i
//             from the same tile transposed in LDS; each workgroup's dW_i is
//             a partial, added in workgroup order
//   output    dW_4 = dZ_4^T A_4 split over the batch in chunks (A_4 is also
//             kept transposed), added in chunk order
// The output layer (width n_out) and the loss run on the vector units, fused
// with the step back to dZ_3.  The grid-feature gradient is accumulated in
// 64-bit fixed point in LDS partitions of the lattice tables.
#include "nat_internal.h"
#include "nat_neural.h"

#include <cmath>

namespace nat {
namespace {

constexpr int kLevels = 4;
constexpr int kBaseRes = 8;
constexpr int kFeat = 4;
constexpr int kTable = 1 << 16;
constexpr int kPeFreqs = 6;
constexpr int kHidden = 128;
constexpr int kLayers = 5;  // 4 hidden + output
constexpr int kRowTile = 128;   // rows per product tile (4 waves x 32)
constexpr int kGemmGrid = 512;  // workgroups of a forward pass (persistent)
constexpr int kTilePitch = kRowTile + 8;  // LDS pitch (bfloat16) of a 128-wide tile row
constexpr int kMaxNv = 16;
constexpr int kMaxOut = 32;
constexpr uint32_t kPrime1 = 2654435761u;
constexpr uint32_t kPrime2 = 805459861u;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__host__ __device__ constexpr int level_res(int l) { return kBaseRes << l; }
__host__ __device__ constexpr int level_n1cube(int l) { return (level_res(l) + 1) * (level_res(l) + 1) * (level_res(l) + 1); }
__host__ __device__ constexpr bool level_hashed(int l) { return level_n1cube(l) > kTable; }
__host__ __device__ constexpr int level_size(int l) { return level_hashed(l) ? kTable : level_n1cube(l); }
__host__ __device__ constexpr int level_base(int l) { return l == 0 ? 0 : level_base(l - 1) + level_size(l - 1) * kFeat; }
// The grid-feature gradient is accumulated in 64-bit fixed point in LDS
// partitions of the four lattices' tables laid end to end (kGridFloats
// values, every partition a whole number of vertices).
constexpr int kGridFloats = level_base(kLevels);
constexpr int kGridPart = 5112 * kFeat;  // 159.75 KB of 64-bit accumulators (the LDS of a CU)
constexpr int kGridParts = (kGridFloats + kGridPart - 1) / kGridPart;
// Row groups per partition: for 2^18 rows, 21 partitions x 36 groups = 756
// workgroups, about three rounds of one per CU, measured best over 8-64
// groups (a training step 0.662 ms against 0.667 with 24 groups, 0.749 with
// 12 and 0.849 with 8, the other kernels as they were at the time).
constexpr int kGridGroupsMax = 36;
// Threads of a partition workgroup: the accumulators fill the LDS, so one
// workgroup runs per CU, and 16 waves keep its loads and atomics in flight
// (286 us with 4 waves, 207 us with 16, for 2^18 rows).
constexpr int kGridThreads = 1024;
static_assert(kGridPart % kFeat == 0, "partitions hold whole vertices");

__device__ __forceinline__ uint16_t to_bf16(float x)
{
    // round to nearest, ties to even (finite inputs)
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }
__device__ __forceinline__ bool bf16_positive(uint16_t h) { return (h & 0x8000u) == 0 && (h & 0x7fffu) != 0; }

__device__ __forceinline__ bf16x8 load8(const uint16_t* p)
{
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}

// Eight bfloat16 values of one LDS column (stride kTilePitch), packed as one
// MFMA operand fragment.
__device__ __forceinline__ bf16x8 lds_col8(const uint16_t* p)
{
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        w[i] = static_cast<uint32_t>(p[(2 * i) * kTilePitch]) |
               (static_cast<uint32_t>(p[(2 * i + 1) * kTilePitch]) << 16);
    return __builtin_bit_cast(bf16x8, make_uint4(w[0], w[1], w[2], w[3]));
}

struct NfDev {
    int32_t n_v, n_out, D, ld_in;
    float r_lo, inv_span;
    const float* grid[kLevels];  // parameter tables [size][4]
};

// Table index of vertex (i, j, k) of lattice l (Section 3.3; spatial hash
// of instant-NGP for the lattices larger than the table).
__device__ __forceinline__ uint32_t vertex_index(int l, uint32_t i, uint32_t j, uint32_t k)
{
    const uint32_t n1 = level_res(l) + 1;
    if (!level_hashed(l))
        return (i * n1 + j) * n1 + k;
    return (i ^ (j * kPrime1) ^ (k * kPrime2)) & (kTable - 1);
}

struct Corners {
    uint32_t idx[8];
    float w[8];
};

// The cell of lattice l holding unit-cube point u, its 8 corners and their
// trilinear weights (coordinates clamped to [0, 1]; the last cell is closed).
__device__ __forceinline__ void cell_corners(const float (&u)[3], int l, Corners& c)
{
    const int n = level_res(l);
    int ci[3];
    float t[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float p = fminf(fmaxf(u[d], 0.0f), 1.0f) * static_cast<float>(n);
        ci[d] = min(static_cast<int>(floorf(p)), n - 1);
        t[d] = p - static_cast<float>(ci[d]);
    }
    int e = 0;
#pragma unroll
    for (int dx = 0; dx < 2; ++dx)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dz = 0; dz < 2; ++dz) {
                c.idx[e] = vertex_index(l, ci[0] + dx, ci[1] + dy, ci[2] + dz);
                c.w[e] = ((dx ? t[0] : 1.0f - t[0]) * (dy ? t[1] : 1.0f - t[1])) * (dz ? t[2] : 1.0f - t[2]);
                ++e;
            }
}

__device__ __forceinline__ void unit_coords(const NfDev& f, const float* row, float (&u)[3])
{
    u[0] = row[0] * static_cast<float>(1.0 / M_PI);
    u[1] = row[1] * static_cast<float>(0.5 / M_PI);
    u[2] = (row[2] - f.r_lo) * f.inv_span;
}

// Forward pass fused over 128-row tiles (persistent): the rows are encoded
// into LDS, the four hidden layers run on the matrix cores with the tile's
// activations kept in LDS (each wave rewrites its own 32 rows in place once
// its operands are in registers; a layer's weights are staged once per
// tile), and then either the output layer is applied (inference: y, two
// half-row sums per output as in the training output step) or the input and
// the four activations are written to HBM for the backward passes.  The
// products are those of the unfused layers, so the values are the same.
struct NfFwd {
    NfDev f;
    const float* in;
    int32_t B, Bp;
    const uint16_t* wb;          // bfloat16 weights, row-major, layer i at offWb[i]
    int64_t offWb[kLayers];
    const float* bias[kLayers];
    uint16_t* X;                 // [Bp][D] (training) or null
    uint16_t* H[4];              // [Bp][128] (training) or null
    float* y;                    // [B][n_out] (inference) or null
};

__device__ __forceinline__ int fwd_pitch(int D) { return (D > kHidden ? D : kHidden) + 8; }

template <int KS>  // K steps of 16 held in registers: max(D, 128) / 16
__global__ void __launch_bounds__(256) k_nf_fwd(NfFwd p)
{
    extern __shared__ uint4 s_raw[];
    const NfDev& f = p.f;
    const int D = f.D;
    const int pitch = fwd_pitch(D);
    uint16_t* sAct = reinterpret_cast<uint16_t*>(s_raw);  // [128][pitch]
    uint16_t* sW = sAct + kRowTile * pitch;               // [128][pitch]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    const int n_tiles = p.Bp / kRowTile;
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int b0 = tile * kRowTile;
        __syncthreads();
        // encode: threads 0..127 the grid features of row tid, threads
        // 128..255 the positional encodings and the padding of row tid - 128
        {
            const int r = tid & (kRowTile - 1);
            const int b = b0 + r;
            uint16_t* dst = sAct + r * pitch;
            const bool live = b < p.B;
            const float* row = p.in + (size_t)(live ? b : 0) * f.ld_in;
            if (tid < kRowTile) {
                float u[3];
                unit_coords(f, row, u);
#pragma unroll
                for (int l = 0; l < kLevels; ++l) {
                    float acc[kFeat] = {0.0f, 0.0f, 0.0f, 0.0f};
                    if (live) {
                        Corners c;
                        cell_corners(u, l, c);
                        // the 8 gathers in flight together, then the sums in
                        // corner order
                        float4 gq[8];
#pragma unroll
                        for (int e = 0; e < 8; ++e)
                            gq[e] = *reinterpret_cast<const float4*>(f.grid[l] + (size_t)c.idx[e] * kFeat);
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            acc[0] = fmaf(c.w[e], gq[e].x, acc[0]);
                            acc[1] = fmaf(c.w[e], gq[e].y, acc[1]);
                            acc[2] = fmaf(c.w[e], gq[e].z, acc[2]);
                            acc[3] = fmaf(c.w[e], gq[e].w, acc[3]);
                        }
                    }
#pragma unroll
                    for (int q = 0; q < kFeat; ++q)
                        dst[l * kFeat + q] = to_bf16(acc[q]);
                }
            } else {
                int col = kLevels * kFeat;
                for (int sv = 0; sv <= f.n_v; ++sv) {
                    const float x = live ? row[3 + sv] : 0.0f;  // v_0 .. v_{n_v-1}, then f
                    for (int m = 0; m < kPeFreqs; ++m) {
                        float sn, cs;
                        sincospif(ldexpf(x, m), &sn, &cs);
                        dst[col++] = to_bf16(live ? sn : 0.0f);
                        dst[col++] = to_bf16(live ? cs : 0.0f);
                    }
                }
                for (; col < D; ++col)
                    dst[col] = 0;
            }
        }
        __syncthreads();
        if (p.X) {
            const int d8 = D / 8;
            for (int task = tid; task < kRowTile * d8; task += 256) {
                const int r = task / d8, c = task - r * d8;
                // 16-byte aligned: the pitch is a multiple of 8 values
                const uint4 v = *reinterpret_cast<const uint4*>(sAct + r * pitch + c * 8);
                *reinterpret_cast<uint4*>(p.X + (size_t)(b0 + r) * D + c * 8) = v;
            }
        }
        for (int i = 0; i < 4; ++i) {
            const int K = i == 0 ? D : kHidden;
            const int k8 = K / 8;
            __syncthreads();  // the previous layer's weights are no longer read
            // row tid / 2 of W_i, its 16-byte runs c = tid % 2 + 2 j (k8 is
            // even): every load in flight before the first LDS write
            const uint16_t* W = p.wb + p.offWb[i];
            const int wr = tid >> 1, wc = tid & 1;
            const uint16_t* wsrc = W + (size_t)wr * K + wc * 8;
            uint16_t* wdst = sW + wr * pitch + wc * 8;
            static_assert(KS <= 16, "at most 16 runs of 8 per thread");
            {
                uint4 wq[KS];
#pragma unroll
                for (int t = 0; t < KS; ++t)  // runs past the row re-read run 0
                    wq[t] = *reinterpret_cast<const uint4*>(wsrc + (2 * t < k8 ? 16 * t : 0));
                // (a run past the row lands in the padding columns K .. 16 KS - 1,
                // which no product reads)
#pragma unroll
                for (int t = 0; t < KS; ++t)
                    *reinterpret_cast<uint4*>(wdst + 16 * t) = wq[t];
            }
            __syncthreads();
            // the wave's A rows for every K step, then the products
            bf16x8 a[KS];
            const uint16_t* ar = sAct + (wave * 32 + l32) * pitch + half * 8;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                if (ks * 16 < K)
                    a[ks] = *reinterpret_cast<const bf16x8*>(ar + ks * 16);
            f32x16 acc[kHidden / 32];
#pragma unroll
            for (int nb = 0; nb < kHidden / 32; ++nb)
                acc[nb] = f32x16{};
            const uint16_t* bp = sW + l32 * pitch + half * 8;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                if (ks * 16 < K) {
#pragma unroll
                    for (int nb = 0; nb < kHidden / 32; ++nb) {
                        const bf16x8 bv = *reinterpret_cast<const bf16x8*>(bp + nb * 32 * pitch + ks * 16);
                        acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ks], bv, acc[nb], 0, 0, 0);
                    }
                }
            }
            // relu(Z + b) into the wave's own rows (its loads are complete:
            // the stores depend on every product)
            const float* bias = p.bias[i];
#pragma unroll
            for (int nb = 0; nb < kHidden / 32; ++nb) {
                const int col = nb * 32 + l32;
                const float bc = bias[col];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int r = wave * 32 + 8 * (q / 4) + 4 * half + (q % 4);
                    sAct[r * pitch + col] = to_bf16(fmaxf(acc[nb][q] + bc, 0.0f));
                }
            }
            if (p.H[i]) {
                __syncthreads();
                for (int task = tid; task < kRowTile * (kHidden / 8); task += 256) {
                    const int r = task >> 4, c = task & 15;
                    const uint4 v = *reinterpret_cast<const uint4*>(sAct + r * pitch + c * 8);
                    *reinterpret_cast<uint4*>(p.H[i] + (size_t)(b0 + r) * kHidden + c * 8) = v;
                }
            }
        }
        if (p.y) {
            // output layer: W_4 as floats into the weight area, two half-row
            // sums per (row, output)
            const int nO = f.n_out;
            float* sW4 = reinterpret_cast<float*>(sW);
            __syncthreads();
            const uint16_t* W4 = p.wb + p.offWb[4];
            for (int e = tid; e < nO * kHidden; e += 256)
                sW4[e] = from_bf16(W4[e]);
            __syncthreads();
            const int r = tid >> 1, hf = tid & 1;
            const int row = b0 + r;
            for (int oi = 0; oi < nO; ++oi) {
                float part = 0.0f;
                const uint16_t* hr = sAct + r * pitch + hf * 64;
                const float* wr = sW4 + oi * kHidden + hf * 64;
#pragma unroll 8
                for (int k = 0; k < 64; ++k)
                    part = fmaf(from_bf16(hr[k]), wr[k], part);
                part += __shfl_xor(part, 1, 64);
                if (hf == 0 && row < p.B)
                    p.y[(size_t)row * nO + oi] = part + p.bias[4][oi];
            }
        }
    }
}

// Fused backward pass of layer i (input width IN <= 32 NB) over 128-row
// tiles (persistent):
//   dH_i^T = W_i^T dZ_i^T: wave w computes rows k = 32 w .. 32 w + 31, its
//            W_i^T fragments held in registers, dZ_i read row-major;
//   dZ_{i-1} = dH_i [A_i > 0] stored row-major (GRID: the 16 grid columns of
//            dH_0 in FP32 instead, and the workgroup's max |dH_0|);
//   dW_i  += dZ_i^T A_i and db_i += column sums of dZ_i, wave w computing
//            rows m = 32 w .. 32 w + 31, from the tile's dZ_i and A_i
//            transposed into LDS (both operands contiguous along the rows).
// Each workgroup writes its dW_i, db_i as one partial.
struct NfBwd {
    const uint16_t* dz;    // dZ_i [Bp][128]
    const uint16_t* act;   // A_i [Bp][in_dim]
    const uint16_t* wt;    // W_i^T [in_dim][128]
    int32_t in_dim, Bp;
    uint16_t* dz_prev;     // dZ_{i-1} [Bp][128]
    float* dh0;            // [Bp][16]
    float* gmax;           // [gridDim.x]
    float* Pw;             // [gridDim.x][128][in_dim]
    float* Pb;             // [gridDim.x][128]
};


template <int NB, bool GRID>
__global__ void __launch_bounds__(256) k_nf_bwd(NfBwd p)
{
    __shared__ uint16_t sDZ[kHidden * kTilePitch];  // dZ tile transposed [m][row]
    __shared__ uint16_t sA[NB * 32 * kTilePitch];   // A tile transposed [k][row]
    __shared__ float s_max[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    const int IN = p.in_dim;
    const bf16x8 zero = __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
    const bool dh_wave = GRID ? wave == 0 : wave * 32 < IN;
    bf16x8 wfr[kHidden / 16];
    {
        const int k = wave * 32 + l32;
#pragma unroll
        for (int kk = 0; kk < kHidden / 16; ++kk)
            wfr[kk] = (dh_wave && k < IN) ? load8(p.wt + (size_t)k * kHidden + kk * 16 + half * 8) : zero;
    }
    f32x16 accW[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
        accW[nb] = f32x16{};
    float gb = 0.0f, vmax = 0.0f;
    const int n_tiles = p.Bp / kRowTile;
    const int in8 = IN / 8;
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int b0 = tile * kRowTile;
        __syncthreads();
        // stage both tiles transposed: a task is a pair of rows and 8 columns,
        // written as 8 packed pairs (consecutive lanes take consecutive pairs)
        for (int task = tid; task < 64 * (kHidden / 8); task += 256) {
            const int rp = task & 63, cj = task >> 6;
            const uint4 r0 = *reinterpret_cast<const uint4*>(p.dz + (size_t)(b0 + 2 * rp) * kHidden + cj * 8);
            const uint4 r1 = *reinterpret_cast<const uint4*>(p.dz + (size_t)(b0 + 2 * rp + 1) * kHidden + cj * 8);
            const uint32_t x0[4] = {r0.x, r0.y, r0.z, r0.w}, x1[4] = {r1.x, r1.y, r1.z, r1.w};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint32_t lo = (x0[e >> 1] >> ((e & 1) * 16)) & 0xffffu;
                const uint32_t hi = (x1[e >> 1] >> ((e & 1) * 16)) & 0xffffu;
                *reinterpret_cast<uint32_t*>(sDZ + (cj * 8 + e) * kTilePitch + 2 * rp) = lo | (hi << 16);
            }
        }
        for (int task = tid; task < 64 * in8; task += 256) {
            const int rp = task & 63, cj = task >> 6;
            const uint4 r0 = *reinterpret_cast<const uint4*>(p.act + (size_t)(b0 + 2 * rp) * IN + cj * 8);
            const uint4 r1 = *reinterpret_cast<const uint4*>(p.act + (size_t)(b0 + 2 * rp + 1) * IN + cj * 8);
            const uint32_t x0[4] = {r0.x, r0.y, r0.z, r0.w}, x1[4] = {r1.x, r1.y, r1.z, r1.w};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint32_t lo = (x0[e >> 1] >> ((e & 1) * 16)) & 0xffffu;
                const uint32_t hi = (x1[e >> 1] >> ((e & 1) * 16)) & 0xffffu;
                *reinterpret_cast<uint32_t*>(sA + (cj * 8 + e) * kTilePitch + 2 * rp) = lo | (hi << 16);
            }
        }
        __syncthreads();
        if (dh_wave) {
            f32x16 acc[kRowTile / 32];
#pragma unroll
            for (int bb = 0; bb < kRowTile / 32; ++bb)
                acc[bb] = f32x16{};
#pragma unroll
            for (int bb = 0; bb < kRowTile / 32; ++bb) {
                // dZ row b0 + bb * 32 + l32, columns kk * 16 + half * 8 + 0..7,
                // gathered from the transposed tile in LDS
                const uint16_t* dr = sDZ + (half * 8) * kTilePitch + bb * 32 + l32;
                bf16x8 bv[kHidden / 16];
#pragma unroll
                for (int kk = 0; kk < kHidden / 16; ++kk)
                    bv[kk] = lds_col8(dr + kk * 16 * kTilePitch);
#pragma unroll
                for (int kk = 0; kk < kHidden / 16; ++kk)
                    acc[bb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wfr[kk], bv[kk], acc[bb], 0, 0, 0);
            }
#pragma unroll
            for (int bb = 0; bb < kRowTile / 32; ++bb) {
                const int b = bb * 32 + l32;  // tile row
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int k0 = wave * 32 + 8 * q + 4 * half;
                    if (GRID) {
                        if (k0 < kLevels * kFeat) {
                            const float4 v = make_float4(acc[bb][4 * q], acc[bb][4 * q + 1], acc[bb][4 * q + 2],
                                                         acc[bb][4 * q + 3]);
                            *reinterpret_cast<float4*>(p.dh0 + (size_t)(b0 + b) * (kLevels * kFeat) + k0) = v;
                            vmax = fmaxf(vmax, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
                        }
                    } else {
                        uint16_t h[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const float v = bf16_positive(sA[(k0 + r) * kTilePitch + b]) ? acc[bb][4 * q + r] : 0.0f;
                            h[r] = to_bf16(v);
                        }
                        const uint2 pk = make_uint2(h[0] | (static_cast<uint32_t>(h[1]) << 16),
                                                    h[2] | (static_cast<uint32_t>(h[3]) << 16));
                        *reinterpret_cast<uint2*>(p.dz_prev + (size_t)(b0 + b) * kHidden + k0) = pk;
                    }
                }
            }
        }
        // dW += dZ^T A and db over the tile's rows
        const uint16_t* ar = sDZ + (wave * 32 + l32) * kTilePitch + half * 8;
#pragma unroll
        for (int kk = 0; kk < kRowTile / 16; ++kk) {
            const bf16x8 av = *reinterpret_cast<const bf16x8*>(ar + kk * 16);
#pragma unroll
            for (int e = 0; e < 8; ++e)
                gb += static_cast<float>(av[e]);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const bf16x8 bv = *reinterpret_cast<const bf16x8*>(sA + (nb * 32 + l32) * kTilePitch + kk * 16 + half * 8);
                accW[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, accW[nb], 0, 0, 0);
            }
        }
    }
    float* Pw = p.Pw + (size_t)blockIdx.x * kHidden * IN;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int k = nb * 32 + l32;
        if (k >= IN)
            continue;
#pragma unroll
        for (int i = 0; i < 16; ++i)
            Pw[(size_t)(wave * 32 + 8 * (i / 4) + 4 * half + (i % 4)) * IN + k] = accW[nb][i];
    }
    gb += __shfl_xor(gb, 32, 64);
    if (half == 0)
        p.Pb[(size_t)blockIdx.x * kHidden + wave * 32 + l32] = gb;
    if (GRID) {
        for (int o = 32; o > 0; o >>= 1)
            vmax = fmaxf(vmax, __shfl_xor(vmax, o, 64));
        if (lane == 0)
            s_max[wave] = vmax;
        __syncthreads();
        if (tid == 0)
            p.gmax[blockIdx.x] = fmaxf(fmaxf(s_max[0], s_max[1]), fmaxf(s_max[2], s_max[3]));
    }
}

// Output layer over 128-row tiles (persistent): y = A_4 W_4^T + b_4, the
// loss, dZ_4 = 2 (y - t) / (B n_out) rounded to bfloat16, and in training
// dZ_3 = (dZ_4 W_4) [A_4 > 0] row-major plus the workgroup's partials of
// dW_4 = dZ_4^T A_4 and db_4 = sums of dZ_4.  Row r's output is the sum of
// two half-rows of 64 products.
struct NfOut {
    const uint16_t* H;   // A_4 [Bp][128]
    const uint16_t* W;   // W_4 [n_out][128] bfloat16
    const float* b;      // b_4
    const float* target; // [B][n_out] (training) or null
    float* y;            // [B][n_out] or null
    int32_t B, Bp, n_out;
    float scale;         // 2 / (B n_out)
    uint16_t* dz3;       // [Bp][128] (training) or null
    float* Pw4;          // [gridDim.x][n_out][128]
    float* Pb4;          // [gridDim.x][n_out]
    double* loss_part;   // [gridDim.x]
};

constexpr int kOutPitch = kHidden + 2;  // bfloat16 per LDS row: an odd number of dwords
constexpr int kOutTasks = kMaxOut * kHidden / 256;

// LDS bytes of the output step for n_out outputs: the tile, W_4 and dZ_4 as
// floats, the loss reduction.
__host__ __device__ constexpr size_t nf_out_lds(int n_out)
{
    return sizeof(uint16_t) * kRowTile * kOutPitch + 2 * sizeof(float) * kHidden * (size_t)n_out +
           sizeof(double) * 256;
}

__global__ void __launch_bounds__(256) k_nf_out(NfOut o)
{
    // sized by n_out (dynamic), so that narrow output layers leave room for
    // more workgroups per CU
    extern __shared__ uint4 s_out_raw[];
    const int nO = o.n_out;
    uint16_t* sH = reinterpret_cast<uint16_t*>(s_out_raw);  // [kRowTile][kOutPitch]
    float* sW = reinterpret_cast<float*>(sH + kRowTile * kOutPitch);  // [n_out][128]
    float* s_dz = sW + nO * kHidden;                                  // [n_out][kRowTile]
    double* s_red = reinterpret_cast<double*>(s_dz + nO * kRowTile);  // [256]
    const int tid = threadIdx.x;
    const bool train = o.dz3 != nullptr;
    for (int e = tid; e < nO * kHidden; e += 256)
        sW[e] = from_bf16(o.W[e]);
    float accw[kOutTasks];
#pragma unroll
    for (int j = 0; j < kOutTasks; ++j)
        accw[j] = 0.0f;
    float accb = 0.0f;
    double lsum = 0.0;
    const int r = tid >> 1, hf = tid & 1;
    const int n_tiles = o.Bp / kRowTile;
    // the next tile's A_4 is loaded into registers while this tile is
    // worked on (eight 16-byte pieces per thread)
    constexpr int kPre = kRowTile * (kHidden / 8) / 256;
    uint4 pre[kPre];
    auto fetch = [&](int t) {
        const int bt = t * kRowTile;
#pragma unroll
        for (int j = 0; j < kPre; ++j) {
            const int task = tid + 256 * j;
            const int rr = task >> 4, c = task & 15;
            pre[j] = *reinterpret_cast<const uint4*>(o.H + (size_t)(bt + rr) * kHidden + c * 8);
        }
    };
    if (static_cast<int>(blockIdx.x) < n_tiles)
        fetch(blockIdx.x);
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int b0 = tile * kRowTile;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kPre; ++j) {
            const int task = tid + 256 * j;
            const int rr = task >> 4, c = task & 15;
            uint32_t* d = reinterpret_cast<uint32_t*>(sH + rr * kOutPitch + c * 8);
            d[0] = pre[j].x;
            d[1] = pre[j].y;
            d[2] = pre[j].z;
            d[3] = pre[j].w;
        }
        __syncthreads();
        const int row = b0 + r;
        const bool live = row < o.B;
        // this tile's first target before the next tile's loads are issued
        // (loads complete in order, so a later target load would wait for
        // them)
        const float tgt0 = (o.target && live && hf == 0) ? o.target[(size_t)row * nO] : 0.0f;
        if (tile + static_cast<int>(gridDim.x) < n_tiles)
            fetch(tile + gridDim.x);
        for (int oi = 0; oi < nO; ++oi) {
            float part = 0.0f;
            const uint16_t* hr = sH + r * kOutPitch + hf * 64;
            const float* wr = sW + oi * kHidden + hf * 64;
#pragma unroll 8
            for (int k = 0; k < 64; ++k)
                part = fmaf(from_bf16(hr[k]), wr[k], part);
            part += __shfl_xor(part, 1, 64);
            if (hf == 0) {
                const float yv = part + o.b[oi];
                float dz = 0.0f;
                if (live) {
                    if (o.y)
                        o.y[(size_t)row * nO + oi] = yv;
                    if (o.target) {
                        const float diff = yv - (oi == 0 ? tgt0 : o.target[(size_t)row * nO + oi]);
                        lsum += static_cast<double>(diff) * diff;
                        dz = o.scale * diff;
                    }
                }
                s_dz[oi * kRowTile + r] = from_bf16(to_bf16(dz));
            }
        }
        if (!train)
            continue;
        __syncthreads();
        // dZ_3, one 8-column piece of a row per task
        for (int task = tid; task < kRowTile * (kHidden / 8); task += 256) {
            const int rr = task >> 4, c = task & 15;
            uint32_t pk[4];
#pragma unroll
            for (int e = 0; e < 8; e += 2) {
                uint32_t two = 0;
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int k = c * 8 + e + u;
                    float dh = 0.0f;
                    for (int oi = 0; oi < nO; ++oi)
                        dh = fmaf(s_dz[oi * kRowTile + rr], sW[oi * kHidden + k], dh);
                    const uint16_t h = to_bf16(bf16_positive(sH[rr * kOutPitch + k]) ? dh : 0.0f);
                    two |= static_cast<uint32_t>(h) << (16 * u);
                }
                pk[e >> 1] = two;
            }
            *reinterpret_cast<uint4*>(o.dz3 + (size_t)(b0 + rr) * kHidden + c * 8) =
                make_uint4(pk[0], pk[1], pk[2], pk[3]);
        }
        // dW_4 and db_4 over the tile's rows
#pragma unroll
        for (int j = 0; j < kOutTasks; ++j) {
            const int e = tid + 256 * j;
            if (e < nO * kHidden) {
                const int oi = e / kHidden, k = e - oi * kHidden;
                float a = accw[j];
                for (int rr = 0; rr < kRowTile; ++rr)
                    a = fmaf(s_dz[oi * kRowTile + rr], from_bf16(sH[rr * kOutPitch + k]), a);
                accw[j] = a;
            }
        }
        if (tid < nO)
            for (int rr = 0; rr < kRowTile; ++rr)
                accb += s_dz[tid * kRowTile + rr];
    }
    if (train) {
#pragma unroll
        for (int j = 0; j < kOutTasks; ++j) {
            const int e = tid + 256 * j;
            if (e < nO * kHidden)
                o.Pw4[(size_t)blockIdx.x * nO * kHidden + e] = accw[j];
        }
        if (tid < nO)
            o.Pb4[(size_t)blockIdx.x * nO + tid] = accb;
    }
    if (o.loss_part) {
        __syncthreads();
        s_red[tid] = lsum;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (tid < h)
                s_red[tid] += s_red[tid + h];
            __syncthreads();
        }
        if (tid == 0)
            o.loss_part[blockIdx.x] = s_red[0];
    }
}

// out = sum of parts[0 .. n) in a fixed order (one workgroup).
__global__ void __launch_bounds__(256) k_nf_sum(const double* __restrict__ parts, int32_t n, double* out)
{
    __shared__ double s[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += 256)
        a += parts[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *out = s[0];
}

// Chunk partials folded in chunk order into the gradient array (one
// segment per blockIdx.y; the loads of 8 chunks are issued together).
struct NfSeg {
    const float* part;
    float* out;
    int32_t n, nch;
};
struct NfReduce {
    NfSeg seg[2 * kLayers];
};

constexpr int kReduceWaves = 16;

__global__ void __launch_bounds__(64 * kReduceWaves) k_nf_reduce(NfReduce r)
{
    // 256 outputs per workgroup, four per lane (one 16-byte load per lane
    // and partial); wave g sums the g-th eighth of the partials in order,
    // then the eight sums are added in order.  Segments whose length is not
    // a multiple of 4 (the biases of a narrow output layer) take one output
    // per lane.
    __shared__ double s_q[kReduceWaves][256];
    const NfSeg& s = r.seg[blockIdx.y];
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int32_t per = (s.nch + kReduceWaves - 1) / kReduceWaves;
    const int32_t c_lo = g * per, c_hi = min(s.nch, c_lo + per);
    const bool vec = (s.n & 3) == 0;
    const int32_t span = vec ? 256 : 64;
    for (int32_t e0 = blockIdx.x * span; e0 < s.n; e0 += gridDim.x * span) {
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        if (vec) {
            const int32_t e = e0 + 4 * lane;
            if (e < s.n) {
                for (int32_t c0 = c_lo; c0 < c_hi; c0 += 8) {
                    // eight loads in flight (past the end: the last partial
                    // again, replaced by zeros)
                    float4 v[8];
#pragma unroll
                    for (int c = 0; c < 8; ++c)
                        v[c] = *reinterpret_cast<const float4*>(s.part + (size_t)min(c0 + c, c_hi - 1) * s.n + e);
#pragma unroll
                    for (int c = 0; c < 8; ++c)
                        if (c0 + c >= c_hi)
                            v[c] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        a[0] += v[c].x;
                        a[1] += v[c].y;
                        a[2] += v[c].z;
                        a[3] += v[c].w;
                    }
                }
            }
        } else {
            const int32_t e = e0 + lane;
            if (e < s.n) {
                for (int32_t c0 = c_lo; c0 < c_hi; c0 += 8) {
                    float v[8];
#pragma unroll
                    for (int c = 0; c < 8; ++c)
                        v[c] = s.part[(size_t)min(c0 + c, c_hi - 1) * s.n + e];
#pragma unroll
                    for (int c = 0; c < 8; ++c)
                        if (c0 + c >= c_hi)
                            v[c] = 0.0f;
#pragma unroll
                    for (int c = 0; c < 8; ++c)
                        a[0] += v[c];
                }
            }
        }
        __syncthreads();
        if (vec) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                s_q[g][4 * lane + k] = a[k];
        } else {
            s_q[g][lane] = a[0];
        }
        __syncthreads();
        for (int t = threadIdx.x; t < span; t += 64 * kReduceWaves) {
            const int32_t e = e0 + t;
            if (e < s.n) {
                double acc = s_q[0][t];
#pragma unroll
                for (int q = 1; q < kReduceWaves; ++q)
                    acc += s_q[q][t];
                s.out[e] = static_cast<float>(acc);
            }
        }
    }
}

// Grid-feature gradient: each row's dH_0 goes to the 8 corners of its cell
// on every lattice with the trilinear weights.  The terms are added as
// 64-bit integers in units of 1/S, S a power of two with B * 8 * max|dH_0|
// * S below 2^62: each term w g S is formed exactly in FP64 and rounded once,
// and integer sums do not depend on their order, so the gradient is the
// same on every run.  Workgroup (p, g) adds the terms of row group g that
// fall in partition p in LDS and writes the partition out as group g's
// partial; the fold adds the partials and scales back.  (Floating-point
// atomic additions, in LDS or in memory, measured 3-8 times slower here.)
__device__ __forceinline__ double grid_scale(float gmax, int32_t B)
{
    // the largest power of two S with B * 8 * gmax * S <= 2^62 and
    // gmax * S <= 2^50 (so every term converts as below)
    const double g = static_cast<double>(gmax);
    const double bound = static_cast<double>(B) * 8.0 * g;
    if (!(bound > 0.0) || !isfinite(bound))
        return 1.0;
    return exp2(floor(fmin(62.0 - log2(bound), 50.0 - log2(g))));
}

// round(x) to a 64-bit integer, ties to even, for |x| < 2^51: adding
// 1.5 * 2^52 leaves the rounded value in the low mantissa bits (three
// instructions instead of the general conversion's seven)
__device__ __forceinline__ long long fixed_rn(double x)
{
    constexpr double kMagic = 6755399441055744.0;  // 1.5 * 2^52
    return __double_as_longlong(x + kMagic) - __double_as_longlong(kMagic);
}

// The largest of the n per-workgroup maxima (every thread of the block).
__device__ float block_max(const float* __restrict__ m, int32_t n)
{
    __shared__ float s[16];
    float a = 0.0f;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        a = fmaxf(a, m[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        a = fmaxf(a, __shfl_xor(a, off, 64));
    if ((threadIdx.x & 63) == 0)
        s[threadIdx.x >> 6] = a;
    __syncthreads();
    float r = 0.0f;
    for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w)
        r = fmaxf(r, s[w]);
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kGridThreads) k_nf_grid_part(NfDev f, const float* __restrict__ in, int32_t B,
                                                      const float* __restrict__ dh0, const float* gmax,
                                                      int32_t n_gmax, long long* __restrict__ part, int32_t G)
{
    __shared__ unsigned long long s_acc[kGridPart];
    // Workgroups go to the 8 XCDs in turn (block b to XCD b mod 8); taking
    // (group, partition) pairs in order within each XCD's share keeps a row
    // group's partitions on one or two XCDs, so its rows are fetched into
    // one or two L2s instead of all eight (a bijection: the grid is a
    // multiple of 8; the workgroups past the last pair have nothing to do)
    const int per_xcd = static_cast<int>(gridDim.x) / 8;
    const int L = static_cast<int>(blockIdx.x % 8) * per_xcd + static_cast<int>(blockIdx.x / 8);
    if (L >= kGridParts * G)
        return;
    const int p = L % kGridParts, g = L / kGridParts;
    const int lo = p * kGridPart;
    const int n = min(kGridPart, kGridFloats - lo);
    const double S = grid_scale(block_max(gmax, n_gmax), B);
    for (int e = threadIdx.x; e < n; e += kGridThreads)
        s_acc[e] = 0ull;
    __syncthreads();
    for (int32_t b = g * kGridThreads + threadIdx.x; b < B; b += G * kGridThreads) {
        const float* row = in + (size_t)b * f.ld_in;
        float u[3];
        unit_coords(f, row, u);
        const float4* dg = reinterpret_cast<const float4*>(dh0 + (size_t)b * (kLevels * kFeat));
#pragma unroll
        for (int l = 0; l < kLevels; ++l) {
            if (level_base(l + 1) <= lo || level_base(l) >= lo + n)
                continue;  // the lattice lies outside this partition
            Corners c;
            cell_corners(u, l, c);
            const float4 gv = dg[l];
            const double gs[4] = {gv.x * S, gv.y * S, gv.z * S, gv.w * S};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int at = level_base(l) + static_cast<int>(c.idx[e]) * kFeat - lo;
                if (at >= 0 && at < n) {
                    const double w = c.w[e];
#pragma unroll
                    for (int q = 0; q < kFeat; ++q)
                        atomicAdd(s_acc + at + q, static_cast<unsigned long long>(fixed_rn(w * gs[q])));
                }
            }
        }
    }
    __syncthreads();
    long long* dst = part + (size_t)g * kGridFloats + lo;
    for (int e = threadIdx.x; e < n; e += kGridThreads)
        dst[e] = static_cast<long long>(s_acc[e]);
}

__global__ void __launch_bounds__(256) k_nf_grid_fold(const long long* __restrict__ part, int32_t G, int32_t B,
                                                      const float* gmax, int32_t n_gmax, float* __restrict__ out)
{
    static_assert(kGridFloats % 2 == 0, "pairs of values");
    const double inv = 1.0 / grid_scale(block_max(gmax, n_gmax), B);
    // two values per thread (16-byte loads), eight row groups' loads in flight
    for (int e = 2 * (blockIdx.x * 256 + threadIdx.x); e < kGridFloats; e += 2 * gridDim.x * 256) {
        long long a0 = 0, a1 = 0;
        for (int g0 = 0; g0 < G; g0 += 8) {
            longlong2 v[8];
#pragma unroll
            for (int c = 0; c < 8; ++c)
                v[c] = *reinterpret_cast<const longlong2*>(part + (size_t)min(g0 + c, G - 1) * kGridFloats + e);
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (g0 + c >= G)
                    v[c] = make_longlong2(0, 0);
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                a0 += v[c].x;
                a1 += v[c].y;
            }
        }
        out[e] = static_cast<float>(static_cast<double>(a0) * inv);
        out[e + 1] = static_cast<float>(static_cast<double>(a1) * inv);
    }
}

// Adam (Kingma & Ba 2015) on the FP32 parameters; c1 = 1 / (1 - beta1^t),
// c2 = 1 / (1 - beta2^t).
__global__ void __launch_bounds__(256) k_nf_adam(float* __restrict__ p, const float* __restrict__ g,
                                                 float* __restrict__ m, float* __restrict__ v, int64_t n,
                                                 float lr, float c1, float c2)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const float ge = g[e];
        const float me = 0.9f * m[e] + 0.1f * ge;
        const float ve = 0.999f * v[e] + 0.001f * (ge * ge);
        m[e] = me;
        v[e] = ve;
        p[e] -= lr * (me * c1) / (sqrtf(ve * c2) + 1e-8f);
    }
}

// bfloat16 copies of the weights, row-major and transposed.
struct NfCast {
    const float* p;
    uint16_t* wb;
    uint16_t* wbt;
    int64_t offW[kLayers], offWb[kLayers + 1];
    int32_t in_dim[kLayers], out_dim[kLayers];
};

__global__ void __launch_bounds__(256) k_nf_cast(NfCast c)
{
    const int64_t total = c.offWb[kLayers];
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        int i = 0;
        while (i + 1 < kLayers && e >= c.offWb[i + 1])
            ++i;
        const int64_t local = e - c.offWb[i];
        const int32_t in = c.in_dim[i], out = c.out_dim[i];
        const int32_t row = static_cast<int32_t>(local / in), col = static_cast<int32_t>(local % in);
        const uint16_t h = to_bf16(c.p[c.offW[i] + local]);
        c.wb[e] = h;
        c.wbt[c.offWb[i] + (int64_t)col * out + row] = h;
    }
}

int grid_for(int64_t work, int per_block, int cap = 4096)
{
    const int64_t g = (work + per_block - 1) / per_block;
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(g, cap)));
}

}  // namespace
}  // namespace nat

// ---------------------------------------------------------------- host side
struct nat_nf {
    nat_ctx* ctx = nullptr;
    int32_t n_v = 0, n_out = 1, D = 0;
    double r_lo = 0.0, r_hi = 1.0;
    int32_t in_dim[nat::kLayers] = {}, out_dim[nat::kLayers] = {};
    int64_t offW[nat::kLayers] = {}, offb[nat::kLayers] = {}, offG[nat::kLevels] = {};
    int64_t offWb[nat::kLayers + 1] = {};
    int64_t n_params = 0;
    float* d_params = nullptr;  // params, grads, Adam m, Adam v
    float* d_grads = nullptr;
    float* d_m = nullptr;
    float* d_v = nullptr;
    uint16_t* d_wb = nullptr;   // bfloat16 weights, row-major, then transposed
    uint16_t* d_wbt = nullptr;
    size_t fixed_bytes = 0;
    void* d_fixed = nullptr;
    // batch workspace, grown on demand
    int32_t cap_rows = 0;
    void* d_ws = nullptr;
    size_t ws_bytes = 0;
};

namespace nat {
namespace {

// Workspace of a batch of Bp rows.
struct NfWs {
    uint16_t* X;
    uint16_t* H[4];           // A_1 .. A_4
    uint16_t* dz[4];          // dZ_0 .. dZ_3
    float* dh0;               // [Bp][16]
    double* loss_part;        // [out_grid]
    double* loss;
    float* Pw[kLayers];       // dW_0 .. dW_4 workgroup partials [bwd_grid, or out_grid for dW_4][out_i][in_i]
    float* Pb[kLayers];       // db_0 .. db_4 workgroup partials [bwd_grid, or out_grid for db_4][out_i]
    long long* gpart;         // grid-gradient partials [grid_groups][kGridFloats]
    float* gmax;              // max |dH_0| of each workgroup of the layer-0 backward
    int32_t n_gmax;
    int32_t grid_groups, bwd_grid, out_grid;
};

constexpr int kBwdGrid = 512;  // workgroups of a fused backward pass (persistent)
constexpr int kOutGrid = 512;  // workgroups of the output step

int32_t nf_grid_groups(int32_t Bp)
{
    return static_cast<int32_t>(std::max<int64_t>(1, std::min<int64_t>(kGridGroupsMax, (Bp + 4095) / 4096)));
}

size_t nf_ws_layout(const nat_nf* nf, int32_t Bp, NfWs* w, void* base)
{
    const size_t bp = static_cast<size_t>(Bp);
    const int32_t G = nf_grid_groups(Bp);
    const int32_t GB = std::min(Bp / kRowTile, kBwdGrid);
    const int32_t OG = std::min(Bp / kRowTile, kOutGrid);
    // the output layer's partials come from the output step, the others
    // from the backward passes
    auto parts = [&](int i) { return static_cast<size_t>(i == kLayers - 1 ? OG : GB); };
    std::vector<size_t> sz;
    sz.push_back(2 * bp * nf->D);                 // X
    for (int i = 0; i < 4; ++i)
        sz.push_back(2 * bp * kHidden);           // H
    for (int i = 0; i < 4; ++i)
        sz.push_back(2 * bp * kHidden);           // dz
    sz.push_back(4 * bp * kLevels * kFeat);       // dh0
    sz.push_back(8 * static_cast<size_t>(OG));    // loss_part
    sz.push_back(8);                              // loss
    for (int i = 0; i < kLayers; ++i)
        sz.push_back(4 * parts(i) * nf->out_dim[i] * nf->in_dim[i]);  // Pw
    for (int i = 0; i < kLayers; ++i)
        sz.push_back(4 * parts(i) * nf->out_dim[i]);                  // Pb
    sz.push_back(8 * static_cast<size_t>(kGridFloats) * G);
    sz.push_back(4 * static_cast<size_t>(GB));
    size_t total = 0;
    for (size_t s : sz)
        total = ((total + 255) & ~size_t(255)) + s;
    total += 256;
    if (w && base) {
        Carver cv(base);
        w->X = cv.take<uint16_t>(bp * nf->D);
        for (int i = 0; i < 4; ++i)
            w->H[i] = cv.take<uint16_t>(bp * kHidden);
        for (int i = 0; i < 4; ++i)
            w->dz[i] = cv.take<uint16_t>(bp * kHidden);
        w->dh0 = cv.take<float>(bp * kLevels * kFeat);
        w->loss_part = cv.take<double>(OG);
        w->loss = cv.take<double>(1);
        for (int i = 0; i < kLayers; ++i)
            w->Pw[i] = cv.take<float>(parts(i) * nf->out_dim[i] * nf->in_dim[i]);
        for (int i = 0; i < kLayers; ++i)
            w->Pb[i] = cv.take<float>(parts(i) * nf->out_dim[i]);
        w->gpart = cv.take<long long>(static_cast<size_t>(kGridFloats) * G);
        w->gmax = cv.take<float>(GB);
        w->n_gmax = GB;
        w->grid_groups = G;
        w->bwd_grid = GB;
        w->out_grid = OG;
    }
    return total;
}

nat_status nf_workspace(nat_nf* nf, int32_t Bp, NfWs* w)
{
    if (Bp > nf->cap_rows) {
        const size_t bytes = nf_ws_layout(nf, Bp, nullptr, nullptr);
        if (nf->d_ws) {
            NAT_HIP(hipDeviceSynchronize());
            dev_free(nf->ctx, nf->d_ws, nf->ws_bytes);
            nf->d_ws = nullptr;
            nf->ws_bytes = 0;
            nf->cap_rows = 0;
        }
        nat_status st = dev_alloc(nf->ctx, bytes, &nf->d_ws);
        if (st != NAT_OK)
            return st;
        nf->ws_bytes = bytes;
        nf->cap_rows = Bp;
    }
    nf_ws_layout(nf, Bp, w, nf->d_ws);
    return NAT_OK;
}

NfDev nf_dev(const nat_nf* nf)
{
    NfDev f{};
    f.n_v = nf->n_v;
    f.n_out = nf->n_out;
    f.D = nf->D;
    f.ld_in = 3 + nf->n_v + 1;
    f.r_lo = static_cast<float>(nf->r_lo);
    f.inv_span = static_cast<float>(1.0 / (nf->r_hi - nf->r_lo));
    for (int l = 0; l < kLevels; ++l)
        f.grid[l] = nf->d_params + nf->offG[l];
    return f;
}

// Forward pass of B rows (padded to Bp); with `train` the output kernel also
// forms the loss, dZ_3 and the partials of dW_4, db_4.
hipError_t nf_forward(nat_nf* nf, const NfWs& w, const float* in, const float* target, int32_t B, int32_t Bp,
                      float* y, bool train, hipStream_t s)
{
    NfFwd p{};
    p.f = nf_dev(nf);
    p.in = in;
    p.B = B;
    p.Bp = Bp;
    p.wb = nf->d_wb;
    for (int i = 0; i < kLayers; ++i) {
        p.offWb[i] = nf->offWb[i];
        p.bias[i] = nf->d_params + nf->offb[i];
    }
    p.X = train ? w.X : nullptr;
    for (int i = 0; i < 4; ++i)
        p.H[i] = train ? w.H[i] : nullptr;
    p.y = train ? nullptr : y;
    const int kmax = std::max(nf->D, kHidden);
    const size_t lds = sizeof(uint16_t) * 2 * kRowTile * (size_t)(kmax + 8);
    const int grid = std::min(Bp / kRowTile, kGemmGrid);
    switch (kmax / 16) {
    case 8: hipLaunchKernelGGL(k_nf_fwd<8>, dim3(grid), dim3(256), lds, s, p); break;
    case 9: hipLaunchKernelGGL(k_nf_fwd<9>, dim3(grid), dim3(256), lds, s, p); break;
    case 10: hipLaunchKernelGGL(k_nf_fwd<10>, dim3(grid), dim3(256), lds, s, p); break;
    case 11: hipLaunchKernelGGL(k_nf_fwd<11>, dim3(grid), dim3(256), lds, s, p); break;
    case 12: hipLaunchKernelGGL(k_nf_fwd<12>, dim3(grid), dim3(256), lds, s, p); break;
    case 13: hipLaunchKernelGGL(k_nf_fwd<13>, dim3(grid), dim3(256), lds, s, p); break;
    case 14: hipLaunchKernelGGL(k_nf_fwd<14>, dim3(grid), dim3(256), lds, s, p); break;
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !train)
        return e;
    NfOut o{};
    o.H = w.H[3];
    o.W = nf->d_wb + nf->offWb[4];
    o.b = nf->d_params + nf->offb[4];
    o.target = target;
    o.y = nullptr;
    o.B = B;
    o.Bp = Bp;
    o.n_out = nf->n_out;
    o.scale = static_cast<float>(2.0 / (static_cast<double>(B) * nf->n_out));
    o.dz3 = w.dz[3];
    o.Pw4 = w.Pw[4];
    o.Pb4 = w.Pb[4];
    o.loss_part = w.loss_part;
    hipLaunchKernelGGL(k_nf_out, dim3(w.out_grid), dim3(256), nf_out_lds(nf->n_out), s, o);
    e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_nf_sum, dim3(1), dim3(256), 0, s, w.loss_part, w.out_grid, w.loss);
        e = hipGetLastError();
    }
    return e;
}

template <bool GRID>
hipError_t launch_bwd(const NfBwd& p, int grid, hipStream_t s)
{
    switch ((p.in_dim + 31) / 32) {
    case 1: hipLaunchKernelGGL((k_nf_bwd<1, GRID>), dim3(grid), dim3(256), 0, s, p); break;
    case 2: hipLaunchKernelGGL((k_nf_bwd<2, GRID>), dim3(grid), dim3(256), 0, s, p); break;
    case 3: hipLaunchKernelGGL((k_nf_bwd<3, GRID>), dim3(grid), dim3(256), 0, s, p); break;
    case 4: hipLaunchKernelGGL((k_nf_bwd<4, GRID>), dim3(grid), dim3(256), 0, s, p); break;
    case 5: hipLaunchKernelGGL((k_nf_bwd<5, GRID>), dim3(grid), dim3(256), 0, s, p); break;
    case 6: hipLaunchKernelGGL((k_nf_bwd<6, GRID>), dim3(grid), dim3(256), 0, s, p); break;
    case 7: hipLaunchKernelGGL((k_nf_bwd<7, GRID>), dim3(grid), dim3(256), 0, s, p); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Gradient of every parameter into d_grads (after nf_forward with train).
hipError_t nf_backward(nat_nf* nf, const NfWs& w, const float* in, int32_t B, int32_t Bp, hipStream_t s)
{
    hipError_t e = hipSuccess;
    // fused passes, layer 3 down to layer 0 (the grid columns of dH_0)
    for (int i = 3; i >= 0 && e == hipSuccess; --i) {
        NfBwd p{};
        p.dz = w.dz[i];
        p.act = i == 0 ? w.X : w.H[i - 1];
        p.wt = nf->d_wbt + nf->offWb[i];  // W_i^T [in_i][128]
        p.in_dim = nf->in_dim[i];
        p.Bp = Bp;
        p.dz_prev = i > 0 ? w.dz[i - 1] : nullptr;
        p.dh0 = w.dh0;
        p.gmax = w.gmax;
        p.Pw = w.Pw[i];
        p.Pb = w.Pb[i];
        e = i > 0 ? launch_bwd<false>(p, w.bwd_grid, s) : launch_bwd<true>(p, w.bwd_grid, s);
    }
    if (e != hipSuccess)
        return e;
    // every layer's workgroup partials folded in workgroup order
    NfReduce red{};
    int32_t max_n = 0;
    for (int i = 0; i < kLayers; ++i) {
        const int32_t n = nf->out_dim[i] * nf->in_dim[i];
        const int32_t nch = i == kLayers - 1 ? w.out_grid : w.bwd_grid;
        red.seg[2 * i] = NfSeg{w.Pw[i], nf->d_grads + nf->offW[i], n, nch};
        red.seg[2 * i + 1] = NfSeg{w.Pb[i], nf->d_grads + nf->offb[i], nf->out_dim[i], nch};
        max_n = std::max(max_n, n);
    }
    hipLaunchKernelGGL(k_nf_reduce, dim3(grid_for(max_n, 256, 1024), 2 * kLayers), dim3(64 * kReduceWaves), 0, s,
                       red);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    // grid-feature gradient: LDS partitions, then the ordered fold
    const NfDev f = nf_dev(nf);
    const int32_t G = w.grid_groups;
    hipLaunchKernelGGL(k_nf_grid_part, dim3((kGridParts * G + 7) / 8 * 8), dim3(kGridThreads), 0, s, f, in, B,
                       w.dh0, w.gmax, w.n_gmax, w.gpart, G);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_nf_grid_fold, dim3(grid_for(kGridFloats / 2, 256, 1024)), dim3(256), 0, s, w.gpart, G, B,
                       w.gmax, w.n_gmax, nf->d_grads + nf->offG[0]);
    return hipGetLastError();
}

hipError_t nf_cast(nat_nf* nf, hipStream_t s)
{
    NfCast c{};
    c.p = nf->d_params;
    c.wb = nf->d_wb;
    c.wbt = nf->d_wbt;
    for (int i = 0; i < kLayers; ++i) {
        c.offW[i] = nf->offW[i];
        c.in_dim[i] = nf->in_dim[i];
        c.out_dim[i] = nf->out_dim[i];
    }
    for (int i = 0; i <= kLayers; ++i)
        c.offWb[i] = nf->offWb[i];
    hipLaunchKernelGGL(k_nf_cast, dim3(grid_for(nf->offWb[kLayers], 256, 1024)), dim3(256), 0, s, c);
    return hipGetLastError();
}

uint64_t splitmix64(uint64_t x)
{
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

// uniform in [-1, 1) from (seed, stream, index)
double uniform_pm1(uint64_t seed, uint64_t stream, uint64_t i)
{
    const uint64_t h = splitmix64(splitmix64(seed ^ (stream << 56)) ^ i);
    return static_cast<double>(h >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

nat_status nf_validate_batch(const nat_nf* nf, const float* in, const float* target, int32_t B, bool need_target,
                             const char* who)
{
    if (!nf)
        return fail(NAT_E_INVALID, "%s: field is NULL", who);
    if (B < 1 || B > (1 << 24))
        return fail(NAT_E_INVALID, "%s: batch of %d rows (1 .. 2^24)", who, B);
    if (!in)
        return fail(NAT_E_INVALID, "%s: inputs is NULL", who);
    if (need_target && !target)
        return fail(NAT_E_INVALID, "%s: targets is NULL", who);
    return NAT_OK;
}

nat_status nf_loss_grad(nat_nf* nf, const float* in, const float* target, int32_t B, hipStream_t s,
                        NfWs* w)
{
    const int32_t Bp = (B + kRowTile - 1) / kRowTile * kRowTile;
    nat_status st = nf_workspace(nf, Bp, w);
    if (st != NAT_OK)
        return st;
    NAT_HIP(nf_forward(nf, *w, in, target, B, Bp, nullptr, true, s));
    NAT_HIP(nf_backward(nf, *w, in, B, Bp, s));
    return NAT_OK;
}

nat_status nf_read_loss(nat_nf* nf, const NfWs& w, int32_t B, double* loss, hipStream_t s)
{
    if (!loss)
        return NAT_OK;
    double sum = 0.0;
    NAT_HIP(hipMemcpyAsync(&sum, w.loss, sizeof(double), hipMemcpyDeviceToHost, s));
    NAT_HIP(hipStreamSynchronize(s));
    *loss = sum / (static_cast<double>(B) * nf->n_out);
    return NAT_OK;
}

}  // namespace
}  // namespace nat

extern "C" {

using nat::fail;

nat_status nat_nf_create(nat_ctx* ctx, int32_t n_v, int32_t n_out, double r_lo, double r_hi, uint64_t seed,
                         nat_nf** out)
{
    using namespace nat;
    if (!out)
        return fail(NAT_E_INVALID, "nat_nf_create: out is NULL");
    *out = nullptr;
    if (!ctx)
        return fail(NAT_E_INVALID, "nat_nf_create: context is NULL");
    if (n_v < 0 || n_v > kMaxNv)
        return fail(NAT_E_INVALID, "nat_nf_create: n_v = %d (0 .. %d)", n_v, kMaxNv);
    if (n_out < 1 || n_out > kMaxOut)
        return fail(NAT_E_INVALID, "nat_nf_create: n_out = %d (1 .. %d)", n_out, kMaxOut);
    if (!std::isfinite(r_lo) || !std::isfinite(r_hi) || !(r_hi > r_lo))
        return fail(NAT_E_INVALID, "nat_nf_create: shell radii %g, %g", r_lo, r_hi);
    nat_status st = set_device(ctx);
    if (st != NAT_OK)
        return st;
    nat_nf* nf = new nat_nf();
    nf->ctx = ctx;
    nf->n_v = n_v;
    nf->n_out = n_out;
    nf->r_lo = r_lo;
    nf->r_hi = r_hi;
    nf->D = (kLevels * kFeat + 2 * kPeFreqs * (n_v + 1) + 15) / 16 * 16;
    int64_t off = 0, offb = 0;
    for (int i = 0; i < kLayers; ++i) {
        nf->in_dim[i] = i == 0 ? nf->D : kHidden;
        nf->out_dim[i] = i == kLayers - 1 ? n_out : kHidden;
        nf->offW[i] = off;
        off += (int64_t)nf->in_dim[i] * nf->out_dim[i];
        nf->offb[i] = off;
        off += nf->out_dim[i];
        nf->offWb[i] = offb;
        offb += (int64_t)nf->in_dim[i] * nf->out_dim[i];
    }
    nf->offWb[kLayers] = offb;
    for (int l = 0; l < kLevels; ++l) {
        nf->offG[l] = off;
        off += (int64_t)level_size(l) * kFeat;
    }
    nf->n_params = off;
    const size_t np = static_cast<size_t>(off);
    const size_t bytes = carve_size<>({4 * np, 4 * np, 4 * np, 4 * np, 2 * (size_t)offb, 2 * (size_t)offb});
    st = dev_alloc(ctx, bytes, &nf->d_fixed);
    if (st != NAT_OK) {
        delete nf;
        return st;
    }
    nf->fixed_bytes = bytes;
    Carver cv(nf->d_fixed);
    nf->d_params = cv.take<float>(np);
    nf->d_grads = cv.take<float>(np);
    nf->d_m = cv.take<float>(np);
    nf->d_v = cv.take<float>(np);
    nf->d_wb = cv.take<uint16_t>(offb);
    nf->d_wbt = cv.take<uint16_t>(offb);
    // initial parameters (Glorot-uniform weights, zero biases, small grid)
    std::vector<float> h(np, 0.0f);
    for (int i = 0; i < kLayers; ++i) {
        const double a = std::sqrt(6.0 / (nf->in_dim[i] + nf->out_dim[i]));
        const int64_t n = (int64_t)nf->in_dim[i] * nf->out_dim[i];
        for (int64_t e = 0; e < n; ++e)
            h[nf->offW[i] + e] = static_cast<float>(a * uniform_pm1(seed, 1 + i, e));
    }
    for (int l = 0; l < kLevels; ++l)
        for (int64_t e = 0; e < (int64_t)level_size(l) * kFeat; ++e)
            h[nf->offG[l] + e] = static_cast<float>(1e-4 * uniform_pm1(seed, 8 + l, e));
    hipError_t e = hipMemcpy(nf->d_params, h.data(), 4 * np, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemset(nf->d_grads, 0, 4 * np);
    if (e == hipSuccess)
        e = hipMemset(nf->d_m, 0, 4 * np);
    if (e == hipSuccess)
        e = hipMemset(nf->d_v, 0, 4 * np);
    if (e == hipSuccess)
        e = nf_cast(nf, nullptr);
    if (e == hipSuccess)
        e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        dev_free(ctx, nf->d_fixed, nf->fixed_bytes);
        delete nf;
        return nat::hip_fail(e, "nat_nf_create");
    }
    *out = nf;
    return NAT_OK;
}

void nat_nf_destroy(nat_nf* nf)
{
    if (!nf)
        return;
    if (nat::set_device(nf->ctx) == NAT_OK)
        (void)hipDeviceSynchronize();
    nat::dev_free(nf->ctx, nf->d_ws, nf->ws_bytes);
    nat::dev_free(nf->ctx, nf->d_fixed, nf->fixed_bytes);
    delete nf;
}

nat_status nat_nf_info(const nat_nf* nf, int32_t* input_dim, int64_t* n_params)
{
    if (!nf)
        return fail(NAT_E_INVALID, "nat_nf_info: field is NULL");
    if (input_dim)
        *input_dim = nf->D;
    if (n_params)
        *n_params = nf->n_params;
    return NAT_OK;
}

static nat_status nf_copy(const nat_nf* nf, const float* src, float* dst, int64_t n, hipMemcpyKind kind,
                          const char* who)
{
    if (!nf)
        return fail(NAT_E_INVALID, "%s: field is NULL", who);
    if (n != nf->n_params)
        return fail(NAT_E_INVALID, "%s: %lld values, the field has %lld parameters", who, (long long)n,
                    (long long)nf->n_params);
    if (!src || !dst)
        return fail(NAT_E_INVALID, "%s: array is NULL", who);
    nat_status st = nat::set_device(nf->ctx);
    if (st != NAT_OK)
        return st;
    NAT_HIP(hipDeviceSynchronize());
    NAT_HIP(hipMemcpy(dst, src, sizeof(float) * n, kind));
    return NAT_OK;
}

nat_status nat_nf_set_params(nat_nf* nf, const float* params, int64_t n)
{
    nat_status st = nf_copy(nf, params, nf ? nf->d_params : nullptr, n, hipMemcpyHostToDevice,
                            "nat_nf_set_params");
    if (st != NAT_OK)
        return st;
    NAT_HIP(hipMemset(nf->d_m, 0, sizeof(float) * n));
    NAT_HIP(hipMemset(nf->d_v, 0, sizeof(float) * n));
    NAT_HIP(nat::nf_cast(nf, nullptr));
    NAT_HIP(hipDeviceSynchronize());
    return NAT_OK;
}

nat_status nat_nf_get_params(const nat_nf* nf, float* params, int64_t n)
{
    return nf_copy(nf, nf ? nf->d_params : nullptr, params, n, hipMemcpyDeviceToHost, "nat_nf_get_params");
}

nat_status nat_nf_get_grads(const nat_nf* nf, float* grads, int64_t n)
{
    return nf_copy(nf, nf ? nf->d_grads : nullptr, grads, n, hipMemcpyDeviceToHost, "nat_nf_get_grads");
}

nat_status nat_nf_loss_grad(nat_nf* nf, const float* inputs, const float* targets, int32_t B, double* loss,
                            void* stream)
{
    nat_status st = nat::nf_validate_batch(nf, inputs, targets, B, true, "nat_nf_loss_grad");
    if (st != NAT_OK)
        return st;
    if ((st = nat::set_device(nf->ctx)) != NAT_OK)
        return st;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    nat::NfWs w{};
    if ((st = nat::nf_loss_grad(nf, inputs, targets, B, s, &w)) != NAT_OK)
        return st;
    return nat::nf_read_loss(nf, w, B, loss, s);
}

nat_status nat_nf_train_step(nat_nf* nf, const float* inputs, const float* targets, int32_t B, int32_t step,
                             int32_t total_steps, double* loss, void* stream)
{
    nat_status st = nat::nf_validate_batch(nf, inputs, targets, B, true, "nat_nf_train_step");
    if (st != NAT_OK)
        return st;
    if (total_steps < 1 || step < 0)
        return fail(NAT_E_INVALID, "nat_nf_train_step: step %d of %d", step, total_steps);
    if ((st = nat::set_device(nf->ctx)) != NAT_OK)
        return st;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    nat::NfWs w{};
    if ((st = nat::nf_loss_grad(nf, inputs, targets, B, s, &w)) != NAT_OK)
        return st;
    const int64_t third = std::min<int64_t>(2, (3 * (int64_t)step) / total_steps);
    const double lr = 1e-3 * std::pow(0.33, static_cast<double>(third));
    const double t = static_cast<double>(step) + 1.0;
    const double c1 = 1.0 / (1.0 - std::pow(0.9, t));
    const double c2 = 1.0 / (1.0 - std::pow(0.999, t));
    hipLaunchKernelGGL(nat::k_nf_adam, dim3(nat::grid_for(nf->n_params, 256, 2048)), dim3(256), 0, s,
                       nf->d_params, nf->d_grads, nf->d_m, nf->d_v, nf->n_params, static_cast<float>(lr),
                       static_cast<float>(c1), static_cast<float>(c2));
    NAT_HIP(hipGetLastError());
    NAT_HIP(nat::nf_cast(nf, s));
    return nat::nf_read_loss(nf, w, B, loss, s);
}

nat_status nat_nf_infer(nat_nf* nf, const float* inputs, int32_t B, float* out, void* stream)
{
    nat_status st = nat::nf_validate_batch(nf, inputs, nullptr, B, false, "nat_nf_infer");
    if (st != NAT_OK)
        return st;
    if (!out)
        return fail(NAT_E_INVALID, "nat_nf_infer: out is NULL");
    if ((st = nat::set_device(nf->ctx)) != NAT_OK)
        return st;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t Bp = (B + nat::kRowTile - 1) / nat::kRowTile * nat::kRowTile;
    // the fused forward pass keeps everything in LDS: no workspace
    const nat::NfWs none{};
    NAT_HIP(nat::nf_forward(nf, none, inputs, nullptr, B, Bp, out, false, s));
    return NAT_OK;
}

}  // extern "C"

// Neural acoustic transfer field (Section 3): the grid encoding of the
// listener position (Section 3.3), the positional encoding of the condition
// variables and the frequency (Section 3.2), the MLP of 4 hidden layers of
// 128 (Section 3.4), its mean-squared-error gradient and the Adam update.
//
// One batch is a set of rows; the batch is padded to a multiple of 128 rows
// with zero inputs and zero loss weight.  Layout of the activations in HBM:
// each layer's input is kept twice in bfloat16, row-major [rows][width]
// (the operand of the forward and the input-gradient products, contiguous
// along the contraction) and transposed [width][rows] (the operand of the
// weight-gradient products, contiguous along the batch).  The products run
// on the matrix cores (32x32x16 bfloat16 MFMA, FP32 accumulation):
//   forward   Z_i  = A_i W_i^T + b_i, A_{i+1} = relu(Z_i)       (i = 0..3)
//   input     dH_i = dZ_i W_i, dZ_{i-1} = dH_i * [A_i > 0]     (i = 3..1),
//             dH_0 = dZ_0 W_0 for the grid features
//   weights   dW_i = dZ_i^T A_i, split over the batch in chunks whose
//             partial products are added in chunk order
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
constexpr int kGemmGrid = 512;  // workgroups of a product launch (persistent)
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
constexpr int kGridPart = 4608 * kFeat;  // 144 KB of 64-bit accumulators
constexpr int kGridParts = (kGridFloats + kGridPart - 1) / kGridPart;
constexpr int kGridGroupsMax = 21;       // row groups per partition
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

// Packs bfloat16 values of one row into 16-byte stores.
struct RowWriter {
    uint16_t* dst;
    uint32_t buf[4] = {0, 0, 0, 0};
    int n = 0;
    __device__ void put(uint16_t h)
    {
        const int w = (n >> 1) & 3;
        buf[w] = (n & 1) ? (buf[w] | (static_cast<uint32_t>(h) << 16)) : static_cast<uint32_t>(h);
        if ((++n & 7) == 0) {
            *reinterpret_cast<uint4*>(dst + n - 8) = make_uint4(buf[0], buf[1], buf[2], buf[3]);
        }
    }
};

// MLP input of each row: [G | P(v) | P(f) | 0], row-major and (when XT is
// given) transposed.  Padding rows are zero.
__global__ void __launch_bounds__(256) k_nf_encode(NfDev f, const float* __restrict__ in, int32_t B, int32_t Bp,
                                                   uint16_t* __restrict__ X, uint16_t* __restrict__ XT)
{
    const int32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b >= Bp)
        return;
    RowWriter wr{X + (size_t)b * f.D};
    int col = 0;
    auto emit = [&](float v) {
        const uint16_t h = to_bf16(v);
        wr.put(h);
        if (XT)
            XT[(size_t)col * Bp + b] = h;
        ++col;
    };
    if (b < B) {
        const float* row = in + (size_t)b * f.ld_in;
        float u[3];
        unit_coords(f, row, u);
        for (int l = 0; l < kLevels; ++l) {
            Corners c;
            cell_corners(u, l, c);
            float acc[kFeat] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float4 g = *reinterpret_cast<const float4*>(f.grid[l] + (size_t)c.idx[e] * kFeat);
                acc[0] = fmaf(c.w[e], g.x, acc[0]);
                acc[1] = fmaf(c.w[e], g.y, acc[1]);
                acc[2] = fmaf(c.w[e], g.z, acc[2]);
                acc[3] = fmaf(c.w[e], g.w, acc[3]);
            }
            for (int q = 0; q < kFeat; ++q)
                emit(acc[q]);
        }
        for (int s = 0; s <= f.n_v; ++s) {
            const float x = row[3 + s];  // v_0 .. v_{n_v-1}, then f
            for (int m = 0; m < kPeFreqs; ++m) {
                float sn, cs;
                sincospif(ldexpf(x, m), &sn, &cs);
                emit(sn);
                emit(cs);
            }
        }
    }
    while (col < f.D)
        emit(0.0f);
}

// C = A B^T with A [M][K] (lda), B [N][K] (ldb), bfloat16, both contiguous
// along K; M a multiple of 128, K of 16, N <= 32 NBLK.  Epilogue: + bias,
// relu, * [mask > 0] (mask given transposed, [N][ldm]), then bfloat16 stores
// row-major (C) and transposed (CT), and FP32 stores of the first nf
// columns (Cf).
struct NfGemm {
    const uint16_t* A;
    int32_t lda;
    const uint16_t* Bm;
    int32_t ldb;
    int32_t M, N, K;
    const float* bias;
    int32_t relu;
    const uint16_t* mask;
    int32_t ldm;
    uint16_t* C;
    int32_t ldc;
    uint16_t* CT;
    int32_t ldct;
    float* Cf;
    int32_t ldcf, nf;
    float* gmax;     // grid epilogue: max |Cf| of each workgroup [gridDim.x]
};

// Epilogue of a product: forward (+ bias, relu), input gradient (* [mask >
// 0]) or the grid-feature columns (FP32).
enum { kEpiFwd = 0, kEpiBwd = 1, kEpiGrid = 2 };

// Each workgroup stages B in LDS once (rows padded by 16 bytes) and walks
// row tiles of 128 (persistent); wave w computes rows 32 w .. 32 w + 31 of
// the tile against all N columns, with the loads of up to 8 K steps of its
// A rows issued before their products.  MFMA 32x32x16 operand layout: lane
// l holds row (or column) l mod 32 and K entries 8 (l / 32) .. 8 (l / 32) + 7
// of the step; accumulator entry i of lane l is row 8 (i / 4) + 4 (l / 32) +
// i mod 4, column l mod 32.
template <int NBLK, int EPI>
__global__ void __launch_bounds__(256) k_nf_gemm(NfGemm g)
{
    extern __shared__ uint4 s_raw[];
    uint16_t* sB = reinterpret_cast<uint16_t*>(s_raw);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int K = g.K, ldsb = K + 8;
    const int k8 = K / 8;
    for (int e = tid; e < NBLK * 32 * k8; e += 256) {
        const int r = e / k8, c = e - r * k8;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (r < g.N)
            v = *reinterpret_cast<const uint4*>(g.Bm + (size_t)r * g.ldb + c * 8);
        *reinterpret_cast<uint4*>(sB + r * ldsb + c * 8) = v;
    }
    __syncthreads();
    const int half = lane >> 5, l32 = lane & 31;
    const int n_tiles = g.M / kRowTile;
    float wmax = 0.0f;
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int row0 = tile * kRowTile + wave * 32;
        f32x16 acc[NBLK];
#pragma unroll
        for (int nb = 0; nb < NBLK; ++nb)
            acc[nb] = f32x16{};
        const uint16_t* ap = g.A + (size_t)(row0 + l32) * g.lda + half * 8;
        const uint16_t* bp = sB + l32 * ldsb + half * 8;
        float vmax = 0.0f;
        for (int kc = 0; kc < K; kc += 128) {
            const int ns = min(8, (K - kc) >> 4);
            bf16x8 a[8];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (j < ns)
                    a[j] = load8(ap + kc + 16 * j);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (j < ns) {
#pragma unroll
                    for (int nb = 0; nb < NBLK; ++nb) {
                        const bf16x8 bv = *reinterpret_cast<const bf16x8*>(bp + nb * 32 * ldsb + kc + 16 * j);
                        acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[j], bv, acc[nb], 0, 0, 0);
                    }
                }
            }
        }
#pragma unroll
        for (int nb = 0; nb < NBLK; ++nb) {
            const int col = nb * 32 + l32;
            if (col >= g.N)
                continue;
            const float bias = EPI == kEpiFwd ? g.bias[col] : 0.0f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int rbase = row0 + 8 * q + 4 * half;
                uint16_t h[4];
                uint2 m4 = make_uint2(0, 0);
                if (EPI == kEpiBwd)  // mask rows rbase .. rbase + 3 of column col (transposed copy)
                    m4 = *reinterpret_cast<const uint2*>(g.mask + (size_t)col * g.ldm + rbase);
                const uint16_t mk[4] = {static_cast<uint16_t>(m4.x), static_cast<uint16_t>(m4.x >> 16),
                                        static_cast<uint16_t>(m4.y), static_cast<uint16_t>(m4.y >> 16)};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = rbase + r;
                    float v = acc[nb][4 * q + r];
                    if (EPI == kEpiFwd)
                        v = fmaxf(v + bias, 0.0f);
                    if (EPI == kEpiBwd && !bf16_positive(mk[r]))
                        v = 0.0f;
                    if (EPI == kEpiGrid) {
                        if (col < g.nf)
                            g.Cf[(size_t)row * g.ldcf + col] = v;
                    } else {
                        h[r] = to_bf16(v);
                        g.C[(size_t)row * g.ldc + col] = h[r];
                    }
                }
                if (EPI == kEpiGrid) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (col < g.nf)
                            vmax = fmaxf(vmax, fabsf(acc[nb][4 * q + r]));
                }
                if (EPI != kEpiGrid && g.CT) {
                    const uint2 pk = make_uint2(h[0] | (static_cast<uint32_t>(h[1]) << 16),
                                                h[2] | (static_cast<uint32_t>(h[3]) << 16));
                    *reinterpret_cast<uint2*>(g.CT + (size_t)col * g.ldct + rbase) = pk;
                }
            }
        }
        if (EPI == kEpiGrid)
            wmax = fmaxf(wmax, vmax);
    }
    if (EPI == kEpiGrid) {
        __shared__ float s_max[4];
        for (int o = 32; o > 0; o >>= 1)
            wmax = fmaxf(wmax, __shfl_xor(wmax, o, 64));
        if (lane == 0)
            s_max[wave] = wmax;
        __syncthreads();
        if (tid == 0)
            g.gmax[blockIdx.x] = fmaxf(fmaxf(s_max[0], s_max[1]), fmaxf(s_max[2], s_max[3]));
    }
}

// Weight gradient partials: P[c] = A[:, chunk c] B[:, chunk c]^T with
// A = dZ^T [Mo][ld] and B = act^T [Ni][ld] (bfloat16, contiguous along
// the batch), Mo <= 128, Ni <= 32 NBLK; and the bias-gradient partials
// Q[c][m] = sum of A[m][chunk c].  The contraction order inside a chunk is
// a fixed permutation shared by both operands: at step s of 64 rows, lane l
// covers rows 32 (l / 32) + 8 j .. + 7 in MFMA j = 0..3, so each lane reads
// 64 contiguous bytes of its operand rows.
struct NfWgrad {
    const uint16_t* A;
    const uint16_t* Bm;
    int64_t ld;
    int32_t Mo, Ni, chunk, n_rows;
    float* P;
    float* Q;
};

template <int NBLK>
__global__ void __launch_bounds__(256) k_nf_wgrad(NfWgrad w)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int half = lane >> 5, l32 = lane & 31;
    const int c = blockIdx.x;
    const int m0 = wave * 32;
    if (m0 >= w.Mo)
        return;
    const int k0 = c * w.chunk;
    const int k1 = min(k0 + w.chunk, w.n_rows);
    const int am = m0 + l32;
    const bool a_ok = am < w.Mo;
    const uint16_t* ap = w.A + (size_t)(a_ok ? am : 0) * w.ld + half * 32;
    const uint16_t* bp[NBLK];
    bool b_ok[NBLK];
#pragma unroll
    for (int nb = 0; nb < NBLK; ++nb) {
        const int bn = nb * 32 + l32;
        b_ok[nb] = bn < w.Ni;
        bp[nb] = w.Bm + (size_t)(b_ok[nb] ? bn : 0) * w.ld + half * 32;
    }
    f32x16 acc[NBLK];
#pragma unroll
    for (int nb = 0; nb < NBLK; ++nb)
        acc[nb] = f32x16{};
    float gsum = 0.0f;
    const bf16x8 zero = __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
    for (int k = k0; k < k1; k += 64) {
        bf16x8 a[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[j] = a_ok ? load8(ap + k + 8 * j) : zero;
#pragma unroll
            for (int e = 0; e < 8; ++e)
                gsum += static_cast<float>(a[j][e]);
        }
#pragma unroll
        for (int nb = 0; nb < NBLK; ++nb) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bf16x8 bv = b_ok[nb] ? load8(bp[nb] + k + 8 * j) : zero;
                acc[nb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[j], bv, acc[nb], 0, 0, 0);
            }
        }
    }
    float* P = w.P + (size_t)c * w.Mo * w.Ni;
#pragma unroll
    for (int nb = 0; nb < NBLK; ++nb) {
        const int col = nb * 32 + l32;
        if (col >= w.Ni)
            continue;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int m = m0 + 8 * (i / 4) + 4 * half + (i % 4);
            if (m < w.Mo)
                P[(size_t)m * w.Ni + col] = acc[nb][i];
        }
    }
    gsum += __shfl_xor(gsum, 32, 64);
    if (half == 0 && a_ok)
        w.Q[(size_t)c * w.Mo + am] = gsum;
}

// Output layer, loss and the step back to dZ_3, one thread per row.
struct NfOut {
    const uint16_t* H;   // A_4 [Bp][128]
    const uint16_t* W;   // W_4 [n_out][128] bfloat16
    const float* b;      // b_4
    const float* target; // [B][n_out] (training) or null
    float* y;            // [B][n_out] (inference) or null
    int32_t B, Bp, n_out;
    float scale;         // 2 / (B n_out)
    uint16_t* dzoT;      // dZ_4^T [n_out][Bp]
    uint16_t* dz3;       // [Bp][128]
    uint16_t* dz3T;      // [128][Bp]
    double* loss_part;   // per workgroup
};

__global__ void __launch_bounds__(256) k_nf_out(NfOut o)
{
    __shared__ float s_dz[kMaxOut][256];
    __shared__ double s_red[256];
    const int tid = threadIdx.x;
    const int32_t b = blockIdx.x * 256 + tid;
    const bool live = b < o.B;
    double lsum = 0.0;
    uint4 hrow[kHidden / 8];
    if (b < o.Bp) {
#pragma unroll
        for (int q = 0; q < kHidden / 8; ++q)
            hrow[q] = reinterpret_cast<const uint4*>(o.H + (size_t)b * kHidden)[q];
    }
    if (b < o.Bp) {
        for (int oi = 0; oi < o.n_out; ++oi) {
            const uint16_t* wr = o.W + (size_t)oi * kHidden;
            float acc = 0.0f;
#pragma unroll
            for (int q = 0; q < kHidden / 8; ++q) {
                const uint32_t hw[4] = {hrow[q].x, hrow[q].y, hrow[q].z, hrow[q].w};
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const uint16_t hv = static_cast<uint16_t>(hw[e >> 1] >> ((e & 1) * 16));
                    acc = fmaf(from_bf16(hv), from_bf16(wr[q * 8 + e]), acc);
                }
            }
            const float yv = acc + o.b[oi];
            float dz = 0.0f;
            if (live) {
                if (o.y)
                    o.y[(size_t)b * o.n_out + oi] = yv;
                if (o.target) {
                    const float diff = yv - o.target[(size_t)b * o.n_out + oi];
                    lsum += static_cast<double>(diff) * diff;
                    dz = o.scale * diff;
                }
            }
            if (o.dzoT) {
                const uint16_t h = to_bf16(dz);
                o.dzoT[(size_t)oi * o.Bp + b] = h;
                s_dz[oi][tid] = from_bf16(h);
            }
        }
        if (o.dz3) {
            RowWriter wr{o.dz3 + (size_t)b * kHidden};
#pragma unroll
            for (int q = 0; q < kHidden / 8; ++q) {
                const uint32_t hw[4] = {hrow[q].x, hrow[q].y, hrow[q].z, hrow[q].w};
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int k = q * 8 + e;
                    const uint16_t hv = static_cast<uint16_t>(hw[e >> 1] >> ((e & 1) * 16));
                    float dh = 0.0f;
                    for (int oi = 0; oi < o.n_out; ++oi)
                        dh = fmaf(s_dz[oi][tid], from_bf16(o.W[(size_t)oi * kHidden + k]), dh);
                    const uint16_t h = to_bf16(bf16_positive(hv) ? dh : 0.0f);
                    wr.put(h);
                    o.dz3T[(size_t)k * o.Bp + b] = h;
                }
            }
        }
    }
    if (o.loss_part) {
        s_red[tid] = lsum;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (tid < s)
                s_red[tid] += s_red[tid + s];
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

__global__ void __launch_bounds__(256) k_nf_reduce(NfReduce r)
{
    const NfSeg& s = r.seg[blockIdx.y];
    for (int32_t e = blockIdx.x * 256 + threadIdx.x; e < s.n; e += gridDim.x * 256) {
        double a = 0.0;
        for (int c0 = 0; c0 < s.nch; c0 += 8) {
            float v[8];
#pragma unroll
            for (int c = 0; c < 8; ++c)
                v[c] = c0 + c < s.nch ? s.part[(size_t)(c0 + c) * s.n + e] : 0.0f;
#pragma unroll
            for (int c = 0; c < 8; ++c)
                a += v[c];
        }
        s.out[e] = static_cast<float>(a);
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
    // the largest power of two S with B * 8 * gmax * S <= 2^62
    const double bound = static_cast<double>(B) * 8.0 * static_cast<double>(gmax);
    if (!(bound > 0.0) || !isfinite(bound))
        return 1.0;
    return exp2(floor(62.0 - log2(bound)));
}

// The largest of the n per-workgroup maxima (every thread of the block).
__device__ float block_max(const float* __restrict__ m, int32_t n)
{
    __shared__ float s[256];
    float a = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256)
        a = fmaxf(a, m[i]);
    s[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            s[threadIdx.x] = fmaxf(s[threadIdx.x], s[threadIdx.x + h]);
        __syncthreads();
    }
    const float r = s[0];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(256) k_nf_grid_part(NfDev f, const float* __restrict__ in, int32_t B,
                                                      const float* __restrict__ dh0, const float* gmax,
                                                      int32_t n_gmax, long long* __restrict__ part, int32_t G)
{
    __shared__ unsigned long long s_acc[kGridPart];
    const int p = blockIdx.x % kGridParts, g = blockIdx.x / kGridParts;
    const int lo = p * kGridPart;
    const int n = min(kGridPart, kGridFloats - lo);
    const double S = grid_scale(block_max(gmax, n_gmax), B);
    for (int e = threadIdx.x; e < n; e += 256)
        s_acc[e] = 0ull;
    __syncthreads();
    for (int32_t b = g * 256 + threadIdx.x; b < B; b += G * 256) {
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
                        atomicAdd(s_acc + at + q, static_cast<unsigned long long>(__double2ll_rn(w * gs[q])));
                }
            }
        }
    }
    __syncthreads();
    long long* dst = part + (size_t)g * kGridFloats + lo;
    for (int e = threadIdx.x; e < n; e += 256)
        dst[e] = static_cast<long long>(s_acc[e]);
}

__global__ void __launch_bounds__(256) k_nf_grid_fold(const long long* __restrict__ part, int32_t G, int32_t B,
                                                      const float* gmax, int32_t n_gmax, float* __restrict__ out)
{
    const double inv = 1.0 / grid_scale(block_max(gmax, n_gmax), B);
    for (int e = blockIdx.x * 256 + threadIdx.x; e < kGridFloats; e += gridDim.x * 256) {
        long long a = 0;
        for (int g = 0; g < G; ++g)
            a += part[(size_t)g * kGridFloats + e];
        out[e] = static_cast<float>(static_cast<double>(a) * inv);
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
    uint16_t *X, *XT;
    uint16_t *H[4], *HT[4];   // A_1 .. A_4
    uint16_t *dz[4], *dzT[4]; // dZ_0 .. dZ_3
    uint16_t* dzoT;           // dZ_4^T
    float* dh0;               // [Bp][16]
    double* loss_part;
    double* loss;
    float* P;                 // weight-gradient chunk partials, every layer
    float* Q;                 // bias-gradient chunk partials, every layer
    long long* gpart;         // grid-gradient partials [grid_groups][kGridFloats]
    float* gmax;              // max |dH_0| of each workgroup of its product
    int32_t n_gmax;
    int64_t offP[kLayers], offQ[kLayers];
    int32_t chunk, nch, grid_groups;
};

int32_t nf_grid_groups(int32_t Bp)
{
    return static_cast<int32_t>(std::max<int64_t>(1, std::min<int64_t>(kGridGroupsMax, (Bp + 4095) / 4096)));
}

void nf_chunks(int32_t Bp, int32_t* chunk, int32_t* nch)
{
    int64_t c = (Bp + 255) / 256;
    c = std::max<int64_t>(kRowTile, (c + kRowTile - 1) / kRowTile * kRowTile);
    *chunk = static_cast<int32_t>(c);
    *nch = static_cast<int32_t>((Bp + c - 1) / c);
}

size_t nf_ws_layout(const nat_nf* nf, int32_t Bp, NfWs* w, void* base)
{
    int32_t chunk, nch;
    nf_chunks(Bp, &chunk, &nch);
    const size_t bp = static_cast<size_t>(Bp);
    size_t sum_pq = 0, sum_q = 0;
    for (int i = 0; i < kLayers; ++i) {
        sum_pq += static_cast<size_t>(nf->out_dim[i]) * nf->in_dim[i];
        sum_q += static_cast<size_t>(nf->out_dim[i]);
    }
    const int32_t G = nf_grid_groups(Bp);
    std::vector<size_t> sz;
    sz.push_back(2 * bp * nf->D);
    sz.push_back(2 * bp * nf->D);
    for (int i = 0; i < 16; ++i)
        sz.push_back(2 * bp * kHidden);
    sz.push_back(2 * bp * nf->n_out);
    sz.push_back(4 * bp * kLevels * kFeat);
    sz.push_back(8 * (bp / 256 + 1));
    sz.push_back(8);
    sz.push_back(4 * sum_pq * nch);
    sz.push_back(4 * sum_q * nch);
    sz.push_back(8 * static_cast<size_t>(kGridFloats) * G);
    sz.push_back(4 * static_cast<size_t>(kGemmGrid));
    size_t total = 0;
    for (size_t s : sz)
        total = ((total + 255) & ~size_t(255)) + s;
    total += 256;
    if (w && base) {
        Carver cv(base);
        w->X = cv.take<uint16_t>(bp * nf->D);
        w->XT = cv.take<uint16_t>(bp * nf->D);
        for (int i = 0; i < 4; ++i)
            w->H[i] = cv.take<uint16_t>(bp * kHidden);
        for (int i = 0; i < 4; ++i)
            w->HT[i] = cv.take<uint16_t>(bp * kHidden);
        for (int i = 0; i < 4; ++i)
            w->dz[i] = cv.take<uint16_t>(bp * kHidden);
        for (int i = 0; i < 4; ++i)
            w->dzT[i] = cv.take<uint16_t>(bp * kHidden);
        w->dzoT = cv.take<uint16_t>(bp * nf->n_out);
        w->dh0 = cv.take<float>(bp * kLevels * kFeat);
        w->loss_part = cv.take<double>(bp / 256 + 1);
        w->loss = cv.take<double>(1);
        w->P = cv.take<float>(sum_pq * nch);
        w->Q = cv.take<float>(sum_q * nch);
        w->gpart = cv.take<long long>(static_cast<size_t>(kGridFloats) * G);
        w->gmax = cv.take<float>(kGemmGrid);
        w->n_gmax = std::min(Bp / kRowTile, kGemmGrid);
        int64_t op = 0, oq = 0;
        for (int i = 0; i < kLayers; ++i) {
            w->offP[i] = op;
            w->offQ[i] = oq;
            op += (int64_t)nf->out_dim[i] * nf->in_dim[i] * nch;
            oq += (int64_t)nf->out_dim[i] * nch;
        }
        w->chunk = chunk;
        w->nch = nch;
        w->grid_groups = G;
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

template <int EPI>
hipError_t launch_gemm_epi(const NfGemm& g, hipStream_t s)
{
    const int nblk = (g.N + 31) / 32;
    const size_t lds = static_cast<size_t>(nblk) * 32 * (g.K + 8) * sizeof(uint16_t);
    // persistent: B is staged once per workgroup
    const int grid = std::min(g.M / kRowTile, kGemmGrid);
    switch (nblk) {
    case 1: hipLaunchKernelGGL((k_nf_gemm<1, EPI>), dim3(grid), dim3(256), lds, s, g); break;
    case 2: hipLaunchKernelGGL((k_nf_gemm<2, EPI>), dim3(grid), dim3(256), lds, s, g); break;
    case 3: hipLaunchKernelGGL((k_nf_gemm<3, EPI>), dim3(grid), dim3(256), lds, s, g); break;
    case 4: hipLaunchKernelGGL((k_nf_gemm<4, EPI>), dim3(grid), dim3(256), lds, s, g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gemm(const NfGemm& g, hipStream_t s)
{
    if (g.Cf)
        return launch_gemm_epi<kEpiGrid>(g, s);
    if (g.mask)
        return launch_gemm_epi<kEpiBwd>(g, s);
    return launch_gemm_epi<kEpiFwd>(g, s);
}

hipError_t launch_wgrad(const NfWgrad& w, int nch, hipStream_t s)
{
    const int nblk = (w.Ni + 31) / 32;
    switch (nblk) {
    case 1: hipLaunchKernelGGL(k_nf_wgrad<1>, dim3(nch), dim3(256), 0, s, w); break;
    case 2: hipLaunchKernelGGL(k_nf_wgrad<2>, dim3(nch), dim3(256), 0, s, w); break;
    case 3: hipLaunchKernelGGL(k_nf_wgrad<3>, dim3(nch), dim3(256), 0, s, w); break;
    case 4: hipLaunchKernelGGL(k_nf_wgrad<4>, dim3(nch), dim3(256), 0, s, w); break;
    case 5: hipLaunchKernelGGL(k_nf_wgrad<5>, dim3(nch), dim3(256), 0, s, w); break;
    case 6: hipLaunchKernelGGL(k_nf_wgrad<6>, dim3(nch), dim3(256), 0, s, w); break;
    case 7: hipLaunchKernelGGL(k_nf_wgrad<7>, dim3(nch), dim3(256), 0, s, w); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Forward pass of B rows (padded to Bp); with `train` the transposed copies
// are written and the output kernel forms the loss and dZ_4, dZ_3.
hipError_t nf_forward(nat_nf* nf, const NfWs& w, const float* in, const float* target, int32_t B, int32_t Bp,
                      float* y, bool train, hipStream_t s)
{
    const NfDev f = nf_dev(nf);
    hipLaunchKernelGGL(k_nf_encode, dim3((Bp + 255) / 256), dim3(256), 0, s, f, in, B, Bp, w.X,
                       train ? w.XT : nullptr);
    hipError_t e = hipGetLastError();
    for (int i = 0; i < 4 && e == hipSuccess; ++i) {
        NfGemm g{};
        g.A = i == 0 ? w.X : w.H[i - 1];
        g.lda = i == 0 ? nf->D : kHidden;
        g.Bm = nf->d_wb + nf->offWb[i];
        g.ldb = nf->in_dim[i];
        g.M = Bp;
        g.N = kHidden;
        g.K = nf->in_dim[i];
        g.bias = nf->d_params + nf->offb[i];
        g.relu = 1;
        g.C = w.H[i];
        g.ldc = kHidden;
        g.CT = train ? w.HT[i] : nullptr;
        g.ldct = Bp;
        e = launch_gemm(g, s);
    }
    if (e != hipSuccess)
        return e;
    NfOut o{};
    o.H = w.H[3];
    o.W = nf->d_wb + nf->offWb[4];
    o.b = nf->d_params + nf->offb[4];
    o.target = train ? target : nullptr;
    o.y = y;
    o.B = B;
    o.Bp = Bp;
    o.n_out = nf->n_out;
    o.scale = static_cast<float>(2.0 / (static_cast<double>(B) * nf->n_out));
    o.dzoT = train ? w.dzoT : nullptr;
    o.dz3 = train ? w.dz[3] : nullptr;
    o.dz3T = train ? w.dzT[3] : nullptr;
    o.loss_part = train ? w.loss_part : nullptr;
    hipLaunchKernelGGL(k_nf_out, dim3((Bp + 255) / 256), dim3(256), 0, s, o);
    e = hipGetLastError();
    if (e == hipSuccess && train) {
        hipLaunchKernelGGL(k_nf_sum, dim3(1), dim3(256), 0, s, w.loss_part, (Bp + 255) / 256, w.loss);
        e = hipGetLastError();
    }
    return e;
}

// Gradient of every parameter into d_grads (after nf_forward with train).
hipError_t nf_backward(nat_nf* nf, const NfWs& w, const float* in, int32_t B, int32_t Bp, hipStream_t s)
{
    hipError_t e = hipSuccess;
    // input gradients: dZ_3 -> dZ_2 -> dZ_1 -> dZ_0 -> dH_0 (grid columns)
    for (int i = 3; i >= 0 && e == hipSuccess; --i) {
        NfGemm g{};
        g.A = w.dz[i];
        g.lda = kHidden;
        g.Bm = nf->d_wbt + nf->offWb[i];  // W_i^T [in_i][128]
        g.ldb = kHidden;
        g.M = Bp;
        g.K = kHidden;
        if (i > 0) {
            g.N = kHidden;
            g.mask = w.HT[i - 1];  // A_i transposed: [128][Bp]
            g.ldm = Bp;
            g.C = w.dz[i - 1];
            g.ldc = kHidden;
            g.CT = w.dzT[i - 1];
            g.ldct = Bp;
        } else {
            g.N = 32;  // the grid features are the first 16 input columns
            g.Cf = w.dh0;
            g.ldcf = kLevels * kFeat;
            g.nf = kLevels * kFeat;
            g.gmax = w.gmax;
        }
        e = launch_gemm(g, s);
    }
    // weight and bias gradients: chunk partials of every layer, then one
    // launch folds them in chunk order
    NfReduce red{};
    int32_t max_n = 0;
    for (int i = 0; i < kLayers && e == hipSuccess; ++i) {
        NfWgrad g{};
        g.A = i == 4 ? w.dzoT : w.dzT[i];
        g.Bm = i == 0 ? w.XT : w.HT[i - 1];
        g.ld = Bp;
        g.Mo = nf->out_dim[i];
        g.Ni = nf->in_dim[i];
        g.chunk = w.chunk;
        g.n_rows = Bp;
        g.P = w.P + w.offP[i];
        g.Q = w.Q + w.offQ[i];
        e = launch_wgrad(g, w.nch, s);
        red.seg[2 * i] = NfSeg{g.P, nf->d_grads + nf->offW[i], nf->out_dim[i] * nf->in_dim[i], w.nch};
        red.seg[2 * i + 1] = NfSeg{g.Q, nf->d_grads + nf->offb[i], nf->out_dim[i], w.nch};
        max_n = std::max(max_n, nf->out_dim[i] * nf->in_dim[i]);
    }
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_nf_reduce, dim3(grid_for(max_n, 256, 64), 2 * kLayers), dim3(256), 0, s, red);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    // grid-feature gradient: LDS partitions, then the ordered fold
    const NfDev f = nf_dev(nf);
    const int32_t G = w.grid_groups;
    hipLaunchKernelGGL(k_nf_grid_part, dim3(kGridParts * G), dim3(256), 0, s, f, in, B, w.dh0, w.gmax, w.n_gmax,
                       w.gpart, G);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_nf_grid_fold, dim3(grid_for(kGridFloats, 256, 512)), dim3(256), 0, s, w.gpart, G, B,
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
    nat::NfWs w{};
    if ((st = nat::nf_workspace(nf, Bp, &w)) != NAT_OK)
        return st;
    NAT_HIP(nat::nf_forward(nf, w, inputs, nullptr, B, Bp, out, false, s));
    return NAT_OK;
}

}  // extern "C"

// Split-BF16 projection GEMMs on the gfx950 BF16 matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation).
//
// Every FP32 operand value x is split while it is staged into LDS as
// x ~ hi + lo with hi = bf16(x) and lo = bf16(x - hi) (|x - hi - lo| <= 2^-16 |x|),
// and each product is formed as hi*hi' + hi*lo' + lo*hi' (the lo*lo' term,
// of relative size 2^-16, is dropped).  The operands in memory stay FP32,
// so the split costs no extra storage and no extra memory traffic.
//
//   coefficients  C[m][n] = sum_k H[m][k] V[n][k]
//   residual      ||H[m] - sum_k C[m][k] V[k]||^2, summed per output tile
//
// Workgroup: 4 waves as 2 x 2, each owning SM x SN tiles of 32 x 32; K in
// chunks of 32 (two MFMA k-steps of 16) through double-buffered LDS.
// 32x32x16 bf16 layout: lane l supplies A[l%32][8(l/32) + j] and
// B[8(l/32) + j][l%32], j = 0..7; result register r of lane l is
// D[8(r/4) + 4(l/32) + r%4][l%32].
#include "lie_internal.h"

#include <algorithm>

namespace lie {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int KC = 32;        // K chunk
constexpr int LDK = KC + 8;   // LDS row stride (bf16 elements), keeps 16-byte alignment

__device__ inline bool aborted(const DevState *st) { return st && (st->done | st->numeric_error | st->full); }

__device__ inline void split(float x, __bf16 &hi, __bf16 &lo)
{
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

// K-contiguous FP32 rows [r0, r0+BR) x [k0, k0+KC) -> split bf16 tiles S[row][k].
template <int BR>
struct SplitRowLoader {
    static constexpr int TOTAL = BR * KC / 4;  // float4 per tile
    static constexpr int PER_THREAD = (TOTAL + 255) / 256;
    float v[PER_THREAD][4];

    __device__ void load(const float *__restrict__ base, int64_t ld, int64_t r0, int64_t rows, int64_t k0, int64_t K,
                         bool vec_ok)
    {
#pragma unroll
        for (int i = 0; i < PER_THREAD; ++i) {
            const int q = threadIdx.x + 256 * i;
            const int r = q / (KC / 4), kv = (q % (KC / 4)) * 4;
            const int64_t row = r0 + r, k = k0 + kv;
            v[i][0] = v[i][1] = v[i][2] = v[i][3] = 0.f;
            if (q < TOTAL && row < rows) {
                const float *p = base + row * ld + k;
                if (vec_ok && k + 4 <= K) {
                    const float4 t = *reinterpret_cast<const float4 *>(p);
                    v[i][0] = t.x;
                    v[i][1] = t.y;
                    v[i][2] = t.z;
                    v[i][3] = t.w;
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (k + u < K)
                            v[i][u] = p[u];
                }
            }
        }
    }
    __device__ void store(__bf16 (*Sh)[LDK], __bf16 (*Sl)[LDK]) const
    {
#pragma unroll
        for (int i = 0; i < PER_THREAD; ++i) {
            const int q = threadIdx.x + 256 * i;
            if (q < TOTAL) {
                const int r = q / (KC / 4), kv = (q % (KC / 4)) * 4;
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    split(v[i][u], Sh[r][kv + u], Sl[r][kv + u]);
            }
        }
    }
};

// Row-major FP32 K x N operand (rows k, contiguous n): [k0, k0+KC) x [n0, n0+BN) -> split bf16 S[n][k].
// A thread takes one column n and 8 consecutive rows k (eight 4-byte loads, each coalesced
// across the wave along n), splits them, and stores each of hi and lo as one 16-byte
// vector at S[n][8g .. 8g+8) -- the layout the MFMA operand reads back.
template <int BN>
struct SplitColLoader {
    static constexpr int GROUPS = KC / 8;
    static constexpr int TOTAL = BN * GROUPS;  // (column, 8-row group) items per tile
    static constexpr int PER_THREAD = (TOTAL + 255) / 256;
    float v[PER_THREAD][8];

    __device__ void load(const float *__restrict__ base, int64_t ld, int64_t k0, int64_t K, int64_t n0, int64_t Ncols,
                         bool)
    {
#pragma unroll
        for (int i = 0; i < PER_THREAD; ++i) {
            const int q = threadIdx.x + 256 * i;
            const int n = q % BN, g = q / BN;
            const int64_t col = n0 + n;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t k = k0 + 8 * g + u;
                v[i][u] = (q < TOTAL && col < Ncols && k < K) ? base[k * ld + col] : 0.f;
            }
        }
    }
    __device__ void store(__bf16 (*Sh)[LDK], __bf16 (*Sl)[LDK]) const
    {
#pragma unroll
        for (int i = 0; i < PER_THREAD; ++i) {
            const int q = threadIdx.x + 256 * i;
            if (q < TOTAL) {
                const int n = q % BN, g = q / BN;
                bf16x8 h, l;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    __bf16 hu, lu;
                    split(v[i][u], hu, lu);
                    h[u] = hu;
                    l[u] = lu;
                }
                *reinterpret_cast<bf16x8 *>(&Sh[n][8 * g]) = h;
                *reinterpret_cast<bf16x8 *>(&Sl[n][8 * g]) = l;
            }
        }
    }
};

template <int SM, int SN>
struct alignas(16) Tiles {
    static constexpr int BM = 2 * SM * 32, BN = 2 * SN * 32;
    __bf16 Ah[2][BM][LDK], Al[2][BM][LDK];
    __bf16 Bh[2][BN][LDK], Bl[2][BN][LDK];
};

// One K chunk of MFMA work for a wave: 3 products per (i, j) tile pair and k-step.
template <int SM, int SN>
__device__ inline void mma_chunk(const Tiles<SM, SN> &t, int buf, int wm, int wn, int lane, f32x16 (&acc)[SM][SN])
{
#pragma unroll
    for (int ks = 0; ks < KC; ks += 16) {
        bf16x8 ah[SM], al[SM], bh[SN], bl[SN];
        const int kq = ks + 8 * (lane >> 5);
#pragma unroll
        for (int i = 0; i < SM; ++i) {
            const int row = wm * SM * 32 + i * 32 + (lane & 31);
            ah[i] = *reinterpret_cast<const bf16x8 *>(&t.Ah[buf][row][kq]);
            al[i] = *reinterpret_cast<const bf16x8 *>(&t.Al[buf][row][kq]);
        }
#pragma unroll
        for (int j = 0; j < SN; ++j) {
            const int col = wn * SN * 32 + j * 32 + (lane & 31);
            bh[j] = *reinterpret_cast<const bf16x8 *>(&t.Bh[buf][col][kq]);
            bl[j] = *reinterpret_cast<const bf16x8 *>(&t.Bl[buf][col][kq]);
        }
#pragma unroll
        for (int i = 0; i < SM; ++i)
#pragma unroll
            for (int j = 0; j < SN; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
            }
    }
}

template <int SM, int SN>
__device__ void bf_dot_body(const GemmArgs &g, int bx0, int by, int gxs)
{
    using TT = Tiles<SM, SN>;
    constexpr int BM = TT::BM, BN = TT::BN;
    if (aborted(g.st))
        return;
    const int64_t N = g.st ? g.st->N : g.N_fixed;
    const int Mrows = g.nrows ? *g.nrows : g.cnt;
    const int m0 = by * BM;
    if ((int64_t)bx0 * BN >= N || m0 >= Mrows)
        return;
    __shared__ TT t;
    const float *H = static_cast<const float *>(g.H);
    const float *V = static_cast<const float *>(g.V);
    const bool vec_ok = (g.D % 4) == 0;
    SplitRowLoader<BM> la;
    SplitRowLoader<BN> lb;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w >> 1, wn = w & 1;
    for (int64_t n0 = (int64_t)bx0 * BN; n0 < N; n0 += (int64_t)gxs * BN) {
        f32x16 acc[SM][SN];
#pragma unroll
        for (int i = 0; i < SM; ++i)
#pragma unroll
            for (int j = 0; j < SN; ++j)
                acc[i][j] = f32x16{};
        const int nchunks = (int)((g.D + KC - 1) / KC);
        la.load(H, g.D, m0, Mrows, 0, g.D, vec_ok);
        lb.load(V, g.D, n0, N, 0, g.D, vec_ok);
        la.store(t.Ah[0], t.Al[0]);
        lb.store(t.Bh[0], t.Bl[0]);
        __syncthreads();
        for (int c = 0; c < nchunks; ++c) {
            const int buf = c & 1;
            if (c + 1 < nchunks) {
                la.load(H, g.D, m0, Mrows, (int64_t)(c + 1) * KC, g.D, vec_ok);
                lb.load(V, g.D, n0, N, (int64_t)(c + 1) * KC, g.D, vec_ok);
            }
            mma_chunk<SM, SN>(t, buf, wm, wn, lane, acc);
            if (c + 1 < nchunks) {
                la.store(t.Ah[buf ^ 1], t.Al[buf ^ 1]);
                lb.store(t.Bh[buf ^ 1], t.Bl[buf ^ 1]);
            }
            __syncthreads();
        }
        float *C = static_cast<float *>(g.C);
#pragma unroll
        for (int i = 0; i < SM; ++i)
#pragma unroll
            for (int j = 0; j < SN; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int m = m0 + wm * SM * 32 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    const int64_t n = n0 + wn * SN * 32 + j * 32 + (lane & 31);
                    if (m < Mrows && n < N)
                        C[(int64_t)m * g.ldc + n] = acc[i][j][r];
                }
    }
}

template <int SM, int SN>
__device__ void bf_sub_body(const GemmArgs &g, int bx, int by, int ntiles)
{
    using TT = Tiles<SM, SN>;
    constexpr int BM = TT::BM, BN = TT::BN;
    if (aborted(g.st))
        return;
    const int64_t N = g.st ? g.st->N : g.N_fixed;
    const int Mrows = g.nrows ? *g.nrows : g.cnt;
    const int64_t j0 = (int64_t)bx * BN;
    const int m0 = by * BM;
    if (m0 >= Mrows)
        return;
    __shared__ TT t;
    __shared__ double red[BM][2][2];
    const float *Cc = static_cast<const float *>(g.C);
    const float *V = static_cast<const float *>(g.V);
    SplitRowLoader<BM> la;  // coefficients, K = basis index
    SplitColLoader<BN> lb;  // basis rows
    const bool vec_c = (g.ldc % 4) == 0;
    const bool vec_v = (g.D % 4) == 0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w >> 1, wn = w & 1;
    f32x16 acc[SM][SN];
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int j = 0; j < SN; ++j)
            acc[i][j] = f32x16{};
    const int nchunks = (int)((N + KC - 1) / KC);
    if (nchunks > 0) {
        la.load(Cc, g.ldc, m0, Mrows, 0, N, vec_c);
        lb.load(V, g.D, 0, N, j0, g.D, vec_v);
        la.store(t.Ah[0], t.Al[0]);
        lb.store(t.Bh[0], t.Bl[0]);
    }
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
        const int buf = c & 1;
        if (c + 1 < nchunks) {
            la.load(Cc, g.ldc, m0, Mrows, (int64_t)(c + 1) * KC, N, vec_c);
            lb.load(V, g.D, (int64_t)(c + 1) * KC, N, j0, g.D, vec_v);
        }
        mma_chunk<SM, SN>(t, buf, wm, wn, lane, acc);
        if (c + 1 < nchunks) {
            la.store(t.Ah[buf ^ 1], t.Al[buf ^ 1]);
            lb.store(t.Bh[buf ^ 1], t.Bl[buf ^ 1]);
        }
        __syncthreads();
    }
    const float *H = static_cast<const float *>(g.H);
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int ml = wm * SM * 32 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const int m = m0 + ml;
            double rs = 0.0, hsq = 0.0;
            if (m < Mrows) {
#pragma unroll
                for (int j = 0; j < SN; ++j) {
                    const int64_t col = j0 + wn * SN * 32 + j * 32 + (lane & 31);
                    if (col < g.D) {
                        const float h = H[(int64_t)m * g.D + col];
                        const float res = h - acc[i][j][r];
                        rs += (double)res * res;
                        hsq += (double)h * h;
                    }
                }
            }
            for (int off = 16; off > 0; off >>= 1) {
                rs += __shfl_xor(rs, off, 64);
                hsq += __shfl_xor(hsq, off, 64);
            }
            if ((lane & 31) == 0) {
                red[ml][wn][0] = rs;
                red[ml][wn][1] = hsq;
            }
        }
    __syncthreads();
    if (threadIdx.x < BM) {
        const int m = m0 + threadIdx.x;
        if (m < Mrows) {
            double *o = g.normpart + ((int64_t)m * ntiles + bx) * 2;
            o[0] = red[threadIdx.x][0][0] + red[threadIdx.x][1][0];
            o[1] = red[threadIdx.x][0][1] + red[threadIdx.x][1][1];
        }
    }
}

template <int SM, int SN>
__global__ void __launch_bounds__(256) k_bf_dot(GemmArgs g)
{
    bf_dot_body<SM, SN>(g, blockIdx.x, blockIdx.y, gridDim.x);
}
template <int SM, int SN>
__global__ void __launch_bounds__(256) k_bf_sub(GemmArgs g)
{
    bf_sub_body<SM, SN>(g, blockIdx.x, blockIdx.y, gridDim.x);
}
template <int SM, int SN>
__global__ void __launch_bounds__(256) k_bf_dot_b(Batch b)
{
    const int p = batch_find(b.start, b.nprob, blockIdx.x);
    const GemmArgs g = static_cast<const GemmArgs *>(b.args)[p];
    const int l = blockIdx.x - b.start[p], gx = b.gx[p];
    bf_dot_body<SM, SN>(g, l % gx, l / gx, gx);
}
template <int SM, int SN>
__global__ void __launch_bounds__(256) k_bf_sub_b(Batch b)
{
    const int p = batch_find(b.start, b.nprob, blockIdx.x);
    const GemmArgs g = static_cast<const GemmArgs *>(b.args)[p];
    const int l = blockIdx.x - b.start[p], gx = b.gx[p];
    bf_sub_body<SM, SN>(g, l % gx, l / gx, gx);
}

}  // namespace

int gemm_sub_tiles_bf16(int64_t D, int tile) { return (int)((D + (tile == 2 ? 128 : 64) - 1) / (tile == 2 ? 128 : 64)); }

hipError_t launch_gemm_dot_bf16x3(const float *Vs, const DevState *st, const float *Hs, int cnt, int64_t D,
                                  int64_t n_hi, int64_t ldc, float *C, int tile, hipStream_t s)
{
    if (cnt <= 0)
        return hipSuccess;
    GemmArgs g{};
    g.H = Hs;
    g.cnt = cnt;
    g.V = Vs;
    g.C = C;
    g.ldc = ldc;
    g.D = D;
    g.st = st;
    n_hi = std::max<int64_t>(n_hi, 1);
    if (tile == 2)
        hipLaunchKernelGGL((k_bf_dot<2, 2>), dim3((unsigned)((n_hi + 127) / 128), (cnt + 127) / 128), dim3(256), 0, s,
                           g);
    else
        hipLaunchKernelGGL((k_bf_dot<1, 1>), dim3((unsigned)((n_hi + 63) / 64), (cnt + 63) / 64), dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_gemm_sub_bf16x3(const float *Vs, const DevState *st, const float *Hs, const float *C, int64_t n_hi,
                                  int64_t ldc, int cnt, int64_t D, double *normpart, int tile, hipStream_t s)
{
    if (cnt <= 0)
        return hipSuccess;
    GemmArgs g{};
    g.H = Hs;
    g.cnt = cnt;
    g.V = Vs;
    g.C = const_cast<float *>(C);
    g.ldc = ldc;
    g.D = D;
    g.st = st;
    g.normpart = normpart;
    const int tiles = gemm_sub_tiles_bf16(D, tile);
    if (tile == 2)
        hipLaunchKernelGGL((k_bf_sub<2, 2>), dim3(tiles, (cnt + 127) / 128), dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL((k_bf_sub<1, 1>), dim3(tiles, (cnt + 63) / 64), dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_gemm_dot_bf16x3_batched(const Batch &b, hipStream_t s)
{
    if (b.total <= 0)
        return hipSuccess;
    hipLaunchKernelGGL((k_bf_dot_b<1, 1>), dim3(b.total), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_gemm_sub_bf16x3_batched(const Batch &b, hipStream_t s)
{
    if (b.total <= 0)
        return hipSuccess;
    hipLaunchKernelGGL((k_bf_sub_b<1, 1>), dim3(b.total), dim3(256), 0, s, b);
    return hipGetLastError();
}

}  // namespace lie

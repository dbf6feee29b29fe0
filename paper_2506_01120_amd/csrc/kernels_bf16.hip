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

constexpr int KC = 32;   // K chunk
constexpr int LDK = KC;  // LDS row: 64 bytes, four 16-byte groups of 8 k, unpadded

// Column of element k of LDS row `row`: the 16-byte group g = k / 8 is stored at position
// g ^ ((row / 2) % 4).  An MFMA fragment read (lanes 0-7 take rows r..r+7 at one group)
// then touches eight distinct 16-byte bank groups, and the staging writes, which cover
// whole consecutive rows, are contiguous -- neither conflicts.
__device__ inline int swz(int row, int k) { return ((((k >> 3) ^ (row >> 1)) & 3) << 3) | (k & 7); }

__device__ inline bool aborted(const DevState *st) { return st && (st->done | st->numeric_error | st->full); }

__device__ inline void split(float x, __bf16 &hi, __bf16 &lo)
{
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

// K-contiguous FP32 rows [r0, r0+BR) x [k0, k0+KC) -> split bf16 tiles S[row][k].
// Loads are unconditional: a row past `rows` or a column past K reads a valid address
// (row rows-1, column 0), and the store replaces such values by zero.  Keeping the
// masking out of the load step lets every load of a chunk be in flight at once.
// VEC: ld and the base are multiples of 4 floats, ld >= K rounded up to 4, and one
// 16-byte load takes four consecutive k.
template <int BR, bool VEC>
struct SplitRowLoader {
    static constexpr int TOTAL = BR * KC / 4;  // float4 per tile
    static_assert(TOTAL % 256 == 0, "tile rows must fill the workgroup");
    static constexpr int PER_THREAD = TOTAL / 256;
    float v[PER_THREAD][4];
    int nv[PER_THREAD];  // leading values of the item that are in range (0..4)

    __device__ void load(const float *__restrict__ base, int64_t ld, int64_t r0, int64_t rows, int64_t k0, int64_t K)
    {
#pragma unroll
        for (int i = 0; i < PER_THREAD; ++i) {
            const int q = threadIdx.x + 256 * i;
            const int r = q / (KC / 4), kv = (q % (KC / 4)) * 4;
            const int64_t row = r0 + r, k = k0 + kv;
            const bool rok = row < rows;
            nv[i] = rok ? (int)min<int64_t>(max<int64_t>(K - k, 0), 4) : 0;
            const float *p = base + (rok ? row : rows - 1) * ld;
            if (VEC) {
                const float4 t = *reinterpret_cast<const float4 *>(p + (k < K ? k : 0));
                v[i][0] = t.x;
                v[i][1] = t.y;
                v[i][2] = t.z;
                v[i][3] = t.w;
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    v[i][u] = p[k + u < K ? k + u : 0];
            }
        }
    }
    __device__ void store(__bf16 (*Sh)[LDK], __bf16 (*Sl)[LDK]) const
    {
#pragma unroll
        for (int i = 0; i < PER_THREAD; ++i) {
            const int q = threadIdx.x + 256 * i;
            const int r = q / (KC / 4), kv = (q % (KC / 4)) * 4;
            const int col = swz(r, kv);  // the four values stay inside one 16-byte group
#pragma unroll
            for (int u = 0; u < 4; ++u)
                split(u < nv[i] ? v[i][u] : 0.f, Sh[r][col + u], Sl[r][col + u]);
        }
    }
};

// Row-major FP32 K x N operand (rows k, contiguous n): [k0, k0+KC) x [n0, n0+BN) -> split bf16 S[n][k].
// A thread takes one column n and 8 consecutive rows k (eight 4-byte loads, each coalesced
// across the wave along n), splits them, and stores each of hi and lo as one 16-byte
// vector at S[n][8g .. 8g+8) -- the layout the MFMA operand reads back.  Out-of-range
// entries read a valid address and are zeroed at the store, as in the row loader.
template <int BN>
struct SplitColLoader {
    static constexpr int GROUPS = KC / 8;
    static constexpr int TOTAL = BN * GROUPS;  // (column, 8-row group) items per tile
    static_assert(TOTAL % 256 == 0, "tile columns must fill the workgroup");
    static constexpr int PER_THREAD = TOTAL / 256;
    float v[PER_THREAD][8];
    int nv[PER_THREAD];  // leading rows of the item that are in range (0..8)

    __device__ void load(const float *__restrict__ base, int64_t ld, int64_t k0, int64_t K, int64_t n0, int64_t Ncols)
    {
#pragma unroll
        for (int i = 0; i < PER_THREAD; ++i) {
            const int q = threadIdx.x + 256 * i;
            const int n = q % BN, g = q / BN;
            const int64_t col = n0 + n, kg = k0 + 8 * g;
            const bool cok = col < Ncols;
            nv[i] = cok ? (int)min<int64_t>(max<int64_t>(K - kg, 0), 8) : 0;
            const float *p = base + (cok ? col : 0);
#pragma unroll
            for (int u = 0; u < 8; ++u)
                v[i][u] = p[(kg + u < K ? kg + u : 0) * ld];
        }
    }
    __device__ void store(__bf16 (*Sh)[LDK], __bf16 (*Sl)[LDK]) const
    {
#pragma unroll
        for (int i = 0; i < PER_THREAD; ++i) {
            const int q = threadIdx.x + 256 * i;
            const int n = q % BN, g = q / BN;
            bf16x8 h, l;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                __bf16 hu, lu;
                split(u < nv[i] ? v[i][u] : 0.f, hu, lu);
                h[u] = hu;
                l[u] = lu;
            }
            *reinterpret_cast<bf16x8 *>(&Sh[n][swz(n, 8 * g)]) = h;
            *reinterpret_cast<bf16x8 *>(&Sl[n][swz(n, 8 * g)]) = l;
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
            ah[i] = *reinterpret_cast<const bf16x8 *>(&t.Ah[buf][row][swz(row, kq)]);
            al[i] = *reinterpret_cast<const bf16x8 *>(&t.Al[buf][row][swz(row, kq)]);
        }
#pragma unroll
        for (int j = 0; j < SN; ++j) {
            const int col = wn * SN * 32 + j * 32 + (lane & 31);
            bh[j] = *reinterpret_cast<const bf16x8 *>(&t.Bh[buf][col][swz(col, kq)]);
            bl[j] = *reinterpret_cast<const bf16x8 *>(&t.Bl[buf][col][swz(col, kq)]);
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

// The K loop over nchunks >= 1 chunks, with two LDS buffers.  fetch(a, b, c) loads chunk c
// into the register stage (a, b); chunk indices past the end are clamped to the last chunk
// (a redundant fetch, never multiplied), which keeps the loop body free of load branches.
// DEPTH 1: chunk c + 1 is fetched while chunk c is multiplied, then split into the other
// buffer.  DEPTH 2: two register stages; chunk c + 2 is fetched while chunk c is multiplied
// and chunk c + 1 is split, so each fetch has two chunk periods to arrive (twice the
// registers of the stage).  Scheduling barriers keep the order fetch, multiply, split: left
// to itself the compiler moves the split of the first fetched values in among the MFMAs,
// and the wave then stalls there for the whole memory latency.
template <int DEPTH, int SM, int SN, class LA, class LB, class Fetch>
__device__ inline void k_loop(Tiles<SM, SN> &t, int nchunks, Fetch fetch, int wm, int wn, int lane,
                              f32x16 (&acc)[SM][SN])
{
    if constexpr (DEPTH == 1) {
        LA a;
        LB b;
        fetch(a, b, 0);
        a.store(t.Ah[0], t.Al[0]);
        b.store(t.Bh[0], t.Bl[0]);
        __syncthreads();
        for (int c = 0; c < nchunks; ++c) {
            const int buf = c & 1;
            fetch(a, b, min(c + 1, nchunks - 1));
            __builtin_amdgcn_sched_barrier(0);
            mma_chunk<SM, SN>(t, buf, wm, wn, lane, acc);
            __builtin_amdgcn_sched_barrier(0);
            a.store(t.Ah[buf ^ 1], t.Al[buf ^ 1]);
            b.store(t.Bh[buf ^ 1], t.Bl[buf ^ 1]);
            __syncthreads();
        }
        return;
    }
    LA a0, a1;
    LB b0, b1;
    fetch(a0, b0, 0);
    fetch(a1, b1, min(1, nchunks - 1));
    a0.store(t.Ah[0], t.Al[0]);
    b0.store(t.Bh[0], t.Bl[0]);
    __syncthreads();
    for (int c = 0; c < nchunks; c += 2) {
        fetch(a0, b0, min(c + 2, nchunks - 1));
        __builtin_amdgcn_sched_barrier(0);
        mma_chunk<SM, SN>(t, 0, wm, wn, lane, acc);
        __builtin_amdgcn_sched_barrier(0);
        a1.store(t.Ah[1], t.Al[1]);
        b1.store(t.Bh[1], t.Bl[1]);
        __syncthreads();
        if (c + 1 >= nchunks)
            break;
        fetch(a1, b1, min(c + 3, nchunks - 1));
        __builtin_amdgcn_sched_barrier(0);
        mma_chunk<SM, SN>(t, 1, wm, wn, lane, acc);
        __builtin_amdgcn_sched_barrier(0);
        a0.store(t.Ah[0], t.Al[0]);
        b0.store(t.Bh[0], t.Bl[0]);
        __syncthreads();
    }
}

template <int SM, int SN, bool VEC>
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
    using LA = SplitRowLoader<BM, VEC>;
    using LB = SplitRowLoader<BN, VEC>;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int nchunks = (int)((g.D + KC - 1) / KC);
    for (int64_t n0 = (int64_t)bx0 * BN; n0 < N; n0 += (int64_t)gxs * BN) {
        f32x16 acc[SM][SN];
#pragma unroll
        for (int i = 0; i < SM; ++i)
#pragma unroll
            for (int j = 0; j < SN; ++j)
                acc[i][j] = f32x16{};
        // depth 1: the second register stage would push the kernel past 256 registers (spills,
        // or one workgroup per CU), and both measured slower
        k_loop<1, SM, SN, LA, LB>(
            t, nchunks,
            [&](LA &a, LB &b, int c) {
                a.load(H, g.D, m0, Mrows, (int64_t)c * KC, g.D);
                b.load(V, g.D, n0, N, (int64_t)c * KC, g.D);
            },
            wm, wn, lane, acc);
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
    // the per-row partial sums of the epilogue reuse the tile storage (64 KB at 128 x 128, so two
    // workgroups fit a CU's LDS); the K loop ends with a barrier, after which the tiles are dead
    __shared__ __attribute__((aligned(16))) char smem[sizeof(TT)];
    static_assert(sizeof(double) * BM * 4 <= sizeof(TT), "partial sums must fit the tile storage");
    TT &t = *reinterpret_cast<TT *>(smem);
    double(*red)[2][2] = reinterpret_cast<double(*)[2][2]>(smem);
    const float *Cc = static_cast<const float *>(g.C);
    const float *V = static_cast<const float *>(g.V);
    using LA = SplitRowLoader<BM, true>;  // coefficients, K = basis index (ldc: a multiple of 4 >= N)
    using LB = SplitColLoader<BN>;        // basis rows
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w >> 1, wn = w & 1;
    f32x16 acc[SM][SN];
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int j = 0; j < SN; ++j)
            acc[i][j] = f32x16{};
    const int nchunks = (int)((N + KC - 1) / KC);
    if (nchunks > 0)
        k_loop<2, SM, SN, LA, LB>(
            t, nchunks,
            [&](LA &a, LB &b, int c) {
                a.load(Cc, g.ldc, m0, Mrows, (int64_t)c * KC, N);
                b.load(V, g.D, (int64_t)c * KC, N, j0, g.D);
            },
            wm, wn, lane, acc);
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

// (256, 2): at most 256 registers per lane, so two workgroups share a CU
template <int SM, int SN, bool VEC>
__global__ void __launch_bounds__(256, 2) k_bf_dot(GemmArgs g)
{
    bf_dot_body<SM, SN, VEC>(g, blockIdx.x, blockIdx.y, gridDim.x);
}
template <int SM, int SN>
__global__ void __launch_bounds__(256, 2) k_bf_sub(GemmArgs g)
{
    bf_sub_body<SM, SN>(g, blockIdx.x, blockIdx.y, gridDim.x);
}
template <int SM, int SN>
__global__ void __launch_bounds__(256) k_bf_dot_b(Batch b)
{
    const int p = batch_find(b.start, b.nprob, blockIdx.x);
    const GemmArgs g = static_cast<const GemmArgs *>(b.args)[p];
    const int l = blockIdx.x - b.start[p], gx = b.gx[p];
    bf_dot_body<SM, SN, false>(g, l % gx, l / gx, gx);
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
    // 16-byte loads need rows of a multiple of 4 floats (the buffers themselves are 256-byte
    // aligned); other rows take the 64 x 64 tile with 4-byte loads
    const bool vec = D % 4 == 0;
    const dim3 g2((unsigned)((n_hi + 127) / 128), (cnt + 127) / 128), g1((unsigned)((n_hi + 63) / 64), (cnt + 63) / 64);
    if (tile == 2 && vec)
        hipLaunchKernelGGL((k_bf_dot<2, 2, true>), g2, dim3(256), 0, s, g);
    else if (vec)
        hipLaunchKernelGGL((k_bf_dot<1, 1, true>), g1, dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL((k_bf_dot<1, 1, false>), g1, dim3(256), 0, s, g);
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

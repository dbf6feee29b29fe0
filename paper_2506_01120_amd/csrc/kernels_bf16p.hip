// Split-BF16 projection GEMMs on pre-split operand planes (gfx950 BF16 matrix
// cores, v_mfma_f32_32x32x16_bf16, FP32 accumulation).
//
// The screening copy of every operand is kept as two BF16 planes, hi = bf16(x)
// and lo = bf16(x - hi) of its FP32 value x, written when the operand is made
// (basis rows when they are appended, candidate rows after the bracket, the
// coefficients in the coefficient GEMM's epilogue).  Each product is formed as
// hi*hi' + hi*lo' + lo*hi' (the lo*lo' term, of relative size 2^-16, is
// dropped).  Staging a tile is then a plain copy of 16-byte groups.
//
// Plane layout ("interleaved planes"): a row of K values is stored as K/8
// groups of 32 bytes, the 8 hi values of the group followed by its 8 lo values;
// K is padded to a multiple of 32 with zeros and rows are padded to whole
// workgroup tiles, so every load of a tile is in bounds and unconditional.
//
//   coefficients  C[m][n] = sum_k H[m][k] V[n][k]       (H planes x basis planes, K = d^2)
//   residual      ||H[m] - sum_k C[m][k] Vt[j][k]||^2    (C planes x transposed basis planes, K = |V|)
//
// Workgroup: WM x WN waves, each owning SM x SN tiles of 32 x 32; K in chunks
// of 32 (two MFMA k-steps of 16) through double-buffered LDS, with the next
// chunks' loads in flight in registers while a chunk is multiplied.  Output
// tiles are renumbered so that the workgroups of one XCD (blocks are dealt to
// the 8 XCDs in turn) cover a compact group of tiles and share operand chunks
// in that XCD's L2.
//
// 32x32x16 bf16 layout: lane l supplies A[l%32][8(l/32) + j] and
// B[8(l/32) + j][l%32], j = 0..7; result register r of lane l is
// D[8(r/4) + 4(l/32) + r%4][l%32].
#include "lie_internal.h"

#include <algorithm>

namespace lie {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int KC = 32;  // K per chunk: four groups of 8

__device__ inline bool aborted(const DevState *st) { return st && (st->done | st->numeric_error | st->full); }

// Position of 16-byte group g in LDS row `row` (four groups per row): rotating the groups
// every two rows makes an MFMA fragment read (32 lanes on 32 rows, one group) and the
// staging writes (whole rows) touch distinct bank groups.
__device__ inline int gpos(int row, int g) { return (g ^ (row >> 1)) & 3; }

template <int WM, int WN, int SM, int SN>
struct PCfg {
    static constexpr int NT = 64 * WM * WN;
    static constexpr int BM = WM * SM * 32, BN = WN * SN * 32;
};

template <int BM, int BN>
struct alignas(16) PTiles {
    bf16x8 Ah[2][BM][4], Al[2][BM][4];
    bf16x8 Bh[2][BN][4], Bl[2][BN][4];
};

// ROWS rows x one K chunk of interleaved planes -> registers -> LDS tiles.  Thread q of
// the workgroup takes 16-byte items q, q + NT, ...; item i covers row i / 8, group
// (i % 8) / 2, plane i % 2, so eight consecutive threads read one row's 128 contiguous bytes.
template <int ROWS, int NT>
struct PlaneLoader {
    static constexpr int ITEMS = ROWS * 8;
    static_assert(ITEMS % NT == 0, "tile rows must fill the workgroup");
    static constexpr int PER = ITEMS / NT;
    u32x4 v[PER];

    __device__ void load(const __bf16 *__restrict__ P, int64_t ld, int64_t r0, int64_t k0)
    {
        const __bf16 *base = P + r0 * ld + 2 * k0;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int q = threadIdx.x + NT * i;
            const int r = q >> 3, x = q & 7;
            v[i] = *reinterpret_cast<const u32x4 *>(base + (int64_t)r * ld + 8 * x);
        }
    }
    __device__ void store(bf16x8 (*Sh)[4], bf16x8 (*Sl)[4]) const
    {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int q = threadIdx.x + NT * i;
            const int r = q >> 3, x = q & 7, g = x >> 1;
            bf16x8 *dst = (x & 1) ? &Sl[r][gpos(r, g)] : &Sh[r][gpos(r, g)];
            *reinterpret_cast<u32x4 *>(dst) = v[i];
        }
    }
};

template <int SM, int SN, int BM, int BN>
__device__ inline void mma_chunk(const PTiles<BM, BN> &t, int buf, int wm, int wn, int lane, f32x16 (&acc)[SM][SN])
{
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
        const int g = 2 * ks + (lane >> 5);
        bf16x8 ah[SM], al[SM], bh[SN], bl[SN];
#pragma unroll
        for (int i = 0; i < SM; ++i) {
            const int row = wm * SM * 32 + i * 32 + (lane & 31);
            ah[i] = t.Ah[buf][row][gpos(row, g)];
            al[i] = t.Al[buf][row][gpos(row, g)];
        }
#pragma unroll
        for (int j = 0; j < SN; ++j) {
            const int col = wn * SN * 32 + j * 32 + (lane & 31);
            bh[j] = t.Bh[buf][col][gpos(col, g)];
            bl[j] = t.Bl[buf][col][gpos(col, g)];
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

// K loop over nchunks >= 1 chunks: two LDS buffers, two register stages (chunk c + 2 is
// fetched while chunk c is multiplied and chunk c + 1 is copied into LDS).  Chunk indices
// past the end are clamped to the last chunk (a redundant fetch, never multiplied).
template <int WM, int WN, int SM, int SN>
__device__ inline void k_loop(PTiles<WM * SM * 32, WN * SN * 32> &t, int nchunks, const __bf16 *A, int64_t lda,
                              int64_t m0, const __bf16 *B, int64_t ldb, int64_t n0, int wm, int wn, int lane,
                              f32x16 (&acc)[SM][SN])
{
    using C = PCfg<WM, WN, SM, SN>;
    using LA = PlaneLoader<C::BM, C::NT>;
    using LB = PlaneLoader<C::BN, C::NT>;
    LA a0, a1;
    LB b0, b1;
    auto fetch = [&](LA &a, LB &b, int c) {
        const int64_t k0 = (int64_t)min(c, nchunks - 1) * KC;
        a.load(A, lda, m0, k0);
        b.load(B, ldb, n0, k0);
    };
    fetch(a0, b0, 0);
    fetch(a1, b1, 1);
    a0.store(t.Ah[0], t.Al[0]);
    b0.store(t.Bh[0], t.Bl[0]);
    __syncthreads();
    for (int c = 0; c < nchunks; c += 2) {
        fetch(a0, b0, c + 2);
        __builtin_amdgcn_sched_barrier(0);
        mma_chunk<SM, SN>(t, 0, wm, wn, lane, acc);
        __builtin_amdgcn_sched_barrier(0);
        a1.store(t.Ah[1], t.Al[1]);
        b1.store(t.Bh[1], t.Bl[1]);
        __syncthreads();
        if (c + 1 >= nchunks)
            break;
        fetch(a1, b1, c + 3);
        __builtin_amdgcn_sched_barrier(0);
        mma_chunk<SM, SN>(t, 1, wm, wn, lane, acc);
        __builtin_amdgcn_sched_barrier(0);
        a0.store(t.Ah[0], t.Al[0]);
        b0.store(t.Bh[0], t.Bl[0]);
        __syncthreads();
    }
}

// Output tile of workgroup `b` in a TM x TN grid of tiles.  Blocks are dealt to the
// 8 XCDs in turn, so block b runs on XCD b % 8: the renumbering gives each XCD a
// contiguous range of tile ids, walked in groups of 8 tile rows (column-major inside a
// group) so that the workgroups resident on one XCD share A rows and B columns.
__device__ inline void tile_of(int b, int TM, int TN, int &tm, int &tn)
{
    const int T = TM * TN;
    const int t = (T % 8 == 0) ? (b % 8) * (T / 8) + b / 8 : b;
    constexpr int GM = 8;
    const int group = t / (GM * TN), first = group * GM;
    const int gm = min(TM - first, GM);
    const int in = t - group * GM * TN;
    tm = first + in % gm;
    tn = in / gm;
}

__device__ inline void split_bf16(float x, __bf16 &hi, __bf16 &lo)
{
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

// Coefficients: C[m][n] = sum_k H[m][k] V[n][k] for m < cnt, n < N, written as interleaved
// planes (row m of C, K index n).
template <int WM, int WN, int SM, int SN>
__global__ void __launch_bounds__(64 * WM * WN, 2) k_bfp_dot(PlaneGemmArgs g)
{
    using C = PCfg<WM, WN, SM, SN>;
    if (aborted(g.st))
        return;
    const int64_t N = g.st->N;
    int tm, tn;
    tile_of(blockIdx.x, g.tm, g.tn, tm, tn);
    const int64_t m0 = (int64_t)tm * C::BM, n0 = (int64_t)tn * C::BN;
    if (n0 >= N || m0 >= g.cnt)
        return;
    __shared__ PTiles<C::BM, C::BN> t;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w / WN, wn = w % WN;
    f32x16 acc[SM][SN];
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int j = 0; j < SN; ++j)
            acc[i][j] = f32x16{};
    k_loop<WM, WN, SM, SN>(t, (int)(g.K / KC), g.A, g.lda, m0, g.B, g.ldb, n0, wm, wn, lane, acc);
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int j = 0; j < SN; ++j) {
            const int64_t n = n0 + wn * SN * 32 + j * 32 + (lane & 31);
            __bf16 *col = g.Cout + 16 * (n >> 3) + (n & 7);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t m = m0 + wm * SM * 32 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (m < g.cnt && n < N) {
                    __bf16 hi, lo;
                    split_bf16(acc[i][j][r], hi, lo);
                    col[m * g.ldcout] = hi;
                    col[m * g.ldcout + 8] = lo;
                }
            }
        }
}

// Residual norms: R[m][j] = H[m][j] - sum_k C[m][k] Vt[j][k] over k < N, for m < cnt and
// j < D; per (row, column tile) the squared norms of R and of H go to normpart.
template <int WM, int WN, int SM, int SN>
__global__ void __launch_bounds__(64 * WM * WN, 2) k_bfp_sub(PlaneGemmArgs g)
{
    using C = PCfg<WM, WN, SM, SN>;
    if (aborted(g.st))
        return;
    const int64_t N = g.st->N;
    int tm, tn;
    tile_of(blockIdx.x, g.tm, g.tn, tm, tn);
    const int64_t m0 = (int64_t)tm * C::BM, j0 = (int64_t)tn * C::BN;
    if (m0 >= g.cnt)
        return;
    __shared__ PTiles<C::BM, C::BN> t;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w / WN, wn = w % WN;
    f32x16 acc[SM][SN];
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int j = 0; j < SN; ++j)
            acc[i][j] = f32x16{};
    const int nchunks = (int)((N + KC - 1) / KC);
    if (nchunks > 0)
        k_loop<WM, WN, SM, SN>(t, nchunks, g.A, g.lda, m0, g.B, g.ldb, j0, wm, wn, lane, acc);
    // the K loop ends with a barrier: the tiles are dead and hold the per-row partial sums
    double(*red)[WN][2] = reinterpret_cast<double(*)[WN][2]>(&t);
    static_assert(sizeof(double) * C::BM * WN * 2 <= sizeof(PTiles<C::BM, C::BN>), "partials must fit the tiles");
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int ml = wm * SM * 32 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const int64_t m = m0 + ml;
            double rs = 0.0, hsq = 0.0;
            if (m < g.cnt) {
                const __bf16 *hrow = g.Hp + m * g.ldh;
#pragma unroll
                for (int j = 0; j < SN; ++j) {
                    const int64_t col = j0 + wn * SN * 32 + j * 32 + (lane & 31);
                    if (col < g.D) {
                        const int64_t o = 16 * (col >> 3) + (col & 7);
                        const float h = (float)hrow[o] + (float)hrow[o + 8];
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
    for (int ml = threadIdx.x; ml < C::BM; ml += C::NT) {
        const int64_t m = m0 + ml;
        if (m < g.cnt) {
            double a = 0.0, b = 0.0;
#pragma unroll
            for (int q = 0; q < WN; ++q) {
                a += red[ml][q][0];
                b += red[ml][q][1];
            }
            double *o = g.normpart + (m * g.tn + tn) * 2;
            o[0] = a;
            o[1] = b;
        }
    }
}

// ------------------------------------------------------------------ plane writers

// FP32 rows [cnt][D] -> interleaved planes [rows][ld], zero past D up to the padded K.
// One thread per group of 8 values.
__global__ void k_split_rows(const float *__restrict__ src, int64_t D, int cnt, int64_t Kp, __bf16 *__restrict__ dst,
                             int64_t ld)
{
    const int64_t groups = Kp / 8;
    const int64_t total = (int64_t)cnt * groups;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / groups, gi = e % groups;
        const float *s = src + r * D + 8 * gi;
        bf16x8 h, l;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float x = 8 * gi + u < D ? s[u] : 0.f;
            __bf16 hi, lo;
            split_bf16(x, hi, lo);
            h[u] = hi;
            l[u] = lo;
        }
        bf16x8 *o = reinterpret_cast<bf16x8 *>(dst + r * ld + 16 * gi);
        o[0] = h;
        o[1] = l;
    }
}

// Basis rows [*done, st->N) -> row planes Vp (row k, K index j) and transposed planes Vt
// (row j, K index k).  A workgroup converts 32 basis rows x 64 columns through LDS; the
// transposed write covers whole 8-row groups (rows past N are written as zeros).
constexpr int kTrK = 32, kTrJ = 64;

__global__ void __launch_bounds__(256) k_planes_refresh(const double *__restrict__ V, int64_t D, const DevState *st,
                                                        const int64_t *done, __bf16 *__restrict__ Vp, int64_t ldp,
                                                        __bf16 *__restrict__ Vt, int64_t ldt)
{
    const int64_t N = st->N, lo = *done;
    if (lo >= N)
        return;
    const int64_t k_first = lo & ~(int64_t)(kTrK - 1);
    const int64_t tk = (N - k_first + kTrK - 1) / kTrK, tj = (D + kTrJ - 1) / kTrJ;
    __shared__ float tile[kTrK][kTrJ + 1];
    for (int64_t t = blockIdx.x; t < tk * tj; t += gridDim.x) {
        const int64_t k0 = k_first + (t / tj) * kTrK, jb = (t % tj) * kTrJ;
        __syncthreads();  // the previous tile's reads are done
        for (int e = threadIdx.x; e < kTrK * kTrJ; e += blockDim.x) {
            const int kk = e / kTrJ, jj = e % kTrJ;
            const int64_t k = k0 + kk, j = jb + jj;
            tile[kk][jj] = (k < N && j < D) ? (float)V[k * D + j] : 0.f;
        }
        __syncthreads();
        // row planes: rows k in [max(lo, k0), min(N, k0 + 32)), groups of 8 columns
        for (int e = threadIdx.x; e < kTrK * (kTrJ / 8); e += blockDim.x) {
            const int kk = e / (kTrJ / 8), gj = e % (kTrJ / 8);
            const int64_t k = k0 + kk, j = jb + 8 * gj;
            if (k < lo || k >= N || j >= D)
                continue;
            bf16x8 h, l;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                __bf16 hi, lw;
                split_bf16(tile[kk][8 * gj + u], hi, lw);
                h[u] = hi;
                l[u] = lw;
            }
            bf16x8 *o = reinterpret_cast<bf16x8 *>(Vp + k * ldp + 16 * (j >> 3));
            o[0] = h;
            o[1] = l;
        }
        // transposed planes: row j, groups of 8 basis rows (whole groups, zeros past N)
        for (int e = threadIdx.x; e < kTrJ * (kTrK / 8); e += blockDim.x) {
            const int jj = e / (kTrK / 8), gk = e % (kTrK / 8);
            const int64_t j = jb + jj;
            if (j >= D)
                continue;
            bf16x8 h, l;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                __bf16 hi, lw;
                split_bf16(tile[8 * gk + u][jj], hi, lw);
                h[u] = hi;
                l[u] = lw;
            }
            bf16x8 *o = reinterpret_cast<bf16x8 *>(Vt + j * ldt + 16 * ((k0 >> 3) + gk));
            o[0] = h;
            o[1] = l;
        }
    }
}

__global__ void k_planes_mark(const DevState *st, int64_t *done)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *done = st->N;
}

}  // namespace

PlaneGeom plane_geom(int64_t D, int64_t cap, int bmax)
{
    PlaneGeom p;
    p.Kp = (D + KC - 1) / KC * KC;
    p.ld = 2 * p.Kp;
    p.cap_rows = (cap + 255) / 256 * 256;
    p.ldt_k = (cap + KC - 1) / KC * KC;
    p.ldt = 2 * p.ldt_k;
    p.d_rows = (D + 255) / 256 * 256;
    p.b_rows = ((int64_t)std::max(bmax, 1) + 255) / 256 * 256;
    return p;
}

int plane_sub_tiles(int64_t D, int tile) { return (int)((D + 127) / 128); }

hipError_t launch_planes_refresh(const double *V64, int64_t D, const DevState *st, int64_t *done, __bf16 *Vp,
                                 __bf16 *Vt, const PlaneGeom &p, hipStream_t s)
{
    hipLaunchKernelGGL(k_planes_refresh, dim3(512), dim3(256), 0, s, V64, D, st, (const int64_t *)done, Vp, p.ld, Vt,
                       p.ldt);
    hipLaunchKernelGGL(k_planes_mark, dim3(1), dim3(64), 0, s, st, done);
    return hipGetLastError();
}

hipError_t launch_split_rows(const float *src, int64_t D, int cnt, __bf16 *dst, const PlaneGeom &p, hipStream_t s)
{
    if (cnt <= 0)
        return hipSuccess;
    const int64_t total = (int64_t)cnt * (p.Kp / 8);
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_split_rows, dim3(blocks), dim3(256), 0, s, src, D, cnt, p.Kp, dst, p.ld);
    return hipGetLastError();
}

hipError_t launch_bfp_dot(const __bf16 *Hp, const __bf16 *Vp, const DevState *st, int cnt, int64_t n_hi,
                          __bf16 *Cp, const PlaneGeom &p, hipStream_t s)
{
    if (cnt <= 0)
        return hipSuccess;
    PlaneGemmArgs g{};
    g.A = Hp;
    g.lda = p.ld;
    g.B = Vp;
    g.ldb = p.ld;
    g.K = p.Kp;
    g.cnt = cnt;
    g.st = st;
    g.Cout = Cp;
    g.ldcout = p.ldt;
    g.tm = (cnt + 127) / 128;
    g.tn = (int)((std::max<int64_t>(n_hi, 1) + 127) / 128);
    hipLaunchKernelGGL((k_bfp_dot<2, 2, 2, 2>), dim3(g.tm * g.tn), dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_bfp_sub(const __bf16 *Cp, const __bf16 *Vt, const __bf16 *Hp, const DevState *st, int cnt,
                          int64_t D, double *normpart, const PlaneGeom &p, hipStream_t s)
{
    if (cnt <= 0)
        return hipSuccess;
    PlaneGemmArgs g{};
    g.A = Cp;
    g.lda = p.ldt;
    g.B = Vt;
    g.ldb = p.ldt;
    g.cnt = cnt;
    g.st = st;
    g.Hp = Hp;
    g.ldh = p.ld;
    g.D = D;
    g.normpart = normpart;
    g.tm = (cnt + 127) / 128;
    g.tn = plane_sub_tiles(D, 0);
    hipLaunchKernelGGL((k_bfp_sub<2, 2, 2, 2>), dim3(g.tm * g.tn), dim3(256), 0, s, g);
    return hipGetLastError();
}

}  // namespace lie

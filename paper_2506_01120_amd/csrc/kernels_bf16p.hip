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
// K is padded to a multiple of 64 with zeros and rows are padded to whole
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

// LDS tile rows hold one row's K chunk as eight 16-byte slots, slot = plane * 4 + group
// (hi groups 0..3, then lo groups 0..3: 128 bytes).  Slot s of row r is stored at position
// s ^ (r & 7) ^ ((r >> 3) & 1).  An MFMA fragment read (lanes on 32 consecutive rows, one slot)
// then puts any 8 consecutive lanes on 8 distinct positions, and any 16 consecutive lanes on
// 16 distinct bank groups across the two row parities; a staging write (eight lanes per row,
// one row's eight slots, consecutive rows) is a permutation of whole rows.  Either way no two
// lanes of a cycle share a bank, whether LDS serves 8 or 16 lanes of a 16-byte access per cycle.
__device__ inline int spos(int row, int slot) { return (slot ^ (row & 7) ^ ((row >> 3) & 1)) & 7; }

template <int WM, int WN, int SM, int SN>
struct PCfg {
    static constexpr int NT = 64 * WM * WN;
    static constexpr int BM = WM * SM * 32, BN = WN * SN * 32;
};

template <int BM, int BN>
struct alignas(16) PTiles {
    bf16x8 A[2][BM][8];
    bf16x8 B[2][BN][8];
};

// ROWS rows x one K chunk of interleaved planes -> registers -> LDS tiles.  Thread q of
// the workgroup takes 16-byte items q, q + NT, ...; item i covers row i / 8 and slot i % 8
// (plane (i % 8) / 4, group i % 4), so eight consecutive threads read one row's 128
// contiguous bytes.
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
            const int r = q >> 3, x = q & 7;  // slot x: plane x / 4, group x % 4
            v[i] = *reinterpret_cast<const u32x4 *>(base + (int64_t)r * ld + 16 * (x & 3) + 8 * (x >> 2));
        }
    }
    __device__ void store(bf16x8 (*S)[8]) const
    {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int q = threadIdx.x + NT * i;
            const int r = q >> 3, x = q & 7;
            *reinterpret_cast<u32x4 *>(&S[r][spos(r, x)]) = v[i];
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
            ah[i] = t.A[buf][row][spos(row, g)];
            al[i] = t.A[buf][row][spos(row, 4 + g)];
        }
#pragma unroll
        for (int j = 0; j < SN; ++j) {
            const int col = wn * SN * 32 + j * 32 + (lane & 31);
            bh[j] = t.B[buf][col][spos(col, g)];
            bl[j] = t.B[buf][col][spos(col, 4 + g)];
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

// K loop over an even number nchunks >= 2 of chunks: two LDS buffers and two register
// stages.  Chunk c + 2 is fetched into registers while chunk c is multiplied, so each fetch
// has two chunks of matrix-core work to arrive; chunk c + 1 is copied into the other buffer
// after chunk c is multiplied.  The loop body covers two chunks and has no exit in between
// (callers pad K to whole chunk pairs with zeros), which keeps the accumulators in place.
// Fetch indices past the end are clamped to the last chunk (redundant, never multiplied).
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
    a0.store(t.A[0]);
    b0.store(t.B[0]);
    __syncthreads();
    for (int c = 0; c < nchunks; c += 2) {
        fetch(a0, b0, c + 2);
        __builtin_amdgcn_sched_barrier(0);
        mma_chunk<SM, SN>(t, 0, wm, wn, lane, acc);
        __builtin_amdgcn_sched_barrier(0);
        a1.store(t.A[1]);
        b1.store(t.B[1]);
        __syncthreads();
        fetch(a1, b1, c + 3);
        __builtin_amdgcn_sched_barrier(0);
        mma_chunk<SM, SN>(t, 1, wm, wn, lane, acc);
        __builtin_amdgcn_sched_barrier(0);
        a0.store(t.A[0]);
        b0.store(t.B[0]);
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
    k_loop<WM, WN, SM, SN>(t, (int)(g.K / KC), g.A, g.lda, m0, g.B, g.ldb, n0, wm, wn, lane, acc);  // K: whole chunk pairs
    // The K loop ends with a barrier: the tiles are dead.  The output tile goes to LDS as
    // interleaved planes (row ml: BN / 8 groups of 32 bytes), then to global memory as
    // 16-byte items, eight consecutive threads per 128 contiguous bytes of a row.  Columns
    // n >= N hold exact zeros (the basis planes are zero there), which is what the residual
    // GEMM's K padding must read; columns past the row's padded K are not written.
    constexpr int RB = C::BN * 4;  // bytes of one output row in LDS
    static_assert(C::BM * RB <= (int)sizeof(PTiles<C::BM, C::BN>), "output tile must fit the LDS tiles");
    unsigned char *ot = reinterpret_cast<unsigned char *>(&t);
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int j = 0; j < SN; ++j) {
            const int nl = wn * SN * 32 + j * 32 + (lane & 31);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int ml = wm * SM * 32 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                __bf16 hi, lo;
                split_bf16(acc[i][j][r], hi, lo);
                __bf16 *o = reinterpret_cast<__bf16 *>(ot + ml * RB) + 16 * (nl >> 3) + (nl & 7);
                o[0] = hi;
                o[8] = lo;
            }
        }
    __syncthreads();
    constexpr int ITEMS = C::BM * (RB / 16), PER = ITEMS / C::NT;
    const int64_t kcols = g.ldcout / 2;  // padded K of a C row
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = threadIdx.x + C::NT * q;
        const int ml = e / (RB / 16), x = e % (RB / 16);  // x: 16-byte item of the row (group x / 2)
        const int64_t m = m0 + ml, n = n0 + 8 * (x >> 1);
        if (m < g.cnt && n < kcols)
            *reinterpret_cast<u32x4 *>(g.Cout + m * g.ldcout + 2 * n0 + 8 * x) =
                *reinterpret_cast<const u32x4 *>(ot + ml * RB + 16 * x);
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
    // K = N rounded up to whole chunk pairs: the C and transposed basis planes are zero there
    const int nchunks = 2 * (int)((N + 2 * KC - 1) / (2 * KC));
    if (nchunks > 0)
        k_loop<WM, WN, SM, SN>(t, nchunks, g.A, g.lda, m0, g.B, g.ldb, j0, wm, wn, lane, acc);
    // The K loop ends with a barrier: the tiles are dead.  The candidate tile H[m0.., j0..]
    // (interleaved planes, 128-byte runs per row) is staged into them with 16-byte loads, all
    // in flight together, instead of two scattered 2-byte loads per element.
    constexpr int RB = C::BN * 4;
    static_assert(C::BM * RB <= (int)sizeof(PTiles<C::BM, C::BN>), "candidate tile must fit the LDS tiles");
    unsigned char *ht = reinterpret_cast<unsigned char *>(&t);
    {
        constexpr int ITEMS = C::BM * (RB / 16), PER = ITEMS / C::NT;
        const int64_t kcols = g.ldh / 2;  // padded K of an H row
        u32x4 v[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + C::NT * q;
            const int ml = e / (RB / 16), x = e % (RB / 16);
            const int64_t jc = j0 + 8 * (x >> 1);
            v[q] = jc < kcols ? *reinterpret_cast<const u32x4 *>(g.Hp + (m0 + ml) * g.ldh + 2 * j0 + 8 * x)
                              : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + C::NT * q;
            const int ml = e / (RB / 16), x = e % (RB / 16);
            *reinterpret_cast<u32x4 *>(ht + ml * RB + 16 * x) = v[q];
        }
    }
    __syncthreads();
    // per-row partial sums, behind the candidate tile in LDS when it fits, else in a small array
    __shared__ double red[C::BM][WN][2];
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int ml = wm * SM * 32 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const int64_t m = m0 + ml;
            double rs = 0.0, hsq = 0.0;
            if (m < g.cnt) {
                const __bf16 *hrow = reinterpret_cast<const __bf16 *>(ht + ml * RB);
#pragma unroll
                for (int j = 0; j < SN; ++j) {
                    const int cl = wn * SN * 32 + j * 32 + (lane & 31);
                    const int64_t col = j0 + cl;
                    if (col < g.D) {
                        const int o = 16 * (cl >> 3) + (cl & 7);
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
    p.Kp = (D + 2 * KC - 1) / (2 * KC) * (2 * KC);  // whole chunk pairs
    p.ld = 2 * p.Kp;
    p.cap_rows = (cap + 255) / 256 * 256;
    p.ldt_k = (cap + 2 * KC - 1) / (2 * KC) * (2 * KC);
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

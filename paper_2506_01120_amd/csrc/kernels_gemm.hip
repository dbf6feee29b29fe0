// Projection GEMMs on the matrix cores, FP32 (v_mfma_f32_32x32x2_f32) and
// FP64 (v_mfma_f64_16x16x4_f64), for the two halves of a projection pass:
//
//   coefficients  C[m][n] = sum_k H[row(m)][k] V[n][k]      (m < M rows, n < N basis rows, k < D)
//   residual      R[m][j] = H[row(m)][j] - sum_k C[m][k] V[k][j]   (j < D, k < N)
//                 with the squared norms of R (and of H) summed per output tile,
//                 R optionally written back over H.
//
// Small passes (a growth-phase block of a few dozen candidates gives only a
// handful of output tiles) split K across workgroups: grid.z = number of K
// slices.  The coefficient slices are summed by the residual kernel as it loads
// them; the residual's own slices (partial products C V) are summed, in slice
// order, by a finishing kernel that forms R and its norms.  Without the split
// such a pass runs on a few compute units and waits on one global-load round
// trip per K chunk.
//
// Workgroup: 4 waves as 2 x 2; each wave owns SM x SN matrix-core tiles.
// K is staged through LDS in chunks of 16 with a register prefetch of the next
// chunk (one barrier per chunk).  Both operands are stored k-major in LDS so
// every fragment read is a run of consecutive addresses.
#include "lie_internal.h"

#include <algorithm>

namespace lie {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mma;

// 32x32x2 f32: lane l supplies A[l%32][l/32] and B[l/32][l%32];
// result register r of lane l is D[8(r/4) + 4(l/32) + r%4][l%32].
template <>
struct Mma<float> {
    static constexpr int E = 32, KS = 2, NR = 16;
    typedef f32x16 Acc;
    __device__ static Acc zero() { return Acc{}; }
    __device__ static Acc mma(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0); }
    __device__ static int frag_row(int lane) { return lane & 31; }
    __device__ static int frag_k(int lane) { return lane >> 5; }
    __device__ static int out_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }
    __device__ static int out_col(int lane) { return lane & 31; }
};

// 16x16x4 f64: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// result register r of lane l is D[4r + l/16][l%16] (measured on gfx950; it
// differs from the FP32 16x16x4 result layout).
template <>
struct Mma<double> {
    static constexpr int E = 16, KS = 4, NR = 4;
    typedef f64x4 Acc;
    __device__ static Acc zero() { return Acc{0.0, 0.0, 0.0, 0.0}; }
    __device__ static Acc mma(double a, double b, Acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int frag_row(int lane) { return lane & 15; }
    __device__ static int frag_k(int lane) { return lane >> 4; }
    __device__ static int out_row(int lane, int r) { return 4 * r + (lane >> 4); }
    __device__ static int out_col(int lane) { return lane & 15; }
};

// K chunk of a tile BT wide: 32 for FP32 64 x 64 tiles (more loads in flight per barrier;
// measured faster), 16 otherwise (FP32 128 x 128 tiles measured slower with 32, and FP64's
// LDS sets its occupancy)
template <typename T, int BT>
constexpr int kKC = sizeof(T) == 4 && BT == 64 ? 32 : 16;
constexpr int KC = 16;  // FP64 (host-side split plans)
constexpr int kMaxSlices = 16;  // K slices of a split pass

__device__ inline bool aborted(const DevState *st) { return st && (st->done | st->numeric_error | st->full); }

// Operand loads are unconditional: an element outside the operand reads a valid
// address (row rows-1 or column 0), and the LDS store replaces it by zero (each item
// keeps the count of its leading in-range values).  With no branch and no use of the
// value at load time, every load of a chunk is in flight at once.  VL (a template
// parameter, so the compiler cannot fold the two load forms into one of 4-byte loads):
// the rows are a multiple of 16 bytes long, so a 16-byte load at an in-range k (a
// multiple of VEC) stays inside the row.

// Tile loader of a K-contiguous operand: rows [r0, r0+BR) x k [k0, k0+KC) into LDS as S[k][row].
// begin() fixes the rows (row pointers through rowmap, computed once per tile).
template <typename T, int BR>
struct KContigLoader {
    static constexpr int VEC = 16 / sizeof(T);           // elements per 16-byte load
    static constexpr int PER_ROW = kKC<T, BR> / VEC;
    static constexpr int TOTAL = BR * PER_ROW;           // vectors per tile
    static constexpr int PER_THREAD = (TOTAL + 255) / 256;
    T v[PER_THREAD][VEC];
    int nv[PER_THREAD];        // leading in-range values of the item
    const T *rp[PER_THREAD];   // row start (a valid row for out-of-range items)
    bool rv[PER_THREAD];       // the item's row is in range

    template <typename RowFn>
    __device__ void begin(const T *__restrict__ base, int64_t ld, int64_t r0, int64_t rows, RowFn rowmap)
    {
#pragma unroll
        for (int i = 0; i < PER_THREAD; ++i) {
            const int q = threadIdx.x + 256 * i;
            const int64_t row = r0 + q / PER_ROW;
            rv[i] = q < TOTAL && row < rows;
            rp[i] = base + (int64_t)rowmap(rv[i] ? row : rows - 1) * ld;
        }
    }
    // chunk k0 of the rows of `geo`, offset by `off` elements (a slice of the operand)
    template <bool VL>
    __device__ void load_from(const KContigLoader &geo, int64_t off, int64_t k0, int64_t K)
    {
#pragma unroll
        for (int i = 0; i < PER_THREAD; ++i) {
            const int q = threadIdx.x + 256 * i;
            const int64_t k = k0 + (q % PER_ROW) * VEC;
            nv[i] = geo.rv[i] ? (int)min<int64_t>(max<int64_t>(K - k, 0), VEC) : 0;
            const T *p = geo.rp[i] + off;
            if constexpr (VL) {
                if constexpr (sizeof(T) == 4) {
                    const float4 t = *reinterpret_cast<const float4 *>(p + (k < K ? k : 0));
                    v[i][0] = t.x;
                    v[i][1] = t.y;
                    v[i][2] = t.z;
                    v[i][3] = t.w;
                } else {
                    const double2 t = *reinterpret_cast<const double2 *>(p + (k < K ? k : 0));
                    v[i][0] = t.x;
                    v[i][1] = t.y;
                }
            } else {
#pragma unroll
                for (int u = 0; u < VEC; ++u)
                    v[i][u] = p[k + u < K ? k + u : 0];
            }
        }
    }
    template <bool VL>
    __device__ void load(int64_t k0, int64_t K)
    {
        load_from<VL>(*this, 0, k0, K);
    }
    template <int LDW>
    __device__ void store(T (*S)[LDW]) const
    {
#pragma unroll
        for (int i = 0; i < PER_THREAD; ++i) {
            const int q = threadIdx.x + 256 * i;
            if (q < TOTAL) {
                const int r = q / PER_ROW, kv = (q % PER_ROW) * VEC;
#pragma unroll
                for (int u = 0; u < VEC; ++u)
                    S[kv + u][r] = u < nv[i] ? v[i][u] : T(0);
            }
        }
    }
};

// Loader of a K-contiguous operand held as `cs` <= CS slices whose sum is the operand
// (coefficients of a split pass): all slices are loaded at once, so their loads are in
// flight together, and added in slice order when the tile is stored.  The slices share
// the row geometry of part[0].
template <typename T, int BR, int CS>
struct SlicedLoader {
    KContigLoader<T, BR> part[CS];
    int cs = 1;
    int64_t stride = 0;

    template <typename RowFn>
    __device__ void begin(const T *__restrict__ base, int64_t ld, int64_t r0, int64_t rows, RowFn rowmap)
    {
        part[0].begin(base, ld, r0, rows, rowmap);
    }
    template <bool VL>
    __device__ void load(int64_t k0, int64_t K)
    {
#pragma unroll
        for (int q = 0; q < CS; ++q)
            if (q < cs)
                part[q].template load_from<VL>(part[0], (int64_t)q * stride, k0, K);
    }
    template <int LDW>
    __device__ void store(T (*S)[LDW])
    {
        // out-of-range values of every slice sit at the same positions; part[0] masks the sum
#pragma unroll
        for (int q = 1; q < CS; ++q)
            if (q < cs)
#pragma unroll
                for (int i = 0; i < KContigLoader<T, BR>::PER_THREAD; ++i)
#pragma unroll
                    for (int u = 0; u < KContigLoader<T, BR>::VEC; ++u)
                        part[0].v[i][u] += part[q].v[i][u];
        part[0].store(S);
    }
};

// Tile loader of a row-major K x N operand (rows k, contiguous n): k [k0, k0+KC) x n [n0, n0+BN) as S[k][n].
// begin() fixes the columns.
template <typename T, int BN>
struct KRowLoader {
    static constexpr int VEC = 16 / sizeof(T);
    static constexpr int PER_ROW = BN / VEC;
    static constexpr int TOTAL = kKC<T, BN> * PER_ROW;
    static constexpr int PER_THREAD = (TOTAL + 255) / 256;
    T v[PER_THREAD][VEC];
    int nv[PER_THREAD];        // leading in-range values of the item
    const T *cp[PER_THREAD];   // column start in row 0 (a valid column for out-of-range items)
    int cv[PER_THREAD];        // in-range columns of the item

    __device__ void begin(const T *__restrict__ base, int64_t n0, int64_t Ncols)
    {
#pragma unroll
        for (int i = 0; i < PER_THREAD; ++i) {
            const int q = threadIdx.x + 256 * i;
            const int64_t n = n0 + (q % PER_ROW) * VEC;
            const bool ok = q < TOTAL && n < Ncols;
            cv[i] = ok ? (int)min<int64_t>(Ncols - n, VEC) : 0;
            cp[i] = base + (ok ? n : 0);
        }
    }
    template <bool VL>
    __device__ void load(int64_t ld, int64_t k0, int64_t K)
    {
#pragma unroll
        for (int i = 0; i < PER_THREAD; ++i) {
            const int q = threadIdx.x + 256 * i;
            const int64_t k = k0 + q / PER_ROW;
            nv[i] = k < K ? cv[i] : 0;
            const T *p = cp[i] + (k < K ? k : 0) * ld;
            if constexpr (VL) {
                if constexpr (sizeof(T) == 4) {
                    const float4 t = *reinterpret_cast<const float4 *>(p);
                    v[i][0] = t.x;
                    v[i][1] = t.y;
                    v[i][2] = t.z;
                    v[i][3] = t.w;
                } else {
                    const double2 t = *reinterpret_cast<const double2 *>(p);
                    v[i][0] = t.x;
                    v[i][1] = t.y;
                }
            } else {
#pragma unroll
                for (int u = 0; u < VEC; ++u)
                    v[i][u] = p[u < cv[i] ? u : 0];
            }
        }
    }
    template <int LDW>
    __device__ void store(T (*S)[LDW]) const
    {
#pragma unroll
        for (int i = 0; i < PER_THREAD; ++i) {
            const int q = threadIdx.x + 256 * i;
            if (q < TOTAL) {
                const int kk = q / PER_ROW, nv0 = (q % PER_ROW) * VEC;
#pragma unroll
                for (int u = 0; u < VEC; ++u)
                    S[kk][nv0 + u] = u < nv[i] ? v[i][u] : T(0);
            }
        }
    }
};

// K chunks [lo, hi) of slice kz out of ks (every chunk in exactly one slice).
__device__ inline void slice_range(int nchunks, int kz, int ks, int &lo, int &hi)
{
    const int per = (nchunks + ks - 1) / ks;
    lo = min(nchunks, kz * per);
    hi = min(nchunks, lo + per);
}

// ---------------------------------------------------------------- coefficients
// VD: rows of D elements take 16-byte loads (D a multiple of 16 bytes)
template <typename T, int SM, int SN, bool VD>
__device__ void gemm_dot_body(const GemmArgs &g, int bx0, int by, int gxs, int kz = 0)
{
    using M = Mma<T>;
    constexpr int BM = 2 * SM * M::E, BN = 2 * SN * M::E;
    constexpr int KCT = kKC<T, BM>;
    static_assert(BM == BN, "the operand loaders take the chunk of their own tile width");
    constexpr int PAD = 16 / sizeof(T);
    if (aborted(g.st))
        return;
    const int64_t N = g.st ? g.st->N : g.N_fixed;
    const int Mrows = g.nrows ? *g.nrows : g.cnt;
    const int m0 = by * BM;
    if ((int64_t)bx0 * BN >= N || m0 >= Mrows)
        return;
    __shared__ T As[2][KCT][BM + PAD];
    __shared__ T Bs[2][KCT][BN + PAD];
    const T *H = static_cast<const T *>(g.H);
    const T *V = static_cast<const T *>(g.V);
    const int *rows = g.rows;
    auto hmap = [rows](int64_t r) -> int64_t { return rows ? rows[r] : r; };
    auto ident = [](int64_t r) -> int64_t { return r; };
    KContigLoader<T, BM> la;
    KContigLoader<T, BN> lb;
    la.begin(H, g.D, m0, Mrows, hmap);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w >> 1, wn = w & 1;
    for (int64_t n0 = (int64_t)bx0 * BN; n0 < N; n0 += (int64_t)gxs * BN) {
        typename M::Acc acc[SM][SN];
#pragma unroll
        for (int i = 0; i < SM; ++i)
#pragma unroll
            for (int j = 0; j < SN; ++j)
                acc[i][j] = M::zero();
        int clo = 0, chi = 0;
        slice_range((int)((g.D + KCT - 1) / KCT), kz, g.ksplit > 1 ? g.ksplit : 1, clo, chi);
        lb.begin(V, g.D, n0, N, ident);
        if (clo < chi) {
            la.template load<VD>((int64_t)clo * KCT, g.D);
            lb.template load<VD>((int64_t)clo * KCT, g.D);
            la.store(As[0]);
            lb.store(Bs[0]);
        }
        __syncthreads();
        for (int c = clo; c < chi; ++c) {
            const int buf = (c - clo) & 1;
            // the next chunk (the last one again at the end: a redundant fetch keeps the loop
            // free of load branches); scheduling barriers keep fetch, multiply, store in order
            const int64_t kn = (int64_t)min(c + 1, chi - 1) * KCT;
            la.template load<VD>(kn, g.D);
            lb.template load<VD>(kn, g.D);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int kk = 0; kk < KCT; kk += M::KS) {
                T a[SM], b[SN];
#pragma unroll
                for (int i = 0; i < SM; ++i)
                    a[i] = As[buf][kk + M::frag_k(lane)][wm * SM * M::E + i * M::E + M::frag_row(lane)];
#pragma unroll
                for (int j = 0; j < SN; ++j)
                    b[j] = Bs[buf][kk + M::frag_k(lane)][wn * SN * M::E + j * M::E + M::frag_row(lane)];
#pragma unroll
                for (int i = 0; i < SM; ++i)
#pragma unroll
                    for (int j = 0; j < SN; ++j)
                        acc[i][j] = M::mma(a[i], b[j], acc[i][j]);
            }
            __builtin_amdgcn_sched_barrier(0);
            la.store(As[buf ^ 1]);
            lb.store(Bs[buf ^ 1]);
            __syncthreads();
        }
        T *C = static_cast<T *>(g.C) + (int64_t)kz * g.cslice;
#pragma unroll
        for (int i = 0; i < SM; ++i)
#pragma unroll
            for (int j = 0; j < SN; ++j)
#pragma unroll
                for (int r = 0; r < M::NR; ++r) {
                    const int m = m0 + wm * SM * M::E + i * M::E + M::out_row(lane, r);
                    const int64_t n = n0 + wn * SN * M::E + j * M::E + M::out_col(lane);
                    if (m < Mrows && n < N)
                        C[(int64_t)m * g.ldc + n] = acc[i][j][r];
                }
    }
}

// ---------------------------------------------------------------- residual + norms
// VD as in the coefficient GEMM (basis rows); the coefficient rows (ldc a multiple of 4)
// always take 16-byte loads.
template <typename T, int SM, int SN, bool VD, int CS = 1>
__device__ void gemm_sub_body(const GemmArgs &g, int bx, int by, int ntiles, int kz = 0)
{
    using M = Mma<T>;
    constexpr int BM = 2 * SM * M::E, BN = 2 * SN * M::E;
    constexpr int KCT = kKC<T, BM>;
    static_assert(BM == BN, "the operand loaders take the chunk of their own tile width");
    constexpr int PAD = 16 / sizeof(T);
    if (aborted(g.st))
        return;
    const int64_t N = g.st ? g.st->N : g.N_fixed;
    const int Mrows = g.nrows ? *g.nrows : g.cnt;
    const int64_t j0 = (int64_t)bx * BN;  // operator columns
    const int m0 = by * BM;
    if (m0 >= Mrows)
        return;
    __shared__ T As[2][KCT][BM + PAD];
    __shared__ T Bs[2][KCT][BN + PAD];
    __shared__ double red[BM][2][2];
    const T *Cc = static_cast<const T *>(g.C);
    const T *V = static_cast<const T *>(g.V);
    auto ident = [](int64_t r) -> int64_t { return r; };
    SlicedLoader<T, BM, CS> la;  // C rows (K = basis index, contiguous), as coefficient slices
    KRowLoader<T, BN> lb;        // V rows
    la.cs = CS > 1 ? min(max(g.cslices, 1), CS) : 1;
    la.stride = g.cslice;
    la.begin(Cc, g.ldc, m0, Mrows, ident);
    lb.begin(V, j0, g.D);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w >> 1, wn = w & 1;
    typename M::Acc acc[SM][SN];
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int j = 0; j < SN; ++j)
            acc[i][j] = M::zero();
    int clo = 0, chi = 0;
    slice_range((int)((N + KCT - 1) / KCT), kz, g.ksplit > 1 ? g.ksplit : 1, clo, chi);
    if (clo < chi) {
        la.template load<true>((int64_t)clo * KCT, N);
        lb.template load<VD>(g.D, (int64_t)clo * KCT, N);
        la.store(As[0]);
        lb.store(Bs[0]);
    }
    __syncthreads();
    for (int c = clo; c < chi; ++c) {
        const int buf = (c - clo) & 1;
        const int64_t kn = (int64_t)min(c + 1, chi - 1) * KCT;  // as in the coefficient GEMM
        la.template load<true>(kn, N);
        lb.template load<VD>(g.D, kn, N);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int kk = 0; kk < KCT; kk += M::KS) {
            T a[SM], b[SN];
#pragma unroll
            for (int i = 0; i < SM; ++i)
                a[i] = As[buf][kk + M::frag_k(lane)][wm * SM * M::E + i * M::E + M::frag_row(lane)];
#pragma unroll
            for (int j = 0; j < SN; ++j)
                b[j] = Bs[buf][kk + M::frag_k(lane)][wn * SN * M::E + j * M::E + M::frag_row(lane)];
#pragma unroll
            for (int i = 0; i < SM; ++i)
#pragma unroll
                for (int j = 0; j < SN; ++j)
                    acc[i][j] = M::mma(a[i], b[j], acc[i][j]);
        }
        __builtin_amdgcn_sched_barrier(0);
        la.store(As[buf ^ 1]);
        lb.store(Bs[buf ^ 1]);
        __syncthreads();
    }
    if (g.ksplit > 1) {
        // one K slice of C V: stored for the finishing kernel
        T *P = static_cast<T *>(g.P) + (int64_t)kz * g.pslice;
#pragma unroll
        for (int i = 0; i < SM; ++i)
#pragma unroll
            for (int j = 0; j < SN; ++j)
#pragma unroll
                for (int r = 0; r < M::NR; ++r) {
                    const int m = m0 + wm * SM * M::E + i * M::E + M::out_row(lane, r);
                    const int64_t col = j0 + wn * SN * M::E + j * M::E + M::out_col(lane);
                    if (m < Mrows && col < g.D)
                        P[(int64_t)m * g.D + col] = acc[i][j][r];
                }
        return;
    }
    // epilogue: R = H - acc, squared norms of R and H summed over this wave's columns.
    // The H values are loaded in groups of RG output rows, every load of a group issued
    // before any is used (out-of-range ones read a valid address and are ignored), so a
    // group costs one memory latency, not one per value.  The group sizes keep the
    // registers, and so the waves per SIMD, of the K loop (FP32: 2 of 16 rows; FP64: all 4).
    T *H = const_cast<T *>(static_cast<const T *>(g.H));
    const int *rows = g.rows;
    constexpr int RG = M::NR <= 4 ? M::NR : 2;
#pragma unroll
    for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int r0 = 0; r0 < M::NR; r0 += RG) {
            int hrow[RG];
            T hv[RG][SN];
#pragma unroll
            for (int q = 0; q < RG; ++q) {
                const int m = m0 + wm * SM * M::E + i * M::E + M::out_row(lane, r0 + q);
                const int mc = m < Mrows ? m : Mrows - 1;
                hrow[q] = rows ? rows[mc] : mc;
            }
#pragma unroll
            for (int q = 0; q < RG; ++q)
#pragma unroll
                for (int j = 0; j < SN; ++j) {
                    const int64_t col = j0 + wn * SN * M::E + j * M::E + M::out_col(lane);
                    hv[q][j] = H[(int64_t)hrow[q] * g.D + (col < g.D ? col : 0)];
                }
#pragma unroll
            for (int q = 0; q < RG; ++q) {
                const int r = r0 + q;
                const int ml = wm * SM * M::E + i * M::E + M::out_row(lane, r);
                const int m = m0 + ml;
                double rs = 0.0, hsq = 0.0;
                if (m < Mrows) {
#pragma unroll
                    for (int j = 0; j < SN; ++j) {
                        const int64_t col = j0 + wn * SN * M::E + j * M::E + M::out_col(lane);
                        if (col < g.D) {
                            const T h = hv[q][j];
                            const T res = h - acc[i][j][r];
                            if (g.write_r)
                                H[(int64_t)hrow[q] * g.D + col] = res;
                            rs += (double)res * (double)res;
                            hsq += (double)h * (double)h;
                        }
                    }
                }
                // sum over the lanes that hold the same output row
                for (int off = M::E / 2; off > 0; off >>= 1) {
                    rs += __shfl_xor(rs, off, 64);
                    hsq += __shfl_xor(hsq, off, 64);
                }
                if (M::out_col(lane) == 0) {
                    red[ml][wn][0] = rs;
                    red[ml][wn][1] = hsq;
                }
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

template <typename T, int SM, int SN, bool VD>
__global__ void __launch_bounds__(256) k_gemm_dot(GemmArgs g)
{
    gemm_dot_body<T, SM, SN, VD>(g, blockIdx.x, blockIdx.y, gridDim.x, blockIdx.z);
}

template <typename T, int SM, int SN, bool VD, int CS = 1>
__global__ void __launch_bounds__(256) k_gemm_sub(GemmArgs g)
{
    gemm_sub_body<T, SM, SN, VD, CS>(g, blockIdx.x, blockIdx.y, gridDim.x, blockIdx.z);
}

// Finishing step of a split residual pass, one workgroup per row m: R = H - sum_z P_z
// (slices added in order), written over H when asked, and the squared norms of R and H.
__global__ void __launch_bounds__(256) k_gemm_sub_finish(GemmArgs g, double *rho2, double *h2)
{
    __shared__ double red[2][4];
    const int m = blockIdx.x;
    const int Mrows = g.nrows ? *g.nrows : g.cnt;
    if (m >= Mrows || aborted(g.st))
        return;
    double *H = const_cast<double *>(static_cast<const double *>(g.H)) + (int64_t)(g.rows ? g.rows[m] : m) * g.D;
    const double *P = static_cast<const double *>(g.P) + (int64_t)m * g.D;
    double rs = 0.0, hs = 0.0;
    for (int64_t j = threadIdx.x; j < g.D; j += blockDim.x) {
        const double acc = ordered_strided_sum(P + j, g.pslice, g.ksplit);
        const double h = H[j], r = h - acc;
        if (g.write_r)
            H[j] = r;
        rs += r * r;
        hs += h * h;
    }
    for (int off = 32; off > 0; off >>= 1) {
        rs += __shfl_xor(rs, off, 64);
        hs += __shfl_xor(hs, off, 64);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][w] = rs;
        red[1][w] = hs;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
        double a = 0.0, b = 0.0;
        for (int q = 0; q < nw; ++q) {
            a += red[0][q];
            b += red[1][q];
        }
        rho2[m] = a;
        if (h2)
            h2[m] = b;
    }
}

template <typename T, int SM, int SN, bool VD>
__global__ void __launch_bounds__(256) k_gemm_dot_b(Batch b)
{
    const int p = batch_find(b.start, b.nprob, blockIdx.x);
    const GemmArgs g = static_cast<const GemmArgs *>(b.args)[p];
    const int l = blockIdx.x - b.start[p], gx = b.gx[p];
    gemm_dot_body<T, SM, SN, VD>(g, l % gx, l / gx, gx);
}

template <typename T, int SM, int SN, bool VD>
__global__ void __launch_bounds__(256) k_gemm_sub_b(Batch b)
{
    const int p = batch_find(b.start, b.nprob, blockIdx.x);
    const GemmArgs g = static_cast<const GemmArgs *>(b.args)[p];
    const int l = blockIdx.x - b.start[p], gx = b.gx[p];
    gemm_sub_body<T, SM, SN, VD>(g, l % gx, l / gx, gx);
}

__device__ void norm_final_body(const NormArgs &a, int bx)
{
    const int m = bx * 256 + threadIdx.x;
    const int Mrows = a.nrows ? *a.nrows : a.cnt;
    if (m >= Mrows || aborted(a.st))
        return;
    const double *np = a.normpart + (int64_t)m * a.tiles * 2;
    const double s0 = ordered_strided_sum(np, 2, a.tiles), s1 = ordered_strided_sum(np + 1, 2, a.tiles);
    a.rho2[m] = s0;
    if (a.h2)
        a.h2[m] = s1;
}

__global__ void __launch_bounds__(256) k_gemm_norm_final(NormArgs a) { norm_final_body(a, blockIdx.x); }

__global__ void __launch_bounds__(256) k_norm_final_b(Batch b)
{
    const int p = batch_find(b.start, b.nprob, blockIdx.x);
    const NormArgs a = static_cast<const NormArgs *>(b.args)[p];
    norm_final_body(a, blockIdx.x - b.start[p]);
}

// 16-byte loads of rows of D elements (buffers are 256-byte aligned, rows a multiple of 16 bytes)
template <typename T>
bool rows_vec(int64_t D)
{
    return D % (16 / (int64_t)sizeof(T)) == 0;
}

template <typename T, int SM, int SN>
hipError_t dot_impl(const GemmArgs &g, int64_t n_hi, hipStream_t s)
{
    constexpr int E = Mma<T>::E;
    constexpr int BM = 2 * SM * E, BN = 2 * SN * E;
    const dim3 grid((unsigned)((n_hi + BN - 1) / BN), (g.cnt + BM - 1) / BM, std::max(g.ksplit, 1));
    if (rows_vec<T>(g.D))
        hipLaunchKernelGGL((k_gemm_dot<T, SM, SN, true>), grid, dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL((k_gemm_dot<T, SM, SN, false>), grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

template <typename T, int SM, int SN>
hipError_t sub_impl(const GemmArgs &g, hipStream_t s)
{
    constexpr int E = Mma<T>::E;
    constexpr int BM = 2 * SM * E, BN = 2 * SN * E;
    const int tiles = (int)((g.D + BN - 1) / BN);
    const dim3 grid(tiles, (g.cnt + BM - 1) / BM, std::max(g.ksplit, 1));
    if (g.ldc % 4 != 0)
        return hipErrorInvalidValue;  // the coefficient rows are read with 16-byte loads
    const bool v = rows_vec<T>(g.D);
    if (g.cslices > 1 && v)
        hipLaunchKernelGGL((k_gemm_sub<T, SM, SN, true, kMaxSlices>), grid, dim3(256), 0, s, g);
    else if (g.cslices > 1)
        hipLaunchKernelGGL((k_gemm_sub<T, SM, SN, false, kMaxSlices>), grid, dim3(256), 0, s, g);
    else if (v)
        hipLaunchKernelGGL((k_gemm_sub<T, SM, SN, true>), grid, dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL((k_gemm_sub<T, SM, SN, false>), grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

// Slices for a K extent of `nchunks` chunks when the output has `tiles` tiles: enough
// to give about 256 workgroups, at most 16, every slice non-empty (one slice: no split).
int slices_for(int64_t tiles, int64_t nchunks)
{
    if (tiles >= 128 || nchunks < 2)
        return 1;
    const int64_t want = std::min<int64_t>({kMaxSlices, nchunks, (256 + tiles - 1) / tiles});
    const int64_t per = (nchunks + want - 1) / want;
    return (int)((nchunks + per - 1) / per);
}


}  // namespace

int64_t coef_ld(int64_t n_hi) { return (std::max<int64_t>(n_hi, 1) + 3) / 4 * 4; }

// Tile choice: the larger workgroup tile when it still yields enough
// workgroups to cover the compute units, the smaller one otherwise.
int gemm_tile_f32(int64_t rows, int64_t cols) { return ((rows + 127) / 128) * ((cols + 127) / 128) >= 192 ? 2 : 1; }

hipError_t launch_gemm_dot_f32(const float *Vs, const DevState *st, const float *Hs, int cnt, int64_t D, int64_t n_hi,
                               int64_t ldc, float *C, int tile, hipStream_t s)
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
    return tile == 2 ? dot_impl<float, 2, 2>(g, n_hi, s) : dot_impl<float, 1, 1>(g, n_hi, s);
}

int gemm_sub_tiles_f32(int64_t D, int tile) { return (int)((D + (tile == 2 ? 128 : 64) - 1) / (tile == 2 ? 128 : 64)); }

hipError_t launch_gemm_sub_f32(const float *Vs, const DevState *st, const float *Hs, const float *C, int64_t n_hi,
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
    g.write_r = 0;
    return tile == 2 ? sub_impl<float, 2, 2>(g, s) : sub_impl<float, 1, 1>(g, s);
}

int gemm_sub_tiles_f64(int64_t D) { return (int)((D + 63) / 64); }

SplitPlan gemm_split_plan_f64(int cnt, int64_t n_hi, int64_t D, int64_t ldc, size_t ws_doubles)
{
    SplitPlan p{1, 1};
    if (cnt <= 0 || cnt > kSplitRows)
        return p;
    n_hi = std::max<int64_t>(n_hi, 1);
    const int64_t mt = (cnt + 63) / 64;
    p.kd = slices_for(((n_hi + 63) / 64) * mt, (D + KC - 1) / KC);
    p.ks = slices_for(((D + 63) / 64) * mt, (n_hi + KC - 1) / KC);
    auto need = [&]() { return (size_t)(p.kd > 1 ? p.kd : 0) * cnt * ldc + (size_t)(p.ks > 1 ? p.ks : 0) * cnt * D; };
    while (need() > ws_doubles && p.ks > 1)
        p.ks = std::max(1, p.ks / 2);
    while (need() > ws_doubles && p.kd > 1)
        p.kd = std::max(1, p.kd / 2);
    return p;
}

size_t gemm_split_ws_doubles(int64_t D, int64_t ldc)
{
    return std::min<size_t>((size_t)8 << 20, (size_t)16 * kSplitRows * (size_t)(ldc + D));
}

hipError_t launch_gemm_dot_f64(const double *V, const DevState *st, const double *H, const int *rows,
                               const int *nrows, int cnt, int64_t D, int64_t n_hi, int64_t ldc, double *C,
                               hipStream_t s, int ksplit)
{
    if (cnt <= 0)
        return hipSuccess;
    GemmArgs g{};
    g.H = H;
    g.rows = rows;
    g.nrows = nrows;
    g.cnt = cnt;
    g.V = V;
    g.C = C;
    g.ldc = ldc;
    g.D = D;
    g.st = st;
    g.ksplit = ksplit;
    g.cslice = (int64_t)cnt * ldc;
    return dot_impl<double, 2, 2>(g, std::max<int64_t>(n_hi, 1), s);
}

hipError_t launch_gemm_sub_f64(const double *V, const DevState *st, double *H, const int *rows, const int *nrows,
                               const double *C, int64_t n_hi, int64_t ldc, int cnt, int64_t D, double *normpart,
                               hipStream_t s, int cslices, int ksplit, double *P)
{
    if (cnt <= 0)
        return hipSuccess;
    GemmArgs g{};
    g.H = H;
    g.rows = rows;
    g.nrows = nrows;
    g.cnt = cnt;
    g.V = V;
    g.C = const_cast<double *>(C);
    g.ldc = ldc;
    g.D = D;
    g.st = st;
    g.normpart = normpart;
    g.write_r = 1;
    g.cslices = cslices;
    g.cslice = (int64_t)cnt * ldc;
    g.ksplit = ksplit > 1 && P ? ksplit : 1;
    g.P = P;
    g.pslice = (int64_t)cnt * D;
    return sub_impl<double, 2, 2>(g, s);
}

hipError_t launch_gemm_sub_finish_f64(const double *P, int ksplit, double *H, const int *rows, const int *nrows,
                                      int cnt, int64_t D, const DevState *st, double *rho2, double *h2, hipStream_t s)
{
    if (cnt <= 0)
        return hipSuccess;
    GemmArgs g{};
    g.H = H;
    g.rows = rows;
    g.nrows = nrows;
    g.cnt = cnt;
    g.D = D;
    g.st = st;
    g.write_r = 1;
    g.ksplit = ksplit;
    g.P = const_cast<double *>(P);
    g.pslice = (int64_t)cnt * D;
    hipLaunchKernelGGL(k_gemm_sub_finish, dim3(cnt), dim3(256), 0, s, g, rho2, h2);
    return hipGetLastError();
}

hipError_t launch_norm_final(const double *normpart, const int *nrows, int cnt, int tiles, const DevState *st,
                             double *rho2, double *h2, hipStream_t s)
{
    if (cnt <= 0)
        return hipSuccess;
    NormArgs a{normpart, nrows, cnt, tiles, st, rho2, h2};
    hipLaunchKernelGGL(k_gemm_norm_final, dim3((cnt + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

int gemm_group_m(bool) { return 64; }
int gemm_group_n(bool) { return 64; }

hipError_t launch_gemm_dot_batched(const Batch &b, bool f32, bool vec, hipStream_t s)
{
    if (b.total <= 0)
        return hipSuccess;
    if (f32 && vec)
        hipLaunchKernelGGL((k_gemm_dot_b<float, 1, 1, true>), dim3(b.total), dim3(256), 0, s, b);
    else if (f32)
        hipLaunchKernelGGL((k_gemm_dot_b<float, 1, 1, false>), dim3(b.total), dim3(256), 0, s, b);
    else if (vec)
        hipLaunchKernelGGL((k_gemm_dot_b<double, 2, 2, true>), dim3(b.total), dim3(256), 0, s, b);
    else
        hipLaunchKernelGGL((k_gemm_dot_b<double, 2, 2, false>), dim3(b.total), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_gemm_sub_batched(const Batch &b, bool f32, bool vec, hipStream_t s)
{
    if (b.total <= 0)
        return hipSuccess;
    if (f32 && vec)
        hipLaunchKernelGGL((k_gemm_sub_b<float, 1, 1, true>), dim3(b.total), dim3(256), 0, s, b);
    else if (f32)
        hipLaunchKernelGGL((k_gemm_sub_b<float, 1, 1, false>), dim3(b.total), dim3(256), 0, s, b);
    else if (vec)
        hipLaunchKernelGGL((k_gemm_sub_b<double, 2, 2, true>), dim3(b.total), dim3(256), 0, s, b);
    else
        hipLaunchKernelGGL((k_gemm_sub_b<double, 2, 2, false>), dim3(b.total), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_norm_final_batched(const Batch &b, hipStream_t s)
{
    if (b.total <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_norm_final_b, dim3(b.total), dim3(256), 0, s, b);
    return hipGetLastError();
}

}  // namespace lie

// Brackets on the matrix cores, FP64 and FP32: large operators (d > 64) as mirrored
// tile pairs, and 16 < d <= 32 with the left operand shared by consecutive candidates.
//
// With A = sqrt(d/2)(Ar + i Ai) read from the packed array (entry (i, k) of Ar and Ai
// both come from p[i][k] and p[k][i]), the bracket is [A, B] = (d/2)(P - P^H) with
// P = (Ar + i Ai)(Br + i Bi), formed as four real products.  Its packed output needs
// P[i][j] and P[j][i] together, and a whole P (2 d^2 values) no longer fits in LDS
// at d = 128, so the work is cut into mirrored 16 x 16 tile pairs {(I, J), (J, I)},
// I <= J: a wave forms both tiles of a pair with 16x16x4 MFMAs, operands gathered
// from the packed rows in L2 four k-steps at a time, puts them in its own LDS buffer
// and writes every output element of the two tiles.  One workgroup per candidate,
// four waves sharing its tile pairs.
#include "lie_internal.h"

#include <type_traits>

#include <algorithm>

namespace lie {

namespace {

// Output element e of a bracket: FP64 rows, FP32 rows, or (FP32 with planes set) split-BF16 planes.
template <typename T>
__device__ inline void put(T *out, __bf16 *plane, int64_t e, T v)
{
    if constexpr (std::is_same<T, float>::value) {
        if (plane) {
            store_plane(plane, e, v);
            return;
        }
    }
    out[e] = v;
}

constexpr int kThreads = 256;
constexpr int kTileLd = 17;  // LDS row stride of a 16 x 16 tile

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct PairMma;

// 16x16x4 f64: result register r of lane l is D[4r + l/16][l%16].
template <>
struct PairMma<double> {
    typedef f64x4 Acc;
    __device__ static Acc mma(double a, double b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int r) { return 4 * r + (lane >> 4); }
};

// 16x16x4 f32: result register r of lane l is D[4(l/16) + r][l%16].
template <>
struct PairMma<float> {
    typedef f32x4 Acc;
    __device__ static Acc mma(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// (x, y) = (p[i][k], p[k][i]); an index outside d x d reads entry (0, 0) and is dropped later.
template <typename T>
struct Raw {
    T x, y;
};
template <typename T>
__device__ inline Raw<T> raw_at(const T *p, int d, int i, int k)
{
    const bool in = i < d && k < d;
    const int ic = in ? i : 0, kc = in ? k : 0;
    return Raw<T>{p[ic * d + kc], p[kc * d + ic]};
}
// Entry (i, k) of Ar and Ai (zero outside d x d).
template <typename T>
__device__ inline void frag(Raw<T> v, int d, int i, int k, T &ar, T &ai)
{
    const bool in = i < d && k < d;
    ar = !in || i == k ? T(0) : (i < k ? v.x : -v.y);
    ai = !in ? T(0) : (i < k ? v.y : (i > k ? v.x : T(1.4142135623730951) * v.x));
}

template <typename T>
__device__ void comm_pairs_body(const CommArgs &A, int c)
{
    using M = PairMma<T>;
    using Acc = typename M::Acc;
    __shared__ T buf[4][4][16 * kTileLd];  // per wave: Pr(I,J), Pi(I,J), Pr(J,I), Pi(J,I)
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const DevState *st = A.st;
    if (c >= (A.ncnt ? *A.ncnt : A.cnt) || (st && (st->done | st->numeric_error | st->full)))
        return;
    const T *V = static_cast<const T *>(A.V);
    const int d = A.d;
    const int64_t D = (int64_t)d * d;
    int64_t l, m;
    decode_pair(A.pair_list ? A.pair_list[c] : (A.dp0 ? *A.dp0 : A.p0) + c, l, m);
    const T *pa = V + l * D, *pb = V + m * D;
    T *out = static_cast<T *>(A.H) + (int64_t)c * D;
    __bf16 *plane = A.Hp ? A.Hp + (int64_t)c * A.ldp : nullptr;
    const T so = (T)sqrt(0.5 * d), sd = (T)sqrt((double)d);
    const int lr = lane & 15, lk = lane >> 4;
    const int TT = (d + 15) / 16, npairs = TT * (TT + 1) / 2;
    T *Pr1 = buf[w][0], *Pi1 = buf[w][1], *Pr2 = buf[w][2], *Pi2 = buf[w][3];
    double sq = 0.0;
    for (int t = w; t < npairs; t += 4) {
        int I = 0, rem = t;  // t -> (I, J), I <= J, row-major over the upper triangle of tiles
        while (rem >= TT - I) {
            rem -= TT - I;
            ++I;
        }
        const int J = I + rem;
        const bool diag = I == J;
        Acc r1, i1, r2, i2;  // tile (I, J) and (J, I)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            r1[r] = i1[r] = r2[r] = i2[r] = T(0);
        for (int k0 = 0; k0 < 16 * TT; k0 += 16) {
            Raw<T> aI[4], aJ[4], bJ[4], bI[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int k = k0 + 4 * s + lk;
                aI[s] = raw_at(pa, d, 16 * I + lr, k);
                bJ[s] = raw_at(pb, d, k, 16 * J + lr);
                if (!diag) {
                    aJ[s] = raw_at(pa, d, 16 * J + lr, k);
                    bI[s] = raw_at(pb, d, k, 16 * I + lr);
                }
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int k = k0 + 4 * s + lk;
                T ar, ai, br, bi;
                frag(aI[s], d, 16 * I + lr, k, ar, ai);
                frag(bJ[s], d, k, 16 * J + lr, br, bi);
                r1 = M::mma(ar, br, r1);
                r1 = M::mma(-ai, bi, r1);
                i1 = M::mma(ar, bi, i1);
                i1 = M::mma(ai, br, i1);
                if (!diag) {
                    frag(aJ[s], d, 16 * J + lr, k, ar, ai);
                    frag(bI[s], d, k, 16 * I + lr, br, bi);
                    r2 = M::mma(ar, br, r2);
                    r2 = M::mma(-ai, bi, r2);
                    i2 = M::mma(ar, bi, i2);
                    i2 = M::mma(ai, br, i2);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = M::row(lane, r);
            Pr1[row * kTileLd + lr] = r1[r];
            Pi1[row * kTileLd + lr] = i1[r];
            Pr2[row * kTileLd + lr] = diag ? r1[r] : r2[r];
            Pi2[row * kTileLd + lr] = diag ? i1[r] : i2[r];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the tiles, read across lanes
        // element (a, b) of tile (I, J) is P[16I + a][16J + b]; its mirror P[16J + b][16I + a]
        // is element (b, a) of tile (J, I)
        for (int e = lane; e < 256; e += 64) {
            const int a = e >> 4, b = e & 15;
            const int i = 16 * I + a, j = 16 * J + b;
            if (i >= d || j >= d || i > j)
                continue;
            if (i < j) {
                const T v1 = so * (Pr1[a * kTileLd + b] - Pr2[b * kTileLd + a]);
                const T v2 = so * (Pi1[a * kTileLd + b] + Pi2[b * kTileLd + a]);
                put(out, plane, (int64_t)i * d + j, v1);
                put(out, plane, (int64_t)j * d + i, v2);
                sq += (double)v1 * v1 + (double)v2 * v2;
            } else {
                const T v = sd * Pi1[a * kTileLd + b];
                put(out, plane, (int64_t)i * d + i, v);
                sq += (double)v * v;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // read before the next pair overwrites
    }
    if (A.hs2) {
        for (int off = 32; off > 0; off >>= 1)
            sq += __shfl_down(sq, off, 64);
        if (lane == 0)
            red[w] = sq;
        __syncthreads();
        if (threadIdx.x == 0)
            A.hs2[c] = red[0] + red[1] + red[2] + red[3];
    }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_comm_pairs(CommArgs a)
{
    comm_pairs_body<T>(a, blockIdx.x);
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_comm_pairs_b(Batch b)
{
    const int p = batch_find(b.start, b.nprob, blockIdx.x);
    const CommArgs a = static_cast<const CommArgs *>(b.args)[p];
    comm_pairs_body<T>(a, blockIdx.x - b.start[p]);
}

// ---- 16 < d <= 32, candidates grouped by their left operand.
//
// Consecutive pair indices p = l(l-1)/2 + m run over m = 0 .. l-1 with l fixed, so
// consecutive candidates of a block share their left operand V_l.  A workgroup takes
// up to kMaxGroup consecutive candidates: the MFMA fragments of A (its row block, every
// k-step) are gathered once per distinct l and stay in registers; per candidate only
// B is staged in LDS (coalesced, row stride 33), and the next candidate's B is fetched
// while this one is multiplied.  Wave w computes the 16 x 16 tile (I, J) = (w % 2, w / 2)
// of P = (Ar + i Ai)(Br + i Bi) (operands zero-padded to 32), P goes to LDS, and the
// packed bracket sqrt(d/2)(P - P^H) (diagonal sqrt(d) Im P_ii) and its squared norm are
// written out as in the other bracket kernels.
constexpr int kMaxGroup = 16;
constexpr int kLo = 33;  // LDS row stride of the staged operand and of P

// (x, y) = (S[i][k], S[k][i]) of an operand staged in LDS; an index outside d x d reads
// entry (0, 0), dropped by frag().
template <typename T>
__device__ inline Raw<T> raw_lds(const T *S, int d, int i, int k)
{
    const bool in = i < d && k < d;
    const int ic = in ? i : 0, kc = in ? k : 0;
    return Raw<T>{S[ic * kLo + kc], S[kc * kLo + ic]};
}

template <typename T>
__device__ void comm_grouped_body(const CommArgs &A, int c0, int G)
{
    using M = PairMma<T>;
    using Acc = typename M::Acc;
    __shared__ T Sa[32 * kLo], Sb[32 * kLo], Pr[32 * kLo], Pi[32 * kLo];
    __shared__ double red[kMaxGroup][4];
    const DevState *st = A.st;
    const int cnt = A.ncnt ? *A.ncnt : A.cnt;
    const int ng = min(G, cnt - c0);
    if (ng <= 0 || (st && (st->done | st->numeric_error | st->full)))
        return;
    const T *V = static_cast<const T *>(A.V);
    const int d = A.d;
    const int D = d * d;  // <= 1024: at most 4 elements per thread
    const int64_t pbase = A.pair_list ? 0 : (A.dp0 ? *A.dp0 : A.p0);
    auto pair_of = [&](int c) -> int64_t { return A.pair_list ? A.pair_list[c] : pbase + c; };
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int I = w & 1, J = w >> 1;
    const int lr = lane & 15, lk = lane >> 4;
    const T so = (T)sqrt(0.5 * d), sd = (T)sqrt((double)d);
    // element e = tid + kThreads j of an operand row: its (row, column) and whether it exists
    int eo[4];
    bool ev[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int e = tid + kThreads * j;
        ev[j] = e < D;
        eo[j] = ev[j] ? (e / d) * kLo + e % d : 0;
    }
    int64_t l, m;
    decode_pair(pair_of(c0), l, m);
    T bnext[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        bnext[j] = V[m * D + (ev[j] ? tid + kThreads * j : 0)];
    int64_t lcur = -1;
    T ar[8], ai[8];  // A fragments of row block I, k-steps 0..7
    for (int g = 0; g < ng; ++g) {
        const bool newa = l != lcur;  // uniform
        if (newa) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (ev[j])
                    Sa[eo[j]] = V[l * D + tid + kThreads * j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (ev[j])
                Sb[eo[j]] = bnext[j];
        __syncthreads();  // Sa (when new) and Sb staged; P of the previous candidate read out
        if (newa) {
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int k = 4 * s + lk;
                frag(raw_lds(Sa, d, 16 * I + lr, k), d, 16 * I + lr, k, ar[s], ai[s]);
            }
            lcur = l;
        }
        int64_t ln = l, mn = m;
        if (g + 1 < ng) {
            decode_pair(pair_of(c0 + g + 1), ln, mn);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                bnext[j] = V[mn * D + (ev[j] ? tid + kThreads * j : 0)];
        }
        Acc pr, pi;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            pr[r] = pi[r] = T(0);
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int k = 4 * s + lk;
            T br, bi;
            frag(raw_lds(Sb, d, k, 16 * J + lr), d, k, 16 * J + lr, br, bi);
            pr = M::mma(ar[s], br, pr);
            pr = M::mma(-ai[s], bi, pr);
            pi = M::mma(ar[s], bi, pi);
            pi = M::mma(ai[s], br, pi);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * I + M::row(lane, r);
            Pr[row * kLo + 16 * J + lr] = pr[r];
            Pi[row * kLo + 16 * J + lr] = pi[r];
        }
        __syncthreads();  // P complete; Sb and Sa reads done
        T *out = static_cast<T *>(A.H) + (int64_t)(c0 + g) * D;
        __bf16 *plane = A.Hp ? A.Hp + (int64_t)(c0 + g) * A.ldp : nullptr;
        double sq = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int e = tid + kThreads * j;
            if (e < D) {
                const int i = e / d, jj = e % d;
                T v;
                if (i < jj)
                    v = so * (Pr[i * kLo + jj] - Pr[jj * kLo + i]);
                else if (i > jj)
                    v = so * (Pi[jj * kLo + i] + Pi[i * kLo + jj]);
                else
                    v = sd * Pi[i * kLo + i];
                put(out, plane, e, v);
                sq += (double)v * (double)v;
            }
        }
        for (int off = 32; off > 0; off >>= 1)
            sq += __shfl_down(sq, off, 64);
        if (lane == 0)
            red[g][w] = sq;
        l = ln;
        m = mn;
    }
    __syncthreads();
    if (A.hs2 && tid < ng)
        A.hs2[c0 + tid] = red[tid][0] + red[tid][1] + red[tid][2] + red[tid][3];
}

// FP32: at most 128 registers, four workgroups per CU (FP64 would spill there)
template <typename T>
__global__ void __launch_bounds__(kThreads, sizeof(T) == 4 ? 4 : 3) k_comm_grouped(CommArgs a, int G)
{
    comm_grouped_body<T>(a, blockIdx.x * G, G);
}

}  // namespace

hipError_t launch_comm_pairs(const CommArgs &a, bool f64, hipStream_t s)
{
    if (a.cnt <= 0)
        return hipSuccess;
    if (f64)
        hipLaunchKernelGGL(k_comm_pairs<double>, dim3(a.cnt), dim3(kThreads), 0, s, a);
    else
        hipLaunchKernelGGL(k_comm_pairs<float>, dim3(a.cnt), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_comm_grouped(const CommArgs &a, bool f64, hipStream_t s)
{
    if (a.cnt <= 0)
        return hipSuccess;
    if (a.d <= 16 || a.d > 32)
        return hipErrorInvalidValue;
    // candidates per workgroup: the sharing grows with the group, but a group runs its
    // candidates one after the other, so keep at least about 1024 workgroups in flight.
    // A pair list (the survivors of a screened block: few, their count on the device,
    // rarely sharing l) takes one candidate per workgroup.
    const int G = a.pair_list ? 1 : std::max(1, std::min(kMaxGroup, a.cnt / 1024));
    const unsigned grid = (unsigned)((a.cnt + G - 1) / G);
    if (f64)
        hipLaunchKernelGGL(k_comm_grouped<double>, dim3(grid), dim3(kThreads), 0, s, a, G);
    else
        hipLaunchKernelGGL(k_comm_grouped<float>, dim3(grid), dim3(kThreads), 0, s, a, G);
    return hipGetLastError();
}

hipError_t launch_comm_pairs_batched(const Batch &b, bool f64, hipStream_t s)
{
    if (b.total <= 0)
        return hipSuccess;
    if (f64)
        hipLaunchKernelGGL(k_comm_pairs_b<double>, dim3(b.total), dim3(kThreads), 0, s, b);
    else
        hipLaunchKernelGGL(k_comm_pairs_b<float>, dim3(b.total), dim3(kThreads), 0, s, b);
    return hipGetLastError();
}

}  // namespace lie

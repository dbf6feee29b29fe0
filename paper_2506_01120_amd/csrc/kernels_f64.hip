// FP64 kernels of the closure engine: layout conversion, the bracket, the
// projection/residual pass (GEMV form), the block cursor and the orthogonality
// check.  The acceptance kernel has a file of its own.
// Operators use the packed anti-Hermitian layout described in lie_internal.h.
#include "lie_internal.h"

#include <algorithm>
#include <cmath>

namespace lie {

namespace {

constexpr int kThreads = 256;

// Sum over a 256-thread workgroup; result valid in thread 0.
__device__ inline double block_sum(double v, double *red /* >= 4 doubles of LDS */)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0)
        red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i)
            s += red[i];
    __syncthreads();
    return s;
}

// ------------------------------------------------------------------ layout

__global__ void k_pack_c128(const double *__restrict__ src, double *__restrict__ dst, int count, int d)
{
    const int64_t D = (int64_t)d * d;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)count * D)
        return;
    const int64_t e = idx / D, r = idx % D;
    const int i = (int)(r / d), j = (int)(r % d);
    const double *x = src + e * D * 2;
    const double s2 = sqrt(2.0 / d), s1 = sqrt(1.0 / d);
    double v;
    // project onto the anti-Hermitian part (X - X^H)/2 while packing
    if (i < j) {
        v = s2 * 0.5 * (x[2 * (i * d + j)] - x[2 * (j * d + i)]);
    } else if (i > j) {
        v = s2 * 0.5 * (x[2 * (j * d + i) + 1] + x[2 * (i * d + j) + 1]);
    } else {
        v = s1 * x[2 * (i * d + i) + 1];
    }
    dst[idx] = v;
}

__global__ void k_unpack_c128(const double *__restrict__ src, double *__restrict__ dst, int64_t count, int d)
{
    const int64_t D = (int64_t)d * d;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= count * D)
        return;
    const int64_t e = idx / D, r = idx % D;
    const int i = (int)(r / d), j = (int)(r % d);
    const double *p = src + e * D;
    const double u2 = sqrt(d / 2.0), u1 = sqrt((double)d);
    double re, im;
    if (i < j) {
        re = u2 * p[i * d + j];
        im = u2 * p[j * d + i];
    } else if (i > j) {
        re = -u2 * p[j * d + i];
        im = u2 * p[i * d + j];
    } else {
        re = 0.0;
        im = u1 * p[i * d + i];
    }
    dst[2 * idx] = re;
    dst[2 * idx + 1] = im;
}

// ------------------------------------------------------------------ bracket
//
// For anti-Hermitian A, B write A = sqrt(d/2) (Ar + i Ai) with Ar antisymmetric
// and Ai symmetric real, read straight from the packed arrays:
//   Ar[i][k] = p[i][k] (i<k), -p[k][i] (i>k), 0 (i=k)
//   Ai[i][k] = p[k][i] (i<k),  p[i][k] (i>k), sqrt(2) p[i][i] (i=k)
// With P = (Ar + i Ai)(Br + i Bi) the bracket is [A,B] = AB - BA = (d/2)(P - P^H)
// because BA = (AB)^H for anti-Hermitian A, B.  Its packed form is
//   out[i][j] = sqrt(d/2) (Pr[i][j] - Pr[j][i]),  out[j][i] = sqrt(d/2) (Pi[i][j] + Pi[j][i])  (i<j)
//   out[i][i] = sqrt(d) Pi[i][i].

__device__ inline double unp_re(const double *p, int d, int i, int k)
{
    return i < k ? p[i * d + k] : (i > k ? -p[k * d + i] : 0.0);
}
__device__ inline double unp_im(const double *p, int d, int i, int k)
{
    return i < k ? p[k * d + i] : (i > k ? p[i * d + k] : 1.4142135623730951 * p[i * d + i]);
}

// One workgroup per candidate; both operands unpacked into LDS (d <= 64).
__device__ void comm_f64_lds_body(const CommArgs &A, int c)
{
    extern __shared__ double lds[];
    const double *V = static_cast<const double *>(A.V);
    const int d = A.d;
    const int64_t p0 = A.dp0 ? *A.dp0 : A.p0;
    const int64_t *pair_list = A.pair_list;
    const int cnt = A.cnt;
    const DevState *st = A.st;
    double *H = static_cast<double *>(A.H);
    if (c >= (A.ncnt ? *A.ncnt : cnt) || (st && (st->done | st->numeric_error | st->full)))
        return;
    const int64_t D = (int64_t)d * d;
    int64_t l, m;
    decode_pair(pair_list ? pair_list[c] : p0 + c, l, m);
    const double *pa = V + l * D, *pb = V + m * D;
    const int ld = d + 1;
    double *Ar = lds, *Ai = Ar + d * ld, *Br = Ai + d * ld, *Bi = Br + d * ld;
    for (int idx = threadIdx.x; idx < d * d; idx += blockDim.x) {
        const int i = idx / d, k = idx % d;
        Ar[i * ld + k] = unp_re(pa, d, i, k);
        Ai[i * ld + k] = unp_im(pa, d, i, k);
        Br[i * ld + k] = unp_re(pb, d, i, k);
        Bi[i * ld + k] = unp_im(pb, d, i, k);
    }
    __syncthreads();
    const double so = sqrt(d / 2.0), sd = sqrt((double)d);
    double *out = H + (int64_t)c * D;
    const int npairs = d * (d + 1) / 2;
    for (int q = threadIdx.x; q < npairs; q += blockDim.x) {
        // q -> (i, j), i <= j, row-major over the upper triangle
        int i = 0, rem = q;
        while (rem >= d - i) {
            rem -= d - i;
            ++i;
        }
        const int j = i + rem;
        double prij = 0, piij = 0, prji = 0, piji = 0;
        for (int k = 0; k < d; ++k) {
            const double ar = Ar[i * ld + k], ai = Ai[i * ld + k];
            const double br = Br[k * ld + j], bi = Bi[k * ld + j];
            prij += ar * br - ai * bi;
            piij += ar * bi + ai * br;
            const double ar2 = Ar[j * ld + k], ai2 = Ai[j * ld + k];
            const double br2 = Br[k * ld + i], bi2 = Bi[k * ld + i];
            prji += ar2 * br2 - ai2 * bi2;
            piji += ar2 * bi2 + ai2 * br2;
        }
        if (i < j) {
            out[i * d + j] = so * (prij - prji);
            out[j * d + i] = so * (piij + piji);
        } else {
            out[i * d + i] = sd * piij;
        }
    }
}

// Same bracket reading operands directly from global memory (any d); scalar, used for
// the occasional raw row that Algorithm 3 rebuilds at d > 64.
__device__ void comm_f64_global_body(const CommArgs &A, int bx, int c)
{
    const double *V = static_cast<const double *>(A.V);
    const int d = A.d;
    const int64_t p0 = A.dp0 ? *A.dp0 : A.p0;
    const int64_t *pair_list = A.pair_list;
    const int cnt = A.cnt;
    const DevState *st = A.st;
    double *H = static_cast<double *>(A.H);
    const int64_t D = (int64_t)d * d;
    if (c >= (A.ncnt ? *A.ncnt : cnt) || (st && (st->done | st->numeric_error | st->full)))
        return;
    int64_t l, m;
    decode_pair(pair_list ? pair_list[c] : p0 + c, l, m);
    const double *pa = V + l * D, *pb = V + m * D;
    const double so = sqrt(d / 2.0), sd = sqrt((double)d);
    double *out = H + (int64_t)c * D;
    const int64_t idx = (int64_t)bx * blockDim.x + threadIdx.x;
    if (idx >= D)
        return;
    const int i = (int)(idx / d), j = (int)(idx % d);
    if (i > j)
        return;
    double prij = 0, piij = 0, prji = 0, piji = 0;
    for (int k = 0; k < d; ++k) {
        const double ar = unp_re(pa, d, i, k), ai = unp_im(pa, d, i, k);
        const double br = unp_re(pb, d, k, j), bi = unp_im(pb, d, k, j);
        prij += ar * br - ai * bi;
        piij += ar * bi + ai * br;
        const double ar2 = unp_re(pa, d, j, k), ai2 = unp_im(pa, d, j, k);
        const double br2 = unp_re(pb, d, k, i), bi2 = unp_im(pb, d, k, i);
        prji += ar2 * br2 - ai2 * bi2;
        piji += ar2 * bi2 + ai2 * br2;
    }
    if (i < j) {
        out[i * d + j] = so * (prij - prji);
        out[j * d + i] = so * (piij + piji);
    } else {
        out[i * d + i] = sd * piij;
    }
}

typedef double f64x4_t __attribute__((ext_vector_type(4)));

// ---- the bracket on the matrix cores (FP64 16x16x4 MFMA)
// P = (Ar + i Ai)(Br + i Bi) as four real products.  Each MFMA operand is gathered
// straight from the packed rows: entry (i, k) of Ar and of Ai both come from the two
// packed values p[i][k] and p[k][i], so one pair of loads serves both (no unpacking
// pass through LDS).  Lane l supplies A[l%16][k0 + l/16] and B[k0 + l/16][l%16]; result
// register r of lane l is P[4r + l/16][l%16].  P goes through LDS only to be read
// transposed for the packed output sqrt(d/2)(P - P^H).

// Entry (i, k) of Ar and Ai (zero outside d x d) from the two packed values x = p[i][k]
// and y = p[k][i].
struct CommRaw {
    double x, y;
};
__device__ inline void comm_frag(CommRaw v, int d, int i, int k, double &ar, double &ai)
{
    const bool in = i < d && k < d;
    ar = !in || i == k ? 0.0 : (i < k ? v.x : -v.y);
    ai = !in ? 0.0 : (i < k ? v.y : (i > k ? v.x : 1.4142135623730951 * v.x));
}

// Packed output element e of the bracket from P = Pr + i Pi held in LDS (row stride ld).
__device__ inline double comm_out(const double *Pr, const double *Pi, int ld, int d, int e)
{
    const int i = e / d, j = e % d;
    if (i < j)
        return sqrt(0.5 * d) * (Pr[i * ld + j] - Pr[j * ld + i]);
    if (i > j)
        return sqrt(0.5 * d) * (Pi[j * ld + i] + Pi[i * ld + j]);
    return sqrt((double)d) * Pi[i * ld + i];
}

// d <= 16: one wave per candidate (four per workgroup).  The wave copies its two packed
// operands into its LDS tile with coalesced loads (row stride 17), gathers the MFMA
// fragments from there, and reuses the tile for P.
__global__ void __launch_bounds__(kThreads) k_comm_f64_mfma16(CommArgs A)
{
    __shared__ double Pbuf[4][2][16 * 17];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int c = blockIdx.x * 4 + w;
    const DevState *st = A.st;
    if (c >= (A.ncnt ? *A.ncnt : A.cnt) || (st && (st->done | st->numeric_error | st->full)))
        return;
    const double *V = static_cast<const double *>(A.V);
    const int d = A.d;
    const int64_t D = (int64_t)d * d;
    int64_t l, m;
    decode_pair(A.pair_list ? A.pair_list[c] : (A.dp0 ? *A.dp0 : A.p0) + c, l, m);
    double *Sa = Pbuf[w][0], *Sb = Pbuf[w][1];
    {
        const double *pa = V + l * D, *pb = V + m * D;
        for (int e = lane; e < D; e += 64) {
            const int i = e / d, k = e % d;
            Sa[i * 17 + k] = pa[e];
            Sb[i * 17 + k] = pb[e];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const int lr = lane & 15, lk = lane >> 4;
    f64x4_t pr = {0.0, 0.0, 0.0, 0.0}, pi = {0.0, 0.0, 0.0, 0.0};
    CommRaw ra[4], rb[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int k = 4 * s + lk;
        const bool ina = lr < d && k < d;
        ra[s] = ina ? CommRaw{Sa[lr * 17 + k], Sa[k * 17 + lr]} : CommRaw{0.0, 0.0};
        rb[s] = ina ? CommRaw{Sb[k * 17 + lr], Sb[lr * 17 + k]} : CommRaw{0.0, 0.0};
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the tile is read; P may overwrite it
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int k0 = 4 * s;
        double ar, ai, br, bi;
        comm_frag(ra[s], d, lr, k0 + lk, ar, ai);
        comm_frag(rb[s], d, k0 + lk, lr, br, bi);
        pr = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, pr, 0, 0, 0);
        pr = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, bi, pr, 0, 0, 0);
        pi = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, pi, 0, 0, 0);
        pi = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, pi, 0, 0, 0);
    }
    double *Pr = Pbuf[w][0], *Pi = Pbuf[w][1];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        Pr[(4 * r + lk) * 17 + lr] = pr[r];
        Pi[(4 * r + lk) * 17 + lr] = pi[r];
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the wave's own LDS writes, read across lanes
    double *out = static_cast<double *>(A.H) + (int64_t)c * D;
    for (int e = lane; e < D; e += 64)
        out[e] = comm_out(Pr, Pi, 17, d, e);
}

// 16 < d <= 16 T: one workgroup per candidate.  The two packed operands are first copied
// into LDS with coalesced loads (row stride d + 1, so that a fragment gather down a
// column does not hit one bank), and the MFMA fragments are gathered from there; wave w
// owns column block J = w % T and row blocks I = w / T, w / T + 4 / T, ...
// Dynamic LDS: max(2 d (d + 1), 2 x 16T x (16T + 1)) doubles (operands, then P).
template <int T>
__device__ void comm_f64_mfma_body(const CommArgs &A, int c)
{
    extern __shared__ double Pl[];
    constexpr int NI = T * T / 4;  // row blocks per wave
    constexpr int ld = 16 * T + 1;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const DevState *st = A.st;
    if (c >= (A.ncnt ? *A.ncnt : A.cnt) || (st && (st->done | st->numeric_error | st->full)))
        return;
    const double *V = static_cast<const double *>(A.V);
    const int d = A.d;
    const int64_t D = (int64_t)d * d;
    int64_t l, m;
    decode_pair(A.pair_list ? A.pair_list[c] : (A.dp0 ? *A.dp0 : A.p0) + c, l, m);
    const int lo = d + 1;  // operand row stride in LDS
    double *Sa = Pl, *Sb = Pl + d * lo;
    {
        const double *pa = V + l * D, *pb = V + m * D;
        for (int64_t e = threadIdx.x; e < D; e += blockDim.x) {
            const int i = (int)(e / d), k = (int)(e % d);
            Sa[i * lo + k] = pa[e];
            Sb[i * lo + k] = pb[e];
        }
    }
    __syncthreads();
    const int lr = lane & 15, lk = lane >> 4;
    const int J = w % T, I0 = w / T;
    f64x4_t pr[NI], pi[NI];
#pragma unroll
    for (int q = 0; q < NI; ++q)
        pr[q] = pi[q] = f64x4_t{0.0, 0.0, 0.0, 0.0};
    auto frag = [&](const double *S, int i, int k, double &ar, double &ai) {
        const bool in = i < d && k < d;
        const int ic = in ? i : 0, kc = in ? k : 0;
        comm_frag(CommRaw{S[ic * lo + kc], S[kc * lo + ic]}, d, i, k, ar, ai);
    };
#pragma unroll 4
    for (int k0 = 0; k0 < 16 * T; k0 += 4) {
        const int k = k0 + lk;
        double br, bi;
        frag(Sb, k, 16 * J + lr, br, bi);
#pragma unroll
        for (int q = 0; q < NI; ++q) {
            double ar, ai;
            frag(Sa, 16 * (I0 + q * (4 / T)) + lr, k, ar, ai);
            pr[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, pr[q], 0, 0, 0);
            pr[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, bi, pr[q], 0, 0, 0);
            pi[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, pi[q], 0, 0, 0);
            pi[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, pi[q], 0, 0, 0);
        }
    }
    __syncthreads();  // the operands are consumed; P takes their place
    double *Pr = Pl, *Pi = Pl + 16 * T * ld;
#pragma unroll
    for (int q = 0; q < NI; ++q) {
        const int I = I0 + q * (4 / T);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Pr[(16 * I + 4 * r + lk) * ld + 16 * J + lr] = pr[q][r];
            Pi[(16 * I + 4 * r + lk) * ld + 16 * J + lr] = pi[q][r];
        }
    }
    __syncthreads();
    double *out = static_cast<double *>(A.H) + (int64_t)c * D;
    for (int e = threadIdx.x; e < D; e += blockDim.x)
        out[e] = comm_out(Pr, Pi, ld, d, e);
}

template <int T>
__global__ void __launch_bounds__(kThreads) k_comm_f64_mfma(CommArgs A)
{
    comm_f64_mfma_body<T>(A, blockIdx.x);
}

// Grouped form: one workgroup per candidate of any problem with d <= 16 T.
template <int T>
__global__ void __launch_bounds__(kThreads) k_comm_f64_mfma_b(Batch b)
{
    const int p = batch_find(b.start, b.nprob, blockIdx.x);
    const CommArgs a = static_cast<const CommArgs *>(b.args)[p];
    comm_f64_mfma_body<T>(a, blockIdx.x - b.start[p]);
}

__global__ void __launch_bounds__(kThreads) k_comm_f64_lds(CommArgs a) { comm_f64_lds_body(a, blockIdx.x); }
__global__ void __launch_bounds__(kThreads) k_comm_f64_lds_b(Batch b)
{
    const int p = batch_find(b.start, b.nprob, blockIdx.x);
    const CommArgs a = static_cast<const CommArgs *>(b.args)[p];
    comm_f64_lds_body(a, blockIdx.x - b.start[p]);
}
// Algorithm 3: raw rows of the elements appended by the last acceptance launch.
// Element e in [st->raw_lo, st->N) came from generator -(src+1) (its packed copy is
// G's row) or from the bracket of raw rows l, m < raw_lo of its source pair.
__global__ void __launch_bounds__(kThreads) k_raw_append(const double *G, double *B, float *Bs, int d,
                                                         const int64_t *elem_src, const DevState *st, int use_lds,
                                                         int normalize)
{
    __shared__ double red[kThreads / 64];
    const int64_t lo = st->raw_lo, hi = st->N;
    const int64_t D = (int64_t)d * d;
    for (int64_t e = lo + blockIdx.x; e < hi; e += gridDim.x) {
        const int64_t src = elem_src[e];
        double *out = B + e * D;
        if (src < 0) {
            const double *g = G + (-src - 1) * D;
            for (int64_t j = threadIdx.x; j < D; j += blockDim.x)
                out[j] = g[j];
        } else {
            const CommArgs A{B, d, 0, elem_src + e, nullptr, nullptr, 1, nullptr, out, nullptr};
            if (use_lds)
                comm_f64_lds_body(A, 0);
            else
                for (int bx = 0; (int64_t)bx * blockDim.x < D; ++bx)
                    comm_f64_global_body(A, bx, 0);
        }
        __syncthreads();  // row e is complete
        if (normalize) {
            // unit norm (the matrix-inversion method keeps unit-norm raw elements)
            double loc = 0.0;
            for (int64_t j = threadIdx.x; j < D; j += blockDim.x)
                loc += out[j] * out[j];
            for (int off = 32; off > 0; off >>= 1)
                loc += __shfl_down(loc, off, 64);
            if ((threadIdx.x & 63) == 0)
                red[threadIdx.x >> 6] = loc;
            __syncthreads();
            double t = 0.0;
            for (int q = 0; q < (int)(blockDim.x >> 6); ++q)
                t += red[q];
            const double inv = t > 0.0 ? 1.0 / sqrt(t) : 0.0;
            __syncthreads();  // red is reused by the next element
            for (int64_t j = threadIdx.x; j < D; j += blockDim.x)
                out[j] *= inv;
            __syncthreads();
        }
        if (Bs)
            for (int64_t j = threadIdx.x; j < D; j += blockDim.x)
                Bs[e * D + j] = (float)out[j];
        __syncthreads();  // the operand LDS is reused by the next element
    }
}


// ------------------------------------------------------------------ projection
//
// Rows of a pass are either H[0..cnt) or, with a row list, H[rows[r]] for
// r < *nrows (survivors of an earlier pass).  Coefficients and partials are
// indexed by the pass row r.

__device__ inline bool aborted(const DevState *st) { return st->done | st->numeric_error | st->full; }

// C[r][k] = <H_row(r), V_k> for k < N (tiled: 16 basis rows x 16 pass rows per workgroup).
// With grid.z = sd > 1 the element range is split in sd slices and slice z of the sums is
// written at C + z * cslice (the consumer adds them); a few workgroups then no longer wait
// on one load round trip per element chunk in turn.
constexpr int kDotT = 16, kDotJ = 32, kMaxDotSlices = 16;

__global__ void __launch_bounds__(kThreads) k_dot_f64(const double *__restrict__ V, const DevState *__restrict__ st,
                                                      int64_t N_fixed, const double *__restrict__ H,
                                                      const int *__restrict__ rows, const int *__restrict__ nrows,
                                                      int cnt, int64_t D, double *__restrict__ C, int64_t ldc,
                                                      int64_t cslice)
{
    if (st && aborted(st))
        return;
    const int64_t N = st ? st->N : N_fixed;
    const int nr = nrows ? *nrows : cnt;
    const int64_t k0 = (int64_t)blockIdx.x * kDotT;
    const int c0 = blockIdx.y * kDotT;
    if (k0 >= N || c0 >= nr)
        return;
    __shared__ double Vs[kDotT][kDotJ + 1];
    __shared__ double Hs[kDotT][kDotJ + 1];
    const int tk = threadIdx.x % kDotT, tc = threadIdx.x / kDotT;
    const int64_t nch = (D + kDotJ - 1) / kDotJ, per = (nch + gridDim.z - 1) / gridDim.z;
    const int64_t jlo = std::min<int64_t>(D, (int64_t)blockIdx.z * per * kDotJ);
    const int64_t jhi = std::min<int64_t>(D, jlo + per * kDotJ);
    double acc = 0.0;
    for (int64_t j0 = jlo; j0 < jhi; j0 += kDotJ) {
        for (int e = threadIdx.x; e < kDotT * kDotJ; e += blockDim.x) {
            const int r = e / kDotJ, jj = e % kDotJ;
            const int64_t j = j0 + jj;
            Vs[r][jj] = (k0 + r < N && j < jhi) ? V[(k0 + r) * D + j] : 0.0;
            double hv = 0.0;
            if (c0 + r < nr && j < jhi) {
                const int hr = rows ? rows[c0 + r] : c0 + r;
                hv = H[(int64_t)hr * D + j];
            }
            Hs[r][jj] = hv;
        }
        __syncthreads();
        for (int jj = 0; jj < kDotJ; ++jj)
            acc += Hs[tc][jj] * Vs[tk][jj];
        __syncthreads();
    }
    if (k0 + tk < N && c0 + tc < nr)
        C[(int64_t)blockIdx.z * cslice + (int64_t)(c0 + tc) * ldc + k0 + tk] = acc;
}

// part[ks][r][j] = sum_{k in chunk ks} C[r][k] V[k][j]  (64 columns x 4 pass rows per workgroup)
constexpr int kSubJ = 64, kSubC = 4, kSubK = 16;

__global__ void __launch_bounds__(kThreads) k_sub_partial_f64(const double *__restrict__ V,
                                                              const DevState *__restrict__ st,
                                                              const double *__restrict__ C, int64_t ldc,
                                                              int cs, int64_t cslice,
                                                              const int *__restrict__ nrows, int cnt, int64_t D,
                                                              int ks_total, double *__restrict__ part)
{
    if (aborted(st))
        return;
    const int64_t N = st->N;
    const int nr = nrows ? *nrows : cnt;
    const int64_t j0 = (int64_t)blockIdx.x * kSubJ;
    const int c0 = blockIdx.y * kSubC;
    if (c0 >= nr)
        return;
    const int ks = blockIdx.z;
    const int tj = threadIdx.x % kSubJ, tc = threadIdx.x / kSubJ;
    const int64_t chunk = (N + ks_total - 1) / ks_total;
    const int64_t kb = ks * chunk, ke = std::min<int64_t>(N, kb + chunk);
    __shared__ double Vt[kSubK][kSubJ];
    __shared__ double Ct[kSubC][kSubK];
    double acc = 0.0;
    for (int64_t k0 = kb; k0 < ke; k0 += kSubK) {
        for (int e = threadIdx.x; e < kSubK * kSubJ; e += blockDim.x) {
            const int r = e / kSubJ, jj = e % kSubJ;
            const int64_t k = k0 + r, j = j0 + jj;
            Vt[r][jj] = (k < ke && j < D) ? V[k * D + j] : 0.0;
        }
        if (threadIdx.x < kSubC * kSubK) {
            const int r = threadIdx.x / kSubK, kk = threadIdx.x % kSubK;
            const int64_t k = k0 + kk;
            double cv = 0.0;
            if (k < ke && c0 + r < nr) {
                // the cs coefficient slices: loaded together, added in slice order
                double sl[kMaxDotSlices];
                const double *p = C + (int64_t)(c0 + r) * ldc + k;
#pragma unroll
                for (int q = 0; q < kMaxDotSlices; ++q)
                    sl[q] = q < cs ? p[(int64_t)q * cslice] : 0.0;
#pragma unroll
                for (int q = 0; q < kMaxDotSlices; ++q)
                    if (q < cs)
                        cv += sl[q];
            }
            Ct[r][kk] = cv;
        }
        __syncthreads();
        for (int kk = 0; kk < kSubK; ++kk)
            acc += Ct[tc][kk] * Vt[kk][tj];
        __syncthreads();
    }
    const int c = c0 + tc;
    const int64_t j = j0 + tj;
    if (c < nr && j < D)
        part[((int64_t)ks * cnt + c) * D + j] = acc;
}

// R = H - sum_ks part, written over H_row(r), and the squared norms of R and H into
// rho2[r], h2[r]: one workgroup per row (these passes have at most a few dozen rows),
// partial sums added in a fixed order.
__global__ void __launch_bounds__(kThreads) k_sub_reduce_f64(double *__restrict__ H, const double *__restrict__ part,
                                                             const int *__restrict__ rows,
                                                             const int *__restrict__ nrows, int cnt, int64_t D,
                                                             int ks_total, const DevState *__restrict__ st,
                                                             double *__restrict__ rho2, double *__restrict__ h2)
{
    __shared__ double red[8];
    const int c = blockIdx.x;
    const int nr = nrows ? *nrows : cnt;
    if (c >= nr || aborted(st))
        return;
    const int hr = rows ? rows[c] : c;
    double r2 = 0.0, hh = 0.0;
    for (int64_t j = threadIdx.x; j < D; j += blockDim.x) {
        const double h = H[(int64_t)hr * D + j];
        const double s = ordered_strided_sum(part + (int64_t)c * D + j, (int64_t)cnt * D, ks_total);
        const double r = h - s;
        H[(int64_t)hr * D + j] = r;
        r2 += r * r;
        hh += h * h;
    }
    r2 = block_sum(r2, red);
    hh = block_sum(hh, red);
    if (threadIdx.x == 0) {
        rho2[c] = r2;
        h2[c] = hh;
    }
}

int split_k(int64_t D, int cnt, int64_t n_hi)
{
    const int64_t jt = (D + kSubJ - 1) / kSubJ;
    const int64_t ct = (cnt + kSubC - 1) / kSubC;
    int64_t ks = (1024 + jt * ct - 1) / (jt * ct);
    ks = std::min<int64_t>(ks, std::max<int64_t>(1, (n_hi + kSubK - 1) / kSubK));
    ks = std::min<int64_t>(ks, 64);
    return (int)std::max<int64_t>(ks, 1);
}

__global__ void k_advance_cursor(int64_t *cursor, int cnt)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *cursor += cnt;
}

__global__ void k_set_cursor(int64_t *cursor, int64_t value)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *cursor = value;
}

__global__ void k_gather_states(const DevState *const *src, int n, DevState *dst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        dst[i] = *src[i];
}

// ------------------------------------------------------------------ orthogonality

__global__ void __launch_bounds__(kThreads) k_gram_loss_part(const double *__restrict__ G, int64_t n,
                                                             double *__restrict__ part)
{
    __shared__ double red[8];
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / n, j = e % n;
        const double g = G[e] - (i == j ? 1.0 : 0.0);
        s += g * g;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0)
        part[blockIdx.x] = s;
}

// Panel form: rows r0 .. r0 + rows of G (row stride n); part[b] receives this panel's sum
// (first panel) or adds it (later panels), so the panels are summed in launch order.
__global__ void __launch_bounds__(kThreads) k_gram_loss_panel(const double *__restrict__ G, int64_t rows, int64_t n,
                                                              int64_t r0, int accumulate, double *__restrict__ part)
{
    __shared__ double red[8];
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < rows * n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = r0 + e / n, j = e % n;
        const double g = G[e] - (i == j ? 1.0 : 0.0);
        s += g * g;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0)
        part[blockIdx.x] = accumulate ? part[blockIdx.x] + s : s;
}

__global__ void k_gram_loss_final(const double *__restrict__ part, int parts, double *__restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < parts; ++i)
            s += part[i];
        *out = sqrt(s);
    }
}

}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t launch_pack_c128(const double *src, double *dst, int count, int d, hipStream_t s)
{
    const int64_t total = (int64_t)count * d * d;
    const int blocks = (int)((total + kThreads - 1) / kThreads);
    if (blocks == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_pack_c128, dim3(blocks), dim3(kThreads), 0, s, src, dst, count, d);
    return hipGetLastError();
}

hipError_t launch_unpack_c128(const double *src, double *dst, int64_t count, int d, hipStream_t s)
{
    const int64_t total = count * d * d;
    const int64_t blocks = (total + kThreads - 1) / kThreads;
    if (blocks == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_unpack_c128, dim3((unsigned)blocks), dim3(kThreads), 0, s, src, dst, count, d);
    return hipGetLastError();
}

hipError_t launch_raw_append(const double *G, double *B, float *Bs, int d, const int64_t *elem_src, const DevState *st,
                             int max_new, hipStream_t s, bool normalize)
{
    if (max_new <= 0)
        return hipSuccess;
    const size_t lds = (size_t)4 * d * (d + 1) * sizeof(double);
    static size_t granted = 65536;
    bool use_lds = d <= 64;
    if (use_lds && lds > granted) {
        if (hipFuncSetAttribute((const void *)k_raw_append, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) ==
            hipSuccess)
            granted = lds;
        else
            (void)hipGetLastError();
    }
    use_lds = use_lds && lds <= granted;
    const int grid = std::min(max_new, 1024);
    hipLaunchKernelGGL(k_raw_append, dim3(grid), dim3(kThreads), use_lds ? lds : 0, s, G, B, Bs, d, elem_src, st,
                       use_lds ? 1 : 0, normalize ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_comm_f64(const double *V, int d, int64_t p0, const int64_t *pair_list, const int *ncnt, int cnt,
                           const DevState *st, double *H, hipStream_t s, const int64_t *dp0)
{
    if (cnt <= 0)
        return hipSuccess;
    const size_t lds = (size_t)4 * d * (d + 1) * sizeof(double);
    static int max_lds = -1;
    static size_t granted = 65536;
    if (max_lds < 0) {
        int dev = 0, v = 65536;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
            max_lds = v;
        else
            max_lds = 65536;
    }
    if (lds > granted && lds + 1024 <= (size_t)max_lds) {
        // raise the dynamic LDS limit of this kernel to what this launch needs
        if (hipFuncSetAttribute((const void *)k_comm_f64_lds, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) ==
            hipSuccess)
            granted = lds;
        else
            (void)hipGetLastError();  // clear the failed request; the fallback kernel is used
    }
    CommArgs a{V, d, p0, pair_list, dp0, ncnt, cnt, st, H, nullptr};
    if (d <= 16) {
        hipLaunchKernelGGL(k_comm_f64_mfma16, dim3((unsigned)((cnt + 3) / 4)), dim3(kThreads), 0, s, a);
        return hipGetLastError();
    }
    if (d <= 32)
        return launch_comm_grouped(a, true, s);
    if (d <= 64) {
        static bool granted64 = false;
        const size_t l64 = (size_t)2 * 64 * 65 * sizeof(double);
        if (!granted64) {
            if (hipFuncSetAttribute((const void *)k_comm_f64_mfma<4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)l64) == hipSuccess)
                granted64 = true;
            else
                (void)hipGetLastError();  // the LDS kernel below is used instead
        }
        if (granted64) {
            hipLaunchKernelGGL(k_comm_f64_mfma<4>, dim3(cnt), dim3(kThreads), l64, s, a);
            return hipGetLastError();
        }
    }
    if (d <= 64 && lds <= granted) {
        hipLaunchKernelGGL(k_comm_f64_lds, dim3(cnt), dim3(kThreads), lds, s, a);
        return hipGetLastError();
    }
    return launch_comm_pairs(a, true, s);
}

bool comm_f64_fits_lds(int d)
{
    if (d > 64)
        return false;
    // the first launch of the single-problem kernel raises the limit; mirror its rule
    int dev = 0, v = 65536;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        v = 65536;
    return (size_t)4 * d * (d + 1) * sizeof(double) + 1024 <= (size_t)v;
}

hipError_t launch_comm_f64_batched(const Batch &b, bool lds_variant, int dmax, hipStream_t s)
{
    if (b.total <= 0)
        return hipSuccess;
    if (lds_variant && dmax <= 32) {
        hipLaunchKernelGGL(k_comm_f64_mfma_b<2>, dim3(b.total), dim3(kThreads), (size_t)2 * 32 * 33 * sizeof(double), s,
                           b);
        return hipGetLastError();
    }
    if (lds_variant && dmax <= 64) {
        static bool granted64 = false;
        const size_t l64 = (size_t)2 * 64 * 65 * sizeof(double);
        if (!granted64) {
            if (hipFuncSetAttribute((const void *)k_comm_f64_mfma_b<4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)l64) == hipSuccess)
                granted64 = true;
            else
                (void)hipGetLastError();  // the LDS kernel below is used instead
        }
        if (granted64) {
            hipLaunchKernelGGL(k_comm_f64_mfma_b<4>, dim3(b.total), dim3(kThreads), l64, s, b);
            return hipGetLastError();
        }
    }
    if (lds_variant) {
        const size_t lds = (size_t)4 * dmax * (dmax + 1) * sizeof(double);
        static size_t granted = 65536;
        if (lds > granted) {
            if (hipFuncSetAttribute((const void *)k_comm_f64_lds_b, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds) != hipSuccess)
                return hipGetLastError();
            granted = lds;
        }
        hipLaunchKernelGGL(k_comm_f64_lds_b, dim3(b.total), dim3(kThreads), lds, s, b);
        return hipGetLastError();
    }
    return launch_comm_pairs_batched(b, true, s);
}

hipError_t launch_advance_cursor(int64_t *cursor, int cnt, hipStream_t s)
{
    hipLaunchKernelGGL(k_advance_cursor, dim3(1), dim3(64), 0, s, cursor, cnt);
    return hipGetLastError();
}

hipError_t launch_set_cursor(int64_t *cursor, int64_t value, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_cursor, dim3(1), dim3(64), 0, s, cursor, value);
    return hipGetLastError();
}

hipError_t launch_gather_states(const DevState *const *src, int n, DevState *dst, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_gather_states, dim3((n + 63) / 64), dim3(64), 0, s, src, n, dst);
    return hipGetLastError();
}

size_t proj_scratch_doubles(int64_t D, int cnt_max, int64_t cap)
{
    size_t best = 0;
    for (int cnt = 1; cnt <= cnt_max; ++cnt) {
        const int ks = split_k(D, cnt, cap);
        best = std::max(best, (size_t)ks * cnt * D);
    }
    return best;
}

int project_split_k(int64_t D, int cnt, int64_t n_hi) { return split_k(D, cnt, std::max<int64_t>(n_hi, 1)); }

int dot_slices_f64(ProjShape sh, size_t ws_doubles)
{
    const int64_t n_hi = std::max<int64_t>(sh.n_hi, 1);
    const int64_t tiles = ((n_hi + kDotT - 1) / kDotT) * ((sh.cnt + kDotT - 1) / kDotT);
    const int64_t nch = (sh.D + kDotJ - 1) / kDotJ;
    if (sh.cnt <= 0 || tiles >= 64 || nch < 2)
        return 1;
    int64_t sd = std::min<int64_t>({(int64_t)kMaxDotSlices, nch, (128 + tiles - 1) / tiles});
    while (sd > 1 && (size_t)sd * sh.cnt * n_hi > ws_doubles)
        --sd;
    return (int)std::max<int64_t>(sd, 1);
}

hipError_t launch_dot_f64(const double *V, const DevState *st, const double *H, const int *rows, const int *nrows,
                          double *C, ProjShape sh, hipStream_t s, int sd)
{
    const int cnt = sh.cnt;
    if (cnt <= 0)
        return hipSuccess;
    const int64_t n_hi = std::max<int64_t>(sh.n_hi, 1);
    sd = std::min(std::max(sd, 1), kMaxDotSlices);
    hipLaunchKernelGGL(k_dot_f64, dim3((unsigned)((n_hi + kDotT - 1) / kDotT), (cnt + kDotT - 1) / kDotT, sd),
                       dim3(kThreads), 0, s, V, st, (int64_t)0, H, rows, nrows, cnt, sh.D, C, n_hi,
                       (int64_t)cnt * n_hi);
    return hipGetLastError();
}

hipError_t launch_sub_f64(const double *V, const DevState *st, const double *C, const int *nrows, double *part,
                          ProjShape sh, hipStream_t s, int cs)
{
    const int cnt = sh.cnt;
    if (cnt <= 0)
        return hipSuccess;
    const int64_t n_hi = std::max<int64_t>(sh.n_hi, 1);
    const int ks = split_k(sh.D, cnt, n_hi);
    hipLaunchKernelGGL(k_sub_partial_f64,
                       dim3((unsigned)((sh.D + kSubJ - 1) / kSubJ), (cnt + kSubC - 1) / kSubC, ks), dim3(kThreads), 0,
                       s, V, st, C, n_hi, std::min(std::max(cs, 1), kMaxDotSlices), (int64_t)cnt * n_hi, nrows, cnt,
                       sh.D, ks, part);
    return hipGetLastError();
}

hipError_t launch_reduce_f64(double *H, const int *rows, const int *nrows, double *part, const DevState *st,
                             double *rho2, double *h2, ProjShape sh, hipStream_t s)
{
    const int cnt = sh.cnt;
    if (cnt <= 0)
        return hipSuccess;
    const int64_t n_hi = std::max<int64_t>(sh.n_hi, 1);
    const int ks = split_k(sh.D, cnt, n_hi);
    hipLaunchKernelGGL(k_sub_reduce_f64, dim3(cnt), dim3(kThreads), 0, s, H, part, rows, nrows, cnt, sh.D, ks, st,
                       rho2, h2);
    return hipGetLastError();
}

hipError_t launch_orth_loss(const double *V, int64_t n, int64_t D, double *work, double *out, hipStream_t s)
{
    if (n <= 0) {
        return hipMemsetAsync(out, 0, sizeof(double), s);
    }
    // G = V V^T through the coefficient kernel (candidates = basis rows)
    double *G = work;
    for (int64_t c0 = 0; c0 < n; c0 += 65535 * kDotT) {
        const int64_t rows = std::min<int64_t>(n - c0, (int64_t)65535 * kDotT);
        hipLaunchKernelGGL(k_dot_f64, dim3((unsigned)((n + kDotT - 1) / kDotT), (unsigned)((rows + kDotT - 1) / kDotT)),
                           dim3(kThreads), 0, s, V, (const DevState *)nullptr, n, V + c0 * D, (const int *)nullptr,
                           (const int *)nullptr, (int)rows, D, G + c0 * n, n, (int64_t)0);
    }
    const int parts = 256;
    double *part = work + n * n;
    hipLaunchKernelGGL(k_gram_loss_part, dim3(parts), dim3(kThreads), 0, s, G, n, part);
    hipLaunchKernelGGL(k_gram_loss_final, dim3(1), dim3(64), 0, s, part, parts, out);
    return hipGetLastError();
}

hipError_t launch_orth_loss_panels(const double *V, int64_t n, int64_t D, double *ws, int64_t ws_doubles,
                                   double *out, hipStream_t s)
{
    const int parts = 256;
    if (n <= 0) {
        hipLaunchKernelGGL(k_gram_loss_final, dim3(1), dim3(64), 0, s, ws, 0, out);  // sqrt(0)
        return hipGetLastError();
    }
    if (ws_doubles < parts + n)
        return hipErrorInvalidValue;
    double *part = ws, *G = ws + parts;
    // rows per panel: as many as the workspace holds, at most the grid's row limit
    const int64_t P = std::min<int64_t>(std::min<int64_t>((ws_doubles - parts) / n, n), (int64_t)65535 * kDotT);
    for (int64_t r0 = 0; r0 < n; r0 += P) {
        const int64_t rows = std::min<int64_t>(P, n - r0);
        hipLaunchKernelGGL(k_dot_f64, dim3((unsigned)((n + kDotT - 1) / kDotT), (unsigned)((rows + kDotT - 1) / kDotT)),
                           dim3(kThreads), 0, s, V, (const DevState *)nullptr, n, V + r0 * D, (const int *)nullptr,
                           (const int *)nullptr, (int)rows, D, G, n, (int64_t)0);
        hipLaunchKernelGGL(k_gram_loss_panel, dim3(parts), dim3(kThreads), 0, s, G, rows, n, r0, r0 > 0 ? 1 : 0,
                           part);
    }
    hipLaunchKernelGGL(k_gram_loss_final, dim3(1), dim3(64), 0, s, part, parts, out);
    return hipGetLastError();
}

}  // namespace lie

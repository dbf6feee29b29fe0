// FP64 kernels of the closure engine: layout conversion, the bracket, the
// projection/residual pass, sequential acceptance and the orthogonality check.
// Operators use the packed anti-Hermitian layout described in lie_internal.h.
#include "lie_internal.h"

#include <algorithm>
#include <cmath>

namespace lie {

namespace {

constexpr int kThreads = 256;

// Workgroup barrier that orders LDS traffic only: it waits for this wave's LDS
// operations (lgkmcnt = 0) but not for outstanding global loads or stores, so a
// prefetch or a result store in flight does not stall every barrier.  Use it
// only where no thread reads global data another thread of the workgroup just wrote.
// s_waitcnt encoding (gfx9): vmcnt[3:0] | expcnt[6:4] | lgkmcnt[11:8] | vmcnt[5:4] << 14.
__device__ inline void lds_barrier()
{
    __builtin_amdgcn_s_waitcnt(0xC07F);  // vmcnt = 63, expcnt = 7, lgkmcnt = 0
    __builtin_amdgcn_s_barrier();
}

__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

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

// ------------------------------------------------------------------ acceptance
//
// One workgroup.  Phase A (parallel over the block's candidates): every
// candidate that is not a survivor is rejected and counted -- exact zeros,
// screen rejects (screened residual) or FP64 rejects (first-pass residual).
// Phase B (sequential over survivors, in candidate order): the survivor's
// FP64 residual R (after the re-orthogonalisation pass against the block's
// basis snapshot) is orthogonalised twice against the elements appended
// earlier in this block, its norm decides, and an accepted residual is
// normalised and appended as V[N] (and its FP32 rounding as Vs[N]).

constexpr int kAccThreads = 1024;
constexpr int kMaxBlock = 16384;



__device__ inline void atomic_max_pos(double *addr, double v)
{
    // values are non-negative, so the IEEE bit pattern orders like a signed integer
    atomicMax(reinterpret_cast<unsigned long long *>(addr), (unsigned long long)__double_as_longlong(v));
}
__device__ inline void atomic_min_pos(double *addr, double v)
{
    atomicMin(reinterpret_cast<unsigned long long *>(addr), (unsigned long long)__double_as_longlong(v));
}


// One 16 x 16 FP64 tile of A B^T over a K-extent of D: lane l supplies row l%16 of
// A through pa and of B through pb (nullptr: a zero row).  Loads are issued 16 at a
// time per operand so that their latencies overlap.
__device__ inline f64x4_t dot_tile_f64(const double *pa, const double *pb, int64_t D, int lane)
{
    f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int64_t k0 = 0; k0 < D; k0 += 64) {
        double av[16], bv[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int64_t k = k0 + 4 * q + (lane >> 4);
            av[q] = (pa && k < D) ? pa[k] : 0.0;
            bv[q] = (pb && k < D) ? pb[k] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[q], acc, 0, 0, 0);
    }
    return acc;
}

// Compiler-level ordering of LDS accesses between the steps of a one-wave
// recurrence (a wavefront's LDS operations complete in issue order).
__device__ inline void wave_order() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// Value of x in lane `src` (uniform) for every lane of the wave.
__device__ inline double lane_bcast(double x, int src)
{
    const int s = __builtin_amdgcn_readfirstlane(src);
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), s);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), s);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Row stride of the small Gram matrix in LDS: odd, so that a column read by
// 64 lanes spreads over the banks, and at least 17.
__host__ __device__ constexpr int gram_ld(int nsv) { return nsv < 17 ? 17 : (nsv | 1); }

// LDS (in doubles) of the block Cholesky-QR pass over nsv survivors with nw >= 16 waves:
// Gram / factor / inverse (nsv x gram_ld) | pivots | verified norms | two index lists
// (ints) | panel products of the inverse (16 x nsv), then per-wave norm partials (nw x nsv).
__host__ __device__ constexpr int64_t bqr_lds(int nsv, int nw)
{
    return (int64_t)nsv * gram_ld(nsv) + 4 * (int64_t)nsv + (int64_t)nw * nsv;
}

struct BqrOut {
    int resume;  // first survivor left to the exact sequential path (nsv: none)
    int u;       // survivors before `resume` accepted by the pass (they are V[N0 .. N0+u))
};

// Block Cholesky-QR of a block's survivors (Algorithm 4's in-block decisions, in
// candidate order).  Survivor rows R_0..R_{s-1} are already orthogonal to the
// basis snapshot; what the sequential loop would measure for R_j is its norm after
// removing the survivors accepted before it, i.e. the Cholesky pivot of the Gram
// matrix G = R R^T restricted to those rows.
//  * A pivot is a certified acceptance when it is at least 0.1 ||R_j|| (the
//    accepted rows stay well conditioned, so the Gram rounding, ~eps ||R_j||^2,
//    cannot matter) and at least 10 thr (rounding cannot flip the decision).
//  * Every other row is provisionally rejected (its column is skipped).  The Gram
//    pivot cannot certify a rejection -- it carries an absolute error of order
//    sqrt(eps) ||R_j|| -- so each provisional rejection is checked with the
//    explicit FP64 residual R_j - sum_c <R_j, Q_c> Q_c over the accepted Q_c that
//    precede it.  The first one found above thr ends the pass there and the
//    exact sequential path resumes at that row; the accepted rows before it stand.
// The accepted rows become Q = L^{-1} R_acc.  Gram, Q and the verification use FP64
// MFMA 16x16x4 (result register r of lane l holds D[4r + l/16][l%16]); the
// factorisation and the triangular inverse are one-wave recurrences in LDS (lane
// i owns row i, resp. column i) that need no workgroup barrier.
__device__ __forceinline__ BqrOut block_qr(const AcceptArgs &a, int nsv, int64_t N0, double *lds, double *cache2, int64_t cslots,
                           double *stat, const double *hn_rows)
{
    const int64_t D = a.D;
    const int ld = gram_ld(nsv);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    double *Gm = lds, *piv = Gm + (int64_t)nsv * ld, *vn = piv + nsv;
    int *acc_idx = reinterpret_cast<int *>(vn + nsv), *rej_idx = acc_idx + nsv, *hrow = rej_idx + nsv;
    double *part = vn + 3 * nsv;  // panel products of the inverse, then per-wave norm partials
    __shared__ int s_u, s_nrej, s_stop, s_resume, s_uk;
    for (int r = threadIdx.x; r < nsv; r += blockDim.x) {
        const int sr = a.rho2 && a.keep ? a.keep[r] : r;  // the caller's survivor order (see sv_of)
        hrow[r] = a.rrow ? a.rrow[sr] : sr;
    }
    __syncthreads();
    auto row = [&](int r) -> const double * { return a.H + (int64_t)hrow[r] * D; };
    // 1. Gram matrix, lower 16 x 16 tiles (I >= J), one tile per wave.  The survivor rows are
    // staged through LDS in chunks of 64 columns with coalesced loads (the next chunk is
    // fetched into registers while the current one is multiplied); without room for the
    // stage the tiles read global memory directly.
    const int T16 = (nsv + 15) / 16;
    const int ntile = T16 * (T16 + 1) / 2;  // <= 10 <= nw
    int tI = 0, tJ = w;
    while (tJ > tI) {
        tJ -= tI + 1;
        ++tI;
    }
    constexpr int KC = 64, KS = KC + 1;
    if (cslots * D >= (int64_t)nsv * KS) {
        double *stage = cache2;
        const int per = (nsv * KC + blockDim.x - 1) / blockDim.x;  // <= 4
        double nxt[4];
        auto fetch = [&](int64_t k0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = threadIdx.x + q * blockDim.x;
                const int r = e / KC, c = e % KC;
                nxt[q] = (q < per && r < nsv && k0 + c < D) ? row(r)[k0 + c] : 0.0;
            }
        };
        fetch(0);
        f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
        for (int64_t k0 = 0; k0 < D; k0 += KC) {
            __syncthreads();  // the previous chunk has been consumed
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = threadIdx.x + q * blockDim.x;
                if (q < per && e < nsv * KC)
                    stage[(e / KC) * KS + e % KC] = nxt[q];
            }
            __syncthreads();
            if (k0 + KC < D)
                fetch(k0 + KC);
            if (w < ntile) {
                const int ia = tI * 16 + (lane & 15), ib = tJ * 16 + (lane & 15);
#pragma unroll
                for (int q = 0; q < KC / 4; ++q) {
                    const int k = 4 * q + (lane >> 4);
                    const double av = ia < nsv ? stage[ia * KS + k] : 0.0;
                    const double bv = ib < nsv ? stage[ib * KS + k] : 0.0;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
                }
            }
        }
        if (w < ntile) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = tI * 16 + 4 * r + (lane >> 4), j = tJ * 16 + (lane & 15);
                if (i < nsv && j <= i)
                    Gm[i * ld + j] = acc[r];
            }
        }
    } else if (w < ntile) {
        const int ia = tI * 16 + (lane & 15), ib = tJ * 16 + (lane & 15);
        const f64x4_t acc = dot_tile_f64(ia < nsv ? row(ia) : nullptr, ib < nsv ? row(ib) : nullptr, D, lane);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = tI * 16 + 4 * r + (lane >> 4), j = tJ * 16 + (lane & 15);
            if (i < nsv && j <= i)
                Gm[i * ld + j] = acc[r];
        }
    }
    __syncthreads();
    if (w == 0) {
        // 2. Cholesky with skipping in candidate order, one wave, panels of 16 candidate
        // columns.  Panel update (left-looking, MFMA): S = G[:, panel] - L[:, :u] L[panel, :u]^T
        // for the rows not yet decided, written back over G.  Panel steps: lane i holds its 16
        // panel values of S in registers; the pivot of row j is lane j's value, and an accepted
        // column's entries are broadcast with readlane for the rank-1 update of the panel.
        // Column c of the compact factor L is stored over column c <= j of G (already consumed).
        const int i = lane;
        const double nrm = i < nsv ? sqrt(Gm[i * ld + i]) : 0.0;
        int u = 0, nrej = 0, stop = nsv;
        bool halt = false;
        int accreg = 0;        // lane r: row index of the r-th accepted survivor
        double pinvreg = 1.0;  // lane r: reciprocal of its pivot
        for (int jb = 0; jb < nsv && !halt; jb += 16) {
            if (u > 0) {
                for (int I = jb / 16; I < T16; ++I) {
                    const int ia = I * 16 + (lane & 15), ib = jb + (lane & 15);
                    f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
                    for (int k0 = 0; k0 < u; k0 += 16) {
                        double av[4], bv[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int k = k0 + 4 * q + (lane >> 4);
                            av[q] = (ia < nsv && k < u) ? Gm[ia * ld + k] : 0.0;
                            bv[q] = (ib < nsv && k < u) ? Gm[ib * ld + k] : 0.0;
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[q], acc, 0, 0, 0);
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = I * 16 + 4 * r + (lane >> 4), col = jb + (lane & 15);
                        if (row < nsv && col <= row)
                            Gm[row * ld + col] -= acc[r];
                    }
                }
                wave_order();
            }
            double sv[16];
#pragma unroll
            for (int t = 0; t < 16; ++t)
                sv[t] = (i < nsv && jb + t <= i) ? Gm[i * ld + jb + t] : 0.0;
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const int j = jb + t;
                if (!halt && j < nsv) {
                    const double dj = lane_bcast(sv[t], j);
                    const double nj = lane_bcast(nrm, j);
                    // 1/sqrt(dj) from the hardware estimate and two Newton steps (quadratic
                    // convergence from ~2^-22 to working precision); rr = dj / sqrt(dj)
                    const bool pos = dj > 1e-200;
                    double rinv = 0.0;
                    if (pos) {
                        double y = __builtin_amdgcn_rsq(dj);
                        y = y * (1.5 - 0.5 * dj * y * y);
                        y = y * (1.5 - 0.5 * dj * y * y);
                        rinv = y;
                    }
                    const double rr = dj * rinv;
                    const bool room = N0 + u < a.ambient && N0 + u < a.cap;
                    const double thr_j = a.rel ? a.tol * hn_rows[j] : a.tol;  // decision threshold of row j
                    if (!isfinite(dj) || !isfinite(nj)) {
                        stop = j;  // the exact path reports the non-finite residual
                        halt = true;
                    } else if (room && pos && rr >= 0.1 * nj && rr >= 10.0 * thr_j) {
                        const double li = i > j ? sv[t] * rinv : 0.0;
                        if (i > j && i < nsv)
                            Gm[i * ld + u] = li;
                        if (i == u) {
                            accreg = j;
                            pinvreg = rinv;
                        }
                        if (i == 0) {
                            piv[u] = rr;
                            acc_idx[u] = j;
                        }
                        wave_order();
#pragma unroll
                        for (int t2 = t + 1; t2 < 16; ++t2)
                            sv[t2] -= li * lane_bcast(li, jb + t2);
                        ++u;
                        if (a.early_exit && N0 + u >= a.ambient) {
                            stop = j + 1;  // nothing after this row is decided
                            halt = true;
                        }
                    } else {
                        if (i == 0)
                            rej_idx[nrej] = j;
                        ++nrej;
                    }
                }
            }
            wave_order();
        }
        // 3. T = L^{-1} in place of L (row acc_idx[r] of the array holds row r of L, then of T),
        // one wave, panels of 16 rows of T: P = L[panel, :pb] T[:pb, :] (MFMA, into part[]), then
        // a 16-step recurrence with lane c holding column c of the panel rows of T in registers.
        for (int pb = 0; pb < u; pb += 16) {
            if (pb > 0) {
                const int ra = pb + (lane & 15);
                const double *arow = ra < u ? Gm + (int64_t)acc_idx[ra] * ld : nullptr;
                for (int J = 0; J * 16 < pb; ++J) {
                    const int cb = J * 16 + (lane & 15);
                    f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
                    for (int k0 = 0; k0 < pb; k0 += 16) {
                        double av[4], bv[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int k = k0 + 4 * q + (lane >> 4);
                            // row index of accepted k: lane k of accreg (k < pb <= 48)
                            const int rk = __shfl(accreg, k < 64 ? k : 0, 64);
                            av[q] = (arow && k < pb) ? arow[k] : 0.0;
                            bv[q] = (k < pb && cb <= k) ? Gm[rk * ld + cb] : 0.0;
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[q], acc, 0, 0, 0);
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int m = 4 * r + (lane >> 4), c = J * 16 + (lane & 15);
                        if (c < nsv)
                            part[m * nsv + c] = acc[r];
                    }
                }
                wave_order();
            }
            const int c = lane;
            double tv[16];
#pragma unroll
            for (int m = 0; m < 16; ++m)
                tv[m] = (pb > 0 && c < pb && pb + m < u) ? part[m * nsv + c] : 0.0;
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                if (pb + m < u) {
                    // row pb + m of L's diagonal block: uniform LDS addresses (broadcast reads)
                    const double *lrow = Gm + (int64_t)acc_idx[pb + m] * ld + pb;
                    double acc = tv[m];
#pragma unroll
                    for (int m2 = 0; m2 < m; ++m2)
                        acc += lrow[m2] * tv[m2];
                    const double pinv = lane_bcast(pinvreg, pb + m);
                    tv[m] = c == pb + m ? pinv : (c < pb + m ? -acc * pinv : 0.0);
                }
            }
            wave_order();
#pragma unroll
            for (int m = 0; m < 16; ++m)
                if (pb + m < u && c <= pb + m)
                    Gm[(int64_t)acc_idx[pb + m] * ld + c] = tv[m];
            wave_order();
        }
        if (lane == 0) {
            s_u = u;
            s_nrej = nrej;
            s_stop = stop;
        }
    }
    __syncthreads();
    const int u = s_u, nrej = s_nrej, stop = s_stop;
    // 4. Q = T R_acc, written as V[N0 + r] (FP64), its FP32 rounding, and the LDS cache.
    // Wave w takes the 16-column tiles J = w, w + nw, ...: the R values of a column tile
    // are loaded once (all at once) and serve every 16-row tile of Q.
    const int64_t JT = (D + 15) / 16;
    const int IT = (u + 15) / 16;
    for (int64_t J = w; J < JT && u > 0; J += nw) {
        const int64_t jc = J * 16 + (lane & 15);
        double bv[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int k = 4 * q + (lane >> 4);
            bv[q] = (k < u && jc < D) ? row(acc_idx[k])[jc] : 0.0;
        }
        for (int I = 0; I < IT; ++I) {
            const int iq = I * 16 + (lane & 15);
            const double *trow = iq < u ? Gm + (int64_t)acc_idx[iq] * ld : nullptr;
            f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                if (4 * q < u) {
                    const int k = 4 * q + (lane >> 4);
                    const double av = (trow && k <= iq) ? trow[k] : 0.0;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[q], acc, 0, 0, 0);
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = I * 16 + 4 * r + (lane >> 4);
                if (i < u && jc < D) {
                    a.V[(N0 + i) * D + jc] = acc[r];
                    if (a.Vs)
                        a.Vs[(N0 + i) * D + jc] = (float)acc[r];
                    if (i < cslots)
                        cache2[(int64_t)i * D + jc] = acc[r];
                }
            }
        }
    }
    __syncthreads();  // Q is complete (global and LDS); T is no longer needed
    // 5. explicit residual norms of the provisional rejections, ||R_rej - C Q|| without storing
    // it.  The coefficients need no pass of their own: for a row i that was not accepted, the
    // factor entry L[i][c] of every accepted c before it (acc_idx[c] < i) is <R_i, Q_c>, and
    // the recurrence left it in row i of the array (the inverse overwrote accepted rows only).
    auto qrow = [&](int c) -> const double * { return c < cslots ? cache2 + (int64_t)c * D : a.V + (N0 + c) * D; };
    if (nrej > 0) {
        // wave w takes the column tiles J = w, w + nw, ... in a fixed order (the Q values of a
        // column tile are loaded once for all rejected rows); the per-wave partial sums are
        // added in wave order, so the result is deterministic
        const int RT = (nrej + 15) / 16;  // <= 4
        double sq[4][4] = {};
        for (int64_t J = w; J < JT; J += nw) {
            const int64_t jc = J * 16 + (lane & 15);
            double bq[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int k = 4 * q + (lane >> 4);
                bq[q] = (k < u && jc < D) ? qrow(k)[jc] : 0.0;
            }
#pragma unroll
            for (int I = 0; I < 4; ++I) {
                if (I < RT) {
                    const int ir = I * 16 + (lane & 15);
                    f64x4_t acc;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = I * 16 + 4 * r + (lane >> 4);
                        acc[r] = (i < nrej && jc < D) ? row(rej_idx[i])[jc] : 0.0;
                    }
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        if (4 * q < u) {
                            const int k = 4 * q + (lane >> 4);
                            const double av =
                                (ir < nrej && k < u && acc_idx[k] < rej_idx[ir]) ? -Gm[rej_idx[ir] * ld + k] : 0.0;
                            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bq[q], acc, 0, 0, 0);
                        }
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        sq[I][r] += acc[r] * acc[r];
                }
            }
        }
#pragma unroll
        for (int I = 0; I < 4; ++I) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double v = sq[I][r];
                for (int off = 1; off < 16; off <<= 1)
                    v += __shfl_xor(v, off, 64);
                const int i = I * 16 + 4 * r + (lane >> 4);
                if ((lane & 15) == 0 && i < nrej)
                    part[w * nsv + i] = v;
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nrej; i += blockDim.x) {
            double t = 0.0;
            for (int q = 0; q < nw; ++q)
                t += part[q * nsv + i];
            vn[i] = sqrt(t);
        }
        __syncthreads();
    }
    // 6. the first provisional rejection above the threshold (or non-finite) ends the pass
    if (threadIdx.x == 0) {
        int resume = stop, uk = u;
        for (int q = 0; q < nrej; ++q) {
            const double v = vn[q];
            if (!(v <= (a.rel ? a.tol * hn_rows[rej_idx[q]] : a.tol))) {
                resume = rej_idx[q];
                break;
            }
        }
        if (resume < stop) {
            uk = 0;
            while (uk < u && acc_idx[uk] < resume)
                ++uk;
        }
        // statistics of the rows decided here: [0] max rejected residual, [1] min accepted
        double mr = 0.0, ma = INFINITY;
        for (int q = 0; q < nrej && rej_idx[q] < resume; ++q)
            mr = fmax(mr, vn[q]);
        for (int q = 0; q < uk; ++q)
            ma = fmin(ma, piv[q]);
        stat[0] = mr;
        stat[1] = ma;
        s_resume = resume;
        s_uk = uk;
        if (a.elem_src)  // Algorithm 3: the source pair of each element appended here
            for (int c = 0; c < uk; ++c) {
                const int sr = a.rho2 && a.keep ? a.keep[acc_idx[c]] : acc_idx[c];
                a.elem_src[N0 + c] = a.surv_pairs ? a.surv_pairs[sr] : -1;
            }
    }
    __syncthreads();
    return BqrOut{s_resume, s_uk};
}

// Dynamic LDS layout of the acceptance kernel: coef[cnt] | R[D] | slots x D
// cached copies of the vectors appended earlier in the block (the rest are
// read from the basis in global memory).
__device__ __forceinline__ void accept_body(const AcceptArgs &a)
{
    extern __shared__ double dyn[];
    __shared__ double red[16];
    __shared__ int64_t sN;
    __shared__ int stop, verdict, ns;
    __shared__ double rr_s;
    __shared__ unsigned long long s_cnt[4];  // zero, screen_rej, fp64_rej, nonfinite
    __shared__ double s_max[2];              // max rejected FP64 residual, max screen-rejected residual
    __shared__ unsigned long long wa_cnt[16][4];  // phase A per-wave counts and maxima
    __shared__ double wa_max[16][2];
    __shared__ double gacc[1024];            // per-group partial sums of the in-block subtraction (G * D <= 1024)
    DevState *st = a.st;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int64_t D = a.D;
    double *coef = dyn;
    double *R = dyn + a.cnt;
    double *cache = R + D;
    const int64_t slots = a.lds_doubles > a.cnt + D ? (a.lds_doubles - a.cnt - D) / D : 0;
    // The state as this launch finds it, read once (all loads in flight together): the
    // statistics are then written back as plain stores of this copy plus the launch's
    // counts, instead of read-modify-write chains on global memory.  Nothing else writes
    // the state while the launch runs.
    __shared__ DevState s0;
    if (threadIdx.x == 0) {
        s0 = *st;
        ns = a.nsurv ? *a.nsurv : 0;
        sN = s0.N;
        stop = s0.done | s0.numeric_error | s0.full;
        if (a.elem_src || a.track_new)
            st->raw_lo = sN;  // the rows appended by this launch start here
        for (int i = 0; i < 4; ++i)
            s_cnt[i] = 0;
        s_max[0] = s_max[1] = 0.0;
    }
    __syncthreads();
    if (stop)
        return;
    // ---- phase A
    {
        unsigned long long k0 = 0, k1 = 0, k2 = 0, k3 = 0;
        double m0 = 0.0, m1 = 0.0;
        for (int c = threadIdx.x; c < a.cnt; c += blockDim.x) {
            if (a.slot[c] >= 0)
                continue;
            const double r = sqrt(a.cand_a2[c]), h = sqrt(a.cand_n2[c]);
            if (!isfinite(r) || !isfinite(h)) {
                ++k3;
            } else if (h == 0.0) {
                ++k0;
            } else if (a.screened) {
                ++k1;
                m1 = fmax(m1, r);
            } else {
                ++k2;
                m0 = fmax(m0, r);
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            k0 += __shfl_down(k0, off, 64);
            k1 += __shfl_down(k1, off, 64);
            k2 += __shfl_down(k2, off, 64);
            k3 += __shfl_down(k3, off, 64);
            m0 = fmax(m0, __shfl_down(m0, off, 64));
            m1 = fmax(m1, __shfl_down(m1, off, 64));
        }
        // per-wave slots, combined by thread 0 (atomics from every wave on the same six
        // LDS words serialise)
        if (lane == 0) {
            wa_cnt[w][0] = k0;
            wa_cnt[w][1] = k1;
            wa_cnt[w][2] = k2;
            wa_cnt[w][3] = k3;
            wa_max[w][0] = m0;
            wa_max[w][1] = m1;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q < nw; ++q) {
            for (int i = 0; i < 4; ++i)
                s_cnt[i] += wa_cnt[q][i];
            s_max[0] = fmax(s_max[0], wa_max[q][0]);
            s_max[1] = fmax(s_max[1], wa_max[q][1]);
        }
        if (a.mode == 1) {
            st->n_cand = (s0.n_cand += a.cnt);
            st->n_zero = (s0.n_zero += (int64_t)s_cnt[0]);
            st->n_screen_rej = (s0.n_screen_rej += (int64_t)s_cnt[1]);
            st->n_fp64 = (s0.n_fp64 += (int64_t)s_cnt[2]);
            st->max_rej = (s0.max_rej = fmax(s0.max_rej, s_max[0]));
            st->max_screen_rej = (s0.max_screen_rej = fmax(s0.max_screen_rej, s_max[1]));
        }
        if (s_cnt[3])
            st->numeric_error = 1;
        stop = s_cnt[3] != 0;
    }
    __syncthreads();
    if (stop)
        return;
    // ---- phase B
    const int64_t N0 = sN;
    __shared__ int64_t l_fp64, l_zero, l_acc, l_gen;
    __shared__ double l_maxrej, l_minacc, l_sdep, l_sind;
    if (threadIdx.x == 0) {
        l_fp64 = l_zero = l_acc = l_gen = 0;
        l_maxrej = 0.0;
        l_minacc = INFINITY;
        l_sdep = 0.0;
        l_sind = INFINITY;
    }
    // Snapshot rejections, in parallel: a survivor whose FP64 residual against the block's
    // basis snapshot is already at or below the threshold stays dependent on every superset
    // of that basis, so it is rejected here; the others (their survivor indices in order)
    // go to a.keep and on to the in-block decisions.
    int nsv = ns;
    const bool use_keep = a.rho2 && a.keep && ns > 0;
    if (use_keep) {
        __shared__ int s_wcnt[16];
        __shared__ int s_base;
        if (threadIdx.x == 0)
            s_base = 0;
        unsigned long long krej = 0;
        double kmax = 0.0, kdep = 0.0;
        for (int r0 = 0; r0 < ns; r0 += blockDim.x) {
            const int r = r0 + threadIdx.x;
            bool kp = false;
            if (r < ns) {
                const int c = a.surv_cand[r];
                const double hn = sqrt(a.h2 ? a.h2[r] : a.cand_n2[c]);
                const double snap = sqrt(a.rho2[r]);
                const double thr = (a.mode == 0 || a.rel) ? a.tol * hn : a.tol;
                const bool rej = snap <= thr && hn > 0.0 && isfinite(hn);  // NaN: left to the exact path
                kp = !rej;
                if (rej && a.mode == 1) {
                    ++krej;
                    kmax = fmax(kmax, snap);
                    kdep = fmax(kdep, sqrt(a.cand_a2[c]));
                }
            }
            const unsigned long long bal = __ballot(kp);
            const int wpre = __popcll(bal & ((1ull << lane) - 1ull));
            __syncthreads();  // s_base and s_wcnt of the previous chunk are settled
            if (lane == 0)
                s_wcnt[w] = __popcll(bal);
            __syncthreads();
            int off = s_base;
            for (int q = 0; q < w; ++q)
                off += s_wcnt[q];
            if (kp)
                a.keep[off + wpre] = r;
            __syncthreads();
            if (threadIdx.x == 0) {
                int t = 0;
                for (int q = 0; q < nw; ++q)
                    t += s_wcnt[q];
                s_base += t;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            krej += __shfl_down(krej, off, 64);
            kmax = fmax(kmax, __shfl_down(kmax, off, 64));
            kdep = fmax(kdep, __shfl_down(kdep, off, 64));
        }
        if (lane == 0 && krej) {
            atomicAdd((unsigned long long *)&l_fp64, krej);
            atomic_max_pos(&l_maxrej, kmax);
            atomic_max_pos(&l_sdep, kdep);
        }
        __syncthreads();
        nsv = s_base;
    }
    // survivor index of the k-th survivor left to decide
    auto sv_of = [&](int k) -> int { return use_keep ? a.keep[k] : k; };
    // per-survivor scalars go to LDS first, counters stay in LDS until the end,
    // and the next survivor's residual is prefetched into registers
    double *hn_a = cache, *rs_a = hn_a + nsv, *sn_a = rs_a + nsv;
    double *cache2 = sn_a + nsv;
    const int64_t slots2 = slots > 0 ? std::max<int64_t>(0, (slots * D - 3 * (int64_t)nsv) / D) : 0;
    const bool meta_in_lds = slots * D >= 3 * (int64_t)nsv;
    for (int k = threadIdx.x; k < nsv && meta_in_lds; k += blockDim.x) {
        const int r = sv_of(k);
        const int c = a.surv_cand[r];
        hn_a[k] = sqrt(a.h2 ? a.h2[r] : a.cand_n2[c]);
        rs_a[k] = sqrt(a.cand_a2[c]);
        sn_a[k] = a.rho2 ? sqrt(a.rho2[r]) : -1.0;
    }
    __syncthreads();
    // block Cholesky-QR pass over the survivors (brackets only, at most 64 survivors)
    const int64_t gram_need = bqr_lds(nsv, nw);
    const bool gram_ok = a.mode == 1 && nsv >= 2 && nsv <= 64 && nw >= 16 && meta_in_lds &&
                         slots * D - 3 * (int64_t)nsv >= gram_need;
    double *gram_base = cache2;
    if (gram_ok)
        cache2 = gram_base + gram_need;
    const int64_t slots3 =
        gram_ok ? std::max<int64_t>(0, (slots * D - 3 * (int64_t)nsv - gram_need) / D) : slots2;
    double *cbase = meta_in_lds ? cache2 : cache;
    const int64_t cslots = meta_in_lds ? slots3 : slots;
    int r_first = 0;
    if (gram_ok) {
        __shared__ double bstat[2];
        const BqrOut b = block_qr(a, nsv, N0, gram_base, cache2, cslots, bstat, hn_a);
        if (threadIdx.x == 0) {
            // rows 0 .. resume-1 are decided: b.u accepted, the rest rejected
            for (int r = 0; r < b.resume; ++r) {
                const double thr = a.rel ? a.tol * hn_a[r] : a.tol;
                if (sn_a[r] >= 0.0) {
                    if (sn_a[r] > thr)
                        l_sind = fmin(l_sind, rs_a[r]);
                    else
                        l_sdep = fmax(l_sdep, rs_a[r]);
                }
            }
            l_fp64 += b.resume;
            l_acc += b.u;
            l_maxrej = fmax(l_maxrej, bstat[0]);
            l_minacc = fmin(l_minacc, bstat[1]);
            st->n_bqr = (s0.n_bqr += b.u);
            sN = N0 + b.u;
            if (a.early_exit && sN >= a.ambient)
                st->done = 1;
        }
        __syncthreads();
        r_first = b.resume;
        if (a.early_exit && sN >= a.ambient)
            r_first = nsv;  // nothing more to decide
    }
    constexpr int PF = 16;  // residual elements prefetched per thread (D <= 16 * blockDim)
    double pf[PF];
    auto row_of = [&](int k) -> const double * {
        const int r = sv_of(k);
        return a.H + (int64_t)(a.rrow ? a.rrow[r] : r) * D;
    };
    if (r_first < nsv) {
        const double *Rg = row_of(r_first);
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int64_t j = threadIdx.x + (int64_t)k * blockDim.x;
            pf[k] = j < D ? Rg[j] : 0.0;
        }
    }
    // thread layout of the in-block subtraction: for D <= 256, G groups of D threads,
    // thread (g, j) owns column j and sums the in-block vectors q = g, g + G, ...;
    // the G partial sums of a column meet in gacc.  Larger D: one group.
    const int G = D <= 256 ? (int)std::min<int64_t>(16, blockDim.x / D) : 1;
    const int gid = G > 1 ? (int)(threadIdx.x / D) : 0;
    const int64_t gt = G > 1 ? (int64_t)(threadIdx.x % D) : 0;
    for (int r = r_first; r < nsv; ++r) {
        lds_barrier();  // everyone has read the previous survivor's verdict and R
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int64_t j = threadIdx.x + (int64_t)k * blockDim.x;
            if (j < D)
                R[j] = pf[k];
        }
        if (r + 1 < nsv) {
            const double *Rg = row_of(r + 1);
#pragma unroll
            for (int k = 0; k < PF; ++k) {
                const int64_t j = threadIdx.x + (int64_t)k * blockDim.x;
                pf[k] = j < D ? Rg[j] : 0.0;
            }
        }
        double hn, rs, snap;
        if (meta_in_lds) {
            hn = hn_a[r];
            rs = rs_a[r];
            snap = sn_a[r];
        } else {
            const int sr = sv_of(r);
            const int c = a.surv_cand[sr];
            hn = sqrt(a.h2 ? a.h2[sr] : a.cand_n2[c]);
            rs = sqrt(a.cand_a2[c]);
            snap = a.rho2 ? sqrt(a.rho2[sr]) : -1.0;
        }
        const double thr = (a.mode == 0 || a.rel) ? a.tol * hn : a.tol;
        if (threadIdx.x == 0 && a.mode == 1 && snap >= 0.0) {
            // audit against the same basis snapshot the screen used
            if (snap > thr)
                l_sind = fmin(l_sind, rs);
            else
                l_sdep = fmax(l_sdep, rs);
        }
        const int64_t A = sN - N0;
        const int64_t AL = A < cslots ? A : cslots;
        double nrm2 = -1.0;  // squared norm of R after the last pass (block-wide, valid in every thread)
        lds_barrier();       // R is complete
        if (A == 0) {
            double loc = 0.0;
            for (int64_t j = threadIdx.x; j < D; j += blockDim.x)
                loc += R[j] * R[j];
            loc = wave_sum(loc);
            if (lane == 0)
                red[w] = loc;
            lds_barrier();
            double t = 0.0;
            for (int i = 0; i < nw; ++i)
                t += red[i];
            nrm2 = t;
        }
        // orthogonalise against the elements appended earlier in this block: one pass,
        // and a second one only if the first removed more than a 1/sqrt(2) fraction of the norm
        double before2 = snap >= 0.0 ? snap * snap : -1.0;
        for (int pass = 0; pass < 2 && A > 0; ++pass) {
            for (int64_t q = w; q < A; q += nw) {
                double sdot = 0.0;
                if (q < AL) {
                    const double *va = cbase + q * D;
                    for (int64_t j = lane; j < D; j += 64)
                        sdot += va[j] * R[j];
                } else {
                    const double *va = a.V + (N0 + q) * D;
                    for (int64_t j = lane; j < D; j += 64)
                        sdot += va[j] * R[j];
                }
                sdot = wave_sum(sdot);
                if (lane == 0)
                    coef[q] = sdot;
            }
            lds_barrier();
            double loc = 0.0;
            if (G > 1) {
                if (gid < G) {
                    double s0 = 0.0;
                    int64_t q = gid;
                    for (; q < AL; q += G)
                        s0 += coef[q] * cbase[q * D + gt];
                    for (; q < A; q += G)
                        s0 += coef[q] * a.V[(N0 + q) * D + gt];
                    gacc[gid * D + gt] = s0;
                }
                lds_barrier();
                for (int64_t j = threadIdx.x; j < D; j += blockDim.x) {
                    double t = 0.0;
                    for (int g2 = 0; g2 < G; ++g2)
                        t += gacc[g2 * D + j];
                    const double v = R[j] - t;
                    R[j] = v;
                    loc += v * v;
                }
            } else {
                for (int64_t j = threadIdx.x; j < D; j += blockDim.x) {
                    double s0 = 0.0, s1 = 0.0;
                    int64_t q = 0;
                    for (; q + 2 <= AL; q += 2) {
                        s0 += coef[q] * cbase[q * D + j];
                        s1 += coef[q + 1] * cbase[(q + 1) * D + j];
                    }
                    if (q < AL) {
                        s0 += coef[q] * cbase[q * D + j];
                        ++q;
                    }
                    const double *vg = a.V + N0 * D;
                    for (; q < A; ++q)
                        s1 += coef[q] * vg[q * D + j];
                    const double v = R[j] - (s0 + s1);
                    R[j] = v;
                    loc += v * v;
                }
            }
            loc = wave_sum(loc);
            if (lane == 0)
                red[w] = loc;
            lds_barrier();
            double t = 0.0;
            for (int i = 0; i < nw; ++i)
                t += red[i];
            nrm2 = t;
            if (before2 >= 0.0 && nrm2 > 0.5 * before2)
                break;  // little was removed: the vector is already orthogonal to working precision
            before2 = nrm2;
            lds_barrier();  // red[] and coef[] are reused by the second pass
        }
        if (threadIdx.x == 0) {
            const double rr = sqrt(nrm2);
            rr_s = rr;
            verdict = 1;
            if (a.mode == 1)
                l_fp64++;
            if (!isfinite(rr) || !isfinite(hn)) {
                st->numeric_error = 1;
                verdict = -1;
            } else if (hn == 0.0 || !(rr > thr)) {
                if (a.mode == 1) {
                    if (hn == 0.0)
                        l_zero++;
                    l_maxrej = fmax(l_maxrej, rr);
                }
                verdict = 0;
            } else if (a.mode == 1 && sN >= a.ambient) {
                st->numeric_error = 2;  // one more independent element than the space holds
                verdict = -1;
            } else if (sN >= a.cap) {
                st->full = 1;
                verdict = -1;
            }
        }
        lds_barrier();
        if (verdict < 0)
            break;
        if (verdict == 0)
            continue;
        const double inv = 1.0 / rr_s;
        const int64_t q_new = sN - N0;
        double *dst = a.V + sN * D;
        double *dstc = q_new < cslots ? cbase + q_new * D : nullptr;
        float *dsts = a.Vs ? a.Vs + sN * D : nullptr;
        for (int64_t j = threadIdx.x; j < D; j += blockDim.x) {
            const double v = R[j] * inv;
            dst[j] = v;
            if (dstc)
                dstc[j] = v;
            if (dsts)
                dsts[j] = (float)v;
        }
        // the appended vector is complete before sN moves; a vector that is not cached
        // in LDS is read back from global memory later, so its stores must be visible
        if (dstc)
            lds_barrier();
        else
            __syncthreads();
        if (threadIdx.x == 0) {
            if (a.elem_src)
                a.elem_src[sN] = a.mode == 0 ? a.src0 : (a.surv_pairs ? a.surv_pairs[sv_of(r)] : -1);
            sN++;
            if (a.mode == 1) {
                l_acc++;
                l_minacc = fmin(l_minacc, rr_s);
            } else {
                l_gen++;
            }
            if (a.early_exit && sN >= a.ambient)
                st->done = 1;
        }
        lds_barrier();
        if (a.early_exit && sN >= a.ambient)
            break;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st->n_rows = s0.n_rows + nsv;
        st->n_fp64 = s0.n_fp64 + l_fp64;
        st->n_zero = s0.n_zero + l_zero;
        st->n_acc = s0.n_acc + l_acc;
        st->n_gen_acc = s0.n_gen_acc + l_gen;
        st->max_rej = fmax(s0.max_rej, l_maxrej);
        st->min_acc = fmin(s0.min_acc, l_minacc);
        st->scr_max_dep = fmax(s0.scr_max_dep, l_sdep);
        st->scr_min_indep = fmin(s0.scr_min_indep, l_sind);
        st->N = sN;
    }
}

__global__ void __launch_bounds__(kAccThreads) k_accept_f64(AcceptArgs a) { accept_body(a); }
__global__ void __launch_bounds__(kAccThreads) k_accept_b(Batch b)
{
    const AcceptArgs a = static_cast<const AcceptArgs *>(b.args)[blockIdx.x];
    accept_body(a);
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

static hipError_t grant_lds(const void *fn, size_t bytes, size_t &granted)
{
    if (bytes <= granted)
        return hipSuccess;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess)
        granted = bytes;
    return e;
}

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

hipError_t launch_accept_batched(const Batch &b, int64_t lds_doubles, hipStream_t s)
{
    if (b.nprob <= 0)
        return hipSuccess;
    static size_t granted = 65536;
    const size_t bytes = (size_t)lds_doubles * sizeof(double);
    hipError_t e = grant_lds((const void *)k_accept_b, bytes, granted);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_accept_b, dim3(b.nprob), dim3(kAccThreads), bytes, s, b);
    return hipGetLastError();
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

// Dynamic LDS of the acceptance kernel: coefficients and the residual always,
// plus as many cached in-block vectors as fit below the device limit.
static int64_t accept_lds_avail()
{
    static int64_t avail = -1;
    if (avail < 0) {
        int dev = 0, v = 65536;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            v = 65536;
        // the dynamic part shares the limit with the kernel's static LDS
        hipFuncAttributes fa{};
        size_t static_bytes = 16384;
        if (hipFuncGetAttributes(&fa, (const void *)k_accept_f64) == hipSuccess)
            static_bytes = fa.sharedSizeBytes + 256;
        else
            (void)hipGetLastError();
        avail = ((int64_t)v - (int64_t)static_bytes) / (int64_t)sizeof(double);
    }
    return avail;
}

int64_t accept_lds_doubles(int cnt, int64_t D)
{
    const int64_t need = cnt + D + (int64_t)cnt * D;
    return std::max<int64_t>(cnt + D, std::min(accept_lds_avail(), need));
}

int accept_max_block(int64_t D) { return (int)std::max<int64_t>(0, std::min<int64_t>(kMaxBlock, accept_lds_avail() - D)); }


hipError_t launch_accept_f64(const AcceptArgs &args, hipStream_t s)
{
    if (args.cnt <= 0)
        return hipSuccess;
    if (args.cnt > kMaxBlock)
        return hipErrorInvalidValue;
    static size_t granted = 65536;
    const size_t bytes = (size_t)args.lds_doubles * sizeof(double);
    hipError_t e = grant_lds((const void *)k_accept_f64, bytes, granted);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_accept_f64, dim3(1), dim3(kAccThreads), bytes, s, args);
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

}  // namespace lie

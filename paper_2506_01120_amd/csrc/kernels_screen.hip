// Screening kernels: the bracket and the projection residual of a candidate
// block in FP32 on the matrix cores (MFMA, FP32 accumulation), and the
// classification / compaction step shared by every precision.
//
// Operators use the packed anti-Hermitian layout of lie_internal.h (d^2 reals,
// Euclidean dot = the paper's inner product); the FP32 shadow basis Vs holds
// the FP32 rounding of the FP64 basis row by row.
#include "lie_internal.h"

#include <algorithm>
#include <cmath>

namespace lie {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;

__device__ inline bool aborted(const DevState *st) { return st->done | st->numeric_error | st->full; }

__device__ inline float wave_sum_f(float v)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

// ------------------------------------------------------------------ bracket (FP32 MFMA)
//
// Same algebra as the FP64 bracket: A = sqrt(d/2)(Ar + i Ai) read from the packed
// array, P = (Ar + i Ai)(Br + i Bi) on the matrix cores as four real products
// (16x16x4 f32 tiles, operands zero-padded to a multiple of 16), then the packed
// bracket sqrt(d/2)(P - P^H) with diagonal sqrt(d) Im P_ii, and the squared norm of
// the output row.  d <= 64 here; larger operators go to the tile-pair kernel.

// ---- gathered variant (d <= 64): the two packed operands are copied into LDS with
// coalesced loads (row stride d + 1 against bank conflicts) and each MFMA operand is
// gathered from there -- entry (i, k) of Ar and Ai both come from p[i][k] and p[k][i],
// so no unpacked copies are written.  P then reuses the LDS to be read transposed.
// FP32 16x16x4: lane l supplies A[l%16][k0 + l/16] and B[k0 + l/16][l%16]; result
// register r of lane l is P[4(l/16) + r][l%16].
struct RawF {
    float x, y;
};
// (x, y) = (S[i][k], S[k][i]) of a staged operand with row stride ls (zero outside d x d).
__device__ inline RawF raw_load(const float *S, int ls, int d, int i, int k)
{
    const bool in = i < d && k < d;
    const int ic = in ? i : 0, kc = in ? k : 0;
    return RawF{S[ic * ls + kc], S[kc * ls + ic]};
}
__device__ inline void raw_frag(RawF v, int d, int i, int k, float &ar, float &ai)
{
    const bool in = i < d && k < d;
    ar = !in || i == k ? 0.f : (i < k ? v.x : -v.y);
    ai = !in ? 0.f : (i < k ? v.y : (i > k ? v.x : 1.41421356237309515f * v.x));
}

// Output element e of the packed bracket from P (row stride ld) in LDS.
__device__ inline float bracket_out(const float *Pr, const float *Pi, int ld, int d, int e, float so, float sd)
{
    const int i = e / d, j = e % d;
    if (i < j)
        return so * (Pr[i * ld + j] - Pr[j * ld + i]);
    if (i > j)
        return so * (Pi[j * ld + i] + Pi[i * ld + j]);
    return sd * Pi[i * ld + i];
}

// d <= 16: one wave per candidate, four candidates per workgroup.
__global__ void __launch_bounds__(kThreads) k_comm_f32_reg16(CommArgs A)
{
    __shared__ float Pbuf[4][2][16 * 17];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int c = blockIdx.x * 4 + w;
    if (c >= A.cnt || aborted(A.st))
        return;
    const float *Vs = static_cast<const float *>(A.V);
    const int d = A.d;
    const int64_t D = (int64_t)d * d;
    int64_t l, m;
    decode_pair((A.dp0 ? *A.dp0 : A.p0) + c, l, m);
    float *Sa = Pbuf[w][0], *Sb = Pbuf[w][1];
    {
        const float *pa = Vs + l * D, *pb = Vs + m * D;
        for (int e = lane; e < D; e += 64) {
            const int i = e / d, k = e % d;
            Sa[i * 17 + k] = pa[e];
            Sb[i * 17 + k] = pb[e];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const int lr = lane & 15, lk = lane >> 4;
    RawF ra[4], rb[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        ra[s] = raw_load(Sa, 17, d, lr, 4 * s + lk);
        rb[s] = raw_load(Sb, 17, d, 4 * s + lk, lr);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the tile is read; P may overwrite it
    f32x4 pr = {0.f, 0.f, 0.f, 0.f}, pi = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        float ar, ai, br, bi;
        raw_frag(ra[s], d, lr, 4 * s + lk, ar, ai);
        raw_frag(rb[s], d, 4 * s + lk, lr, br, bi);
        pr = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br, pr, 0, 0, 0);
        pr = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai, bi, pr, 0, 0, 0);
        pi = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, bi, pi, 0, 0, 0);
        pi = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, br, pi, 0, 0, 0);
    }
    float *Pr = Pbuf[w][0], *Pi = Pbuf[w][1];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        Pr[(4 * lk + r) * 17 + lr] = pr[r];
        Pi[(4 * lk + r) * 17 + lr] = pi[r];
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the wave's own LDS writes, read across lanes
    const float so = sqrtf(0.5f * d), sd = sqrtf((float)d);
    float *out = static_cast<float *>(A.H) + (int64_t)c * D;
    float sq = 0.f;
    for (int e = lane; e < D; e += 64) {
        const float v = bracket_out(Pr, Pi, 17, d, e, so, sd);
        if (A.Hp)
            store_plane(A.Hp + (int64_t)c * A.ldp, e, v);
        else
            out[e] = v;
        sq += v * v;
    }
    sq = wave_sum_f(sq);
    if (lane == 0)
        A.hs2[c] = (double)sq;
}

// 16 < d <= 16 T: one workgroup per candidate; wave w owns column block J = w % T and
// row blocks I = w / T, w / T + 4 / T, ...  Dynamic LDS: 2 x 16T x (16T + 1) floats
// (the operands, then P).
template <int T>
__device__ void comm_f32_reg_body(const CommArgs &A, int c)
{
    extern __shared__ float Pl[];
    __shared__ float red[4];
    constexpr int NI = T * T / 4;
    constexpr int ld = 16 * T + 1;
    constexpr int G = T == 2 ? 8 : 4;  // k-steps per load group
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (c >= A.cnt || aborted(A.st))
        return;
    const float *Vs = static_cast<const float *>(A.V);
    const int d = A.d;
    const int64_t D = (int64_t)d * d;
    int64_t l, m;
    decode_pair((A.dp0 ? *A.dp0 : A.p0) + c, l, m);
    const int lo = d + 1;
    float *Sa = Pl, *Sb = Pl + d * lo;
    {
        const float *pa = Vs + l * D, *pb = Vs + m * D;
        for (int64_t e = threadIdx.x; e < D; e += blockDim.x) {
            const int i = (int)(e / d), k = (int)(e % d);
            Sa[i * lo + k] = pa[e];
            Sb[i * lo + k] = pb[e];
        }
    }
    __syncthreads();
    const int lr = lane & 15, lk = lane >> 4;
    const int J = w % T, I0 = w / T;
    f32x4 pr[NI], pi[NI];
#pragma unroll
    for (int q = 0; q < NI; ++q)
        pr[q] = pi[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int g0 = 0; g0 < 4 * T; g0 += G) {
        RawF ra[NI][G], rb[G];
#pragma unroll
        for (int s = 0; s < G; ++s) {
            const int k = 4 * (g0 + s) + lk;
            rb[s] = raw_load(Sb, lo, d, k, 16 * J + lr);
#pragma unroll
            for (int q = 0; q < NI; ++q)
                ra[q][s] = raw_load(Sa, lo, d, 16 * (I0 + q * (4 / T)) + lr, k);
        }
#pragma unroll
        for (int s = 0; s < G; ++s) {
            const int k = 4 * (g0 + s) + lk;
            float br, bi;
            raw_frag(rb[s], d, k, 16 * J + lr, br, bi);
#pragma unroll
            for (int q = 0; q < NI; ++q) {
                float ar, ai;
                raw_frag(ra[q][s], d, 16 * (I0 + q * (4 / T)) + lr, k, ar, ai);
                pr[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br, pr[q], 0, 0, 0);
                pr[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai, bi, pr[q], 0, 0, 0);
                pi[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, bi, pi[q], 0, 0, 0);
                pi[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, br, pi[q], 0, 0, 0);
            }
        }
    }
    __syncthreads();  // the operands are consumed; P takes their place
    float *Pr = Pl, *Pi = Pl + 16 * T * ld;
#pragma unroll
    for (int q = 0; q < NI; ++q) {
        const int I = I0 + q * (4 / T);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Pr[(16 * I + 4 * lk + r) * ld + 16 * J + lr] = pr[q][r];
            Pi[(16 * I + 4 * lk + r) * ld + 16 * J + lr] = pi[q][r];
        }
    }
    __syncthreads();
    const float so = sqrtf(0.5f * d), sd = sqrtf((float)d);
    float *out = static_cast<float *>(A.H) + (int64_t)c * D;
    float sq = 0.f;
    for (int e = threadIdx.x; e < D; e += blockDim.x) {
        const float v = bracket_out(Pr, Pi, ld, d, e, so, sd);
        if (A.Hp)
            store_plane(A.Hp + (int64_t)c * A.ldp, e, v);
        else
            out[e] = v;
        sq += v * v;
    }
    sq = wave_sum_f(sq);
    if (lane == 0)
        red[w] = sq;
    __syncthreads();
    if (threadIdx.x == 0)
        A.hs2[c] = (double)red[0] + red[1] + red[2] + red[3];
}

template <int T>
__global__ void __launch_bounds__(kThreads) k_comm_f32_reg(CommArgs A)
{
    comm_f32_reg_body<T>(A, blockIdx.x);
}

// Grouped form: one workgroup per candidate of any problem with d <= 16 T.
template <int T>
__global__ void __launch_bounds__(kThreads) k_comm_f32_reg_b(Batch b)
{
    const int p = batch_find(b.start, b.nprob, blockIdx.x);
    const CommArgs a = static_cast<const CommArgs *>(b.args)[p];
    comm_f32_reg_body<T>(a, blockIdx.x - b.start[p]);
}

// ------------------------------------------------------------------ classification and compaction
//
// One workgroup of 1024 threads walks the block in chunks of 1024 candidates.
// Survivors are written in candidate order: rows[r] = c, pairs[r] = p0 + c,
// and slot[c] = r (or -1); *nsurv receives their count.
//
// Certified screening (A.certify = 1).  A screened residual carries rounding of
// order 1e-7 (FP32) to 1e-5 (split BF16) of the candidate's scale, far above the
// FP64 threshold tol, so a small screened residual does not prove that the FP64
// residual is at most tol: a direction of the closure that couples only weakly
// screens as small as rounding noise.  What does prove dependence is the basis
// size: once |V| equals the ambient bound (d^2 - 1 for traceless operators,
// d^2 otherwise) V spans every operator a bracket can produce, so every
// candidate is dependent.  With certify set, the policy therefore rejects only
// while st->N >= ambient; there its threshold only separates the candidates
// whose screen looks healthy from those re-checked in FP64.  Below the bound
// every candidate survives to the FP64 decision.
__device__ void classify_body(const ClassifyArgs &A)
{
    const double *a2 = A.a2, *n2 = A.n2;
    const int cnt = A.cnt;
    const int64_t p0 = A.dp0 ? *A.dp0 : A.p0;
    const int policy = A.policy;
    const double thr = A.thr;
    const DevState *st = A.st;
    int *rows = A.rows;
    int64_t *pairs = A.pairs;
    int *slot = A.slot;
    int *nsurv = A.nsurv;
    __shared__ int wcount[16];
    __shared__ int wbase[16];
    __shared__ int running;
    const bool ab = aborted(st);
    const bool below_bound = A.certify && st->N < A.ambient;  // no rejection can be certified yet
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0)
        running = 0;
    __syncthreads();
    for (int c0 = 0; c0 < cnt; c0 += blockDim.x) {
        const int c = c0 + threadIdx.x;
        bool keep = false;
        if (c < cnt && !ab) {
            const double r = sqrt(a2[c]), h = sqrt(n2[c]);
            if (!isfinite(r) || !isfinite(h)) {
                keep = true;  // the acceptance kernel reports the numeric failure
            } else {
                switch (policy) {
                case POL_ALL: keep = true; break;
                case POL_ABS: keep = h > 0.0 && r > thr; break;
                case POL_REL: keep = h > 0.0 && r > thr * h; break;
                case POL_GE: keep = h > 0.0 && r >= thr; break;
                case POL_GE_REL: keep = h > 0.0 && r >= thr * h; break;
                }
                keep = keep || below_bound;
            }
        }
        const unsigned long long mask = __ballot(keep);
        if (lane == 0)
            wcount[w] = __popcll(mask);
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = running;
            for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
                wbase[i] = t;
                t += wcount[i];
            }
            running = t;
        }
        __syncthreads();
        if (c < cnt) {
            if (keep) {
                const int r = wbase[w] + __popcll(mask & ((1ull << lane) - 1ull));
                rows[r] = c;
                pairs[r] = p0 + c;
                slot[c] = r;
            } else {
                slot[c] = -1;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *nsurv = ab ? 0 : running;
}

__global__ void __launch_bounds__(1024) k_classify(ClassifyArgs a) { classify_body(a); }
__global__ void __launch_bounds__(1024) k_classify_b(Batch b)
{
    const ClassifyArgs a = static_cast<const ClassifyArgs *>(b.args)[blockIdx.x];
    classify_body(a);
}

}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t launch_comm_f32(const float *Vs, int d, int64_t p0, int cnt, const DevState *st, float *Hs, double *hs2,
                           hipStream_t s, const int64_t *dp0, __bf16 *Hp, int64_t ldp)
{
    if (cnt <= 0)
        return hipSuccess;
    CommArgs a{Vs, d, p0, nullptr, dp0, nullptr, cnt, st, Hs, hs2, Hp, ldp};
    if (d <= 16)
        hipLaunchKernelGGL(k_comm_f32_reg16, dim3((unsigned)((cnt + 3) / 4)), dim3(kThreads), 0, s, a);
    else if (d <= 32)
        return launch_comm_grouped(a, false, s);
    else if (d <= 64)
        hipLaunchKernelGGL(k_comm_f32_reg<4>, dim3(cnt), dim3(kThreads), (size_t)2 * 64 * 65 * sizeof(float), s, a);
    else
        return launch_comm_pairs(a, false, s);
    return hipGetLastError();
}

bool comm_f32_fits_lds(int d) { return d <= 64; }

hipError_t launch_comm_f32_batched(const Batch &b, bool lds_variant, int dmax, hipStream_t s)
{
    if (b.total <= 0)
        return hipSuccess;
    if (!lds_variant)
        return launch_comm_pairs_batched(b, false, s);
    if (dmax <= 32)
        hipLaunchKernelGGL(k_comm_f32_reg_b<2>, dim3(b.total), dim3(kThreads), (size_t)2 * 32 * 33 * sizeof(float), s,
                           b);
    else
        hipLaunchKernelGGL(k_comm_f32_reg_b<4>, dim3(b.total), dim3(kThreads), (size_t)2 * 64 * 65 * sizeof(float), s,
                           b);
    return hipGetLastError();
}

hipError_t launch_classify(const double *a2, const double *n2, int cnt, int64_t p0, int policy, double thr,
                           const DevState *st, int *rows, int64_t *pairs, int *slot, int *nsurv, hipStream_t s,
                           const int64_t *dp0, int64_t ambient, int certify)
{
    if (cnt <= 0)
        return hipSuccess;
    const int threads = cnt >= 1024 ? 1024 : ((cnt + 63) / 64) * 64;
    ClassifyArgs a{a2, n2, cnt, p0, dp0, policy, thr, st, rows, pairs, slot, nsurv, ambient, certify};
    hipLaunchKernelGGL(k_classify, dim3(1), dim3(threads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_classify_batched(const Batch &b, hipStream_t s)
{
    if (b.nprob <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_classify_b, dim3(b.nprob), dim3(1024), 0, s, b);
    return hipGetLastError();
}

}  // namespace lie

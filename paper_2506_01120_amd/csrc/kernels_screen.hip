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
// Same algebra as the FP64 bracket: A = sqrt(d/2)(Ar + i Ai) read from the
// packed array, P = (Ar + i Ai)(Br + i Bi) on the matrix cores as four real
// products (16x16x4 f32 tiles, operands zero-padded to a multiple of 16),
// then the packed bracket sqrt(d/2)(P - P^H) with diagonal sqrt(d) Im P_ii.
// One workgroup per candidate; operands and P live in LDS (d <= 64).

__global__ void __launch_bounds__(kThreads) k_comm_f32_mfma(const float *__restrict__ Vs, int d, int64_t p0,
                                                            int cnt, const DevState *__restrict__ st,
                                                            float *__restrict__ Hs, double *__restrict__ hs2)
{
    extern __shared__ float smem[];
    const int c = blockIdx.x;
    if (c >= cnt || aborted(st))
        return;
    const int D = d * d;
    const int dp = (d + 15) & ~15;
    const int ld = dp + 1;
    float *Ar = smem, *Ai = Ar + dp * ld, *Br = Ai + dp * ld, *Bi = Br + dp * ld, *Pr = Bi + dp * ld,
          *Pi = Pr + dp * ld;
    __shared__ float red[4];
    int64_t l, m;
    decode_pair(p0 + c, l, m);
    const float *pa = Vs + l * (int64_t)D, *pb = Vs + m * (int64_t)D;
    const float r2 = 1.41421356237309515f;
    for (int idx = threadIdx.x; idx < dp * dp; idx += blockDim.x) {
        const int i = idx / dp, k = idx % dp;
        float ar = 0.f, ai = 0.f, br = 0.f, bi = 0.f;
        if (i < d && k < d) {
            if (i < k) {
                ar = pa[i * d + k];
                ai = pa[k * d + i];
                br = pb[i * d + k];
                bi = pb[k * d + i];
            } else if (i > k) {
                ar = -pa[k * d + i];
                ai = pa[i * d + k];
                br = -pb[k * d + i];
                bi = pb[i * d + k];
            } else {
                ai = r2 * pa[i * d + i];
                bi = r2 * pb[i * d + i];
            }
        }
        Ar[i * ld + k] = ar;
        Ai[i * ld + k] = ai;
        Br[i * ld + k] = br;
        Bi[i * ld + k] = bi;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int T = dp / 16;
    const int lr = lane & 15, lk = lane >> 4;
    for (int t = w; t < 2 * T * T; t += 4) {
        const int part = t / (T * T);  // 0: real part, 1: imaginary part
        const int I = (t % (T * T)) / T, J = t % T;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        const int row = I * 16 + lr, col = J * 16 + lr;
        for (int k0 = 0; k0 < dp; k0 += 4) {
            const int k = k0 + lk;
            const float ar = Ar[row * ld + k], ai = Ai[row * ld + k];
            const float br = Br[k * ld + col], bi = Bi[k * ld + col];
            if (part == 0) {
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai, bi, acc, 0, 0, 0);
            } else {
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, bi, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, br, acc, 0, 0, 0);
            }
        }
        float *P = part == 0 ? Pr : Pi;
        for (int r = 0; r < 4; ++r)
            P[(I * 16 + 4 * lk + r) * ld + J * 16 + lr] = acc[r];
    }
    __syncthreads();
    const float so = sqrtf(0.5f * d), sd = sqrtf((float)d);
    float *out = Hs + (int64_t)c * D;
    float sq = 0.f;
    for (int e = threadIdx.x; e < D; e += blockDim.x) {
        const int i = e / d, j = e % d;
        float v;
        if (i < j)
            v = so * (Pr[i * ld + j] - Pr[j * ld + i]);
        else if (i > j)
            v = so * (Pi[j * ld + i] + Pi[i * ld + j]);
        else
            v = sd * Pi[i * ld + i];
        out[e] = v;
        sq += v * v;
    }
    sq = wave_sum_f(sq);
    if (lane == 0)
        red[w] = sq;
    __syncthreads();
    if (threadIdx.x == 0)
        hs2[c] = (double)red[0] + red[1] + red[2] + red[3];
}

// FP32 bracket straight from global memory, for d beyond the LDS kernel.
__global__ void __launch_bounds__(kThreads) k_comm_f32_global(const float *__restrict__ Vs, int d, int64_t p0,
                                                              int cnt, const DevState *__restrict__ st,
                                                              float *__restrict__ Hs)
{
    const int c = blockIdx.y;
    if (c >= cnt || aborted(st))
        return;
    const int64_t D = (int64_t)d * d;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= D)
        return;
    const int i = (int)(idx / d), j = (int)(idx % d);
    if (i > j)
        return;
    int64_t l, m;
    decode_pair(p0 + c, l, m);
    const float *pa = Vs + l * D, *pb = Vs + m * D;
    auto re = [d](const float *p, int a, int b) { return a < b ? p[a * d + b] : (a > b ? -p[b * d + a] : 0.f); };
    auto im = [d](const float *p, int a, int b) {
        return a < b ? p[b * d + a] : (a > b ? p[a * d + b] : 1.41421356237309515f * p[a * d + a]);
    };
    float prij = 0, piij = 0, prji = 0, piji = 0;
    for (int k = 0; k < d; ++k) {
        const float ar = re(pa, i, k), ai = im(pa, i, k), br = re(pb, k, j), bi = im(pb, k, j);
        prij += ar * br - ai * bi;
        piij += ar * bi + ai * br;
        const float ar2 = re(pa, j, k), ai2 = im(pa, j, k), br2 = re(pb, k, i), bi2 = im(pb, k, i);
        prji += ar2 * br2 - ai2 * bi2;
        piji += ar2 * bi2 + ai2 * br2;
    }
    const float so = sqrtf(0.5f * d), sd = sqrtf((float)d);
    float *out = Hs + (int64_t)c * D;
    if (i < j) {
        out[i * d + j] = so * (prij - prji);
        out[j * d + i] = so * (piij + piji);
    } else {
        out[i * d + i] = sd * piij;
    }
}

__global__ void __launch_bounds__(kThreads) k_rownorm_f32(const float *__restrict__ Hs, int cnt, int64_t D,
                                                          const DevState *__restrict__ st, double *__restrict__ hs2)
{
    __shared__ double red[4];
    const int c = blockIdx.x;
    if (c >= cnt || aborted(st))
        return;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < D; j += blockDim.x) {
        const double v = Hs[(int64_t)c * D + j];
        s += v * v;
    }
    for (int off = 32; off > 0; off >>= 1)
        s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0)
        hs2[c] = red[0] + red[1] + red[2] + red[3];
}

// ------------------------------------------------------------------ projection (FP32 MFMA)
//
// Workgroup tile 64 x 64 of the output, four waves each owning a 32 x 32
// quarter computed with v_mfma_f32_32x32x2_f32; K streamed in chunks of 32
// through LDS.  32x32x2 operand layout: lane l supplies A[l%32][l/32] and
// B[l/32][l%32]; result register r of lane l is D[8(r/4) + 4(l/32) + r%4][l%32].

constexpr int kT = 64;   // output tile edge
constexpr int kKC = 32;  // K chunk

// C[c][k] = <Hs_c, Vs_k> for c < cnt, k < N.
__global__ void __launch_bounds__(kThreads) k_dot_f32_mfma(const float *__restrict__ Vs,
                                                           const DevState *__restrict__ st,
                                                           const float *__restrict__ Hs, int cnt, int64_t D,
                                                           float *__restrict__ C, int64_t ldc)
{
    if (aborted(st))
        return;
    const int64_t N = st->N;
    const int64_t k0 = (int64_t)blockIdx.x * kT;  // basis rows
    const int c0 = blockIdx.y * kT;               // candidates
    if (k0 >= N || c0 >= cnt)
        return;
    __shared__ float As[kT][kKC + 1];  // candidates x K
    __shared__ float Bs[kT][kKC + 1];  // basis rows x K
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w >> 1, wn = w & 1;
    f32x16 acc = {};
    const bool vec4 = (D % 4) == 0;
    for (int64_t j0 = 0; j0 < D; j0 += kKC) {
        // 64 rows x 32 columns per operand: 512 float4, two per thread
        for (int q = threadIdx.x; q < kT * kKC / 4; q += blockDim.x) {
            const int r = q / (kKC / 4), c4 = (q % (kKC / 4)) * 4;
            const int64_t j = j0 + c4;
            float4 a = {0.f, 0.f, 0.f, 0.f}, b = {0.f, 0.f, 0.f, 0.f};
            if (vec4 && j + 3 < D) {
                if (c0 + r < cnt)
                    a = *reinterpret_cast<const float4 *>(Hs + (int64_t)(c0 + r) * D + j);
                if (k0 + r < N)
                    b = *reinterpret_cast<const float4 *>(Vs + (k0 + r) * D + j);
            } else {
                float ta[4] = {0.f, 0.f, 0.f, 0.f}, tb[4] = {0.f, 0.f, 0.f, 0.f};
                for (int u = 0; u < 4; ++u)
                    if (j + u < D) {
                        if (c0 + r < cnt)
                            ta[u] = Hs[(int64_t)(c0 + r) * D + j + u];
                        if (k0 + r < N)
                            tb[u] = Vs[(k0 + r) * D + j + u];
                    }
                a = {ta[0], ta[1], ta[2], ta[3]};
                b = {tb[0], tb[1], tb[2], tb[3]};
            }
            As[r][c4] = a.x;
            As[r][c4 + 1] = a.y;
            As[r][c4 + 2] = a.z;
            As[r][c4 + 3] = a.w;
            Bs[r][c4] = b.x;
            Bs[r][c4 + 1] = b.y;
            Bs[r][c4 + 2] = b.z;
            Bs[r][c4 + 3] = b.w;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kKC; kk += 2) {
            const float a = As[wm * 32 + (lane & 31)][kk + (lane >> 5)];
            const float b = Bs[wn * 32 + (lane & 31)][kk + (lane >> 5)];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    const int64_t kb = k0 + wn * 32 + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int c = c0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (c < cnt && kb < N)
            C[(int64_t)c * ldc + kb] = acc[r];
    }
}

// normpart[c][jt] = sum over the tile's columns j of (Hs[c][j] - sum_k C[c][k] Vs[k][j])^2
__global__ void __launch_bounds__(kThreads) k_sub_f32_mfma(const float *__restrict__ Vs,
                                                           const DevState *__restrict__ st,
                                                           const float *__restrict__ Hs, const float *__restrict__ C,
                                                           int64_t ldc, int cnt, int64_t D,
                                                           double *__restrict__ normpart)
{
    if (aborted(st))
        return;
    const int64_t N = st->N;
    const int64_t j0 = (int64_t)blockIdx.x * kT;  // columns of the operator
    const int c0 = blockIdx.y * kT;               // candidates
    if (c0 >= cnt)
        return;
    __shared__ float As[kT][kKC + 1];   // C chunk: candidates x basis rows
    __shared__ float Bs[kKC][kT + 4];   // V chunk: basis rows x columns
    __shared__ float rsum[kT][2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w >> 1, wn = w & 1;
    f32x16 acc = {};
    const bool vec4 = (D % 4) == 0;
    for (int64_t k0 = 0; k0 < N; k0 += kKC) {
        for (int q = threadIdx.x; q < kT * kKC; q += blockDim.x) {
            const int r = q / kKC, kk = q % kKC;
            As[r][kk] = (c0 + r < cnt && k0 + kk < N) ? C[(int64_t)(c0 + r) * ldc + k0 + kk] : 0.f;
        }
        for (int q = threadIdx.x; q < kKC * kT / 4; q += blockDim.x) {
            const int kk = q / (kT / 4), c4 = (q % (kT / 4)) * 4;
            const int64_t k = k0 + kk, j = j0 + c4;
            float4 b = {0.f, 0.f, 0.f, 0.f};
            if (k < N) {
                if (vec4 && j + 3 < D) {
                    b = *reinterpret_cast<const float4 *>(Vs + k * D + j);
                } else {
                    float tb[4] = {0.f, 0.f, 0.f, 0.f};
                    for (int u = 0; u < 4; ++u)
                        if (j + u < D)
                            tb[u] = Vs[k * D + j + u];
                    b = {tb[0], tb[1], tb[2], tb[3]};
                }
            }
            Bs[kk][c4] = b.x;
            Bs[kk][c4 + 1] = b.y;
            Bs[kk][c4 + 2] = b.z;
            Bs[kk][c4 + 3] = b.w;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kKC; kk += 2) {
            const float a = As[wm * 32 + (lane & 31)][kk + (lane >> 5)];
            const float b = Bs[kk + (lane >> 5)][wn * 32 + (lane & 31)];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // epilogue: residual, squares, row sums over the 32 columns of this wave
    const int64_t j = j0 + wn * 32 + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int cl = wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int c = c0 + cl;
        float v = 0.f;
        if (c < cnt && j < D)
            v = Hs[(int64_t)c * D + j] - acc[r];
        v = v * v;
        for (int off = 16; off > 0; off >>= 1)
            v += __shfl_xor(v, off, 64);
        if ((lane & 31) == 0)
            rsum[cl][wn] = v;
    }
    __syncthreads();
    if (threadIdx.x < kT) {
        const int c = c0 + threadIdx.x;
        if (c < cnt)
            normpart[(int64_t)c * gridDim.x + blockIdx.x] = (double)rsum[threadIdx.x][0] + rsum[threadIdx.x][1];
    }
}

__global__ void k_norm_final_s(const double *__restrict__ normpart, int cnt, int tiles,
                               const DevState *__restrict__ st, double *__restrict__ rs2)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cnt || aborted(st))
        return;
    double s = 0.0;
    for (int t = 0; t < tiles; ++t)
        s += normpart[(int64_t)c * tiles + t];
    rs2[c] = s;
}

// ------------------------------------------------------------------ classification and compaction
//
// One workgroup of up to 1024 threads, thread c owns candidate c.  Survivors
// are written in candidate order: rows[r] = c, pairs[r] = p0 + c, and
// slot[c] = r (or -1); *nsurv receives their count.
__global__ void __launch_bounds__(1024) k_classify(const double *__restrict__ a2, const double *__restrict__ n2,
                                                   int cnt, int64_t p0, int policy, double thr,
                                                   const DevState *__restrict__ st, int *__restrict__ rows,
                                                   int64_t *__restrict__ pairs, int *__restrict__ slot,
                                                   int *__restrict__ nsurv)
{
    __shared__ int wcount[16];
    __shared__ int wbase[16];
    const int c = threadIdx.x;
    const bool ab = aborted(st);
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
            }
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned long long mask = __ballot(keep);
    if (lane == 0)
        wcount[w] = __popcll(mask);
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            wbase[i] = s;
            s += wcount[i];
        }
        *nsurv = ab ? 0 : s;
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
}

// Vs[row] = fp32(V64[row]) for rows [from, to) (to read from the device state if negative)
__global__ void k_shadow_f32(const double *__restrict__ V64, float *__restrict__ Vs, int64_t D, int64_t from,
                             const DevState *__restrict__ st)
{
    const int64_t to = st->N;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + from * D;
    if (e < to * D)
        Vs[e] = (float)V64[e];
}

}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t launch_comm_f32(const float *Vs, int d, int64_t p0, int cnt, const DevState *st, float *Hs, double *hs2,
                           hipStream_t s)
{
    if (cnt <= 0)
        return hipSuccess;
    const int dp = (d + 15) & ~15;
    const size_t lds = (size_t)6 * dp * (dp + 1) * sizeof(float);
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
        if (hipFuncSetAttribute((const void *)k_comm_f32_mfma, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) ==
            hipSuccess)
            granted = lds;
        else
            (void)hipGetLastError();  // clear the failed request; the fallback kernel is used
    }
    if (lds <= granted) {
        hipLaunchKernelGGL(k_comm_f32_mfma, dim3(cnt), dim3(kThreads), lds, s, Vs, d, p0, cnt, st, Hs, hs2);
    } else {
        const int64_t D = (int64_t)d * d;
        hipLaunchKernelGGL(k_comm_f32_global, dim3((unsigned)((D + kThreads - 1) / kThreads), cnt), dim3(kThreads), 0,
                           s, Vs, d, p0, cnt, st, Hs);
        hipLaunchKernelGGL(k_rownorm_f32, dim3(cnt), dim3(kThreads), 0, s, Hs, cnt, D, st, hs2);
    }
    return hipGetLastError();
}

hipError_t launch_dot_f32(const float *Vs, const DevState *st, const float *Hs, int cnt, int64_t D, int64_t n_hi,
                          float *C, hipStream_t s)
{
    if (cnt <= 0)
        return hipSuccess;
    n_hi = std::max<int64_t>(n_hi, 1);
    hipLaunchKernelGGL(k_dot_f32_mfma, dim3((unsigned)((n_hi + kT - 1) / kT), (cnt + kT - 1) / kT), dim3(kThreads), 0,
                       s, Vs, st, Hs, cnt, D, C, n_hi);
    return hipGetLastError();
}

int sub_f32_tiles(int64_t D) { return (int)((D + kT - 1) / kT); }

hipError_t launch_sub_f32(const float *Vs, const DevState *st, const float *Hs, const float *C, int64_t n_hi, int cnt,
                          int64_t D, double *normpart, double *rs2, hipStream_t s)
{
    if (cnt <= 0)
        return hipSuccess;
    n_hi = std::max<int64_t>(n_hi, 1);
    const int tiles = sub_f32_tiles(D);
    hipLaunchKernelGGL(k_sub_f32_mfma, dim3(tiles, (cnt + kT - 1) / kT), dim3(kThreads), 0, s, Vs, st, Hs, C, n_hi,
                       cnt, D, normpart);
    hipLaunchKernelGGL(k_norm_final_s, dim3((cnt + kThreads - 1) / kThreads), dim3(kThreads), 0, s, normpart, cnt,
                       tiles, st, rs2);
    return hipGetLastError();
}

hipError_t launch_classify(const double *a2, const double *n2, int cnt, int64_t p0, int policy, double thr,
                           const DevState *st, int *rows, int64_t *pairs, int *slot, int *nsurv, hipStream_t s)
{
    if (cnt <= 0 || cnt > 1024)
        return cnt <= 0 ? hipSuccess : hipErrorInvalidValue;
    const int threads = ((cnt + 63) / 64) * 64;
    hipLaunchKernelGGL(k_classify, dim3(1), dim3(threads), 0, s, a2, n2, cnt, p0, policy, thr, st, rows, pairs, slot,
                       nsurv);
    return hipGetLastError();
}

hipError_t launch_shadow_f32(const double *V64, float *Vs, int64_t D, int64_t from, int64_t to_hi, const DevState *st,
                             hipStream_t s)
{
    const int64_t n = (to_hi - from) * D;
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_shadow_f32, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, V64, Vs, D,
                       from, st);
    return hipGetLastError();
}

}  // namespace lie

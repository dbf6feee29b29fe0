// Inverse Gram matrix of the matrix-inversion method (Algorithm 2, Section 3.1).
//
// The method keeps a raw basis B of unit-norm elements and the inverse of their
// Gram matrix A_ij = <B_i, B_j>.  A candidate h is tested through
// beta = (<B_0, h>, ..., <B_{N-1}, h>), x = A^{-1} beta and the explicit
// residual h - sum_k x_k B_k.  Packed real coordinates make every inner
// product a Euclidean dot, so A is real symmetric.
//
// Expanding A by an appended element b (Algorithm 2's "Expand A": the new row
// and column are beta_i = <B_i, b>, the new diagonal entry is 1) and computing
// the inverse of the expanded matrix goes through the Cholesky factor A = L L^T,
// kept as its inverse T = L^{-1} (lower triangular).  Bordering A by (beta, 1)
// borders L by the row (l^T, delta) with l = T beta and delta^2 = 1 - l^T l (the
// row-by-row Cholesky factorisation), and T by the row (-(l^T T) / delta, 1/delta):
// O(N^2) per appended element, no refactorisation.  A^{-1} = T^T T is applied to a
// block of candidates as two products, y = T beta and x = T^T y.  A non-positive or
// non-finite delta^2 means the expanded A is not numerically positive definite --
// the ill-conditioning the paper warns about -- and is reported.  Everything here is
// the library's own FP64 kernels: the inner products of the new elements, the
// bordered factor updates, and the two products on the FP64 matrix cores.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>

#include "lie_internal.h"

namespace lie {

namespace {

typedef double f64x4_t __attribute__((ext_vector_type(4)));

constexpr int kNewRows = 64;  // new elements whose inner products are formed per launch

// G[r][k] = <B_{n0 + r}, B_k> for r < rows, k < n0 + r (the entries the bordered updates
// of the rows' elements read).  One wave per (r, k) dot product of length D.
__global__ void __launch_bounds__(256) k_new_inner(const double *__restrict__ B, int64_t D, int64_t n0, int rows,
                                                   double *__restrict__ G, int64_t ldg)
{
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t total = (int64_t)rows * (n0 + rows);
    for (int64_t e = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); e < total; e += nwaves) {
        const int64_t r = e / (n0 + rows), k = e % (n0 + rows);
        if (k >= n0 + r)
            continue;
        const double *a = B + (n0 + r) * D, *b = B + k * D;
        double s = 0.0;
        for (int64_t j = lane; j < D; j += 64)
            s += a[j] * b[j];
        s = wave_sum(s);
        if (lane == 0)
            G[r * ldg + k] = s;
    }
}

// l = T beta over the leading n x n block of T (one wave per row; row i of T is zero past i).
__global__ void __launch_bounds__(256) k_factor_l(const double *__restrict__ T, int64_t ldt, int64_t n,
                                                  const double *__restrict__ beta, double *__restrict__ l)
{
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < n; i += nwaves) {
        const double *t = T + i * ldt;
        double s = 0.0;
        for (int64_t k = lane; k <= i; k += 64)
            s += t[k] * beta[k];
        s = wave_sum(s);
        if (lane == 0)
            l[i] = s;
    }
}

// Row n of T for the bordered factor: delta^2 = 1 - l^T l (every workgroup forms the same
// sum in the same order), T[n][k] = -(sum_{i=k}^{n-1} l_i T[i][k]) / delta for k < n and
// T[n][n] = 1 / delta.  A non-positive or non-finite delta^2 is flagged in *bad (element
// index + 1) and T is left as it was.
__global__ void __launch_bounds__(256) k_factor_row(double *__restrict__ T, int64_t ldt, int64_t n,
                                                    const double *__restrict__ l, int *__restrict__ bad)
{
    __shared__ double red[4];
    __shared__ double s_sh;
    double p = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x)
        p += l[k] * l[k];
    p = wave_sum(p);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = p;
    __syncthreads();
    if (threadIdx.x == 0)
        s_sh = 1.0 - (red[0] + red[1] + red[2] + red[3]);
    __syncthreads();
    const double d2 = s_sh;
    if (!(d2 > 0.0) || !isfinite(d2)) {
        if (blockIdx.x == 0 && threadIdx.x == 0)
            atomicCAS(bad, 0, (int)n + 1);
        return;
    }
    const double inv = 1.0 / sqrt(d2);
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k <= n; k += (int64_t)gridDim.x * blockDim.x) {
        if (k == n) {
            T[n * ldt + n] = inv;
            continue;
        }
        double w = 0.0;
        for (int64_t i = k; i < n; ++i)
            w += l[i] * T[i * ldt + k];
        T[n * ldt + k] = -w * inv;
    }
}

// X[m][n] = sum_k Y[m][k] M(n, k) for m < cnt, n < N, k < N, with M(n, k) = Tm[n][k]
// (TRANS = false: rows of y are T beta) or Tm[k][n] (TRANS = true: x = T^T y).  Workgroup
// tile 64 x 64 (4 waves of 32 x 32, each 2 x 2 MFMA f64 16x16x4 tiles), K in chunks of 16
// through LDS.  f64 16x16x4: lane l supplies A[l%16][l/16] and B[l/16][l%16]; result
// register r of lane l is D[4r + l/16][l%16].
constexpr int kAT = 64, kAK = 16;

template <bool TRANS>
__global__ void __launch_bounds__(256) k_apply_factor(const double *__restrict__ beta, int64_t ldb,
                                                      const double *__restrict__ Ai, int64_t lda, int64_t N, int cnt,
                                                      double *__restrict__ X, int64_t ldx)
{
    const int64_t m0 = (int64_t)blockIdx.y * kAT, n0 = (int64_t)blockIdx.x * kAT;
    if (m0 >= cnt || n0 >= N)
        return;
    __shared__ double As[kAT][kAK + 1], Bs[kAT][kAK + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w >> 1, wn = w & 1;
    f64x4_t acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            acc[i][j] = f64x4_t{0.0, 0.0, 0.0, 0.0};
    for (int64_t k0 = 0; k0 < N; k0 += kAK) {
        for (int e = threadIdx.x; e < kAT * kAK; e += blockDim.x) {
            const int r = e / kAK, kk = e % kAK;
            const int64_t k = k0 + kk;
            As[r][kk] = (m0 + r < cnt && k < N) ? beta[(m0 + r) * ldb + k] : 0.0;
            if (!TRANS)
                Bs[r][kk] = (n0 + r < N && k < N) ? Ai[(n0 + r) * lda + k] : 0.0;
        }
        if (TRANS)  // column n0 + r of row k: consecutive threads take consecutive columns
            for (int e = threadIdx.x; e < kAT * kAK; e += blockDim.x) {
                const int r = e % kAT, kk = e / kAT;
                const int64_t k = k0 + kk;
                Bs[r][kk] = (n0 + r < N && k < N) ? Ai[k * lda + n0 + r] : 0.0;
            }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kAK; ks += 4) {
            double a[2], b[2];
            for (int i = 0; i < 2; ++i)
                a[i] = As[wm * 32 + i * 16 + (lane & 15)][ks + (lane >> 4)];
            for (int j = 0; j < 2; ++j)
                b[j] = Bs[wn * 32 + j * 16 + (lane & 15)][ks + (lane >> 4)];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 4; ++r) {
                const int64_t m = m0 + wm * 32 + i * 16 + 4 * r + (lane >> 4);
                const int64_t n = n0 + wn * 32 + j * 16 + (lane & 15);
                if (m < cnt && n < N)
                    X[m * ldx + n] = acc[i][j][r];
            }
}

}  // namespace

struct GramInverse {
    hipStream_t stream = nullptr;
    int64_t cap = 0, D = 0;
    int max_rows = 0;        // candidates per application
    int64_t n = 0;           // elements the factor covers
    double *T = nullptr;     // cap x cap, row-major: inverse Cholesky factor (zero above the diagonal)
    double *G = nullptr;     // kNewRows x cap: inner products of new elements
    double *l = nullptr;     // cap
    double *Y = nullptr;     // max_rows x cap: T beta of a block of candidates
    int *bad = nullptr;      // first element whose delta^2 failed (+1), or 0
};

hipError_t gram_inverse_create(GramInverse **out, int64_t cap, int64_t D, int max_rows, hipStream_t s)
{
    auto *g = new (std::nothrow) GramInverse();
    if (!g)
        return hipErrorOutOfMemory;
    g->stream = s;
    g->cap = cap;
    g->D = D;
    g->max_rows = std::max(max_rows, 1);
    hipError_t e;
    if ((e = hipMalloc(&g->T, (size_t)cap * cap * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&g->G, (size_t)kNewRows * cap * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&g->l, (size_t)cap * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&g->Y, (size_t)g->max_rows * cap * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&g->bad, sizeof(int))) != hipSuccess ||
        (e = hipMemsetAsync(g->T, 0, (size_t)cap * cap * sizeof(double), s)) != hipSuccess ||
        (e = hipMemsetAsync(g->bad, 0, sizeof(int), s)) != hipSuccess) {
        gram_inverse_destroy(g);
        return e;
    }
    *out = g;
    return hipSuccess;
}

void gram_inverse_destroy(GramInverse *g)
{
    if (!g)
        return;
    for (void *p : {(void *)g->T, (void *)g->G, (void *)g->l, (void *)g->Y, (void *)g->bad})
        if (p)
            (void)hipFree(p);
    delete g;
}

hipError_t gram_inverse_update(GramInverse *g, const double *B, int64_t N, int *info_host)
{
    *info_host = 0;
    if (N > g->cap)
        return hipErrorInvalidValue;
    const int64_t cap = g->cap;
    for (int64_t n0 = g->n; n0 < N; n0 += kNewRows) {
        const int rows = (int)std::min<int64_t>(kNewRows, N - n0);
        hipLaunchKernelGGL(k_new_inner, dim3(1024), dim3(256), 0, g->stream, B, g->D, n0, rows, g->G, cap);
        for (int r = 0; r < rows; ++r) {
            const int64_t n = n0 + r;  // border the n x n factor to (n + 1) x (n + 1)
            const double *beta = g->G + (int64_t)r * cap;
            if (n > 0) {
                const unsigned wb = (unsigned)std::min<int64_t>(1024, (n + 3) / 4);
                hipLaunchKernelGGL(k_factor_l, dim3(wb), dim3(256), 0, g->stream, (const double *)g->T, cap, n, beta,
                                   g->l);
            }
            const unsigned ub = (unsigned)std::min<int64_t>(256, (n + 256) / 256);
            hipLaunchKernelGGL(k_factor_row, dim3(ub), dim3(256), 0, g->stream, g->T, cap, n, (const double *)g->l,
                               g->bad);
        }
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(info_host, g->bad, sizeof(int), hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(g->stream);
    if (e == hipSuccess)
        g->n = N;
    return e;
}

hipError_t gram_inverse_apply(GramInverse *g, const double *beta, int64_t ldb, int64_t N, int cnt, double *X,
                              int64_t ldx)
{
    if (N <= 0 || cnt <= 0)
        return hipSuccess;
    if (cnt > g->max_rows)
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)((N + kAT - 1) / kAT), (unsigned)((cnt + kAT - 1) / kAT));
    // y = T beta, then x = T^T y = A^{-1} beta
    hipLaunchKernelGGL(k_apply_factor<false>, grid, dim3(256), 0, g->stream, beta, ldb, (const double *)g->T, g->cap,
                       N, cnt, g->Y, g->cap);
    hipLaunchKernelGGL(k_apply_factor<true>, grid, dim3(256), 0, g->stream, (const double *)g->Y, g->cap,
                       (const double *)g->T, g->cap, N, cnt, X, ldx);
    return hipGetLastError();
}

}  // namespace lie

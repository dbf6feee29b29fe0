// Rank test of the standard algorithm (Algorithm 1 with the rank computed by an SVD).
//
// The standard construction keeps a raw basis B and accepts a candidate h iff
// rank([B; h]) > rank(B).  The paper times this against the orthonormalization
// method; here it is the comparison baseline on the same device.  For a block of
// candidates, each matrix [B_0 .. B_{N-1}, h_c] (packed real coordinates, whose
// Euclidean products are the paper's inner products) goes through one batched
// singular-value decomposition (rocSOLVER, values only); the candidate raises
// the rank iff its smallest singular value exceeds max(m, n) * eps * sigma_max,
// the usual numerical-rank tolerance.  B has full rank N by construction.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cfloat>
#include <cmath>

#include "lie_internal.h"

namespace lie {

namespace {

// A[c] = [B (N x D) ; H_c (D)], column-major D x (N+1): column j is vector j.
__global__ void k_rank_gather(const double *__restrict__ B, int64_t N, const double *__restrict__ H, int cnt,
                              int64_t D, double *__restrict__ A)
{
    const int c = blockIdx.y;
    if (c >= cnt)
        return;
    const int64_t per = (N + 1) * D;
    double *out = A + (int64_t)c * per;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < per; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = i < N * D ? B[i] : H[(int64_t)c * D + (i - N * D)];
}

// flags[c] = 1 iff sigma_N > max(D, N+1) * eps * sigma_0 (the rank rose) and the SVD converged.
__global__ void k_rank_decide(const double *__restrict__ S, int64_t N, int64_t D, const int *__restrict__ info,
                              int cnt, unsigned char *__restrict__ flags)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cnt)
        return;
    const double *s = S + (int64_t)c * (N + 1);
    const double smax = s[0], smin = s[N];
    const double tau = (double)std::max<int64_t>(D, N + 1) * DBL_EPSILON * smax;
    flags[c] = (info[c] == 0 && smax > 0.0 && smin > tau) ? 1 : 0;
}

}  // namespace

struct RankTester {
    rocblas_handle handle = nullptr;
    hipStream_t stream = nullptr;
    int64_t D = 0;
    int max_batch = 0;
    double *A = nullptr, *S = nullptr, *E = nullptr;
    int *info = nullptr;
    unsigned char *flags = nullptr, *flags_host = nullptr;
};

hipError_t rank_tester_create(RankTester **out, int64_t D, int max_batch, hipStream_t s)
{
    auto *t = new (std::nothrow) RankTester();
    if (!t)
        return hipErrorOutOfMemory;
    t->stream = s;
    t->D = D;
    t->max_batch = max_batch;
    hipError_t e;
    const size_t mats = (size_t)max_batch * D * D;  // (N + 1) <= D columns of length D
    if ((e = hipMalloc(&t->A, mats * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&t->S, (size_t)max_batch * D * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&t->E, (size_t)max_batch * D * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&t->info, (size_t)max_batch * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&t->flags, (size_t)max_batch)) != hipSuccess ||
        (e = hipHostMalloc((void **)&t->flags_host, (size_t)max_batch, hipHostMallocDefault)) != hipSuccess) {
        rank_tester_destroy(t);
        return e;
    }
    if (rocblas_create_handle(&t->handle) != rocblas_status_success ||
        rocblas_set_stream(t->handle, s) != rocblas_status_success) {
        rank_tester_destroy(t);
        return hipErrorUnknown;
    }
    *out = t;
    return hipSuccess;
}

void rank_tester_destroy(RankTester *t)
{
    if (!t)
        return;
    if (t->handle)
        (void)rocblas_destroy_handle(t->handle);
    for (void *p : {(void *)t->A, (void *)t->S, (void *)t->E, (void *)t->info, (void *)t->flags})
        if (p)
            (void)hipFree(p);
    if (t->flags_host)
        (void)hipHostFree(t->flags_host);
    delete t;
}

hipError_t rank_tester_run(RankTester *t, const double *B, int64_t N, const double *H, int cnt, unsigned char *flags)
{
    if (cnt <= 0)
        return hipSuccess;
    if (cnt > t->max_batch || N + 1 > t->D)
        return hipErrorInvalidValue;
    const int64_t D = t->D;
    const int64_t per = (N + 1) * D;
    const unsigned gx = (unsigned)std::min<int64_t>(1024, (per + 255) / 256);
    hipLaunchKernelGGL(k_rank_gather, dim3(gx, cnt), dim3(256), 0, t->stream, B, N, H, cnt, D, t->A);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const rocblas_status rs = rocsolver_dgesvd_strided_batched(
        t->handle, rocblas_svect_none, rocblas_svect_none, (rocblas_int)D, (rocblas_int)(N + 1), t->A,
        (rocblas_int)D, (rocblas_stride)per, t->S, (rocblas_stride)(N + 1), nullptr, 1, 0, nullptr, 1, 0, t->E,
        (rocblas_stride)std::max<int64_t>(N, 1), rocblas_outofplace, t->info, cnt);
    if (rs != rocblas_status_success)
        return hipErrorUnknown;
    hipLaunchKernelGGL(k_rank_decide, dim3((cnt + 255) / 256), dim3(256), 0, t->stream, t->S, N, D, t->info, cnt,
                       t->flags);
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = hipMemcpyAsync(t->flags_host, t->flags, (size_t)cnt, hipMemcpyDeviceToHost, t->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(t->stream)) != hipSuccess)
        return e;
    std::copy(t->flags_host, t->flags_host + cnt, flags);
    return hipSuccess;
}

}  // namespace lie

// Inverse Gram matrix of the matrix-inversion method (Algorithm 2, Section 3.1).
//
// The method keeps a raw basis B of unit-norm elements and the inverse of its
// Gram matrix A_ij = <B_i, B_j>.  A candidate h is tested through
// beta = (<B_0, h>, ..., <B_{N-1}, h>), x = A^{-1} beta and the explicit
// residual h - sum_k x_k B_k.  After elements are appended, A^{-1} is computed
// again (the method's "compute A^{-1} and store"): A = B B^T, a Cholesky
// factorisation and the inverse from it (rocSOLVER), symmetrised.  Packed real
// coordinates make every inner product a Euclidean dot, so A is real symmetric.
// A failed factorisation means A lost positive definiteness in floating point --
// the ill-conditioning the paper warns about -- and is reported.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>

#include "lie_internal.h"

namespace lie {

namespace {

// The inverse is complete in the lower triangle (column-major); mirror it.
__global__ void k_symmetrize(double *A, int64_t n, int64_t ld)
{
    const int64_t total = n * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e % n, c = e / n;  // element (r, c) at A[c * ld + r]
        if (r < c)
            A[c * ld + r] = A[r * ld + c];
    }
}

}  // namespace

struct GramInverse {
    rocblas_handle handle = nullptr;
    hipStream_t stream = nullptr;
    int64_t cap = 0, D = 0;
    double *Ainv = nullptr;  // cap x cap, leading dimension cap
    int *info = nullptr;
};

hipError_t gram_inverse_create(GramInverse **out, int64_t cap, int64_t D, hipStream_t s)
{
    auto *g = new (std::nothrow) GramInverse();
    if (!g)
        return hipErrorOutOfMemory;
    g->stream = s;
    g->cap = cap;
    g->D = D;
    hipError_t e;
    if ((e = hipMalloc(&g->Ainv, (size_t)cap * cap * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&g->info, sizeof(int))) != hipSuccess) {
        gram_inverse_destroy(g);
        return e;
    }
    if (rocblas_create_handle(&g->handle) != rocblas_status_success ||
        rocblas_set_stream(g->handle, s) != rocblas_status_success) {
        gram_inverse_destroy(g);
        return hipErrorUnknown;
    }
    *out = g;
    return hipSuccess;
}

void gram_inverse_destroy(GramInverse *g)
{
    if (!g)
        return;
    if (g->handle)
        (void)rocblas_destroy_handle(g->handle);
    for (void *p : {(void *)g->Ainv, (void *)g->info})
        if (p)
            (void)hipFree(p);
    delete g;
}

hipError_t gram_inverse_update(GramInverse *g, const double *B, int64_t N, int *info_host)
{
    *info_host = 0;
    if (N <= 0)
        return hipSuccess;
    if (N > g->cap)
        return hipErrorInvalidValue;
    // column-major view of B (row-major N x D) is B^T (D x N, ld D): A = (B^T)^T B^T = B B^T
    const double one = 1.0, zero = 0.0;
    if (rocblas_dgemm(g->handle, rocblas_operation_transpose, rocblas_operation_none, (rocblas_int)N, (rocblas_int)N,
                      (rocblas_int)g->D, &one, B, (rocblas_int)g->D, B, (rocblas_int)g->D, &zero, g->Ainv,
                      (rocblas_int)g->cap) != rocblas_status_success)
        return hipErrorUnknown;
    if (rocsolver_dpotrf(g->handle, rocblas_fill_lower, (rocblas_int)N, g->Ainv, (rocblas_int)g->cap, g->info) !=
        rocblas_status_success)
        return hipErrorUnknown;
    hipError_t e = hipMemcpyAsync(info_host, g->info, sizeof(int), hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess || *info_host != 0)
        return e;
    if (rocsolver_dpotri(g->handle, rocblas_fill_lower, (rocblas_int)N, g->Ainv, (rocblas_int)g->cap, g->info) !=
        rocblas_status_success)
        return hipErrorUnknown;
    const unsigned blocks = (unsigned)std::min<int64_t>(4096, (N * N + 255) / 256);
    hipLaunchKernelGGL(k_symmetrize, dim3(blocks), dim3(256), 0, g->stream, g->Ainv, N, g->cap);
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = hipMemcpyAsync(info_host, g->info, sizeof(int), hipMemcpyDeviceToHost, g->stream)) != hipSuccess)
        return e;
    return hipStreamSynchronize(g->stream);
}

hipError_t gram_inverse_apply(GramInverse *g, const double *beta, int64_t ldb, int64_t N, int cnt, double *X,
                              int64_t ldx)
{
    if (N <= 0 || cnt <= 0)
        return hipSuccess;
    // row-major beta (cnt x N, stride ldb) is beta^T column-major (N x cnt, ld ldb);
    // X^T = A^{-1} beta^T (A^{-1} symmetric), stored as row-major X (cnt x N, stride ldx)
    const double one = 1.0, zero = 0.0;
    if (rocblas_dgemm(g->handle, rocblas_operation_none, rocblas_operation_none, (rocblas_int)N, (rocblas_int)cnt,
                      (rocblas_int)N, &one, g->Ainv, (rocblas_int)g->cap, beta, (rocblas_int)ldb, &zero, X,
                      (rocblas_int)ldx) != rocblas_status_success)
        return hipErrorUnknown;
    return hipSuccess;
}

}  // namespace lie

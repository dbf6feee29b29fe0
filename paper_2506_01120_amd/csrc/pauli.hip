// Pauli-sum representation of the operators (the paper's sparse representation,
// Sections 3 and 4.2).
//
// On n qubits (d = 2^n) every anti-Hermitian operator is a real combination of
// the 4^n operators iP_s, P_s = i^{|x&z|} X^x Z^z for the string s = (x, z) of
// two n-bit masks (index s = x * 2^n + z; X^x flips the basis-index bits in x,
// Z^z is the sign (-1)^{popcount(z & j)}).  Since <iP_s, iP_t> = tr(P_s P_t)/d =
// delta_st, the coefficient vectors are orthonormal coordinates: the projection,
// the residual norms and the acceptance run on them unchanged.  What changes is
// the bracket: from P_a P_b = i^{|x_a&z_a| + |x_b&z_b| - |x_c&z_c| + 2|z_a&x_b|} P_c
// (c = a xor b) it follows that [iP_a, iP_b] is 0 for commuting strings and
// 2 i^{e+1} iP_c (a sign, since e is odd) for anticommuting ones.  A bracket is
// then a sparse product: for each output string c, sum over the support of the
// sparser operand, the partner string being fixed by c -- nnz * 4^n work instead
// of the dense 8 d^3.  Each element's support (indices of its non-negligible
// coefficients) is recorded when it is appended.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "lie_internal.h"

namespace lie {

namespace {

constexpr int kThreads = 256;

__device__ inline bool aborted(const DevState *st) { return st && (st->done | st->numeric_error | st->full); }

// Coefficient of iP_{a^b} in [iP_a, iP_b]: 0 (commuting) or +-2.
__device__ inline double bracket_coef(uint32_t a, uint32_t b, int n)
{
    const uint32_t mask = (1u << n) - 1u;
    const uint32_t xa = a >> n, za = a & mask, xb = b >> n, zb = b & mask;
    if (((__popc(xa & zb) + __popc(za & xb)) & 1) == 0)
        return 0.0;
    const uint32_t xc = xa ^ xb, zc = za ^ zb;
    const int e = __popc(xa & za) + __popc(xb & zb) - __popc(xc & zc) + 2 * __popc(za & xb);
    return ((e + 1) & 3) == 0 ? 2.0 : -2.0;
}

// H[c] = [V_l, V_m] for the pairs p0 + c: each output coordinate sums over the
// support of the sparser operand.  grid = (coordinate tiles, candidates).
__global__ void __launch_bounds__(kThreads) k_comm_pauli(const double *__restrict__ V, const int *__restrict__ sup_cnt,
                                                         const int *__restrict__ sup_idx, int n, int64_t D, int64_t p0,
                                                         const int64_t *dp0, int cnt, const DevState *st,
                                                         double *__restrict__ H)
{
    const int c = blockIdx.y;
    if (c >= cnt || aborted(st))
        return;
    int64_t l, m;
    decode_pair((dp0 ? *dp0 : p0) + c, l, m);
    const int nl = sup_cnt[l], nm = sup_cnt[m];
    const bool lsparse = nl <= nm;
    const int64_t ra = lsparse ? l : m, rb = lsparse ? m : l;
    const int na = lsparse ? nl : nm;
    const int *ia = sup_idx + ra * D;
    const double *va = V + ra * D, *vb = V + rb * D;
    const double sign = lsparse ? 1.0 : -1.0;  // [V_l, V_m] = -[V_m, V_l]
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < D; s += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int t = 0; t < na; ++t) {
            const uint32_t a = (uint32_t)ia[t], b = a ^ (uint32_t)s;
            const double k = bracket_coef(a, b, n);
            if (k != 0.0)
                acc += k * va[a] * vb[b];
        }
        H[(int64_t)c * D + s] = sign * acc;
    }
}

// Support of the rows appended by the last acceptance launch ([st->raw_lo, st->N)):
// indices of the coefficients above thr * ||row||, in increasing order (ballot prefix).
__global__ void __launch_bounds__(1024) k_pauli_support(const double *__restrict__ V, int64_t D, const DevState *st,
                                                        double rel_thr, int *__restrict__ sup_cnt,
                                                        int *__restrict__ sup_idx)
{
    __shared__ double red[16];
    __shared__ int wcount[16];
    __shared__ int running;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int64_t lo = st->raw_lo, hi = st->N;
    for (int64_t e = lo + blockIdx.x; e < hi; e += gridDim.x) {
        const double *row = V + e * D;
        double loc = 0.0;
        for (int64_t j = threadIdx.x; j < D; j += blockDim.x)
            loc += row[j] * row[j];
        for (int off = 32; off > 0; off >>= 1)
            loc += __shfl_down(loc, off, 64);
        if (lane == 0)
            red[w] = loc;
        if (threadIdx.x == 0)
            running = 0;
        __syncthreads();
        double t2 = 0.0;
        for (int q = 0; q < nw; ++q)
            t2 += red[q];
        const double thr = rel_thr * sqrt(t2);
        int *out = sup_idx + e * D;
        for (int64_t j0 = 0; j0 < D; j0 += blockDim.x) {
            const int64_t j = j0 + threadIdx.x;
            const bool keep = j < D && fabs(row[j]) > thr;
            const unsigned long long bal = __ballot(keep);
            if (lane == 0)
                wcount[w] = __popcll(bal);
            __syncthreads();
            int base = running;
            for (int q = 0; q < w; ++q)
                base += wcount[q];
            if (keep)
                out[base + __popcll(bal & ((1ull << lane) - 1ull))] = (int)j;
            __syncthreads();
            if (threadIdx.x == 0) {
                int t = 0;
                for (int q = 0; q < nw; ++q)
                    t += wcount[q];
                running += t;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0)
            sup_cnt[e] = running;
        __syncthreads();
    }
}

// In-place fast Walsh-Hadamard transform: f(z) <- sum_k (-1)^{popcount(z & k)} f(k).
void wht(std::complex<double> *f, int d)
{
    for (int h = 1; h < d; h <<= 1)
        for (int i = 0; i < d; i += 2 * h)
            for (int j = i; j < i + h; ++j) {
                const std::complex<double> u = f[j], v = f[j + h];
                f[j] = u + v;
                f[j + h] = u - v;
            }
}

std::complex<double> ipow(int k)
{
    switch (k & 3) {
    case 0: return {1.0, 0.0};
    case 1: return {0.0, 1.0};
    case 2: return {-1.0, 0.0};
    default: return {0.0, -1.0};
    }
}

}  // namespace

hipError_t launch_comm_pauli(const double *V, const int *sup_cnt, const int *sup_idx, int n, int64_t p0, int cnt,
                             const DevState *st, double *H, hipStream_t s, const int64_t *dp0)
{
    if (cnt <= 0)
        return hipSuccess;
    const int64_t D = (int64_t)1 << (2 * n);
    const unsigned gx = (unsigned)std::min<int64_t>(64, (D + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_comm_pauli, dim3(gx, cnt), dim3(kThreads), 0, s, V, sup_cnt, sup_idx, n, D, p0, dp0, cnt, st,
                       H);
    return hipGetLastError();
}

hipError_t launch_pauli_support(const double *V, int64_t D, const DevState *st, int max_new, int *sup_cnt,
                                int *sup_idx, hipStream_t s)
{
    if (max_new <= 0)
        return hipSuccess;
    // coefficients below 1e-14 of the row norm are round-off of the orthogonalisation
    hipLaunchKernelGGL(k_pauli_support, dim3(std::min(max_new, 1024)), dim3(1024), 0, s, V, D, st, 1e-14, sup_cnt,
                       sup_idx);
    return hipGetLastError();
}

void pauli_from_dense(const double *g, int n, double *out)
{
    const int d = 1 << n;
    const double *c = g;  // interleaved (re, im), row-major d x d
    std::vector<std::complex<double>> f(d);
    for (int x = 0; x < d; ++x) {
        for (int k = 0; k < d; ++k) {
            const int64_t e = (int64_t)k * d + (k ^ x);
            f[k] = {c[2 * e], c[2 * e + 1]};
        }
        wht(f.data(), d);
        for (int z = 0; z < d; ++z) {
            // a_s = -i tr(P_s g) / d with tr(P_s g) = i^{|x&z|} T_x(z)
            const std::complex<double> a = std::complex<double>(0.0, -1.0) * ipow(__builtin_popcount(x & z)) * f[z];
            out[((int64_t)x << n) | z] = a.real() / d;
        }
    }
}

void pauli_to_dense(const double *a, int n, double *g)
{
    const int d = 1 << n;
    std::vector<std::complex<double>> u(d);
    for (int x = 0; x < d; ++x) {
        for (int z = 0; z < d; ++z)
            u[z] = a[((int64_t)x << n) | z] * ipow(1 + __builtin_popcount(x & z));
        wht(u.data(), d);
        for (int j = 0; j < d; ++j) {
            const int64_t e = (int64_t)(j ^ x) * d + j;  // G[j^x][j]
            g[2 * e] = u[j].real();
            g[2 * e + 1] = u[j].imag();
        }
    }
}

}  // namespace lie

// Internal declarations shared by the engine's translation units.
//
// Operator storage ("packed anti-Hermitian" layout).  Every operator the
// engine handles is anti-Hermitian (generators, brackets of anti-Hermitian
// operators, and real combinations of them), so d^2 real numbers describe it.
// Element X is stored as a d x d real array p, row-major, with
//     p[i][j] = sqrt(2/d) Re X_ij   (i < j)
//     p[j][i] = sqrt(2/d) Im X_ij   (i < j)
//     p[i][i] = sqrt(1/d) Im X_ii
// With this scaling the Euclidean dot product of two packed arrays equals the
// paper's inner product <X,Y> = tr(X^H Y)/d (Section 2.2), which is real for
// anti-Hermitian X, Y.  So projections, residuals and norms are plain real
// dot products of length D = d^2, and a unit-norm element has unit 2-norm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lie {

// Device-resident counters of one closure problem.  Written only by the
// single-workgroup acceptance kernel (no atomics), read back by the host.
struct DevState {
    int64_t N;               // current |V|
    int64_t n_cand;          // bracket candidates decided
    int64_t n_zero;          // exactly zero brackets
    int64_t n_screen_rej;    // rejected from the screened residual
    int64_t n_fp64;          // decided from an FP64 residual
    int64_t n_acc;           // appended by the bracket loop
    int64_t n_gen_acc;       // appended by the generator phase
    double min_acc;          // smallest accepted FP64 residual (bracket loop)
    double max_rej;          // largest rejected FP64 residual (bracket loop)
    double max_screen_rej;   // largest screened residual among screen rejects
    int32_t numeric_error;   // 1: non-finite residual; 2: |V| would pass the ambient bound
    int32_t full;            // 1: an append was refused because the capacity is reached
    int32_t done;            // 1: early-exit bound reached
    int32_t pad;
};

// Pair index p <-> (l, m) with 0 <= m < l: p = l(l-1)/2 + m.  Row l holds the
// brackets of element l with every earlier element, so consecutive indices
// visit the pairs in the order of the bracket loop.
__host__ __device__ inline void decode_pair(int64_t p, int64_t &l, int64_t &m)
{
    double s = sqrt(8.0 * (double)p + 1.0);
    int64_t L = (int64_t)((1.0 + s) * 0.5);
    while (L > 1 && L * (L - 1) / 2 > p) --L;
    while ((L + 1) * L / 2 <= p) ++L;
    l = L;
    m = p - L * (L - 1) / 2;
}

inline int64_t pairs_below(int64_t n) { return n * (n - 1) / 2; }

// ------------------------------------------------------------- FP64 kernels
// All pointers are device pointers.  `dN` points at DevState::N; kernels read
// the current basis size from the device so that a host loop can enqueue
// several block steps without a round trip.  Grids are sized on the host for
// an upper bound `n_hi` of N; workgroups beyond N exit.

// Pack complex128 operators (interleaved re,im; d x d row-major) into the packed layout.
hipError_t launch_pack_c128(const double *src, double *dst, int count, int d, hipStream_t s);
// Unpack packed operators back to complex128 d x d.
hipError_t launch_unpack_c128(const double *src, double *dst, int64_t count, int d, hipStream_t s);

// H[c] = pack([V_l, V_m]) for the pair of index p0 + c (pair_list == nullptr)
// or pair_list[c], c < cnt.  FP64.
hipError_t launch_comm_f64(const double *V, int d, int64_t p0, const int64_t *pair_list, int cnt, double *H,
                           hipStream_t s);

// Projection pass on rows H[0..cnt):  C = H V^T (N columns), R = H - C V written over H,
// and per-row squared norms of R and of the input H into rho2[c], h2[c] (FP64).
// `part` is split-K scratch of at least proj_scratch_doubles(...) doubles.
struct ProjShape {
    int64_t D;      // elements per operator (d*d)
    int cnt;        // rows in this call
    int64_t n_hi;   // host upper bound of N (grid sizing)
};
size_t proj_scratch_doubles(int64_t D, int cnt_max, int64_t cap);
int project_split_k(int64_t D, int cnt, int64_t n_hi);
// C[c][k] = <H_c, V_k>, ldc = n_hi
hipError_t launch_dot_f64(const double *V, const int64_t *dN, const double *H, double *C, ProjShape sh, hipStream_t s);
// split-K partial products of C V into `part`
hipError_t launch_sub_f64(const double *V, const int64_t *dN, const double *C, double *part, ProjShape sh,
                          hipStream_t s);
// R = H - sum(part) over H, and the squared norms of R and H
hipError_t launch_reduce_f64(double *H, double *part, double *rho2, double *h2, ProjShape sh, hipStream_t s);

// Sequential acceptance of a block (one workgroup): candidate c in order, FP64.
// mode 0: generator (accept iff ||R|| > tol*||H||); mode 1: bracket (||R|| > tol).
// Survivors are orthogonalised twice against elements accepted earlier in the
// same call, normalised and appended at V[N]; N and the counters advance.
hipError_t launch_accept_f64(double *V, DevState *st, double *H, const double *rho2, const double *h2, int cnt,
                             int64_t D, int64_t cap, int64_t ambient, double tol, int mode, int early_exit,
                             hipStream_t s);

// G = V V^T (n x n) then ||G - I||_F into *out (device), using `work` of n*n doubles.
hipError_t launch_orth_loss(const double *V, int64_t n, int64_t D, double *work, double *out, hipStream_t s);

}  // namespace lie

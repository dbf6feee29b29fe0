// The FP64 acceptance kernel: the decisions of a block step.
//
// One workgroup of 1024 threads per block (per problem, grouped).  Phase A counts and
// rejects, in parallel, every candidate that did not survive the classification.
// Phase B decides the survivors in candidate order: snapshot rejections in parallel,
// then a block Cholesky-QR of up to 64 kept survivors (certified acceptances, explicit
// residual checks of the provisional rejections, Q = L^-1 R appended to the basis), and
// the exact sequential path (two-pass Gram-Schmidt against the elements appended
// earlier in the block) from the first row the block pass leaves undecided.
#include "lie_internal.h"

#include <algorithm>
#include <cmath>

namespace lie {

namespace {

typedef double f64x4_t __attribute__((ext_vector_type(4)));

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
                           double *stage, int64_t stage_cap, double *stat, const double *hn_rows)
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
    // staged through LDS (`stage`, stage_cap doubles) in chunks of 64 columns with coalesced
    // loads (the next chunk is fetched into registers while the current one is multiplied);
    // without room for the stage the tiles read global memory directly.
    const int T16 = (nsv + 15) / 16;
    const int ntile = T16 * (T16 + 1) / 2;  // <= 10 <= nw
    int tI = 0, tJ = w;
    while (tJ > tI) {
        tJ -= tI + 1;
        ++tI;
    }
    if (stage_cap >= (int64_t)nsv * 65) {
        // chunk width KC = 2^kcs >= 64 columns: as wide as four values per thread and the
        // stage allow, so few survivors over a long row take few chunks (each chunk costs a
        // global-load round trip and two barriers)
        int kcs = 6;
        while ((nsv << (kcs + 1)) <= 4 * (int)blockDim.x && (int64_t)nsv * ((2 << kcs) + 1) <= stage_cap &&
               (int64_t)(1 << kcs) < D)
            ++kcs;
        const int KC = 1 << kcs, KS = KC + 1;
        const int per = (nsv * KC + blockDim.x - 1) / blockDim.x;  // <= 4
        double nxt[4];
        auto fetch = [&](int64_t k0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = threadIdx.x + q * blockDim.x;
                const int r = e >> kcs, c = e & (KC - 1);
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
                    stage[(e >> kcs) * KS + (e & (KC - 1))] = nxt[q];
            }
            __syncthreads();
            if (k0 + KC < D)
                fetch(k0 + KC);
            if (w < ntile) {
                const int ia = tI * 16 + (lane & 15), ib = tJ * 16 + (lane & 15);
                for (int q0 = 0; q0 < KC / 4; q0 += 16) {
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const int k = 4 * (q0 + q) + (lane >> 4);
                        const double av = ia < nsv ? stage[ia * KS + k] : 0.0;
                        const double bv = ib < nsv ? stage[ib * KS + k] : 0.0;
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
                    }
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

// A further projection pass of the residual R (LDS, D values) against the whole basis: the
// snapshot rows V[0, N0) and the elements appended earlier in the block, V[N0, nall), the
// first AL of them cached in LDS at cbase.  Chunks of one element per wave: the chunk's
// coefficients against the current R, then their subtraction.  Returns ||R||^2 (every
// thread).  Kept out of line: it runs rarely, and inlined it would cost the acceptance
// kernel's hot path registers.
__device__ __noinline__ double reorth_whole_basis(double *R, const double *V, const double *cbase, int64_t AL,
                                                  int64_t N0, int64_t nall, int64_t D, double *red)
{
    __shared__ double scoef[16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int64_t q0 = 0; q0 < nall; q0 += nw) {
        const int64_t q = q0 + w;
        if (q < nall) {
            const int64_t qb = q - N0;
            const double *va = (qb >= 0 && qb < AL) ? cbase + qb * D : V + q * D;
            double sdot = 0.0;
            for (int64_t j = lane; j < D; j += 64)
                sdot += va[j] * R[j];
            sdot = wave_sum(sdot);
            if (lane == 0)
                scoef[w] = sdot;
        }
        lds_barrier();  // the chunk's coefficients are complete, R is no longer read
        const int nq = (int)std::min<int64_t>(nw, nall - q0);
        for (int64_t j = threadIdx.x; j < D; j += blockDim.x) {
            double t = 0.0;
            for (int i = 0; i < nq; ++i) {
                const int64_t qb = q0 + i - N0;
                const double *va = (qb >= 0 && qb < AL) ? cbase + qb * D : V + (q0 + i) * D;
                t += scoef[i] * va[j];
            }
            R[j] -= t;
        }
        lds_barrier();  // R is updated and scoef[] may be overwritten
    }
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
    return t;
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
    __shared__ int64_t l_fp64, l_zero, l_acc, l_gen, l_reorth;
    __shared__ double l_maxrej, l_minacc, l_sdep, l_sind;
    if (threadIdx.x == 0) {
        l_fp64 = l_zero = l_acc = l_gen = l_reorth = 0;
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
    // LDS after R, in doubles (whole cached rows need not fit for the per-survivor scalars
    // and the block pass's workspace)
    const int64_t free_d = a.lds_doubles > a.cnt + D ? a.lds_doubles - a.cnt - D : 0;
    const bool meta_in_lds = free_d >= 3 * (int64_t)nsv;
    const int64_t rest = meta_in_lds ? free_d - 3 * (int64_t)nsv : 0;
    const int64_t slots2 = rest / D;
    for (int k = threadIdx.x; k < nsv && meta_in_lds; k += blockDim.x) {
        const int r = sv_of(k);
        const int c = a.surv_cand[r];
        hn_a[k] = sqrt(a.h2 ? a.h2[r] : a.cand_n2[c]);
        rs_a[k] = sqrt(a.cand_a2[c]);
        sn_a[k] = a.rho2 ? sqrt(a.rho2[r]) : -1.0;
    }
    __syncthreads();
    // block Cholesky-QR pass over the survivors (brackets only, at most 64 survivors).  Its
    // workspace goes after the scalars when it fits there; otherwise (large D: R alone takes
    // most of the LDS) into R, which the pass does not use -- the sequential path after it
    // refills R -- with the Gram staging behind it.
    // The block pass takes the first 64 survivors at most; with more, the exact sequential
    // path decides the rest against everything the pass appended.
    const int nb = nsv < 64 ? nsv : 64;
    const int64_t gram_need = bqr_lds(nb, nw);
    // (in R only from 8 survivors on: at such D the pass has a fixed cost of a few hundred
    // microseconds in latency-bound sweeps over the columns, while the sequential path
    // takes a few tens per survivor)
    const bool gram_free = rest >= gram_need, gram_in_r = !gram_free && D >= gram_need && nb >= 8;
    const bool gram_ok = a.mode == 1 && nb >= 2 && nw >= 16 && meta_in_lds && (gram_free || gram_in_r);
    double *gram_base = gram_in_r ? R : cache2;
    if (gram_ok && gram_free)
        cache2 = gram_base + gram_need;
    const int64_t slots3 = gram_ok && gram_free ? (rest - gram_need) / D : slots2;
    double *cbase = meta_in_lds ? cache2 : cache;
    const int64_t cslots = meta_in_lds ? slots3 : slots;
    int r_first = 0;
    if (gram_ok) {
        __shared__ double bstat[2];
        double *stage = gram_in_r ? R + gram_need : cache2;
        const int64_t stage_cap = gram_in_r ? D - gram_need : cslots * D;
        const BqrOut b = block_qr(a, nb, N0, gram_base, cache2, cslots, stage, stage_cap, bstat, hn_a);
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
        // R_j left the snapshot passes with components along the snapshot of order
        // eps * ||R_j|| (their rounding).  When the in-block elements then take away
        // nearly all of its norm, normalisation magnifies those components by
        // ||R_j|| / ||r||: a weakly coupled direction would come out orthogonal to the
        // snapshot only to eps times that ratio.  Past a ratio of 64 a further pass runs
        // against the whole basis (snapshot and in-block elements, in chunks of one
        // element per wave), which brings the components back to rounding of ||r||.
        // (Only for a vector that would be accepted: a further pass cannot lengthen it, so one
        // already at or below the threshold is rejected either way.)
        if (A > 0 && snap > 0.0 && nrm2 > thr * thr && nrm2 * 4096.0 < snap * snap) {
            nrm2 = reorth_whole_basis(R, a.V, cbase, AL, N0, sN, D, red);
            if (threadIdx.x == 0)
                l_reorth++;
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
        st->n_reorth = s0.n_reorth + l_reorth;
        st->max_rej = fmax(s0.max_rej, l_maxrej);
        st->min_acc = fmin(s0.min_acc, l_minacc);
        st->scr_max_dep = fmax(s0.scr_max_dep, l_sdep);
        st->scr_min_indep = fmin(s0.scr_min_indep, l_sind);
        // work of the FP64 verification of this block's ns survivors against the N0-element
        // snapshot: per projection pass 2 N0 D flops for the coefficients and 2 N0 D for the
        // subtraction; bytes per pass: the basis streamed by both GEMMs, the rows read by both
        // and written once, the coefficients written and read; the recomputed bracket (one
        // complex product, 8 d^3 flops) reads two operands and writes one row
        if (a.vpasses > 0 && ns > 0) {
            const double n = (double)ns, Nd = (double)N0, Dd = (double)D, dd = (double)a.d;
            const double br = a.vbracket ? 1.0 : 0.0;
            st->vfy_flops = s0.vfy_flops + n * (a.vpasses * 4.0 * Nd * Dd + br * 8.0 * dd * dd * dd);
            st->vfy_bytes = s0.vfy_bytes + 8.0 * (a.vpasses * (2.0 * Nd * Dd + 3.0 * n * Dd + 2.0 * n * Nd) +
                                                  br * 3.0 * n * Dd);
        }
        st->N = sN;
    }
}

__global__ void __launch_bounds__(kAccThreads) k_accept_f64(AcceptArgs a) { accept_body(a); }
__global__ void __launch_bounds__(kAccThreads) k_accept_b(Batch b)
{
    const AcceptArgs a = static_cast<const AcceptArgs *>(b.args)[blockIdx.x];
    accept_body(a);
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

}  // namespace lie

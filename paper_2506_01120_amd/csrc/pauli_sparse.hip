// Sparse Pauli-sum representation (the paper's sparse representation of operators,
// Sections 3 and 4.2): elements stored as their supports only.
//
// An anti-Hermitian operator on n qubits is a real combination sum_s c_s iP_s of the
// Pauli strings P_s = i^{|x&z|} X^x Z^z, s = (x, z) two n-bit masks, here the 64-bit key
// (x << 32) | z.  Distinct strings are orthonormal in the paper's inner product, so an
// element is kept as the sorted list of its (key, c_s) terms, with memory proportional to
// its support, and every step of Algorithm 4 works on such lists:
//
//   bracket     [iP_a, iP_b] = 0 for commuting strings, +-2 iP_{a xor b} otherwise, so the
//               bracket of two lists is the list of the |S_l| |S_m| products, sorted by key
//               and summed over equal keys;
//   projection  <V_k, h> = sum over the keys the two supports share (a join of two sorted
//               lists), then h - sum_k <V_k, h> V_k as a list (the terms of h and of every
//               V_k with a nonzero coefficient, sorted and summed), twice (CGS2);
//   decision    the residual norm against tol (tol * ||g|| for a generator), as for dense
//               operators; an accepted residual is normalised and appended to the pool.
//
// Terms whose magnitude falls to 1e-14 of the candidate's norm after a summation are
// dropped (cancellation leaves rounding residue that would otherwise grow the supports).
// Candidates are processed one at a time in Algorithm 4's order, with every size held on
// the device, so the host enqueues many candidates between synchronisations.  Sorting is
// a bitonic network inside one workgroup: in LDS up to 4096 terms, in the scratch arrays
// in global memory beyond that.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "lie_internal.h"

namespace lie {

namespace {

constexpr uint64_t kNoKey = ~0ull;  // sorts last; not a string for n <= 31
constexpr int kSortThreads = 1024;
constexpr int kLdsTerms = 4096;

__device__ inline bool sp_aborted(const DevState *st) { return st->done | st->numeric_error | st->full; }

// Coefficient of iP_{a^b} in [iP_a, iP_b]: 0 for commuting strings, else +-2.
__device__ inline double sp_bracket_coef(uint64_t a, uint64_t b)
{
    const uint32_t xa = (uint32_t)(a >> 32), za = (uint32_t)a, xb = (uint32_t)(b >> 32), zb = (uint32_t)b;
    if (((__popc(xa & zb) + __popc(za & xb)) & 1) == 0)
        return 0.0;
    const uint32_t xc = xa ^ xb, zc = za ^ zb;
    const int e = __popc(xa & za) + __popc(xb & zb) - __popc(xc & zc) + 2 * __popc(za & xb);
    return ((e + 1) & 3) == 0 ? 2.0 : -2.0;
}

__device__ inline double block_sum_1024(double v, double *red /* 16 */)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0)
        red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i)
        s += red[i];
    __syncthreads();
    return s;
}

// Products of the supports of elements l and m of pair p: slot i * |S_m| + j holds the key
// and coefficient of [c_i iP_{a_i}, c_j iP_{b_j}] (kNoKey for commuting strings).
__global__ void __launch_bounds__(256) k_sp_bracket(const uint64_t *__restrict__ pk, const double *__restrict__ pc,
                                                    const int64_t *__restrict__ off, int64_t p, DevState *st,
                                                    uint64_t *__restrict__ tk, double *__restrict__ tc, int64_t *tn,
                                                    int64_t cap)
{
    if (sp_aborted(st))
        return;
    int64_t l, m;
    decode_pair(p, l, m);
    const int64_t la = off[l], na = off[l + 1] - la, lb = off[m], nb = off[m + 1] - lb;
    const int64_t total = na * nb;
    if (total > cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->full = 2;  // a bracket's product list exceeds the scratch
            *tn = 0;
        }
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *tn = total;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / nb, j = e % nb;
        const uint64_t a = pk[la + i], b = pk[lb + j];
        const double c = sp_bracket_coef(a, b) * pc[la + i] * pc[lb + j];
        tk[e] = c != 0.0 ? (a ^ b) : kNoKey;
        tc[e] = c;
    }
}

// Bitonic sort of n <= P entries (P a power of two, entries [n, P) are kNoKey) by key.
template <bool LDS>
__device__ void bitonic(uint64_t *k, double *c, int64_t P)
{
    for (int64_t size = 2; size <= P; size <<= 1) {
        for (int64_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (int64_t i = threadIdx.x; i < P / 2; i += blockDim.x) {
                const int64_t lo = 2 * i - (i & (stride - 1)), hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t a = k[lo], b = k[hi];
                if ((a > b) == up) {
                    k[lo] = b;
                    k[hi] = a;
                    const double t = c[lo];
                    c[lo] = c[hi];
                    c[hi] = t;
                }
            }
            if (LDS)
                __syncthreads();
            else {
                __threadfence_block();
                __syncthreads();
            }
        }
    }
}

// Sort the list (tk, tc, *tn) by key, sum equal keys, drop terms whose magnitude is at most
// 1e-14 of the reference norm, and write the result to (ok, oc, *on).  The reference norm is
// the norm of this result when `first` (it is then stored in *hn), else *hn.  One workgroup.
// Entries [n, P) of the scratch (P the next power of two) are overwritten.
__global__ void __launch_bounds__(kSortThreads) k_sp_sort_reduce(uint64_t *__restrict__ tk, double *__restrict__ tc,
                                                                 const int64_t *tn, int64_t tcap,
                                                                 uint64_t *__restrict__ ok, double *__restrict__ oc,
                                                                 int64_t *on, double *hn, int first, DevState *st)
{
    __shared__ uint64_t sk[kLdsTerms];
    __shared__ double sc[kLdsTerms];
    __shared__ double red[16];
    __shared__ int64_t s_base;
    if (sp_aborted(st))
        return;
    const int64_t n = *tn;
    int64_t P = 1;
    while (P < n)
        P <<= 1;
    if (P > tcap) {  // cannot happen for lists the scratch holds (tcap is a power of two)
        if (threadIdx.x == 0)
            st->full = 2;
        return;
    }
    if (P <= kLdsTerms) {
        for (int64_t i = threadIdx.x; i < P; i += blockDim.x) {
            sk[i] = i < n ? tk[i] : kNoKey;
            sc[i] = i < n ? tc[i] : 0.0;
        }
        __syncthreads();
        bitonic<true>(sk, sc, P);
        for (int64_t i = threadIdx.x; i < P; i += blockDim.x) {
            tk[i] = sk[i];
            tc[i] = sc[i];
        }
    } else {
        for (int64_t i = n + threadIdx.x; i < P; i += blockDim.x) {
            tk[i] = kNoKey;
            tc[i] = 0.0;
        }
        __threadfence_block();
        __syncthreads();
        bitonic<false>(tk, tc, P);
    }
    __threadfence_block();
    __syncthreads();
    // run sums at the run heads (into ok/oc), kNoKey elsewhere
    double sq = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint64_t key = tk[i];
        const bool head = key != kNoKey && (i == 0 || tk[i - 1] != key);
        double s = 0.0;
        if (head)
            for (int64_t j = i; j < n && tk[j] == key; ++j)
                s += tc[j];
        ok[i] = head ? key : kNoKey;
        oc[i] = head ? s : 0.0;
        sq += s * s;
    }
    const double nrm = sqrt(block_sum_1024(sq, red));
    if (first && threadIdx.x == 0)
        *hn = nrm;
    const double ref = first ? nrm : *hn;
    const double thr = 1e-14 * ref;
    __threadfence_block();
    __syncthreads();
    // compaction in place, chunk by chunk (a chunk's values are read before any is written)
    if (threadIdx.x == 0)
        s_base = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < n; c0 += blockDim.x) {
        const int64_t i = c0 + threadIdx.x;
        uint64_t key = kNoKey;
        double v = 0.0;
        if (i < n) {
            key = ok[i];
            v = oc[i];
        }
        const bool keep = key != kNoKey && fabs(v) > thr;
        const unsigned long long bal = __ballot(keep);
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        __shared__ int wcnt[16];
        if (lane == 0)
            wcnt[w] = __popcll(bal);
        __syncthreads();
        int64_t pos = s_base;
        for (int q = 0; q < w; ++q)
            pos += wcnt[q];
        pos += __popcll(bal & ((1ull << lane) - 1ull));
        __syncthreads();  // every read of this chunk is done
        if (keep) {
            ok[pos] = key;
            oc[pos] = v;
        }
        if (threadIdx.x == 0) {
            int64_t t = 0;
            for (int q = 0; q < (int)(blockDim.x >> 6); ++q)
                t += wcnt[q];
            s_base += t;
        }
        __threadfence_block();
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *on = s_base;
}

// c[k] = <V_k, h> for k < N: the terms of the shorter list looked up in the longer one by
// binary search, summed in the shorter list's order.  One wave per element.
__global__ void __launch_bounds__(256) k_sp_coef(const uint64_t *__restrict__ pk, const double *__restrict__ pc,
                                                 const int64_t *__restrict__ off, const DevState *st,
                                                 const uint64_t *__restrict__ hk, const double *__restrict__ hc,
                                                 const int64_t *hnum, double *__restrict__ coef)
{
    if (sp_aborted(st))
        return;
    const int64_t N = st->N, nh = *hnum;
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t k = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); k < N; k += nwaves) {
        const int64_t a0 = off[k], na = off[k + 1] - a0;
        const bool vshort = na <= nh;
        const uint64_t *sk = vshort ? pk + a0 : hk, *lk = vshort ? hk : pk + a0;
        const double *sc = vshort ? pc + a0 : hc, *lc = vshort ? hc : pc + a0;
        const int64_t ns = vshort ? na : nh, nl = vshort ? nh : na;
        double s = 0.0;
        for (int64_t i = lane; i < ns; i += 64) {
            const uint64_t key = sk[i];
            int64_t lo = 0, hi = nl;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (lk[mid] < key)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            if (lo < nl && lk[lo] == key)
                s += sc[i] * lc[lo];
        }
        s = wave_sum(s);
        if (lane == 0)
            coef[k] = s;
    }
}

// Offsets of the gathered list h - sum_k c_k V_k: the terms of h first, then those of every
// V_k with c_k != 0 in k order.  One workgroup (exclusive scan over k).
__global__ void __launch_bounds__(kSortThreads) k_sp_gather_plan(const int64_t *__restrict__ off, const DevState *st,
                                                                 const double *__restrict__ coef, const int64_t *hnum,
                                                                 int64_t *__restrict__ goff, int64_t *gn, int64_t cap,
                                                                 DevState *stw)
{
    __shared__ int64_t s_base;
    __shared__ int64_t wsum[16];
    if (sp_aborted(st))
        return;
    const int64_t N = st->N;
    if (threadIdx.x == 0)
        s_base = *hnum;
    __syncthreads();
    for (int64_t c0 = 0; c0 < N; c0 += blockDim.x) {
        const int64_t k = c0 + threadIdx.x;
        const int64_t len = (k < N && coef[k] != 0.0) ? off[k + 1] - off[k] : 0;
        // block exclusive scan of len
        int64_t x = len;
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(x, o, 64);
            if (lane >= o)
                x += y;
        }
        if (lane == 63)
            wsum[w] = x;
        __syncthreads();
        int64_t pre = s_base;
        for (int q = 0; q < w; ++q)
            pre += wsum[q];
        if (k < N)
            goff[k] = pre + x - len;
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t t = 0;
            for (int q = 0; q < (int)(blockDim.x >> 6); ++q)
                t += wsum[q];
            s_base += t;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (s_base > cap) {
            stw->full = 2;  // the gathered list exceeds the scratch
            *gn = 0;
        } else {
            *gn = s_base;
        }
    }
}

// Copy the gathered list: h's terms, then -c_k times V_k's terms (one wave per element).
__global__ void __launch_bounds__(256) k_sp_gather(const uint64_t *__restrict__ pk, const double *__restrict__ pc,
                                                   const int64_t *__restrict__ off, const DevState *st,
                                                   const double *__restrict__ coef, const int64_t *__restrict__ goff,
                                                   const uint64_t *__restrict__ hk, const double *__restrict__ hc,
                                                   const int64_t *hnum, const int64_t *gn, uint64_t *__restrict__ tk,
                                                   double *__restrict__ tc)
{
    if (sp_aborted(st) || *gn == 0)
        return;
    const int64_t N = st->N, nh = *hnum;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nh; i += (int64_t)gridDim.x * blockDim.x) {
        tk[i] = hk[i];
        tc[i] = hc[i];
    }
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t k = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); k < N; k += nwaves) {
        const double ck = coef[k];
        if (ck == 0.0)
            continue;
        const int64_t a0 = off[k], na = off[k + 1] - a0, g0 = goff[k];
        for (int64_t i = lane; i < na; i += 64) {
            tk[g0 + i] = pk[a0 + i];
            tc[g0 + i] = -ck * pc[a0 + i];
        }
    }
}

// The decision for the candidate (hk, hc, *hnum) after its projection passes: keep iff its
// norm exceeds tol (bracket) or tol * ||g|| (generator, rel = 1); a kept candidate is
// normalised and appended as element N.  One workgroup.
__global__ void __launch_bounds__(kSortThreads) k_sp_finalize(const uint64_t *__restrict__ hk,
                                                              const double *__restrict__ hc, const int64_t *hnum,
                                                              const double *hn, double tol, int rel, int early_exit,
                                                              int64_t ambient, int64_t cap, int64_t max_terms,
                                                              uint64_t *__restrict__ pk, double *__restrict__ pc,
                                                              int64_t *__restrict__ off, DevState *st)
{
    __shared__ double red[16];
    __shared__ int verdict;
    __shared__ double s_inv;
    if (sp_aborted(st))
        return;
    const int64_t n = *hnum, N = st->N;
    double sq = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
        sq += hc[i] * hc[i];
    const double rr = sqrt(block_sum_1024(sq, red));
    if (threadIdx.x == 0) {
        const double h0 = *hn;
        const double thr = rel ? tol * h0 : tol;
        verdict = 0;
        if (!rel)
            st->n_cand++;
        if (!isfinite(rr) || !isfinite(h0)) {
            st->numeric_error = 1;
        } else if (h0 == 0.0 || !(rr > thr)) {
            if (!rel) {
                if (h0 == 0.0)
                    st->n_zero++;
                st->max_rej = fmax(st->max_rej, rr);
            }
        } else if (!rel && N >= ambient) {
            st->numeric_error = 2;  // one more independent element than the space holds
        } else if (N >= cap) {
            st->full = 1;
        } else if (off[N] + n > max_terms) {
            st->full = 3;  // the term pool is exhausted
        } else {
            verdict = 1;
            s_inv = 1.0 / rr;
            if (rel) {
                st->n_gen_acc++;
            } else {
                st->n_acc++;
                st->min_acc = fmin(st->min_acc, rr);
            }
        }
    }
    __syncthreads();
    if (!verdict)
        return;
    const int64_t base = off[N];
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        pk[base + i] = hk[i];
        pc[base + i] = hc[i] * s_inv;
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        off[N + 1] = base + n;
        st->N = N + 1;
        if (early_exit && N + 1 >= ambient)
            st->done = 1;
    }
}

// The list of generator g (terms [t0, t1) of the staged generators) into the scratch.
__global__ void k_sp_load(const uint64_t *__restrict__ gk, const double *__restrict__ gc, int64_t t0, int64_t t1,
                          uint64_t *__restrict__ tk, double *__restrict__ tc, int64_t *tn)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < t1 - t0; i += (int64_t)gridDim.x * blockDim.x) {
        tk[i] = gk[t0 + i];
        tc[i] = gc[t0 + i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *tn = t1 - t0;
}

}  // namespace

struct SparsePauli {
    int nq = 0;
    int64_t cap = 0, max_terms = 0, scratch = 0;
    uint64_t *pk = nullptr;  // term pool: keys
    double *pc = nullptr;    //            coefficients
    int64_t *off = nullptr;  // cap + 1 element offsets into the pool
    uint64_t *tk = nullptr, *hk = nullptr;  // scratch list, candidate list
    double *tc = nullptr, *hc = nullptr;
    int64_t *cnt = nullptr;  // [0] scratch count, [1] candidate count, [2] gathered count
    double *hn = nullptr;    // reference norm of the current candidate
    double *coef = nullptr;  // cap coefficients
    int64_t *goff = nullptr; // cap gather offsets
    uint64_t *gk = nullptr;  // staged generator terms
    double *gc = nullptr;
    std::vector<int64_t> gen_off;  // host: generator term offsets
};

void sparse_pauli_destroy(SparsePauli *s)
{
    if (!s)
        return;
    for (void *p : {(void *)s->pk, (void *)s->pc, (void *)s->off, (void *)s->tk, (void *)s->hk, (void *)s->tc,
                    (void *)s->hc, (void *)s->cnt, (void *)s->hn, (void *)s->coef, (void *)s->goff, (void *)s->gk,
                    (void *)s->gc})
        if (p)
            (void)hipFree(p);
    delete s;
}

hipError_t sparse_pauli_create(SparsePauli **out, int nq, int64_t cap, int64_t max_terms, int64_t scratch,
                               const int64_t *gen_off, int n_gen, const uint64_t *keys, const double *coefs,
                               hipStream_t s)
{
    auto *sp = new (std::nothrow) SparsePauli();
    if (!sp)
        return hipErrorOutOfMemory;
    sp->nq = nq;
    sp->cap = cap;
    sp->max_terms = max_terms;
    int64_t P = 1;
    while (P < scratch)
        P <<= 1;
    sp->scratch = P;
    sp->gen_off.assign(gen_off, gen_off + n_gen + 1);
    const int64_t gt = std::max<int64_t>(gen_off[n_gen], 1);
    hipError_t e;
    if ((e = hipMalloc(&sp->pk, (size_t)max_terms * 8)) != hipSuccess ||
        (e = hipMalloc(&sp->pc, (size_t)max_terms * 8)) != hipSuccess ||
        (e = hipMalloc(&sp->off, (size_t)(cap + 1) * 8)) != hipSuccess ||
        (e = hipMalloc(&sp->tk, (size_t)P * 8)) != hipSuccess || (e = hipMalloc(&sp->tc, (size_t)P * 8)) != hipSuccess ||
        (e = hipMalloc(&sp->hk, (size_t)P * 8)) != hipSuccess || (e = hipMalloc(&sp->hc, (size_t)P * 8)) != hipSuccess ||
        (e = hipMalloc(&sp->cnt, 4 * 8)) != hipSuccess || (e = hipMalloc(&sp->hn, 8)) != hipSuccess ||
        (e = hipMalloc(&sp->coef, (size_t)std::max<int64_t>(cap, 1) * 8)) != hipSuccess ||
        (e = hipMalloc(&sp->goff, (size_t)std::max<int64_t>(cap, 1) * 8)) != hipSuccess ||
        (e = hipMalloc(&sp->gk, (size_t)gt * 8)) != hipSuccess || (e = hipMalloc(&sp->gc, (size_t)gt * 8)) != hipSuccess ||
        (e = hipMemsetAsync(sp->off, 0, (size_t)(cap + 1) * 8, s)) != hipSuccess ||
        (e = hipMemsetAsync(sp->cnt, 0, 4 * 8, s)) != hipSuccess ||
        (e = hipMemcpyAsync(sp->gk, keys, (size_t)gen_off[n_gen] * 8, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(sp->gc, coefs, (size_t)gen_off[n_gen] * 8, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess) {
        sparse_pauli_destroy(sp);
        return e;
    }
    *out = sp;
    return hipSuccess;
}

// Projection passes and decision of the candidate in the scratch list (count cnt[0]).
static hipError_t sp_decide(SparsePauli *sp, DevState *st, double tol, bool generator, int early_exit, int64_t ambient,
                            hipStream_t s)
{
    int64_t *tn = sp->cnt, *hnum = sp->cnt + 1, *gn = sp->cnt + 2;
    const unsigned wg = (unsigned)std::min<int64_t>(256, (sp->cap + 3) / 4);
    hipLaunchKernelGGL(k_sp_sort_reduce, dim3(1), dim3(kSortThreads), 0, s, sp->tk, sp->tc, (const int64_t *)tn,
                       sp->scratch, sp->hk, sp->hc, hnum, sp->hn, 1, st);
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_sp_coef, dim3(wg), dim3(256), 0, s, (const uint64_t *)sp->pk, (const double *)sp->pc,
                           (const int64_t *)sp->off, (const DevState *)st, (const uint64_t *)sp->hk,
                           (const double *)sp->hc, (const int64_t *)hnum, sp->coef);
        hipLaunchKernelGGL(k_sp_gather_plan, dim3(1), dim3(kSortThreads), 0, s, (const int64_t *)sp->off,
                           (const DevState *)st, (const double *)sp->coef, (const int64_t *)hnum, sp->goff, gn,
                           sp->scratch, st);
        hipLaunchKernelGGL(k_sp_gather, dim3(wg), dim3(256), 0, s, (const uint64_t *)sp->pk, (const double *)sp->pc,
                           (const int64_t *)sp->off, (const DevState *)st, (const double *)sp->coef,
                           (const int64_t *)sp->goff, (const uint64_t *)sp->hk, (const double *)sp->hc,
                           (const int64_t *)hnum, (const int64_t *)gn, sp->tk, sp->tc);
        hipLaunchKernelGGL(k_sp_sort_reduce, dim3(1), dim3(kSortThreads), 0, s, sp->tk, sp->tc, (const int64_t *)gn,
                           sp->scratch, sp->hk, sp->hc, hnum, sp->hn, 0, st);
    }
    hipLaunchKernelGGL(k_sp_finalize, dim3(1), dim3(kSortThreads), 0, s, (const uint64_t *)sp->hk,
                       (const double *)sp->hc, (const int64_t *)hnum, (const double *)sp->hn, tol, generator ? 1 : 0,
                       early_exit, ambient, sp->cap, sp->max_terms, sp->pk, sp->pc, sp->off, st);
    return hipGetLastError();
}

hipError_t sparse_pauli_generator(SparsePauli *sp, int g, DevState *st, double tol, int64_t ambient, hipStream_t s)
{
    const int64_t t0 = sp->gen_off[g], t1 = sp->gen_off[g + 1];
    if (t1 - t0 > sp->scratch)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sp_load, dim3(64), dim3(256), 0, s, (const uint64_t *)sp->gk, (const double *)sp->gc, t0, t1,
                       sp->tk, sp->tc, sp->cnt);
    return sp_decide(sp, st, tol, true, 0, ambient, s);
}

hipError_t sparse_pauli_candidate(SparsePauli *sp, int64_t p, DevState *st, double tol, int early_exit,
                                  int64_t ambient, hipStream_t s)
{
    hipLaunchKernelGGL(k_sp_bracket, dim3(64), dim3(256), 0, s, (const uint64_t *)sp->pk, (const double *)sp->pc,
                       (const int64_t *)sp->off, p, st, sp->tk, sp->tc, sp->cnt, sp->scratch);
    return sp_decide(sp, st, tol, false, early_exit, ambient, s);
}

hipError_t sparse_pauli_terms(const SparsePauli *sp, int64_t N, int64_t *terms, hipStream_t s)
{
    *terms = 0;
    if (N <= 0)
        return hipSuccess;
    hipError_t e = hipMemcpyAsync(terms, sp->off + N, 8, hipMemcpyDeviceToHost, s);
    return e == hipSuccess ? hipStreamSynchronize(s) : e;
}

hipError_t sparse_pauli_basis(const SparsePauli *sp, int64_t N, int64_t *offsets, uint64_t *keys, double *coefs,
                              int64_t capacity, int64_t *written, hipStream_t s)
{
    int64_t terms = 0;
    hipError_t e = sparse_pauli_terms(sp, N, &terms, s);
    *written = terms;
    if (e != hipSuccess || terms > capacity)
        return e;
    if ((e = hipMemcpyAsync(offsets, sp->off, (size_t)(N + 1) * 8, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return e;
    if (terms > 0 && ((e = hipMemcpyAsync(keys, sp->pk, (size_t)terms * 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
                      (e = hipMemcpyAsync(coefs, sp->pc, (size_t)terms * 8, hipMemcpyDeviceToHost, s)) != hipSuccess))
        return e;
    return hipStreamSynchronize(s);
}

}  // namespace lie

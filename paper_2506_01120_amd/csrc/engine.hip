// Host control loop and C ABI of the closure engine (see include/lie_closure.h).
//
// The host loop owns one problem's device state: the FP64 basis V64 in the
// packed anti-Hermitian layout, the candidate block buffer, coefficient and
// scratch buffers, and the DevState counters.  It runs the generator phase and
// then the bracket loop of the dimension-only orthonormalization algorithm as a
// sequence of block steps over consecutive pair indices.
#include "lie_internal.h"
#include "../../include/lie_closure.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <type_traits>
#include <string>
#include <vector>

namespace {

thread_local std::string g_last_error;

lie_status fail(lie_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                                                     \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess)                                                                             \
            return fail(e_ == hipErrorOutOfMemory ? LIE_ERR_OOM : LIE_ERR_DEVICE, "%s failed: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                                \
    } while (0)

// Blocks of at most this many rows use the split-K GEMV projection; larger ones the matrix-core GEMMs.
constexpr int kGemvRows = 4;
// Set while the batch API creates its problems: their passes are grouped launches that
// need no split-K workspace.
thread_local bool t_batch_member = false;
// Block steps enqueued between two synchronisations: growth-size blocks, saturated blocks.
constexpr int kGrowthQueued = 4;
// SCREEN threshold on the FP32-screened residual (paper norm) once the basis is at the ambient
// bound: below it a candidate is rejected without FP64 work (every candidate is dependent there),
// at or above it the candidate is re-checked in FP64.  It lies far above the screen's rounding
// (dependent candidates screen at <= 2e-6) and far below the residual of any candidate that is
// independent of a basis short of the bound; with config.tau_rej > 0 the given value is applied
// at every basis size instead (an uncertified, approximate screen).
constexpr double kDefaultTauFp32 = 1e-4;
// The same threshold for the split-BF16 screen (dependent candidates screen at <= 2e-5).
constexpr double kDefaultTauBf16x3 = 1e-2;
constexpr int kMaxBlock = 16384;
constexpr int kMaxD = 128;

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Per-kernel-class launch counters, algorithmic work, and (optionally) HIP-event
// durations.  Events bracket single kernel launches on the handle's stream and
// are harvested at the host loop's synchronisation points.
struct KernelTimer {
    bool on = false;
    struct Pending {
        int k;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    int64_t n[LIE_K_COUNT] = {};
    double ms[LIE_K_COUNT] = {};
    double flops[LIE_K_COUNT] = {};
    double bytes[LIE_K_COUNT] = {};
    hipEvent_t cur_a = nullptr;

    hipEvent_t get()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess)
            return nullptr;
        return e;
    }
    void begin(hipStream_t s)
    {
        cur_a = nullptr;
        if (!on)
            return;
        cur_a = get();
        if (cur_a)
            (void)hipEventRecord(cur_a, s);
    }
    void end(int k, hipStream_t s, double f, double b)
    {
        n[k]++;
        flops[k] += f;
        bytes[k] += b;
        if (!on || !cur_a)
            return;
        hipEvent_t e = get();
        if (!e)
            return;
        (void)hipEventRecord(e, s);
        pending.push_back({k, cur_a, e});
        cur_a = nullptr;
    }
    // Call only after the stream has been synchronised.
    void harvest()
    {
        for (auto &p : pending) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess)
                ms[p.k] += t;
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pending.clear();
    }
    ~KernelTimer()
    {
        for (auto &p : pending) {
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        for (hipEvent_t e : pool)
            (void)hipEventDestroy(e);
    }
};

}  // namespace

struct lie_closure {
    // problem
    int d = 0;
    int64_t D = 0;
    double tol = 0;
    int n_gen = 0;
    int64_t cap = 0;
    int64_t ambient = 0;
    lie_closure_config cfg{};
    int block = 1;           // fixed block size, or 0: adaptive (growth / saturated sizes below)
    int block_growth = 32;   // adaptive: block size while most candidates are accepted
    int block_sat = 1024;    // adaptive: block size once acceptances are rare
    int tile_dot = 0, tile_sub = 0;  // screening GEMM tiles of full saturated blocks (0: heuristic)
    int autotuned = 0;       // 1: timed at init, 2: from the tune cache
    int bmax = 1;            // allocation bound of any block
    bool screened = false;   // FP32 screening pass in front of the FP64 decisions
    int policy = lie::POL_ALL;
    double policy_thr = 0.0;
    bool certify = false;    // screen rejections only at the ambient bound (see classify_body)
    // device
    int device = -1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *pool = nullptr;        // one device allocation holding every buffer below that init sets up
    double *V64 = nullptr;       // cap x D, FP64 basis
    float *Vs = nullptr;         // cap x D, FP32 rounding of V64 (screened modes)
    double *H64 = nullptr;       // block x D, FP64 candidates, then residuals
    float *Hs = nullptr;         // block x D, FP32 screened candidates
    double *C = nullptr;         // block x cap FP64 coefficients
    float *Cs = nullptr;         // block x cap FP32 coefficients
    double *part = nullptr;      // FP64 split-K scratch + norm partials
    double *splitws = nullptr;   // K slices of small matrix-core passes
    size_t splitws_n = 0;
    double *normpart_s = nullptr;// block x tiles, screened residual partial norms
    // split-BF16 screen (single problems): pre-split interleaved hi/lo planes of the basis
    // (rows, and transposed), of the candidate block and of its coefficients
    bool planes = false;
    lie::PlaneGeom pg{};
    __bf16 *Vp = nullptr;        // cap_rows x ld
    __bf16 *Vt = nullptr;        // d_rows x ldt
    __bf16 *Hp = nullptr;        // b_rows x ld
    __bf16 *Cp = nullptr;        // b_rows x ldt
    int64_t *planes_n = nullptr; // basis rows already in Vp / Vt
    double *cand_a2 = nullptr;   // block: squared residual of the first pass (screen or FP64)
    double *cand_n2 = nullptr;   // block: squared candidate norm of the first pass
    double *rho2 = nullptr;      // block: squared FP64 residuals of survivors
    double *h2 = nullptr;        // block: squared FP64 candidate norms of survivors
    double *h2b = nullptr;       // block: scratch norms
    int *surv_rows = nullptr;    // block: survivor -> candidate
    int64_t *surv_pairs = nullptr;  // block: survivor -> pair index
    int *slot = nullptr;         // block: candidate -> survivor or -1
    int *keep = nullptr;         // block: survivors left to the in-block decisions (acceptance kernel)
    // Algorithm 3 (config.raw_basis): raw elements and where each came from
    bool raw = false;
    double *B64 = nullptr;       // cap x D, raw elements (packed), FP64
    float *Bs = nullptr;         // cap x D, their FP32 rounding (screened modes)
    double *Graw = nullptr;      // n_gen x D, packed generators as given
    int64_t *elem_src = nullptr; // cap: pair index of each element, or -(generator + 1)
    // comparison baseline (config.method = LIE_METHOD_RANK_SVD): standard algorithm, SVD rank test
    int method = LIE_METHOD_ORTHONORMALIZATION;
    lie::RankTester *rank = nullptr;
    // Pauli-sum representation (config.representation = LIE_REP_PAULI): rows are coordinates over
    // the 4^nq strings; each element's support is recorded for the sparse bracket
    bool pauli = false;
    int nq = 0;
    int *sup_cnt = nullptr;      // cap
    int *sup_idx = nullptr;      // cap x D
    // sparse Pauli-sum representation (lie_closure_init_pauli_sparse): elements as term lists
    bool sparse = false;
    lie::SparsePauli *sp = nullptr;
    // matrix-inversion method (config.method = LIE_METHOD_MATRIX_INVERSION)
    bool inv = false;
    lie::GramInverse *ginv = nullptr;
    double *Xc = nullptr;        // block x cap: x = A^{-1} beta of every candidate
    int *nsurv = nullptr;        // 1: survivor count
    lie::DevState *st = nullptr;
    double *scalar = nullptr;    // one double of device scratch
    // host mirror
    lie::DevState hs{};
    int64_t cursor = 0;  // next pair index
    bool done = false;
    bool failed = false;
    int64_t blocks = 0;
    int64_t host_syncs = 0;
    double run_ms = 0;
    KernelTimer timer;
    // captured steady-state block step (hipGraph), replayed with a device pair cursor
    int64_t *d_cursor = nullptr;
    bool cursor_on_device = false;
    struct {
        hipGraphExec_t exec = nullptr;
        int cnt = 0;
        int64_t n_hi = -1;
        bool screen = false;
        int64_t n[LIE_K_COUNT] = {};
        double flops[LIE_K_COUNT] = {}, bytes[LIE_K_COUNT] = {};
    } graph;
    int64_t graph_replays = 0;
    // bookkeeping of the grouped (batched) executor
    int64_t b_nlo = 0, b_qrows = 0, b_lastc = 0, b_lasta = 0;
    int b_cur = 0;

    ~lie_closure()
    {
        if (device >= 0)
            (void)hipSetDevice(device);
        if (stream)
            (void)hipStreamSynchronize(stream);
        if (graph.exec)
            (void)hipGraphExecDestroy(graph.exec);
        lie::rank_tester_destroy(rank);
        lie::sparse_pauli_destroy(sp);
        lie::gram_inverse_destroy(ginv);
        if (pool) {
            (void)hipFree(pool);  // every buffer of a dense handle is a slice of it
        } else {
            for (void *p : {(void *)Xc, (void *)sup_cnt, (void *)sup_idx})
                if (p)
                    (void)hipFree(p);
        }
        for (void *p : {(void *)d_cursor, (void *)V64, (void *)Vs, (void *)H64, (void *)Hs, (void *)C, (void *)Cs,
                        (void *)part, (void *)splitws,
                        (void *)normpart_s, (void *)cand_a2, (void *)cand_n2, (void *)rho2, (void *)h2, (void *)h2b,
                        (void *)surv_rows, (void *)surv_pairs, (void *)slot, (void *)keep, (void *)nsurv,
                        (void *)st, (void *)scalar, (void *)B64, (void *)Bs, (void *)Graw, (void *)elem_src,
                        (void *)Vp, (void *)Vt, (void *)Hp, (void *)Cp, (void *)planes_n})
            if (p && !pool)
                (void)hipFree(p);
        if (own_stream && stream)
            (void)hipStreamDestroy(stream);
    }

    lie_status sync_state()
    {
        HIP_TRY(hipMemcpyAsync(&hs, st, sizeof hs, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        ++host_syncs;
        timer.harvest();
        return LIE_OK;
    }

    lie_status check_state()
    {
        if (hs.numeric_error == 1) {
            failed = true;
            return fail(LIE_ERR_NUMERIC, "non-finite residual norm encountered");
        }
        if (hs.numeric_error == 2) {
            failed = true;
            return fail(LIE_ERR_NUMERIC,
                        "an independent candidate was found with |V| already at the ambient bound %lld (spurious "
                        "element from round-off)",
                        (long long)ambient);
        }
        if (hs.full == 2) {
            failed = true;
            return fail(LIE_ERR_CAPACITY, "a bracket's or projection's term list exceeds the scratch lists");
        }
        if (hs.full == 3) {
            failed = true;
            return fail(LIE_ERR_CAPACITY, "the term pool of the sparse representation is exhausted");
        }
        if (hs.full) {
            failed = true;
            return fail(LIE_ERR_CAPACITY, "basis capacity %lld reached", (long long)cap);
        }
        return LIE_OK;
    }

    // One FP64 projection pass R = H - V^T V H over rows of H64 (all `cnt`, or
    // the survivor list when `rows`/`nrows` are given).  n_lo: known |V| (for the
    // work accounting); n_hi: an upper bound (grid, leading dimension).
    // Algorithmic work per row: 2*N*D flops for the coefficients and 2*N*D for
    // the subtraction; bytes: the basis streamed once per kernel, the row read
    // once and the residual written once.
    lie_status project(const int *rows, const int *nrows, double *rho2_out, double *h2_out, int cnt, int64_t n_lo,
                       int64_t n_hi, int kid_dot, int kid_sub, int kid_red)
    {
        lie::ProjShape sh{D, cnt, std::min(std::max<int64_t>(n_hi, 1), cap)};
        // verification passes run over the device-side survivor count: their work is accounted
        // by the acceptance kernel from that count (DevState::vfy_flops / vfy_bytes)
        const double acc = kid_dot == LIE_K_VERIFY ? 0.0 : 1.0;
        const double N = acc * (double)n_lo, Dd = (double)D, c = acc * cnt, w = sizeof(double);
        if (cnt > kGemvRows) {
            // matrix-core path: coefficients, then residual with fused norms, then the norm sums;
            // the coefficient rows span the capacity so that any basis size fits
            const int64_t ldc = lie::coef_ld(cap);
            // small passes split K over workgroups (coefficient slices first in the workspace,
            // then the residual's partial products)
            const lie::SplitPlan sp = lie::gemm_split_plan_f64(cnt, sh.n_hi, D, ldc, splitws ? splitws_n : 0);
            double *Cd = sp.kd > 1 ? splitws : C;
            double *P = splitws + (sp.kd > 1 ? (size_t)sp.kd * cnt * ldc : 0);
            timer.begin(stream);
            HIP_TRY(lie::launch_gemm_dot_f64(V64, st, H64, rows, nrows, cnt, D, sh.n_hi, ldc, Cd, stream, sp.kd));
            timer.end(kid_dot, stream, 2.0 * N * Dd * c, (N * Dd + c * Dd + c * N) * w);
            timer.begin(stream);
            HIP_TRY(lie::launch_gemm_sub_f64(V64, st, H64, rows, nrows, Cd, sh.n_hi, ldc, cnt, D, part, stream, sp.kd,
                                             sp.ks, P));
            timer.end(kid_sub, stream, 2.0 * N * Dd * c, (N * Dd + c * N + 2.0 * c * Dd) * w);
            timer.begin(stream);
            if (sp.ks > 1)
                HIP_TRY(lie::launch_gemm_sub_finish_f64(P, sp.ks, H64, rows, nrows, cnt, D, st, rho2_out, h2_out,
                                                        stream));
            else
                HIP_TRY(lie::launch_norm_final(part, nrows, cnt, lie::gemm_sub_tiles_f64(D), st, rho2_out, h2_out,
                                               stream));
            timer.end(kid_red, stream, 0, 0);
            return LIE_OK;
        }
        const int sd = lie::dot_slices_f64(sh, splitws ? splitws_n : 0);
        double *Cd = sd > 1 ? splitws : C;
        timer.begin(stream);
        HIP_TRY(lie::launch_dot_f64(V64, st, H64, rows, nrows, Cd, sh, stream, sd));
        timer.end(kid_dot, stream, 2.0 * N * Dd * c, (N * Dd + c * Dd + c * N) * w);
        timer.begin(stream);
        HIP_TRY(lie::launch_sub_f64(V64, st, Cd, nrows, part, sh, stream, sd));
        timer.end(kid_sub, stream, 2.0 * N * Dd * c, (N * Dd + c * N + c * Dd) * w);
        const int ks = lie::project_split_k(D, cnt, sh.n_hi);
        timer.begin(stream);
        HIP_TRY(lie::launch_reduce_f64(H64, rows, nrows, part, st, rho2_out, h2_out, sh, stream));
        timer.end(kid_red, stream, 3.0 * c * Dd, (ks + 2.0) * c * Dd * w);
        return LIE_OK;
    }

    lie_status classify(int cnt, int64_t p0, int pol, double thr, const int64_t *dp0 = nullptr, bool cert = false)
    {
        timer.begin(stream);
        HIP_TRY(lie::launch_classify(cand_a2, cand_n2, cnt, p0, pol, thr, st, surv_rows, surv_pairs, slot, nsurv,
                                     stream, dp0, ambient, cert ? 1 : 0));
        timer.end(LIE_K_REDUCE, stream, 0, 0);
        return LIE_OK;
    }

    // vpasses / vbracket: the FP64 verification the survivors went through before this launch
    // (projection passes, recomputed bracket), accounted by the kernel from the survivor count.
    lie_status accept(int cnt, int mode, bool screen_first, const int *rrow, const double *h2_surv, int kid,
                      int64_t src0 = 0, int vpasses = 0, int vbracket = 0)
    {
        lie::AcceptArgs a{};
        a.V = V64;
        a.Vs = Vs;
        a.st = st;
        a.H = H64;
        a.rrow = rrow;
        a.cand_a2 = cand_a2;
        a.cand_n2 = cand_n2;
        a.slot = slot;
        a.nsurv = nsurv;
        a.surv_cand = surv_rows;
        a.keep = keep;
        a.surv_pairs = surv_pairs;
        a.elem_src = raw ? elem_src : nullptr;
        a.src0 = src0;
        a.rel = raw && mode == 1 ? 1 : 0;
        a.track_new = pauli ? 1 : 0;
        a.h2 = h2_surv;
        a.rho2 = inv ? nullptr : rho2;  // the matrix-inversion step has no second projection pass
        a.cnt = cnt;
        a.D = D;
        a.cap = cap;
        a.ambient = ambient;
        a.tol = tol;
        a.mode = mode;
        a.screened = screen_first ? 1 : 0;
        a.early_exit = mode == 1 ? cfg.early_exit : 0;
        a.lds_doubles = lie::accept_lds_doubles(cnt, D);
        a.vpasses = vpasses;
        a.vbracket = vbracket;
        a.d = d;
        timer.begin(stream);
        HIP_TRY(lie::launch_accept_f64(a, stream));
        timer.end(kid, stream, 0, 0);
        if (pauli) {
            timer.begin(stream);
            HIP_TRY(lie::launch_pauli_support(V64, D, st, cnt, sup_cnt, sup_idx, stream));
            timer.end(LIE_K_OTHER, stream, 0, 0);
        }
        if (raw) {
            // Algorithm 3: the raw rows of this launch's appends (brackets of raw rows)
            timer.begin(stream);
            HIP_TRY(lie::launch_raw_append(Graw, B64, Bs, d, elem_src, st, cnt, stream, inv));
            timer.end(LIE_K_OTHER, stream, 0, 0);
        }
        return LIE_OK;
    }

    // Generator phase: every generator in input order, FP64, relative threshold.
    // Generator phase of the standard algorithm: each generator is kept iff it raises the
    // rank of the raw basis.
    lie_status generators_rank(const double *packed)
    {
        unsigned char flag = 0;
        for (int g = 0; g < n_gen; ++g) {
            const int64_t N = hs.N;
            if (N >= D || N >= cap)
                break;
            HIP_TRY(lie::rank_tester_run(rank, B64, N, packed + (size_t)g * D, 1, &flag));
            if (flag) {
                HIP_TRY(hipMemcpyAsync(B64 + N * D, packed + (size_t)g * D, D * sizeof(double),
                                       hipMemcpyDeviceToDevice, stream));
                hs.N = N + 1;
                hs.n_gen_acc++;
            }
        }
        HIP_TRY(hipStreamSynchronize(stream));
        return LIE_OK;
    }

    lie_status generators(const double *gens_host)
    {
        double *staging = nullptr;
        const size_t bytes = (size_t)n_gen * D * 2 * sizeof(double);
        HIP_TRY(hipMalloc(&staging, bytes));
        struct Guard {
            double *p;
            ~Guard() { (void)hipFree(p); }
        } guard{staging};
        double *packed = raw ? Graw : nullptr;  // Algorithm 3 keeps the packed generators
        if (!raw)
            HIP_TRY(hipMalloc(&packed, (size_t)n_gen * D * sizeof(double)));
        Guard guard2{raw ? nullptr : packed};
        if (pauli) {
            // Pauli coordinates of each generator (fast Walsh-Hadamard transforms on the host)
            std::vector<double> coords((size_t)n_gen * D);
            for (int g = 0; g < n_gen; ++g)
                lie::pauli_from_dense(gens_host + (size_t)g * D * 2, nq, coords.data() + (size_t)g * D);
            HIP_TRY(hipMemcpyAsync(packed, coords.data(), (size_t)n_gen * D * sizeof(double), hipMemcpyHostToDevice,
                                   stream));
            HIP_TRY(hipStreamSynchronize(stream));
        } else {
            HIP_TRY(hipMemcpyAsync(staging, gens_host, bytes, hipMemcpyHostToDevice, stream));
            HIP_TRY(lie::launch_pack_c128(staging, packed, n_gen, d, stream));
        }
        if (method == LIE_METHOD_RANK_SVD)
            return generators_rank(packed);
        lie_status s;
        if (inv) {
            // Algorithm 2's generator phase: each generator against B through A^{-1}, unit-normalised
            for (int g = 0; g < n_gen; ++g) {
                HIP_TRY(hipMemcpyAsync(H64, packed + (size_t)g * D, D * sizeof(double), hipMemcpyDeviceToDevice,
                                       stream));
                const int64_t N = hs.N;
                if ((s = step_inv(1, true, -(int64_t)g - 1)) != LIE_OK || (s = sync_state()) != LIE_OK ||
                    (s = check_state()) != LIE_OK)
                    return s;
                if (hs.N > N && (s = refresh_inverse()) != LIE_OK)
                    return s;
            }
            return LIE_OK;
        }
        for (int g = 0; g < n_gen; ++g) {
            HIP_TRY(hipMemcpyAsync(H64, packed + (size_t)g * D, D * sizeof(double), hipMemcpyDeviceToDevice, stream));
            if ((s = project(nullptr, nullptr, cand_a2, cand_n2, 1, g, g, LIE_K_OTHER, LIE_K_OTHER, LIE_K_OTHER)) !=
                LIE_OK)
                return s;
            if ((s = classify(1, 0, lie::POL_REL, tol)) != LIE_OK)
                return s;
            if ((s = project(surv_rows, nsurv, rho2, h2b, 1, g, g, LIE_K_OTHER, LIE_K_OTHER, LIE_K_OTHER)) != LIE_OK)
                return s;
            if ((s = accept(1, 0, false, surv_rows, nullptr, LIE_K_OTHER, -(int64_t)g - 1)) != LIE_OK)
                return s;
        }
        if ((s = sync_state()) != LIE_OK)
            return s;
        return check_state();
    }

    // FP64 block step over pair indices [cursor, cursor + cnt).
    // Bracket work per candidate: one complex d x d product (8 d^3 flops), since
    // [a,b] = ab - (ab)^H for anti-Hermitian a, b; bytes: two operands read, one result written.
    lie_status step_fp64(int cnt, int64_t n_lo, int64_t n_hi, const int64_t *dp0 = nullptr)
    {
        const double c = cnt, Dd = (double)D, dd = d;
        // in a screened run these FP64 blocks are the growth phase: a class of their own, so that
        // the screen-precision classes hold the screen's kernels only
        const int kc = screened ? LIE_K_GROWTH : LIE_K_COMM, kd = screened ? LIE_K_GROWTH : LIE_K_DOT,
                  ks = screened ? LIE_K_GROWTH : LIE_K_SUB, kr = screened ? LIE_K_GROWTH : LIE_K_REDUCE;
        timer.begin(stream);
        if (pauli)
            HIP_TRY(lie::launch_comm_pauli(V64, sup_cnt, sup_idx, nq, cursor, cnt, st, H64, stream, dp0));
        else
            HIP_TRY(lie::launch_comm_f64(raw ? B64 : V64, d, cursor, nullptr, nullptr, cnt, st, H64, stream, dp0));
        timer.end(kc, stream, pauli ? 0.0 : 8.0 * dd * dd * dd * c, 3.0 * c * Dd * sizeof(double));
        lie_status s;
        if ((s = project(nullptr, nullptr, cand_a2, cand_n2, cnt, n_lo, n_hi, kd, ks, kr)) != LIE_OK)
            return s;
        if ((s = classify(cnt, cursor, raw ? lie::POL_REL : lie::POL_ABS, tol, dp0)) != LIE_OK)
            return s;
        // re-orthogonalisation pass for the survivors only (twice is enough)
        if ((s = project(surv_rows, nsurv, rho2, h2b, cnt, 0, n_hi, LIE_K_VERIFY, LIE_K_VERIFY, LIE_K_VERIFY)) !=
            LIE_OK)
            return s;
        return accept(cnt, 1, false, surv_rows, nullptr, LIE_K_ACCEPT, 0, 1, 0);
    }

    // Screened block step: FP32 bracket and projection on MFMA, classification,
    // then FP64 recomputation (bracket + two projection passes) of the survivors.
    lie_status step_screen(int cnt, int64_t n_lo, int64_t n_hi, const int64_t *dp0 = nullptr)
    {
        const double c = cnt, Dd = (double)D, dd = d, N = (double)n_lo, w = sizeof(float);
        const int64_t nh = std::min(std::max<int64_t>(n_hi, 1), cap);
        timer.begin(stream);
        // split BF16 on planes: the bracket writes the candidate rows as hi/lo planes itself
        HIP_TRY(lie::launch_comm_f32(raw ? Bs : Vs, d, cursor, cnt, st, Hs, cand_n2, stream, dp0, planes ? Hp : nullptr,
                                     pg.ld));
        timer.end(LIE_K_COMM, stream, 8.0 * dd * dd * dd * c, 3.0 * c * Dd * w);
        const bool tuned = cnt == block_sat && tile_dot > 0;
        const int tile_d = tuned ? tile_dot : lie::gemm_tile_f32(cnt, nh);
        const int tile_s = tuned ? tile_sub : lie::gemm_tile_f32(cnt, D);
        const bool bf = cfg.precision == LIE_PREC_BF16X3;
        const int64_t ldc = lie::coef_ld(cap);
        if (planes) {
            // new basis rows into planes, then the two GEMMs on planes
            timer.begin(stream);
            HIP_TRY(lie::launch_planes_refresh(V64, D, st, planes_n, Vp, Vt, pg, stream));
            timer.end(LIE_K_OTHER, stream, 0.0, 0.0);
            timer.begin(stream);
            HIP_TRY(lie::launch_bfp_dot(Hp, Vp, st, cnt, cap, Cp, pg, stream));  // tiles up to the capacity: N may grow
            timer.end(LIE_K_DOT, stream, 2.0 * N * Dd * c, (N * Dd + c * Dd + c * N) * w);
            timer.begin(stream);
            HIP_TRY(lie::launch_bfp_sub(Cp, Vt, Hp, st, cnt, D, normpart_s, pg, stream));
            timer.end(LIE_K_SUB, stream, 2.0 * N * Dd * c, (N * Dd + c * N + c * Dd) * w);
            timer.begin(stream);
            HIP_TRY(lie::launch_norm_final(normpart_s, nullptr, cnt, lie::plane_sub_tiles(D, 0), st, cand_a2, nullptr,
                                           stream));
            timer.end(LIE_K_REDUCE, stream, 0, 0);
            return step_screen_verify(cnt, n_hi, dp0);
        }
        timer.begin(stream);
        HIP_TRY(bf ? lie::launch_gemm_dot_bf16x3(Vs, st, Hs, cnt, D, nh, ldc, Cs, tile_d, stream)
                   : lie::launch_gemm_dot_f32(Vs, st, Hs, cnt, D, nh, ldc, Cs, tile_d, stream));
        timer.end(LIE_K_DOT, stream, 2.0 * N * Dd * c, (N * Dd + c * Dd + c * N) * w);
        timer.begin(stream);
        HIP_TRY(bf ? lie::launch_gemm_sub_bf16x3(Vs, st, Hs, Cs, nh, ldc, cnt, D, normpart_s, tile_s, stream)
                   : lie::launch_gemm_sub_f32(Vs, st, Hs, Cs, nh, ldc, cnt, D, normpart_s, tile_s, stream));
        timer.end(LIE_K_SUB, stream, 2.0 * N * Dd * c, (N * Dd + c * N + c * Dd) * w);
        timer.begin(stream);
        HIP_TRY(lie::launch_norm_final(normpart_s, nullptr, cnt,
                                       bf ? lie::gemm_sub_tiles_bf16(D, tile_s) : lie::gemm_sub_tiles_f32(D, tile_s),
                                       st, cand_a2, nullptr, stream));
        timer.end(LIE_K_REDUCE, stream, 0, 0);
        return step_screen_verify(cnt, n_hi, dp0);
    }

    // The rest of a screened block step: classification, then the FP64 recomputation
    // (bracket + two projection passes) of the survivors and their acceptance.
    lie_status step_screen_verify(int cnt, int64_t n_hi, const int64_t *dp0)
    {
        lie_status s;
        if ((s = classify(cnt, cursor, policy, policy_thr, dp0, certify)) != LIE_OK)
            return s;
        timer.begin(stream);
        HIP_TRY(lie::launch_comm_f64(raw ? B64 : V64, d, 0, surv_pairs, nsurv, cnt, st, H64, stream));
        timer.end(LIE_K_VERIFY, stream, 0, 0);
        if ((s = project(nullptr, nsurv, rho2, h2, cnt, 0, n_hi, LIE_K_VERIFY, LIE_K_VERIFY, LIE_K_VERIFY)) != LIE_OK)
            return s;
        if ((s = project(nullptr, nsurv, rho2, h2b, cnt, 0, n_hi, LIE_K_VERIFY, LIE_K_VERIFY, LIE_K_VERIFY)) != LIE_OK)
            return s;
        return accept(cnt, 1, policy != lie::POL_ALL, nullptr, h2, LIE_K_ACCEPT, 0, 2, 1);
    }

    // Capture one block step (kernels reading the pair cursor from d_cursor, then
    // the cursor advance) and instantiate it; the work counters of the captured
    // launches are kept so that each replay can be accounted.
    lie_status capture(int cnt, int64_t n_lo, int64_t n_hi, bool screen)
    {
        if (graph.exec) {
            HIP_TRY(hipGraphExecDestroy(graph.exec));
            graph.exec = nullptr;
        }
        int64_t n0[LIE_K_COUNT];
        double f0[LIE_K_COUNT], b0[LIE_K_COUNT];
        std::memcpy(n0, timer.n, sizeof n0);
        std::memcpy(f0, timer.flops, sizeof f0);
        std::memcpy(b0, timer.bytes, sizeof b0);
        HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        lie_status s = screen ? step_screen(cnt, n_lo, n_hi, d_cursor) : step_fp64(cnt, n_lo, n_hi, d_cursor);
        hipError_t e = s == LIE_OK ? lie::launch_advance_cursor(d_cursor, cnt, stream) : hipSuccess;
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(stream, &g);
        for (int k = 0; k < LIE_K_COUNT; ++k) {
            graph.n[k] = timer.n[k] - n0[k];
            graph.flops[k] = timer.flops[k] - f0[k];
            graph.bytes[k] = timer.bytes[k] - b0[k];
        }
        std::memcpy(timer.n, n0, sizeof n0);  // capture executes nothing
        std::memcpy(timer.flops, f0, sizeof f0);
        std::memcpy(timer.bytes, b0, sizeof b0);
        if (s != LIE_OK) {
            if (g)
                (void)hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g)
                (void)hipGraphDestroy(g);
            return fail(LIE_ERR_DEVICE, "graph capture failed: %s",
                        hipGetErrorString(e != hipSuccess ? e : e2));
        }
        hipError_t e3 = hipGraphInstantiate(&graph.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e3 != hipSuccess) {
            graph.exec = nullptr;
            return fail(LIE_ERR_DEVICE, "graph instantiation failed: %s", hipGetErrorString(e3));
        }
        graph.cnt = cnt;
        graph.n_hi = n_hi;
        graph.screen = screen;
        return LIE_OK;
    }

    lie_status replay(int cnt, int64_t n_lo, int64_t n_hi, bool screen)
    {
        if (!graph.exec || graph.cnt != cnt || graph.n_hi != n_hi || graph.screen != screen) {
            lie_status s = capture(cnt, n_lo, n_hi, screen);
            if (s != LIE_OK)
                return s;
        }
        if (!cursor_on_device) {
            HIP_TRY(lie::launch_set_cursor(d_cursor, cursor, stream));
            cursor_on_device = true;
        }
        HIP_TRY(hipGraphLaunch(graph.exec, stream));
        for (int k = 0; k < LIE_K_COUNT; ++k) {
            timer.n[k] += graph.n[k];
            timer.flops[k] += graph.flops[k];
            timer.bytes[k] += graph.bytes[k];
        }
        ++graph_replays;
        return LIE_OK;
    }

    // Standard algorithm (Algorithm 1) with the SVD rank test, host-driven: each batch of
    // brackets [B_l, B_m] (pair order of the paper) is tested against the raw basis B; the
    // first candidate that raises the rank is appended and the candidates before it are
    // final (dependent on B, hence on every superset).  Batches grow while nothing is
    // accepted and restart at one candidate after an acceptance.
    lie_status run_rank(int64_t budget)
    {
        const auto t0 = std::chrono::steady_clock::now();
        constexpr int kRankBatch = 64;
        int64_t spent = 0;
        int cnt = 1;
        unsigned char flags[kRankBatch];
        lie_status s = LIE_OK;
        for (;;) {
            const int64_t N = hs.N;
            const int64_t avail = lie::pairs_below(N);
            if ((cfg.early_exit && N >= ambient) || cursor >= avail) {
                done = true;
                break;
            }
            if (budget >= 0 && spent >= budget) {
                s = LIE_INCOMPLETE;
                break;
            }
            const int c = (int)std::min<int64_t>(cnt, avail - cursor);
            int j = -1;
            if (N < D) {
                const double dd = d, cc = c, n1 = (double)N + 1.0, Dd = (double)D;
                timer.begin(stream);
                hipError_t e = lie::launch_comm_f64(B64, d, cursor, nullptr, nullptr, c, st, H64, stream);
                timer.end(LIE_K_COMM, stream, 8.0 * dd * dd * dd * cc, 3.0 * cc * Dd * sizeof(double));
                // singular values of c matrices D x (N+1): bidiagonalisation 4 m n^2 - 4 n^3 / 3 flops each
                timer.begin(stream);
                if (e == hipSuccess)
                    e = lie::rank_tester_run(rank, B64, N, H64, c, flags);
                timer.end(LIE_K_OTHER, stream, cc * (4.0 * Dd * n1 * n1 - 4.0 * n1 * n1 * n1 / 3.0),
                          cc * n1 * Dd * sizeof(double) * 2.0);
                if (e != hipSuccess) {
                    s = fail(LIE_ERR_DEVICE, "rank test failed: %s", hipGetErrorString(e));
                    failed = true;
                    break;
                }
                for (int q = 0; q < c && j < 0; ++q)
                    if (flags[q])
                        j = q;
            }
            const int processed = j >= 0 ? j + 1 : c;
            if (j >= 0) {
                if (N >= cap) {
                    hs.full = 1;
                    s = fail(LIE_ERR_CAPACITY, "basis capacity %lld reached", (long long)cap);
                    failed = true;
                    break;
                }
                const hipError_t e = hipMemcpyAsync(B64 + N * D, H64 + (int64_t)j * D, D * sizeof(double),
                                                    hipMemcpyDeviceToDevice, stream);
                if (e != hipSuccess) {
                    s = fail(LIE_ERR_DEVICE, "append failed: %s", hipGetErrorString(e));
                    failed = true;
                    break;
                }
                hs.N = N + 1;
                hs.n_acc++;
                cnt = 1;
            } else {
                cnt = std::min(2 * cnt, kRankBatch);
            }
            hs.n_cand += processed;
            hs.n_fp64 += processed;
            cursor += processed;
            spent += processed;
            ++blocks;
        }
        run_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return s;
    }

    // Matrix-inversion method (Algorithm 2): one block of candidates (brackets of unit-norm raw
    // rows, or one generator) tested against the raw basis B through x = A^{-1} beta and the
    // explicit residual h - B x (relative to ||h||, i.e. absolute for the unit-norm candidate);
    // survivors are then decided in candidate order against the elements appended earlier in
    // the block, and the new raw rows are appended unit-normalised.  N = hs.N is current.
    lie_status step_inv(int cnt, bool generator, int64_t src0)
    {
        const int64_t N = hs.N;
        const int64_t ldc = lie::coef_ld(cap);
        const double c = cnt, Dd = (double)D, Nd = (double)N, dd = d, w = sizeof(double);
        if (!generator) {
            timer.begin(stream);
            HIP_TRY(lie::launch_comm_f64(B64, d, cursor, nullptr, nullptr, cnt, st, H64, stream));
            timer.end(LIE_K_COMM, stream, 8.0 * dd * dd * dd * c, 3.0 * c * Dd * w);
        }
        timer.begin(stream);
        HIP_TRY(lie::launch_gemm_dot_f64(B64, st, H64, nullptr, nullptr, cnt, D, std::max<int64_t>(N, 1), ldc, C,
                                         stream));
        HIP_TRY(lie::gram_inverse_apply(ginv, C, ldc, N, cnt, Xc, ldc));
        timer.end(LIE_K_DOT, stream, 2.0 * Nd * Dd * c + 2.0 * Nd * Nd * c, (Nd * Dd + c * Dd + Nd * Nd + 2 * c * Nd) * w);
        timer.begin(stream);
        HIP_TRY(lie::launch_gemm_sub_f64(B64, st, H64, nullptr, nullptr, Xc, std::max<int64_t>(N, 1), ldc, cnt, D, part,
                                         stream));
        timer.end(LIE_K_SUB, stream, 2.0 * Nd * Dd * c, (Nd * Dd + c * Nd + 2.0 * c * Dd) * w);
        timer.begin(stream);
        HIP_TRY(lie::launch_norm_final(part, nullptr, cnt, lie::gemm_sub_tiles_f64(D), st, cand_a2, cand_n2, stream));
        timer.end(LIE_K_REDUCE, stream, 0, 0);
        lie_status s;
        if ((s = classify(cnt, generator ? 0 : cursor, lie::POL_REL, tol)) != LIE_OK)
            return s;
        return accept(cnt, generator ? 0 : 1, false, surv_rows, nullptr, LIE_K_ACCEPT, src0);
    }

    // A^{-1} expanded by the elements appended since the last call (bordered updates in element
    // order); a Schur complement that is not positive is the method's numerical failure.
    lie_status refresh_inverse()
    {
        int info = 0;
        const hipError_t e = lie::gram_inverse_update(ginv, B64, hs.N, &info);
        if (e != hipSuccess)
            return fail(LIE_ERR_DEVICE, "inverse Gram update failed: %s", hipGetErrorString(e));
        if (info != 0)
            return fail(LIE_ERR_NUMERIC, "Gram matrix of %lld elements is not numerically positive definite "
                                         "(bordered Cholesky pivot of element %d not positive); the matrix-inversion "
                                         "method lost accuracy",
                        (long long)hs.N, info - 1);
        return LIE_OK;
    }

    lie_status run_inv(int64_t budget)
    {
        const auto t0 = std::chrono::steady_clock::now();
        int64_t spent = 0;
        int cur = block_growth;
        lie_status s = LIE_OK;
        for (;;) {
            const int64_t N = hs.N;
            const int64_t avail = lie::pairs_below(N);
            if ((cfg.early_exit && N >= ambient) || cursor >= avail) {
                done = true;
                break;
            }
            if (budget >= 0 && spent >= budget) {
                s = LIE_INCOMPLETE;
                break;
            }
            const int cnt = (int)std::min<int64_t>(cur, avail - cursor);
            if ((s = step_inv(cnt, false, 0)) != LIE_OK || (s = sync_state()) != LIE_OK ||
                (s = check_state()) != LIE_OK)
                break;
            if (hs.N > N) {
                if ((s = refresh_inverse()) != LIE_OK)
                    break;
                cur = block_growth;
            } else {
                cur = block_sat;
            }
            cursor += cnt;
            spent += cnt;
            ++blocks;
        }
        if (s < 0)
            failed = true;
        run_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return s;
    }

    // Sparse Pauli-sum elements: one candidate at a time in Algorithm 4's order, every list
    // size on the device; the host learns |V| every kSparseQueued candidates.
    lie_status run_sparse(int64_t budget)
    {
        constexpr int64_t kSparseQueued = 256;
        const auto t0 = std::chrono::steady_clock::now();
        int64_t spent = 0;
        lie_status s = LIE_OK;
        for (;;) {
            const int64_t N = hs.N;
            const int64_t avail = lie::pairs_below(N);
            if (hs.done || (cfg.early_exit && N >= ambient) || cursor >= avail) {
                done = true;
                break;
            }
            if (budget >= 0 && spent >= budget) {
                s = LIE_INCOMPLETE;
                break;
            }
            int64_t q = std::min<int64_t>(kSparseQueued, avail - cursor);
            if (budget >= 0)
                q = std::min<int64_t>(q, budget - spent);
            for (int64_t i = 0; i < q; ++i)
                HIP_TRY(lie::sparse_pauli_candidate(sp, cursor + i, st, tol, cfg.early_exit, ambient, stream));
            cursor += q;
            spent += q;
            blocks += q;
            if ((s = sync_state()) != LIE_OK || (s = check_state()) != LIE_OK)
                break;
        }
        if (s < 0)
            failed = true;
        run_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return s;
    }

    lie_status run(int64_t budget)
    {
        if (sparse) {
            if (failed)
                return fail(LIE_ERR_STATE, "a previous run of this handle failed");
            if (done)
                return LIE_OK;
            HIP_TRY(hipSetDevice(device));
            return run_sparse(budget);
        }
        if (method == LIE_METHOD_MATRIX_INVERSION) {
            if (failed)
                return fail(LIE_ERR_STATE, "a previous run of this handle failed");
            if (done)
                return LIE_OK;
            HIP_TRY(hipSetDevice(device));
            return run_inv(budget);
        }
        if (method == LIE_METHOD_RANK_SVD) {
            if (failed)
                return fail(LIE_ERR_STATE, "a previous run of this handle failed");
            if (done)
                return LIE_OK;
            HIP_TRY(hipSetDevice(device));
            return run_rank(budget);
        }
        if (failed)
            return fail(LIE_ERR_STATE, "a previous run of this handle failed");
        if (done)
            return LIE_OK;
        HIP_TRY(hipSetDevice(device));
        const auto t0 = std::chrono::steady_clock::now();
        constexpr int kMaxQueued = 64;
        int64_t spent = 0;
        int queued = 0;
        int64_t queued_rows = 0;  // candidates enqueued since the last synchronisation
        int64_t n_lo = hs.N;  // |V| at the last synchronisation (a lower bound of the device value)
        int cur = block > 0 ? block : block_growth;
        int64_t last_cand = hs.n_cand, last_acc = hs.n_acc;
        lie_status s = LIE_OK;
        for (;;) {
            int64_t avail = lie::pairs_below(n_lo);
            const bool over_budget = budget >= 0 && spent >= budget;
            // growth and ramp-size blocks are re-evaluated often; saturated ones can queue deep
            const int max_queued = (block == 0 && cur < block_sat) ? kGrowthQueued : kMaxQueued;
            if (cursor >= avail || queued >= max_queued || over_budget) {
                if ((s = sync_state()) != LIE_OK || (s = check_state()) != LIE_OK)
                    break;
                queued = 0;
                queued_rows = 0;
                n_lo = hs.N;
                if (block == 0) {
                    // adaptive block: small while candidates are mostly accepted, growing fourfold per
                    // synchronisation while few are (a block's survivors that are new to the basis
                    // snapshot are decided in sequence, so a large block early on pays for every
                    // in-block duplicate); a basis at the ambient bound cannot grow, so it is saturated
                    // at once
                    const int64_t dc = hs.n_cand - last_cand, da = hs.n_acc - last_acc;
                    if (dc > 0)
                        cur = 8 * da > dc ? block_growth : std::min(block_sat, 4 * std::max(cur, block_growth));
                    if (n_lo >= ambient)
                        cur = block_sat;
                    last_cand = hs.n_cand;
                    last_acc = hs.n_acc;
                }
                avail = lie::pairs_below(n_lo);
                if (hs.done || (cfg.early_exit && n_lo >= ambient) || cursor >= avail) {
                    done = true;
                    break;
                }
                if (over_budget) {
                    s = LIE_INCOMPLETE;
                    break;
                }
            }
            const int cnt = (int)std::min<int64_t>(cur, avail - cursor);
            const int64_t n_hi = std::min<int64_t>(cap, n_lo + queued_rows);
            // while most candidates are accepted the screen filters nothing: decide in FP64 directly;
            // a certified screen rejects nothing below the ambient bound, so it waits for it too
            const bool growth = block == 0 && cur == block_growth;
            const bool screen_step = screened && !growth && (!certify || n_lo >= ambient);
            // full-size steps of the steady state replay a captured graph; the grid bound
            // is the synchronised basis size (the coefficient GEMMs stride beyond it)
            const bool steady = cnt == cur && !growth && cnt > kGemvRows && cfg.use_graphs && !timer.on;
            if (steady) {
                s = replay(cnt, n_lo, std::max<int64_t>(n_lo, 1), screen_step);
            } else {
                s = screen_step ? step_screen(cnt, n_lo, n_hi) : step_fp64(cnt, n_lo, n_hi);
                cursor_on_device = false;
            }
            if (s != LIE_OK)
                break;
            cursor += cnt;
            spent += cnt;
            ++queued;
            queued_rows += cnt;
            ++blocks;
        }
        run_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (s < 0)
            failed = true;
        return s;
    }
};

// ------------------------------------------------------------------ validation (host, before any HIP call)

namespace {

lie_status validate_generators(const double *g, int32_t n_gen, int32_t d, double tol, int64_t *ambient_out)
{
    if (!g)
        return fail(LIE_ERR_ARG, "generators is NULL");
    if (n_gen < 1)
        return fail(LIE_ERR_ARG, "n_gen must be >= 1 (got %d)", n_gen);
    if (d < 1 || d > kMaxD)
        return fail(LIE_ERR_ARG, "d must be in [1, %d] (got %d)", kMaxD, d);
    if (!(tol > 0.0 && tol < 1.0))
        return fail(LIE_ERR_ARG, "tol must satisfy 0 < tol < 1 (got %g)", tol);
    const int64_t D = (int64_t)d * d;
    bool traceless = true;
    for (int32_t k = 0; k < n_gen; ++k) {
        const double *x = g + (size_t)k * D * 2;
        double nrm2 = 0.0, defect2 = 0.0, tr_re = 0.0, tr_im = 0.0;
        for (int64_t e = 0; e < 2 * D; ++e)
            if (!std::isfinite(x[e]))
                return fail(LIE_ERR_NONFINITE, "generator %d has a non-finite entry", k);
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                const double re = x[2 * (i * d + j)], im = x[2 * (i * d + j) + 1];
                const double tre = x[2 * (j * d + i)], tim = x[2 * (j * d + i) + 1];
                nrm2 += re * re + im * im;
                // (g + g^H)_ij = g_ij + conj(g_ji)
                const double sre = re + tre, sim = im - tim;
                defect2 += sre * sre + sim * sim;
            }
        for (int i = 0; i < d; ++i) {
            tr_re += x[2 * (i * d + i)];
            tr_im += x[2 * (i * d + i) + 1];
        }
        const double nrm = std::sqrt(nrm2);
        if (std::sqrt(defect2) > 1e-12 * std::max(1.0, nrm))
            return fail(LIE_ERR_NOT_ANTIHERMITIAN,
                        "generator %d is not anti-Hermitian (||g + g^H||_F = %.3e); pass i*H for a Hermitian H", k,
                        std::sqrt(defect2));
        if (std::hypot(tr_re, tr_im) > 1e-12 * std::max(1.0, nrm))
            traceless = false;
    }
    *ambient_out = traceless ? D - 1 : D;
    if (D == 1)
        *ambient_out = traceless ? 0 : 1;
    return LIE_OK;
}

lie_status resolve_config(const lie_closure_config *in, lie_closure_config *out)
{
    lie_closure_config_default(out);
    if (!in)
        return LIE_OK;
    if (in->struct_size != sizeof(lie_closure_config))
        return fail(LIE_ERR_ARG, "config.struct_size must be %zu", sizeof(lie_closure_config));
    *out = *in;
    if (out->precision < LIE_PREC_FP64 || out->precision > LIE_PREC_BF16X3)
        return fail(LIE_ERR_ARG, "unknown precision %d", out->precision);
    if (out->decide < LIE_DECIDE_FP64 || out->decide > LIE_DECIDE_SCREEN)
        return fail(LIE_ERR_ARG, "unknown decide mode %d", out->decide);
    if (out->block < 0 || out->block > kMaxBlock)
        return fail(LIE_ERR_ARG, "block must be in [0, %d]", kMaxBlock);
    if (out->max_dim < 0)
        return fail(LIE_ERR_ARG, "max_dim must be >= 0");
    if (out->tau_rej < 0 || !std::isfinite(out->tau_rej))
        return fail(LIE_ERR_ARG, "tau_rej must be finite and >= 0");
    if (out->reserved0 != 0)
        return fail(LIE_ERR_ARG, "config.reserved0 must be zero");
    if (out->raw_basis != 0 && out->raw_basis != 1)
        return fail(LIE_ERR_ARG, "config.raw_basis must be 0 or 1");
    if (out->method != LIE_METHOD_ORTHONORMALIZATION && out->method != LIE_METHOD_RANK_SVD &&
        out->method != LIE_METHOD_MATRIX_INVERSION)
        return fail(LIE_ERR_ARG, "unknown method %d", out->method);
    if (out->method != LIE_METHOD_ORTHONORMALIZATION && out->precision != LIE_PREC_FP64)
        return fail(LIE_ERR_ARG, "the rank-test and matrix-inversion methods run in FP64 only");
    if (out->representation != LIE_REP_DENSE && out->representation != LIE_REP_PAULI)
        return fail(LIE_ERR_ARG, "unknown representation %d", out->representation);
    if (out->representation == LIE_REP_PAULI &&
        (out->precision != LIE_PREC_FP64 || out->method != LIE_METHOD_ORTHONORMALIZATION || out->raw_basis))
        return fail(LIE_ERR_ARG, "the Pauli representation runs the orthonormalization method in FP64 without raw_basis");
    for (int r : out->reserved)
        if (r != 0)
            return fail(LIE_ERR_ARG, "config.reserved must be zero");
    if (out->gemm_tile < 0 || out->gemm_tile > 2 || (out->gemm_tile != 0 && out->precision == LIE_PREC_FP64))
        return fail(LIE_ERR_ARG, "config.gemm_tile %d: screened precisions take 1 or 2, FP64 takes 0",
                    out->gemm_tile);
    if (out->autotune != 0 && out->autotune != 1)
        return fail(LIE_ERR_ARG, "config.autotune must be 0 or 1");
    out->tune_cache = nullptr;  // read at init only (see lie_closure_init), never kept
    return LIE_OK;
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

lie_status lie_closure_config_default(lie_closure_config *cfg)
{
    if (!cfg)
        return fail(LIE_ERR_ARG, "cfg is NULL");
    std::memset(cfg, 0, sizeof *cfg);
    cfg->struct_size = sizeof(lie_closure_config);
    cfg->precision = LIE_PREC_FP64;
    cfg->decide = LIE_DECIDE_SCREEN;
    cfg->block = 0;
    cfg->early_exit = 0;
    cfg->device = -1;
    cfg->use_graphs = 1;
    return LIE_OK;
}

lie_status lie_closure_init(lie_closure **out, const double *generators, int32_t n_gen, int32_t d, double tol,
                            const lie_closure_config *cfg_in)
{
    g_last_error.clear();
    if (!out)
        return fail(LIE_ERR_ARG, "out is NULL");
    *out = nullptr;
    int64_t ambient = 0;
    lie_status s = validate_generators(generators, n_gen, d, tol, &ambient);
    if (s != LIE_OK)
        return s;
    lie_closure_config cfg;
    if ((s = resolve_config(cfg_in, &cfg)) != LIE_OK)
        return s;
    if (cfg.representation == LIE_REP_PAULI && (d < 2 || (d & (d - 1)) != 0 || d > 128))
        return fail(LIE_ERR_ARG, "the Pauli representation needs d = 2^n with 1 <= n <= 7 (got %d)", d);
    if (cfg.method == LIE_METHOD_RANK_SVD) {
        if (d > 16)
            return fail(LIE_ERR_ARG, "the rank-test method is limited to d <= 16 (got %d)", d);
        cfg.block = 0;  // its batches are sized by the host loop
    }

    lie_closure *h = new (std::nothrow) lie_closure();
    if (!h)
        return fail(LIE_ERR_OOM, "host allocation failed");
    h->d = d;
    h->D = (int64_t)d * d;
    h->tol = tol;
    h->n_gen = n_gen;
    h->ambient = ambient;
    h->cfg = cfg;
    h->block = cfg.block;
    if (h->block == 0) {
        // adaptive sizes: the growth size bounds the sequential in-block work
        // (about block^2/2 * d^2 * 32 bytes through one compute unit per block)
        const int64_t D0 = (int64_t)d * d;
        h->block_growth = D0 <= 256 ? 64 : (D0 <= 1024 ? 32 : 16);
        // saturated size: enough 128-row candidate tiles that the coefficient GEMM
        // (candidates x basis rows) spans about 256 workgroups
        const int64_t ntiles = std::max<int64_t>(1, (std::max<int64_t>(ambient, 1) + 127) / 128);
        const int64_t want = ((256 + ntiles - 1) / ntiles) * 128;
        h->block_sat = (int)std::min<int64_t>(kMaxBlock, std::max<int64_t>(1024, want));
    }
    h->timer.on = cfg.profile != 0;
    h->screened = cfg.precision != LIE_PREC_FP64;
    if (h->screened) {
        switch (cfg.decide) {
        case LIE_DECIDE_FP64:
            h->policy = lie::POL_ALL;
            break;
        case LIE_DECIDE_STRICT:
            // certified; at the ambient bound only screened residuals below 100 * tol skip FP64
            h->policy = lie::POL_GE;
            h->policy_thr = 100.0 * tol;
            h->certify = true;
            break;
        default:
            h->policy = lie::POL_GE;
            h->policy_thr = cfg.tau_rej > 0 ? cfg.tau_rej
                                            : (cfg.precision == LIE_PREC_BF16X3 ? kDefaultTauBf16x3 : kDefaultTauFp32);
            h->certify = !(cfg.tau_rej > 0);  // an explicit threshold is applied uncertified
            break;
        }
    }
    h->method = cfg.method;
    h->pauli = cfg.representation == LIE_REP_PAULI;
    if (h->pauli)
        while ((1 << h->nq) < d)
            ++h->nq;
    h->inv = cfg.method == LIE_METHOD_MATRIX_INVERSION;
    h->raw = cfg.raw_basis != 0 || cfg.method != LIE_METHOD_ORTHONORMALIZATION;  // the other methods keep B
    if (h->raw) {
        // Algorithm 3: raw brackets have no fixed scale, so every threshold is relative to ||h||
        if (h->policy == lie::POL_GE)
            h->policy = lie::POL_GE_REL;
    }
    h->cap = cfg.max_dim > 0 ? std::min<int64_t>(cfg.max_dim, h->D) : std::max<int64_t>(ambient, 1);
    h->device = -1;

    auto bail = [&](lie_status st) {
        delete h;
        return st;
    };
    int dev = cfg.device;
    if (dev < 0) {
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess)
            return bail(fail(LIE_ERR_DEVICE, "hipGetDevice failed: %s", hipGetErrorString(e)));
    }
    h->device = dev;
    {
        hipError_t e = hipSetDevice(dev);
        if (e != hipSuccess)
            return bail(fail(LIE_ERR_DEVICE, "hipSetDevice(%d) failed: %s", dev, hipGetErrorString(e)));
        // the fixed workspace of the allocation-free entry points, once per device
        e = lie::noalloc_setup(dev);
        if (e != hipSuccess)
            return bail(fail(LIE_ERR_DEVICE, "workspace lookup on device %d failed: %s", dev, hipGetErrorString(e)));
    }
    if (cfg.stream) {
        h->stream = (hipStream_t)cfg.stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess)
            return bail(fail(LIE_ERR_DEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e)));
        h->own_stream = true;
    }
    const int64_t D = h->D;
    {
        const int maxb = lie::accept_max_block(D);
        if (h->block > maxb)
            return bail(fail(LIE_ERR_ARG, "block %d is too large for d = %d (at most %d)", h->block, d, maxb));
        if (h->block == 0) {
            h->block_sat = std::min(h->block_sat, maxb);
            h->block_growth = std::min(h->block_growth, h->block_sat);
        }
        if (h->block == 0 && cfg.autotune) {
            lie::TuneChoice tc{};
            bool cached = false;
            const hipError_t e = lie::autotune_block_step(dev, cfg.precision, d, ambient, maxb,
                                                          cfg_in ? cfg_in->tune_cache : nullptr, h->stream, &tc,
                                                          &cached);
            if (e != hipSuccess)
                return bail(fail(LIE_ERR_DEVICE, "autotuning failed: %s", hipGetErrorString(e)));
            h->block_sat = tc.block_sat;
            h->tile_dot = tc.tile_dot;
            h->tile_sub = tc.tile_sub;
            h->block_growth = std::min(h->block_growth, h->block_sat);
            h->autotuned = cached ? 2 : 1;
        }
        if (h->block == 0 && cfg.gemm_tile > 0)
            h->tile_dot = h->tile_sub = cfg.gemm_tile;  // an explicit tile replaces the timed or heuristic one
    }
    const int b = h->block > 0 ? h->block : std::max(h->block_growth, h->block_sat);
    h->bmax = b;
    // Every buffer is a 256-byte aligned slice of one device allocation: the layout is laid out
    // twice, once to size the allocation and once to place the slices.  A handle then costs one
    // hipMalloc instead of some thirty, which dominates the set-up of many live handles (a batch).
    size_t pool_off = 0;
    bool sizing = true;
    auto alloc = [&](auto **p, size_t n) -> lie_status {
        using T = std::remove_pointer_t<std::remove_reference_t<decltype(*p)>>;
        pool_off = (pool_off + 255) & ~size_t(255);
        if (!sizing)
            *p = reinterpret_cast<T *>(h->pool + pool_off);
        pool_off += std::max<size_t>(n, 1) * sizeof(T);
        return LIE_OK;
    };
    const int bmax = std::max(b, 1);
    const size_t capr = (size_t)lie::coef_ld(h->cap);
    const bool planes = h->screened && cfg.precision == LIE_PREC_BF16X3 && !t_batch_member;
    if (planes)
        h->pg = lie::plane_geom(D, h->cap, bmax);
    auto layout = [&]() -> lie_status {
        lie_status s;
        if ((s = alloc(&h->V64, (size_t)h->cap * D)) != LIE_OK || (s = alloc(&h->H64, (size_t)bmax * D)) != LIE_OK ||
            (s = alloc(&h->C, (size_t)bmax * capr)) != LIE_OK ||
            (s = alloc(&h->part, std::max(lie::proj_scratch_doubles(D, std::min(bmax, 64), h->cap),
                                           (size_t)bmax * lie::gemm_sub_tiles_f64(D) * 2))) != LIE_OK ||
            (s = alloc(&h->cand_a2, bmax)) != LIE_OK || (s = alloc(&h->cand_n2, bmax)) != LIE_OK ||
            (s = alloc(&h->rho2, bmax)) != LIE_OK || (s = alloc(&h->h2, bmax)) != LIE_OK ||
            (s = alloc(&h->h2b, bmax)) != LIE_OK || (s = alloc(&h->surv_rows, bmax)) != LIE_OK ||
            (s = alloc(&h->surv_pairs, bmax)) != LIE_OK || (s = alloc(&h->slot, bmax)) != LIE_OK ||
            (s = alloc(&h->keep, bmax)) != LIE_OK ||
            (!t_batch_member &&
             (s = alloc(&h->splitws, h->splitws_n = lie::gemm_split_ws_doubles(D, (int64_t)capr))) != LIE_OK) ||
            (s = alloc(&h->nsurv, 1)) != LIE_OK || (s = alloc(&h->scalar, 1)) != LIE_OK ||
            (s = alloc(&h->d_cursor, 1)) != LIE_OK || (s = alloc(&h->st, 1)) != LIE_OK)
            return s;
        if (h->raw) {
            if ((s = alloc(&h->B64, (size_t)h->cap * D)) != LIE_OK ||
                (s = alloc(&h->Graw, (size_t)n_gen * D)) != LIE_OK ||
                (s = alloc(&h->elem_src, (size_t)h->cap)) != LIE_OK ||
                (h->screened && (s = alloc(&h->Bs, (size_t)h->cap * D)) != LIE_OK))
                return s;
        }
        if (h->screened) {
            if ((s = alloc(&h->Vs, (size_t)h->cap * D)) != LIE_OK || (s = alloc(&h->Hs, (size_t)bmax * D)) != LIE_OK ||
                (s = alloc(&h->Cs, (size_t)bmax * capr)) != LIE_OK ||
                (s = alloc(&h->normpart_s, (size_t)bmax * lie::gemm_sub_tiles_f32(D, 1) * 2)) != LIE_OK)
                return s;
        }
        if (planes) {
            const lie::PlaneGeom &g = h->pg;
            if ((s = alloc(&h->Vp, (size_t)(g.cap_rows * g.ld))) != LIE_OK ||
                (s = alloc(&h->Vt, (size_t)(g.d_rows * g.ldt))) != LIE_OK ||
                (s = alloc(&h->Hp, (size_t)(g.b_rows * g.ld))) != LIE_OK ||
                (s = alloc(&h->Cp, (size_t)(g.b_rows * g.ldt))) != LIE_OK || (s = alloc(&h->planes_n, 1)) != LIE_OK)
                return s;
        }
        if (h->pauli) {
            if ((s = alloc(&h->sup_cnt, (size_t)h->cap)) != LIE_OK ||
                (s = alloc(&h->sup_idx, (size_t)h->cap * D)) != LIE_OK)
                return s;
        }
        if (h->inv && (s = alloc(&h->Xc, (size_t)bmax * capr)) != LIE_OK)
            return s;
        return LIE_OK;
    };
    if ((s = layout()) != LIE_OK)
        return bail(s);
    {
        const hipError_t e = hipMalloc((void **)&h->pool, pool_off);
        if (e != hipSuccess)
            return bail(fail(e == hipErrorOutOfMemory ? LIE_ERR_OOM : LIE_ERR_DEVICE,
                             "hipMalloc of the handle's %zu bytes failed: %s", pool_off, hipGetErrorString(e)));
    }
    sizing = false;
    pool_off = 0;
    if ((s = layout()) != LIE_OK)
        return bail(s);
    if (planes) {
        // the split-BF16 screen of single problems runs on pre-split planes; their padding
        // must read as zeros, so every plane starts cleared
        h->planes = true;
        const lie::PlaneGeom &g = h->pg;
        hipError_t e = hipSuccess;
        for (auto pz : {std::make_pair((void *)h->Vp, (size_t)(g.cap_rows * g.ld) * 2),
                        std::make_pair((void *)h->Vt, (size_t)(g.d_rows * g.ldt) * 2),
                        std::make_pair((void *)h->Hp, (size_t)(g.b_rows * g.ld) * 2),
                        std::make_pair((void *)h->Cp, (size_t)(g.b_rows * g.ldt) * 2),
                        std::make_pair((void *)h->planes_n, sizeof(int64_t))})
            if (e == hipSuccess)
                e = hipMemsetAsync(pz.first, 0, pz.second, h->stream);
        if (e != hipSuccess)
            return bail(fail(LIE_ERR_DEVICE, "clearing the screen planes failed: %s", hipGetErrorString(e)));
    }
    if (h->method == LIE_METHOD_RANK_SVD) {
        const hipError_t e = lie::rank_tester_create(&h->rank, D, 64, h->stream);
        if (e != hipSuccess)
            return bail(fail(LIE_ERR_DEVICE, "rank tester setup failed: %s", hipGetErrorString(e)));
    }
    if (h->inv) {
        const hipError_t e = lie::gram_inverse_create(&h->ginv, h->cap, D, bmax, h->stream);
        if (e != hipSuccess)
            return bail(fail(LIE_ERR_DEVICE, "inverse Gram setup failed: %s", hipGetErrorString(e)));
    }
    h->hs = lie::DevState{};
    h->hs.min_acc = INFINITY;
    h->hs.scr_min_indep = INFINITY;
    {
        hipError_t e = hipMemcpyAsync(h->st, &h->hs, sizeof h->hs, hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess)
            return bail(fail(LIE_ERR_DEVICE, "state upload failed: %s", hipGetErrorString(e)));
    }
    if ((s = h->generators(generators)) != LIE_OK)
        return bail(s);
    *out = h;
    return LIE_OK;
}

lie_status lie_closure_run(lie_closure *h)
{
    if (!h)
        return fail(LIE_ERR_ARG, "handle is NULL");
    return h->run(-1);
}

lie_status lie_closure_run_budget(lie_closure *h, int64_t max_candidates)
{
    if (!h)
        return fail(LIE_ERR_ARG, "handle is NULL");
    if (max_candidates < 0)
        return fail(LIE_ERR_ARG, "max_candidates must be >= 0");
    return h->run(max_candidates);
}

lie_status lie_closure_dim(const lie_closure *h, int64_t *dim)
{
    if (!h || !dim)
        return fail(LIE_ERR_ARG, "NULL argument");
    *dim = h->hs.N;
    return LIE_OK;
}

static lie_status basis_common(const lie_closure *h, void *dst, int64_t capacity, int64_t *written, bool device_dst)
{
    if (!h || !written || (!dst && capacity > 0))
        return fail(LIE_ERR_ARG, "NULL argument");
    if (h->sparse)
        return fail(LIE_ERR_STATE, "a sparse Pauli-sum handle returns its basis through lie_closure_basis_pauli_sparse");
    if (h->method != LIE_METHOD_ORTHONORMALIZATION)
        return fail(LIE_ERR_STATE, "this method keeps only the raw basis (lie_closure_raw_basis)");
    const int64_t n = h->hs.N;
    *written = n;
    if (capacity < n)
        return fail(LIE_ERR_CAPACITY, "output holds %lld elements, basis has %lld", (long long)capacity,
                    (long long)n);
    if (n == 0)
        return LIE_OK;
    HIP_TRY(hipSetDevice(h->device));
    if (h->pauli) {
        // coordinates to dense matrices on the host
        std::vector<double> coords((size_t)n * h->D), dense((size_t)n * h->D * 2);
        HIP_TRY(hipMemcpyAsync(coords.data(), h->V64, coords.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        for (int64_t k = 0; k < n; ++k)
            lie::pauli_to_dense(coords.data() + k * h->D, h->nq, dense.data() + k * h->D * 2);
        if (device_dst) {
            HIP_TRY(hipMemcpyAsync(dst, dense.data(), dense.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
            HIP_TRY(hipStreamSynchronize(h->stream));
        } else {
            std::memcpy(dst, dense.data(), dense.size() * sizeof(double));
        }
        return LIE_OK;
    }
    if (device_dst) {
        HIP_TRY(lie::launch_unpack_c128(h->V64, (double *)dst, n, h->d, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        return LIE_OK;
    }
    double *tmp = nullptr;
    HIP_TRY(hipMalloc(&tmp, (size_t)n * h->D * 2 * sizeof(double)));
    hipError_t e = lie::launch_unpack_c128(h->V64, tmp, n, h->d, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dst, tmp, (size_t)n * h->D * 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(h->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess)
        return fail(LIE_ERR_DEVICE, "basis copy failed: %s", hipGetErrorString(e));
    return LIE_OK;
}

lie_status lie_closure_basis(const lie_closure *h, double *out, int64_t capacity, int64_t *written)
{
    return basis_common(h, out, capacity, written, false);
}

lie_status lie_closure_basis_device(const lie_closure *h, void *dst, int64_t capacity, int64_t *written)
{
    return basis_common(h, dst, capacity, written, true);
}

static int pauli_qubits(int32_t d)
{
    if (d < 2 || d > 128 || (d & (d - 1)) != 0)
        return -1;
    int n = 0;
    while ((1 << n) < d)
        ++n;
    return n;
}

lie_status lie_pauli_coordinates(int32_t d, const double *matrix, double *coords)
{
    const int n = pauli_qubits(d);
    if (n < 0 || !matrix || !coords)
        return fail(LIE_ERR_ARG, "need d = 2^n (1 <= n <= 7) and non-NULL buffers");
    lie::pauli_from_dense(matrix, n, coords);
    return LIE_OK;
}

lie_status lie_pauli_matrix(int32_t d, const double *coords, double *matrix)
{
    const int n = pauli_qubits(d);
    if (n < 0 || !matrix || !coords)
        return fail(LIE_ERR_ARG, "need d = 2^n (1 <= n <= 7) and non-NULL buffers");
    lie::pauli_to_dense(coords, n, matrix);
    return LIE_OK;
}

lie_status lie_closure_raw_basis(const lie_closure *h, double *out, int64_t capacity, int64_t *written)
{
    if (!h || !written || (!out && capacity > 0))
        return fail(LIE_ERR_ARG, "NULL argument");
    if (!h->raw)
        return fail(LIE_ERR_STATE, "the handle was not created with config.raw_basis = 1");
    const int64_t n = h->hs.N;
    *written = n;
    if (capacity < n)
        return fail(LIE_ERR_CAPACITY, "output holds %lld elements, raw basis has %lld", (long long)capacity,
                    (long long)n);
    if (n == 0)
        return LIE_OK;
    HIP_TRY(hipSetDevice(h->device));
    double *tmp = nullptr;
    HIP_TRY(hipMalloc(&tmp, (size_t)n * h->D * 2 * sizeof(double)));
    hipError_t e = lie::launch_unpack_c128(h->B64, tmp, n, h->d, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, tmp, (size_t)n * h->D * 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(h->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess)
        return fail(LIE_ERR_DEVICE, "raw basis copy failed: %s", hipGetErrorString(e));
    return LIE_OK;
}

lie_status lie_closure_orthogonality(lie_closure *h, double *loss)
{
    if (!h || !loss)
        return fail(LIE_ERR_ARG, "NULL argument");
    if (h->sparse)
        return fail(LIE_ERR_STATE, "a sparse Pauli-sum handle keeps no dense basis");
    if (h->method != LIE_METHOD_ORTHONORMALIZATION)
        return fail(LIE_ERR_STATE, "this method keeps no orthonormal basis");
    const int64_t n = h->hs.N;
    HIP_TRY(hipSetDevice(h->device));
    double *work = nullptr;
    HIP_TRY(hipMalloc(&work, ((size_t)n * n + 256) * sizeof(double)));
    hipError_t e = lie::launch_orth_loss(h->V64, n, h->D, work, h->scalar, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(loss, h->scalar, sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(h->stream);
    (void)hipFree(work);
    if (e != hipSuccess)
        return fail(LIE_ERR_DEVICE, "orthogonality check failed: %s", hipGetErrorString(e));
    return LIE_OK;
}

lie_status lie_closure_orthogonality_noalloc(lie_closure *h, double *loss_dev)
{
    if (!h || !loss_dev)
        return fail(LIE_ERR_ARG, "NULL argument");
    if (h->sparse)
        return fail(LIE_ERR_STATE, "a sparse Pauli-sum handle keeps no dense basis");
    if (h->method != LIE_METHOD_ORTHONORMALIZATION)
        return fail(LIE_ERR_STATE, "this method keeps no orthonormal basis");
    const int64_t n = h->hs.N;
    double *ws = lie::noalloc_scratch(h->device);
    if (!ws)
        return fail(LIE_ERR_STATE, "no workspace on device %d", h->device);
    if (n + 256 > lie::kNoallocScratchDoubles)
        return fail(LIE_ERR_CAPACITY, "basis of %lld elements exceeds the fixed workspace (at most %lld)",
                    (long long)n, (long long)(lie::kNoallocScratchDoubles - 256));
    HIP_TRY(hipSetDevice(h->device));
    const hipError_t e = lie::launch_orth_loss_panels(h->V64, n, h->D, ws, lie::kNoallocScratchDoubles, loss_dev,
                                                      h->stream);
    if (e != hipSuccess)
        return fail(LIE_ERR_DEVICE, "orthogonality check failed: %s", hipGetErrorString(e));
    return LIE_OK;
}

lie_status lie_closure_stats_get(const lie_closure *h, lie_closure_stats *out)
{
    if (!h || !out)
        return fail(LIE_ERR_ARG, "NULL argument");
    if (out->struct_size != sizeof(lie_closure_stats))
        return fail(LIE_ERR_ARG, "stats.struct_size must be %zu", sizeof(lie_closure_stats));
    std::memset(out, 0, sizeof *out);
    out->struct_size = sizeof(lie_closure_stats);
    out->done = h->done ? 1 : 0;
    out->dim = h->hs.N;
    out->ambient = h->ambient;
    out->candidates = h->hs.n_cand;
    out->generator_checks = h->n_gen;
    out->zero_brackets = h->hs.n_zero;
    out->screen_rejected = h->hs.n_screen_rej;
    out->fp64_decided = h->hs.n_fp64;
    out->accepted = h->hs.n_acc;
    out->block_qr_accepted = h->hs.n_bqr;
    out->reorth_passes = h->hs.n_reorth;
    if (h->sparse) {
        int64_t terms = 0;
        if (lie::sparse_pauli_terms(h->sp, h->hs.N, &terms, h->stream) != hipSuccess)
            return fail(LIE_ERR_DEVICE, "reading the term count failed");
        out->pauli_terms = terms;
    }
    out->blocks = h->blocks;
    out->host_syncs = h->host_syncs;
    out->min_accepted_residual = h->hs.min_acc;
    out->max_rejected_residual = h->hs.max_rej;
    out->max_screen_rejected = h->hs.max_screen_rej;
    out->screen_max_dependent = h->hs.scr_max_dep;
    out->screen_min_independent = h->hs.scr_min_indep;
    out->run_ms = h->run_ms;
    out->precision = h->cfg.precision;
    out->decide = h->cfg.decide;
    out->block = h->block > 0 ? h->block : -h->block_sat;
    out->early_exit = h->cfg.early_exit;
    out->tile_dot = h->tile_dot;
    out->tile_sub = h->tile_sub;
    out->autotuned = h->autotuned;
    out->block_growth = h->block > 0 ? h->block : h->block_growth;
    for (int k = 0; k < LIE_K_COUNT; ++k) {
        out->kernel_launches[k] = h->timer.n[k];
        out->kernel_ms[k] = h->timer.ms[k];
        out->kernel_flops[k] = h->timer.flops[k];
        out->kernel_bytes[k] = h->timer.bytes[k];
    }
    // The acceptance kernel's work depends on device-side survivor counts, so its
    // algorithmic bytes are formed from the run's counters: per candidate its
    // classification record (an int and two doubles), per survivor left to the
    // in-block decisions its residual row, per appended element its FP64 row (and
    // FP32 shadow when screened).
    {
        const double D = (double)h->D;
        out->kernel_bytes[LIE_K_ACCEPT] = 20.0 * (double)h->hs.n_cand + 8.0 * D * (double)h->hs.n_rows +
                                          (8.0 + (h->screened ? 4.0 : 0.0)) * D * (double)h->hs.n_acc;
        // the FP64 verification passes run over device-side survivor counts as well
        out->kernel_flops[LIE_K_VERIFY] = h->hs.vfy_flops;
        out->kernel_bytes[LIE_K_VERIFY] = h->hs.vfy_bytes;
    }
    return LIE_OK;
}

lie_status lie_closure_init_pauli_sparse(lie_closure **out, int32_t n_qubits, int32_t n_gen,
                                        const int64_t *term_offsets, const uint64_t *strings, const double *coefs,
                                        double tol, int64_t max_terms, const lie_closure_config *cfg_in)
{
    g_last_error.clear();
    if (!out)
        return fail(LIE_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (n_qubits < 1 || n_qubits > 31)
        return fail(LIE_ERR_ARG, "n_qubits must be in 1..31 (got %d)", n_qubits);
    if (n_gen < 1 || !term_offsets || !strings || !coefs)
        return fail(LIE_ERR_ARG, "NULL argument or n_gen < 1");
    if (!(tol > 0.0 && tol < 1.0))
        return fail(LIE_ERR_ARG, "tol must be in (0, 1)");
    if (max_terms < 0)
        return fail(LIE_ERR_ARG, "max_terms must be >= 0");
    if (term_offsets[0] != 0)
        return fail(LIE_ERR_ARG, "term_offsets[0] must be 0");
    const uint64_t mask = (1ull << n_qubits) - 1ull;
    bool identity = false;
    for (int g = 0; g < n_gen; ++g) {
        if (term_offsets[g + 1] < term_offsets[g])
            return fail(LIE_ERR_ARG, "term_offsets must be non-decreasing");
        for (int64_t t = term_offsets[g]; t < term_offsets[g + 1]; ++t) {
            const uint64_t x = strings[t] >> 32, z = strings[t] & 0xffffffffull;
            if ((x & ~mask) || (z & ~mask))
                return fail(LIE_ERR_ARG, "term %lld names a qubit beyond n_qubits", (long long)t);
            if (!std::isfinite(coefs[t]))
                return fail(LIE_ERR_NONFINITE, "coefficient %lld is not finite", (long long)t);
            if (strings[t] == 0 && coefs[t] != 0.0)
                identity = true;
        }
    }
    lie_closure_config cfg;
    lie_status s;
    if ((s = resolve_config(cfg_in, &cfg)) != LIE_OK)
        return s;
    if (cfg.precision != LIE_PREC_FP64 || cfg.method != LIE_METHOD_ORTHONORMALIZATION || cfg.raw_basis)
        return fail(LIE_ERR_ARG, "the sparse Pauli-sum representation runs Algorithm 4 in FP64 only");
    lie_closure *h = new (std::nothrow) lie_closure();
    if (!h)
        return fail(LIE_ERR_OOM, "host allocation failed");
    auto bail = [&](lie_status st) {
        delete h;
        return st;
    };
    h->sparse = true;
    h->d = 0;
    h->D = 0;
    h->tol = tol;
    h->n_gen = n_gen;
    h->nq = n_qubits;
    // traceless generators (no identity term) stay traceless: 4^n - 1 strings, else 4^n
    h->ambient = (int64_t)1 << (2 * n_qubits);
    if (!identity)
        h->ambient -= 1;
    h->cfg = cfg;
    h->cap = cfg.max_dim > 0 ? std::min<int64_t>(cfg.max_dim, h->ambient) : std::min<int64_t>(h->ambient, 1 << 20);
    int dev = cfg.device;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess)
        return bail(fail(LIE_ERR_DEVICE, "hipGetDevice failed"));
    h->device = dev;
    if (hipSetDevice(dev) != hipSuccess)
        return bail(fail(LIE_ERR_DEVICE, "hipSetDevice(%d) failed", dev));
    if (cfg.stream) {
        h->stream = (hipStream_t)cfg.stream;
    } else {
        if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(LIE_ERR_DEVICE, "hipStreamCreate failed"));
        h->own_stream = true;
    }
    if (hipMalloc(&h->st, sizeof(lie::DevState)) != hipSuccess)
        return bail(fail(LIE_ERR_OOM, "device allocation failed"));
    hipError_t e = lie::sparse_pauli_create(&h->sp, n_qubits, h->cap, max_terms > 0 ? max_terms : (int64_t)1 << 24,
                                            (int64_t)1 << 20, term_offsets, n_gen, strings, coefs, h->stream);
    if (e != hipSuccess)
        return bail(fail(e == hipErrorOutOfMemory ? LIE_ERR_OOM : LIE_ERR_DEVICE, "sparse pool setup failed: %s",
                         hipGetErrorString(e)));
    h->hs = lie::DevState{};
    h->hs.min_acc = INFINITY;
    h->hs.scr_min_indep = INFINITY;
    if (hipMemcpyAsync(h->st, &h->hs, sizeof h->hs, hipMemcpyHostToDevice, h->stream) != hipSuccess)
        return bail(fail(LIE_ERR_DEVICE, "state upload failed"));
    // Algorithm 4's generator phase: each generator against the basis, relative threshold
    for (int g = 0; g < n_gen; ++g) {
        if (term_offsets[g + 1] - term_offsets[g] > ((int64_t)1 << 20))
            return bail(fail(LIE_ERR_CAPACITY, "generator %d has more terms than the scratch lists hold", g));
        if ((e = lie::sparse_pauli_generator(h->sp, g, h->st, tol, h->ambient, h->stream)) != hipSuccess)
            return bail(fail(LIE_ERR_DEVICE, "generator phase failed: %s", hipGetErrorString(e)));
    }
    if ((s = h->sync_state()) != LIE_OK || (s = h->check_state()) != LIE_OK)
        return bail(s);
    *out = h;
    return LIE_OK;
}

lie_status lie_closure_basis_pauli_sparse(const lie_closure *h, int64_t *offsets, uint64_t *strings, double *coefs,
                                          int64_t capacity_terms, int64_t *terms_written)
{
    if (!h || !terms_written || !offsets || (capacity_terms > 0 && (!strings || !coefs)))
        return fail(LIE_ERR_ARG, "NULL argument");
    if (!h->sparse)
        return fail(LIE_ERR_STATE, "the handle was not created by lie_closure_init_pauli_sparse");
    HIP_TRY(hipSetDevice(h->device));
    const hipError_t e = lie::sparse_pauli_basis(h->sp, h->hs.N, offsets, strings, coefs, capacity_terms,
                                                 terms_written, h->stream);
    if (e != hipSuccess)
        return fail(LIE_ERR_DEVICE, "basis copy failed: %s", hipGetErrorString(e));
    if (*terms_written > capacity_terms)
        return fail(LIE_ERR_CAPACITY, "output holds %lld terms, basis has %lld", (long long)capacity_terms,
                    (long long)*terms_written);
    return LIE_OK;
}

void lie_closure_free(lie_closure *h) { delete h; }

const char *lie_status_string(lie_status s)
{
    switch (s) {
    case LIE_OK: return "LIE_OK";
    case LIE_INCOMPLETE: return "LIE_INCOMPLETE";
    case LIE_ERR_ARG: return "LIE_ERR_ARG";
    case LIE_ERR_NOT_ANTIHERMITIAN: return "LIE_ERR_NOT_ANTIHERMITIAN";
    case LIE_ERR_NONFINITE: return "LIE_ERR_NONFINITE";
    case LIE_ERR_OOM: return "LIE_ERR_OOM";
    case LIE_ERR_DEVICE: return "LIE_ERR_DEVICE";
    case LIE_ERR_STATE: return "LIE_ERR_STATE";
    case LIE_ERR_CAPACITY: return "LIE_ERR_CAPACITY";
    case LIE_ERR_NUMERIC: return "LIE_ERR_NUMERIC";
    }
    return "unknown lie_status";
}

const char *lie_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------------------ batched form (problems advanced together)

}  // extern "C"

// Grouped executor: every round advances each live problem by one block step,
// and each stage of the step is one launch for all problems of the round
// (workgroups find their problem through a prefix table).  Problems leave the
// batch when they complete; the host loop synchronises once for all problems when
// any of them runs out of known pairs (or after 64 rounds).
struct lie_closure_batch {
    std::vector<lie_closure *> probs;
    int device = -1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // staging ring for the per-round argument tables (pinned host -> device)
    static constexpr int kSlots = 65;
    size_t slot_bytes = 0;
    char *host_ring = nullptr, *dev_ring = nullptr;
    int slot = 0;
    size_t used = 0;
    hipEvent_t slot_free[kSlots] = {};
    // state read-back
    lie::DevState **d_stptrs = nullptr;
    lie::DevState *d_states = nullptr, *h_states = nullptr;
    KernelTimer timer;
    int64_t rounds = 0, host_syncs = 0;
    double run_ms = 0;
    bool done = false;
    lie_status first_status = LIE_OK;
    std::string first_error;

    ~lie_closure_batch()
    {
        if (device >= 0)
            (void)hipSetDevice(device);
        if (stream)
            (void)hipStreamSynchronize(stream);
        for (auto *p : probs)
            delete p;
        for (hipEvent_t e : slot_free)
            if (e)
                (void)hipEventDestroy(e);
        if (host_ring)
            (void)hipHostFree(host_ring);
        if (h_states)
            (void)hipHostFree(h_states);
        for (void *p : {(void *)dev_ring, (void *)d_stptrs, (void *)d_states})
            if (p)
                (void)hipFree(p);
        if (own_stream && stream)
            (void)hipStreamDestroy(stream);
    }

    lie_status setup()
    {
        const int n = (int)probs.size();
        // argument tables of one round: at most ~24 stage tables of n entries each
        slot_bytes = (size_t)n * 32 * 256 + 64 * 1024;
        HIP_TRY(hipHostMalloc((void **)&host_ring, slot_bytes * kSlots, hipHostMallocDefault));
        HIP_TRY(hipMalloc(&dev_ring, slot_bytes * kSlots));
        for (auto &e : slot_free)
            HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        HIP_TRY(hipMalloc(&d_stptrs, n * sizeof(lie::DevState *)));
        HIP_TRY(hipMalloc(&d_states, n * sizeof(lie::DevState)));
        HIP_TRY(hipHostMalloc((void **)&h_states, n * sizeof(lie::DevState), hipHostMallocDefault));
        std::vector<lie::DevState *> ptrs(n);
        for (int i = 0; i < n; ++i)
            ptrs[i] = probs[i]->st;
        HIP_TRY(hipMemcpyAsync(d_stptrs, ptrs.data(), n * sizeof(lie::DevState *), hipMemcpyHostToDevice, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        return LIE_OK;
    }

    // Append a table to the current round's slot; returns its device address.
    template <typename T>
    const T *put(const std::vector<T> &v)
    {
        used = (used + 15) & ~size_t(15);
        const size_t bytes = v.size() * sizeof(T);
        if (used + bytes > slot_bytes)
            return nullptr;
        std::memcpy(host_ring + (size_t)slot * slot_bytes + used, v.data(), bytes);
        const T *dev = reinterpret_cast<const T *>(dev_ring + (size_t)slot * slot_bytes + used);
        used += bytes;
        return dev;
    }

    // A grouped launch under construction.
    template <typename A>
    struct Group {
        std::vector<A> args;
        std::vector<int> start{0};
        std::vector<int> gx;
        void add(const A &a, int wgs, int gridx)
        {
            args.push_back(a);
            start.push_back(start.back() + std::max(wgs, 0));
            gx.push_back(std::max(gridx, 1));
        }
        bool empty() const { return args.empty(); }
    };

    template <typename A>
    lie_status make(const Group<A> &g, lie::Batch *out)
    {
        out->args = put(g.args);
        out->start = put(g.start);
        out->gx = put(g.gx);
        out->nprob = (int)g.args.size();
        out->total = g.start.back();
        if (!out->args || !out->start || !out->gx)
            return fail(LIE_ERR_OOM, "batched launch table exceeds its staging slot");
        return LIE_OK;
    }

    lie_status sync_all()
    {
        const int n = (int)probs.size();
        HIP_TRY(lie::launch_gather_states(d_stptrs, n, d_states, stream));
        HIP_TRY(hipMemcpyAsync(h_states, d_states, n * sizeof(lie::DevState), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        ++host_syncs;
        timer.harvest();
        for (int i = 0; i < n; ++i) {
            lie_closure *h = probs[i];
            if (h->done || h->failed)
                continue;
            h->hs = h_states[i];
            ++h->host_syncs;
            lie_status s = h->check_state();
            if (s != LIE_OK) {
                if (first_status == LIE_OK) {
                    first_status = s;
                    first_error = "problem " + std::to_string(i) + ": " + g_last_error;
                }
                continue;
            }
            h->b_nlo = h->hs.N;
            h->b_qrows = 0;
            if (h->block == 0) {
                const int64_t dc = h->hs.n_cand - h->b_lastc, da = h->hs.n_acc - h->b_lasta;
                if (dc > 0)
                    h->b_cur = 8 * da > dc ? h->block_growth
                                           : std::min(h->block_sat, 4 * std::max(h->b_cur, h->block_growth));
                if (h->b_nlo >= h->ambient)
                    h->b_cur = h->block_sat;
                h->b_lastc = h->hs.n_cand;
                h->b_lasta = h->hs.n_acc;
            }
            if (h->hs.done || (h->cfg.early_exit && h->b_nlo >= h->ambient) ||
                h->cursor >= lie::pairs_below(h->b_nlo))
                h->done = true;
        }
        return LIE_OK;
    }

    struct Item {
        lie_closure *h;
        int cnt;
        int64_t n_hi;
    };

    lie_status run()
    {
        if (done)
            return LIE_OK;
        if (first_status != LIE_OK)
            return fail(LIE_ERR_STATE, "a previous run of this batch failed");
        HIP_TRY(hipSetDevice(device));
        const auto t0 = std::chrono::steady_clock::now();
        constexpr int kMaxQueued = 64;
        for (lie_closure *h : probs) {
            h->b_nlo = h->hs.N;
            h->b_qrows = 0;
            h->b_cur = h->block > 0 ? h->block : h->block_growth;
            h->b_lastc = h->hs.n_cand;
            h->b_lasta = h->hs.n_acc;
            if (h->cursor >= lie::pairs_below(h->b_nlo) || (h->cfg.early_exit && h->b_nlo >= h->ambient))
                h->done = true;
        }
        int queued = 0;
        lie_status s = LIE_OK;
        for (;;) {
            bool need = queued >= kMaxQueued;
            bool growing = false;
            for (lie_closure *h : probs) {
                if (h->done || h->failed)
                    continue;
                if (h->cursor >= lie::pairs_below(h->b_nlo))
                    need = true;
                if (h->block == 0 && h->b_cur < h->block_sat)
                    growing = true;
            }
            if (growing && queued >= kGrowthQueued)
                need = true;
            if (need) {
                if ((s = sync_all()) != LIE_OK)
                    break;
                queued = 0;
            }
            std::vector<Item> f64, scr;
            for (lie_closure *h : probs) {
                if (h->done || h->failed)
                    continue;
                const int64_t avail = lie::pairs_below(h->b_nlo);
                if (h->cursor >= avail)
                    continue;
                const int cnt = (int)std::min<int64_t>(h->b_cur, avail - h->cursor);
                const int64_t n_hi = std::min<int64_t>(h->cap, h->b_nlo + h->b_qrows);
                const bool growth = h->block == 0 && h->b_cur == h->block_growth;
                const bool screen = h->screened && !growth && (!h->certify || h->b_nlo >= h->ambient);
                (screen ? scr : f64).push_back(Item{h, cnt, n_hi});
            }
            if (f64.empty() && scr.empty())
                break;
            // a slot is reused kSlots rounds later; its event proves the copy out of it has run
            HIP_TRY(hipEventSynchronize(slot_free[slot]));
            if ((s = build_and_launch(f64, scr)) != LIE_OK)
                break;
            for (auto *v : {&f64, &scr})
                for (const Item &it : *v) {
                    it.h->cursor += it.cnt;
                    it.h->b_qrows += it.cnt;
                    ++it.h->blocks;
                }
            ++queued;
            ++rounds;
        }
        if (s == LIE_OK && first_status == LIE_OK) {
            if ((s = sync_all()) == LIE_OK && first_status == LIE_OK)
                done = true;
        }
        run_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (s == LIE_OK && first_status != LIE_OK) {
            std::string msg = first_error;
            return fail(first_status, "%s", msg.c_str());
        }
        return s;
    }

    // A recorded grouped launch of the round being built.
    enum Kind { COMM_F64, COMM_F32, DOT_F64, DOT_F32, DOT_BF, SUB_F64, SUB_F32, SUB_BF, NORM, CLASSIFY,
                ACCEPT };
    struct Rec {
        Kind kind;
        lie::Batch b;
        bool lds;
        int dmax;
        int kid;
        double flops;
        int64_t lds_doubles;
        bool vec;  // projection GEMMs: every problem's rows take 16-byte loads
    };
    std::vector<Rec> recs;

    template <typename A>
    lie_status record(Kind kind, const Group<A> &g, bool lds, int dmax, int kid, double flops, bool vec = false)
    {
        if (g.empty())
            return LIE_OK;
        Rec r{kind, {}, lds, dmax, kid, flops, 0, vec};
        if constexpr (std::is_same<A, lie::AcceptArgs>::value)
            r.lds_doubles = g.args.front().lds_doubles;
        lie_status s = make(g, &r.b);
        if (s != LIE_OK)
            return s;
        recs.push_back(r);
        return LIE_OK;
    }

    // FP64 bracket of the block (or of the survivors) into H64 of each item.
    lie_status group_comm_f64(const std::vector<Item> &items, bool from_survivors)
    {
        Group<lie::CommArgs> lds, glob;
        int dmax = 1;
        double fl = 0;
        for (const Item &it : items) {
            lie_closure *h = it.h;
            lie::CommArgs a{h->V64,          h->d,        from_survivors ? 0 : h->cursor,
                            from_survivors ? h->surv_pairs : nullptr, nullptr,
                            from_survivors ? h->nsurv : nullptr,      it.cnt, h->st, h->H64, nullptr};
            if (lie::comm_f64_fits_lds(h->d)) {
                lds.add(a, it.cnt, 1);
                dmax = std::max(dmax, h->d);
            } else {
                glob.add(a, it.cnt, 1);  // one workgroup per candidate (tile-pair kernel)
            }
            if (!from_survivors)
                fl += 8.0 * h->d * h->d * (double)h->d * it.cnt;
        }
        const int kid = from_survivors ? LIE_K_VERIFY : LIE_K_COMM;
        lie_status s = record(COMM_F64, lds, true, dmax, kid, fl);
        if (s == LIE_OK)
            s = record(COMM_F64, glob, false, 0, kid, lds.empty() ? fl : 0);
        return s;
    }

    // FP64 projection pass over H64 rows (all cnt, or the survivor list / count).
    lie_status group_project_f64(const std::vector<Item> &items, bool survivors_rows, bool survivors_count,
                                 bool first, bool verify)
    {
        Group<lie::GemmArgs> dot, sub;
        Group<lie::NormArgs> nrm;
        double fl = 0;
        bool vec = true;
        const int bm = lie::gemm_group_m(false), bn = lie::gemm_group_n(false);
        for (const Item &it : items) {
            lie_closure *h = it.h;
            vec = vec && h->D % 2 == 0;
            const int64_t nh = std::min(std::max<int64_t>(it.n_hi, 1), h->cap);
            lie::GemmArgs g{};
            g.H = h->H64;
            g.rows = survivors_rows ? h->surv_rows : nullptr;
            g.nrows = survivors_count ? h->nsurv : nullptr;
            g.cnt = it.cnt;
            g.V = h->V64;
            g.C = h->C;
            g.ldc = lie::coef_ld(h->cap);
            g.D = h->D;
            g.st = h->st;
            const int mt = (it.cnt + bm - 1) / bm;
            const int nt = (int)((nh + bn - 1) / bn);
            dot.add(g, nt * mt, nt);
            g.normpart = h->part;
            g.write_r = 1;
            const int jt = (int)((h->D + bn - 1) / bn);
            sub.add(g, jt * mt, jt);
            double *r2 = first ? h->cand_a2 : h->rho2;
            double *n2 = first ? h->cand_n2 : (verify_first_ ? h->h2 : h->h2b);
            nrm.add(lie::NormArgs{h->part, g.nrows, it.cnt, jt, h->st, r2, n2}, (it.cnt + 255) / 256, 1);
            if (!verify)
                fl += 2.0 * (double)h->b_nlo * (double)h->D * it.cnt;
        }
        lie_status s = record(DOT_F64, dot, false, 0, verify ? LIE_K_VERIFY : LIE_K_DOT, fl, vec);
        if (s == LIE_OK)
            s = record(SUB_F64, sub, false, 0, verify ? LIE_K_VERIFY : LIE_K_SUB, fl, vec);
        if (s == LIE_OK)
            s = record(NORM, nrm, false, 0, verify ? LIE_K_VERIFY : LIE_K_REDUCE, 0);
        return s;
    }
    bool verify_first_ = false;  // screened verification: first FP64 pass keeps the candidate norms in h2

    lie_status group_classify(const std::vector<Item> &items, bool screen)
    {
        Group<lie::ClassifyArgs> g;
        for (const Item &it : items) {
            lie_closure *h = it.h;
            const int pol = screen ? h->policy : lie::POL_ABS;
            const double thr = screen ? h->policy_thr : h->tol;
            g.add(lie::ClassifyArgs{h->cand_a2, h->cand_n2, it.cnt, h->cursor, nullptr, pol, thr, h->st,
                                    h->surv_rows, h->surv_pairs, h->slot, h->nsurv, h->ambient,
                                    screen && h->certify ? 1 : 0},
                  1, 1);
        }
        return record(CLASSIFY, g, false, 0, LIE_K_REDUCE, 0);
    }

    lie_status group_accept(const std::vector<Item> &items, bool screen)
    {
        Group<lie::AcceptArgs> g;
        int64_t lds_acc = 0;
        for (const Item &it : items) {
            lie_closure *h = it.h;
            lie::AcceptArgs a{};
            a.V = h->V64;
            a.Vs = h->Vs;
            a.st = h->st;
            a.H = h->H64;
            a.rrow = screen ? nullptr : h->surv_rows;
            a.cand_a2 = h->cand_a2;
            a.cand_n2 = h->cand_n2;
            a.slot = h->slot;
            a.nsurv = h->nsurv;
            a.surv_cand = h->surv_rows;
            a.keep = h->keep;
            a.h2 = screen ? h->h2 : nullptr;
            a.rho2 = h->rho2;
            a.cnt = it.cnt;
            a.D = h->D;
            a.cap = h->cap;
            a.ambient = h->ambient;
            a.tol = h->tol;
            a.mode = 1;
            a.screened = screen && h->policy != lie::POL_ALL ? 1 : 0;
            a.early_exit = h->cfg.early_exit;
            a.vpasses = screen ? 2 : 1;
            a.vbracket = screen ? 1 : 0;
            a.d = h->d;
            a.lds_doubles = 0;  // set below to the launch-wide size
            g.add(a, 1, 1);
            lds_acc = std::max<int64_t>(lds_acc, lie::accept_lds_doubles(it.cnt, h->D));
        }
        for (auto &a : g.args)
            a.lds_doubles = lds_acc;
        return record(ACCEPT, g, false, 0, LIE_K_ACCEPT, 0);
    }

    lie_status round_fp64(const std::vector<Item> &items)
    {
        if (items.empty())
            return LIE_OK;
        lie_status s;
        if ((s = group_comm_f64(items, false)) != LIE_OK)
            return s;
        if ((s = group_project_f64(items, false, false, true, false)) != LIE_OK)
            return s;
        if ((s = group_classify(items, false)) != LIE_OK)
            return s;
        verify_first_ = false;
        if ((s = group_project_f64(items, true, true, false, true)) != LIE_OK)
            return s;
        return group_accept(items, false);
    }

    bool bf_items = false;  // the screened items of this round use split-BF16 GEMMs

    lie_status round_screen(const std::vector<Item> &items)
    {
        if (items.empty())
            return LIE_OK;
        Group<lie::CommArgs> lds, glob;
        Group<lie::GemmArgs> dot, sub;
        Group<lie::NormArgs> nrm;
        int dmax = 1;
        double flc = 0, flp = 0;
        bool vec = true;
        const int bm = lie::gemm_group_m(true), bn = lie::gemm_group_n(true);
        for (const Item &it : items) {
            lie_closure *h = it.h;
            lie::CommArgs a{h->Vs, h->d, h->cursor, nullptr, nullptr, nullptr, it.cnt, h->st, h->Hs, h->cand_n2};
            if (lie::comm_f32_fits_lds(h->d)) {
                lds.add(a, it.cnt, 1);
                dmax = std::max(dmax, h->d);
            } else {
                glob.add(a, it.cnt, 1);  // one workgroup per candidate (tile-pair kernel, row norms included)
            }
            vec = vec && h->D % 4 == 0;
            const int64_t nh = std::min(std::max<int64_t>(it.n_hi, 1), h->cap);
            lie::GemmArgs g{};
            g.H = h->Hs;
            g.cnt = it.cnt;
            g.V = h->Vs;
            g.C = h->Cs;
            g.ldc = lie::coef_ld(h->cap);
            g.D = h->D;
            g.st = h->st;
            const int mt = (it.cnt + bm - 1) / bm;
            const int nt = (int)((nh + bn - 1) / bn);
            dot.add(g, nt * mt, nt);
            g.normpart = h->normpart_s;
            g.write_r = 0;
            const int jt = (int)((h->D + bn - 1) / bn);
            sub.add(g, jt * mt, jt);
            nrm.add(lie::NormArgs{h->normpart_s, nullptr, it.cnt, jt, h->st, h->cand_a2, nullptr}, (it.cnt + 255) / 256,
                    1);
            flc += 8.0 * h->d * h->d * (double)h->d * it.cnt;
            flp += 2.0 * (double)h->b_nlo * (double)h->D * it.cnt;
        }
        lie_status s = LIE_OK;
        if ((s = record(COMM_F32, lds, true, dmax, LIE_K_COMM, flc)) != LIE_OK ||
            (s = record(COMM_F32, glob, false, 0, LIE_K_COMM, lds.empty() ? flc : 0)) != LIE_OK ||
            (s = record(bf_items ? DOT_BF : DOT_F32, dot, false, 0, LIE_K_DOT, flp, vec)) != LIE_OK ||
            (s = record(bf_items ? SUB_BF : SUB_F32, sub, false, 0, LIE_K_SUB, flp, vec)) != LIE_OK ||
            (s = record(NORM, nrm, false, 0, LIE_K_REDUCE, 0)) != LIE_OK)
            return s;
        if ((s = group_classify(items, true)) != LIE_OK)
            return s;
        if ((s = group_comm_f64(items, true)) != LIE_OK)
            return s;
        verify_first_ = true;  // first FP64 pass: candidate norms into h2
        if ((s = group_project_f64(items, false, true, false, true)) != LIE_OK)
            return s;
        verify_first_ = false;  // second pass: norms into h2b
        if ((s = group_project_f64(items, false, true, false, true)) != LIE_OK)
            return s;
        return group_accept(items, true);
    }

    lie_status execute(const Rec &r)
    {
        switch (r.kind) {
        case COMM_F64: return status_of(lie::launch_comm_f64_batched(r.b, r.lds, r.dmax, stream));
        case COMM_F32: return status_of(lie::launch_comm_f32_batched(r.b, r.lds, r.dmax, stream));
        case DOT_F64: return status_of(lie::launch_gemm_dot_batched(r.b, false, r.vec, stream));
        case DOT_F32: return status_of(lie::launch_gemm_dot_batched(r.b, true, r.vec, stream));
        case DOT_BF: return status_of(lie::launch_gemm_dot_bf16x3_batched(r.b, stream));
        case SUB_BF: return status_of(lie::launch_gemm_sub_bf16x3_batched(r.b, stream));
        case SUB_F64: return status_of(lie::launch_gemm_sub_batched(r.b, false, r.vec, stream));
        case SUB_F32: return status_of(lie::launch_gemm_sub_batched(r.b, true, r.vec, stream));
        case NORM: return status_of(lie::launch_norm_final_batched(r.b, stream));
        case CLASSIFY: return status_of(lie::launch_classify_batched(r.b, stream));
        case ACCEPT: return status_of(lie::launch_accept_batched(r.b, r.lds_doubles, stream));
        }
        return LIE_OK;
    }
    static lie_status status_of(hipError_t e)
    {
        if (e == hipSuccess)
            return LIE_OK;
        return fail(LIE_ERR_DEVICE, "grouped launch failed: %s", hipGetErrorString(e));
    }

    // Build every table of the round into the current slot, copy the slot once,
    // then launch the recorded stages in order.
    lie_status build_and_launch(const std::vector<Item> &f64, const std::vector<Item> &scr)
    {
        recs.clear();
        used = 0;
        lie_status s = round_fp64(f64);
        // screened problems share the batch configuration, hence one precision
        bf_items = !scr.empty() && scr.front().h->cfg.precision == LIE_PREC_BF16X3;
        if (s == LIE_OK)
            s = round_screen(scr);
        if (s != LIE_OK)
            return s;
        HIP_TRY(hipMemcpyAsync(dev_ring + (size_t)slot * slot_bytes, host_ring + (size_t)slot * slot_bytes, used,
                               hipMemcpyHostToDevice, stream));
        for (const Rec &r : recs) {
            timer.begin(stream);
            if ((s = execute(r)) != LIE_OK)
                return s;
            timer.end(r.kid, stream, r.flops, 0);
        }
        HIP_TRY(hipEventRecord(slot_free[slot], stream));
        slot = (slot + 1) % kSlots;
        return LIE_OK;
    }
};

extern "C" {

lie_status lie_closure_batch_init(lie_closure_batch **out, int32_t n_problems, const double *const *generators,
                                  const int32_t *n_gen, const int32_t *d, const double *tol,
                                  const lie_closure_config *cfg_in)
{
    g_last_error.clear();
    if (!out || !generators || !n_gen || !d || !tol)
        return fail(LIE_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (n_problems < 1)
        return fail(LIE_ERR_ARG, "n_problems must be >= 1");
    lie_closure_config cfg;
    lie_status s = resolve_config(cfg_in, &cfg);
    if (s != LIE_OK)
        return s;
    if (cfg.raw_basis || cfg.method != LIE_METHOD_ORTHONORMALIZATION || cfg.representation != LIE_REP_DENSE)
        return fail(LIE_ERR_ARG, "config.raw_basis, the comparison methods and the Pauli representation are "
                                 "supported for single problems only");
    // validate every problem before any device work
    for (int32_t i = 0; i < n_problems; ++i) {
        int64_t amb = 0;
        if ((s = validate_generators(generators[i], n_gen[i], d[i], tol[i], &amb)) != LIE_OK) {
            std::string msg = g_last_error;
            return fail(s, "problem %d: %s", i, msg.c_str());
        }
    }
    auto *b = new (std::nothrow) lie_closure_batch();
    if (!b)
        return fail(LIE_ERR_OOM, "host allocation failed");
    int dev = cfg.device;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess) {
        delete b;
        return fail(LIE_ERR_DEVICE, "hipGetDevice failed");
    }
    b->device = dev;
    if (hipSetDevice(dev) != hipSuccess) {
        delete b;
        return fail(LIE_ERR_DEVICE, "hipSetDevice(%d) failed", dev);
    }
    if (cfg.stream) {
        b->stream = (hipStream_t)cfg.stream;
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            delete b;
            return fail(LIE_ERR_DEVICE, "hipStreamCreate failed");
        }
        b->own_stream = true;
    }
    lie_closure_config pc = cfg;
    pc.stream = b->stream;  // every problem runs on the batch's stream
    pc.device = dev;
    pc.tune_cache = cfg_in ? cfg_in->tune_cache : nullptr;  // resolve_config drops the pointer
    for (int32_t i = 0; i < n_problems; ++i) {
        lie_closure *h = nullptr;
        t_batch_member = true;  // the grouped launches need no split-K workspace
        s = lie_closure_init(&h, generators[i], n_gen[i], d[i], tol[i], &pc);
        t_batch_member = false;
        if (s != LIE_OK) {
            std::string msg = g_last_error;
            delete b;
            return fail(s, "problem %d: %s", i, msg.c_str());
        }
        h->timer.on = false;  // grouped launches are timed by the batch
        b->probs.push_back(h);
    }
    b->timer.on = cfg.profile != 0;
    if ((s = b->setup()) != LIE_OK) {
        delete b;
        return s;
    }
    *out = b;
    return LIE_OK;
}

lie_status lie_closure_batch_run(lie_closure_batch *b)
{
    if (!b)
        return fail(LIE_ERR_ARG, "batch is NULL");
    return b->run();
}

lie_status lie_closure_batch_dim(const lie_closure_batch *b, int32_t i, int64_t *dim)
{
    if (!b || i < 0 || i >= (int32_t)b->probs.size())
        return fail(LIE_ERR_ARG, "bad batch index");
    return lie_closure_dim(b->probs[i], dim);
}

lie_status lie_closure_batch_basis(const lie_closure_batch *b, int32_t i, double *out, int64_t capacity,
                                   int64_t *written)
{
    if (!b || i < 0 || i >= (int32_t)b->probs.size())
        return fail(LIE_ERR_ARG, "bad batch index");
    return lie_closure_basis(b->probs[i], out, capacity, written);
}

lie_status lie_closure_batch_stats_get(const lie_closure_batch *b, int32_t i, lie_closure_stats *out)
{
    if (!b || i < -1 || i >= (int32_t)b->probs.size())
        return fail(LIE_ERR_ARG, "bad batch index");
    if (i >= 0)
        return lie_closure_stats_get(b->probs[i], out);
    // aggregate over the batch: summed counters, the batch's own launch timers
    if (!out || out->struct_size != sizeof(lie_closure_stats))
        return fail(LIE_ERR_ARG, "stats.struct_size must be %zu", sizeof(lie_closure_stats));
    lie_closure_stats agg;
    std::memset(&agg, 0, sizeof agg);
    agg.struct_size = sizeof agg;
    agg.done = b->done ? 1 : 0;
    agg.min_accepted_residual = INFINITY;
    agg.screen_min_independent = INFINITY;
    double acc_bytes = 0.0, vfy_flops = 0.0, vfy_bytes = 0.0;  // from each problem's device counters
    for (lie_closure *h : b->probs) {
        lie_closure_stats one;
        one.struct_size = sizeof one;
        lie_closure_stats_get(h, &one);
        agg.dim += one.dim;
        agg.ambient += one.ambient;
        agg.candidates += one.candidates;
        agg.generator_checks += one.generator_checks;
        agg.zero_brackets += one.zero_brackets;
        agg.screen_rejected += one.screen_rejected;
        agg.fp64_decided += one.fp64_decided;
        agg.accepted += one.accepted;
        agg.block_qr_accepted += one.block_qr_accepted;
        agg.reorth_passes += one.reorth_passes;
        agg.min_accepted_residual = std::min(agg.min_accepted_residual, one.min_accepted_residual);
        agg.max_rejected_residual = std::max(agg.max_rejected_residual, one.max_rejected_residual);
        agg.max_screen_rejected = std::max(agg.max_screen_rejected, one.max_screen_rejected);
        agg.screen_max_dependent = std::max(agg.screen_max_dependent, one.screen_max_dependent);
        agg.screen_min_independent = std::min(agg.screen_min_independent, one.screen_min_independent);
        agg.precision = one.precision;
        agg.decide = one.decide;
        agg.block = one.block;
        agg.early_exit = one.early_exit;
        agg.block_growth = one.block_growth;  // per-problem values: those of the last problem
        agg.tile_dot = one.tile_dot;
        agg.tile_sub = one.tile_sub;
        agg.autotuned = std::max(agg.autotuned, one.autotuned);
        acc_bytes += one.kernel_bytes[LIE_K_ACCEPT];
        vfy_flops += one.kernel_flops[LIE_K_VERIFY];
        vfy_bytes += one.kernel_bytes[LIE_K_VERIFY];
    }
    agg.blocks = b->rounds;
    agg.host_syncs = b->host_syncs;
    agg.run_ms = b->run_ms;
    for (int k = 0; k < LIE_K_COUNT; ++k) {
        agg.kernel_launches[k] = b->timer.n[k];
        agg.kernel_ms[k] = b->timer.ms[k];
        agg.kernel_flops[k] = b->timer.flops[k];
        agg.kernel_bytes[k] = b->timer.bytes[k];
    }
    agg.kernel_bytes[LIE_K_ACCEPT] = acc_bytes;
    agg.kernel_flops[LIE_K_VERIFY] = vfy_flops;
    agg.kernel_bytes[LIE_K_VERIFY] = vfy_bytes;
    *out = agg;
    return LIE_OK;
}

void lie_closure_batch_free(lie_closure_batch *b) { delete b; }

}  // extern "C"

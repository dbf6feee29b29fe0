// Host driver and C ABI of the closure engine (see include/lie_closure.h).
//
// The driver owns one problem's device state: the FP64 basis V64 in the
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
constexpr int kGemvRows = 16;
// Default SCREEN reject threshold on the FP32-screened residual (paper norm).
constexpr double kDefaultTauFp32 = 1e-4;
constexpr int kMaxBlock = 1024;
constexpr int kMaxD = 128;

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Per-kernel-class launch counters, algorithmic work, and (optionally) HIP-event
// durations.  Events bracket single kernel launches on the handle's stream and
// are harvested at the driver's synchronisation points.
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
    int bmax = 1;            // allocation bound of any block
    bool screened = false;   // FP32 screening pass in front of the FP64 decisions
    int policy = lie::POL_ALL;
    double policy_thr = 0.0;
    // device
    int device = -1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    double *V64 = nullptr;       // cap x D, FP64 basis
    float *Vs = nullptr;         // cap x D, FP32 rounding of V64 (screened modes)
    double *H64 = nullptr;       // block x D, FP64 candidates, then residuals
    float *Hs = nullptr;         // block x D, FP32 screened candidates
    double *C = nullptr;         // block x cap FP64 coefficients
    float *Cs = nullptr;         // block x cap FP32 coefficients
    double *part = nullptr;      // FP64 split-K scratch + norm partials
    double *normpart_s = nullptr;// block x tiles, screened residual partial norms
    double *cand_a2 = nullptr;   // block: squared residual of the first pass (screen or FP64)
    double *cand_n2 = nullptr;   // block: squared candidate norm of the first pass
    double *rho2 = nullptr;      // block: squared FP64 residuals of survivors
    double *h2 = nullptr;        // block: squared FP64 candidate norms of survivors
    double *h2b = nullptr;       // block: scratch norms
    int *surv_rows = nullptr;    // block: survivor -> candidate
    int64_t *surv_pairs = nullptr;  // block: survivor -> pair index
    int *slot = nullptr;         // block: candidate -> survivor or -1
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

    ~lie_closure()
    {
        if (device >= 0)
            (void)hipSetDevice(device);
        if (stream)
            (void)hipStreamSynchronize(stream);
        for (void *p : {(void *)V64, (void *)Vs, (void *)H64, (void *)Hs, (void *)C, (void *)Cs, (void *)part,
                        (void *)normpart_s, (void *)cand_a2, (void *)cand_n2, (void *)rho2, (void *)h2, (void *)h2b,
                        (void *)surv_rows, (void *)surv_pairs, (void *)slot, (void *)nsurv, (void *)st,
                        (void *)scalar})
            if (p)
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
        const double N = (double)n_lo, Dd = (double)D, c = cnt, w = sizeof(double);
        if (cnt > kGemvRows) {
            // matrix-core path: coefficients, then residual with fused norms, then the norm sums
            timer.begin(stream);
            HIP_TRY(lie::launch_gemm_dot_f64(V64, st, H64, rows, nrows, cnt, D, sh.n_hi, C, stream));
            timer.end(kid_dot, stream, 2.0 * N * Dd * c, (N * Dd + c * Dd + c * N) * w);
            timer.begin(stream);
            HIP_TRY(lie::launch_gemm_sub_f64(V64, st, H64, rows, nrows, C, sh.n_hi, cnt, D, part, stream));
            timer.end(kid_sub, stream, 2.0 * N * Dd * c, (N * Dd + c * N + 2.0 * c * Dd) * w);
            timer.begin(stream);
            HIP_TRY(lie::launch_norm_final(part, nrows, cnt, lie::gemm_sub_tiles_f64(D), st, rho2_out, h2_out, stream));
            timer.end(kid_red, stream, 0, 0);
            return LIE_OK;
        }
        timer.begin(stream);
        HIP_TRY(lie::launch_dot_f64(V64, st, H64, rows, nrows, C, sh, stream));
        timer.end(kid_dot, stream, 2.0 * N * Dd * c, (N * Dd + c * Dd + c * N) * w);
        timer.begin(stream);
        HIP_TRY(lie::launch_sub_f64(V64, st, C, nrows, part, sh, stream));
        timer.end(kid_sub, stream, 2.0 * N * Dd * c, (N * Dd + c * N + c * Dd) * w);
        const int ks = lie::project_split_k(D, cnt, sh.n_hi);
        timer.begin(stream);
        HIP_TRY(lie::launch_reduce_f64(H64, rows, nrows, part, st, rho2_out, h2_out, sh, stream));
        timer.end(kid_red, stream, 3.0 * c * Dd, (ks + 2.0) * c * Dd * w);
        return LIE_OK;
    }

    lie_status classify(int cnt, int64_t p0, int pol, double thr)
    {
        timer.begin(stream);
        HIP_TRY(lie::launch_classify(cand_a2, cand_n2, cnt, p0, pol, thr, st, surv_rows, surv_pairs, slot, nsurv,
                                     stream));
        timer.end(LIE_K_REDUCE, stream, 0, 0);
        return LIE_OK;
    }

    lie_status accept(int cnt, int mode, bool screen_first, const int *rrow, const double *h2_surv, int kid)
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
        a.h2 = h2_surv;
        a.rho2 = rho2;
        a.cnt = cnt;
        a.D = D;
        a.cap = cap;
        a.ambient = ambient;
        a.tol = tol;
        a.mode = mode;
        a.screened = screen_first ? 1 : 0;
        a.early_exit = mode == 1 ? cfg.early_exit : 0;
        timer.begin(stream);
        HIP_TRY(lie::launch_accept_f64(a, stream));
        timer.end(kid, stream, 0, 0);
        return LIE_OK;
    }

    // Generator phase: every generator in input order, FP64, relative threshold.
    lie_status generators(const double *gens_host)
    {
        double *staging = nullptr;
        const size_t bytes = (size_t)n_gen * D * 2 * sizeof(double);
        HIP_TRY(hipMalloc(&staging, bytes));
        struct Guard {
            double *p;
            ~Guard() { (void)hipFree(p); }
        } guard{staging};
        double *packed = nullptr;
        HIP_TRY(hipMalloc(&packed, (size_t)n_gen * D * sizeof(double)));
        Guard guard2{packed};
        HIP_TRY(hipMemcpyAsync(staging, gens_host, bytes, hipMemcpyHostToDevice, stream));
        HIP_TRY(lie::launch_pack_c128(staging, packed, n_gen, d, stream));
        lie_status s;
        for (int g = 0; g < n_gen; ++g) {
            HIP_TRY(hipMemcpyAsync(H64, packed + (size_t)g * D, D * sizeof(double), hipMemcpyDeviceToDevice, stream));
            if ((s = project(nullptr, nullptr, cand_a2, cand_n2, 1, g, g, LIE_K_OTHER, LIE_K_OTHER, LIE_K_OTHER)) !=
                LIE_OK)
                return s;
            if ((s = classify(1, 0, lie::POL_REL, tol)) != LIE_OK)
                return s;
            if ((s = project(surv_rows, nsurv, rho2, h2b, 1, g, g, LIE_K_OTHER, LIE_K_OTHER, LIE_K_OTHER)) != LIE_OK)
                return s;
            if ((s = accept(1, 0, false, surv_rows, nullptr, LIE_K_OTHER)) != LIE_OK)
                return s;
        }
        if ((s = sync_state()) != LIE_OK)
            return s;
        return check_state();
    }

    // FP64 block step over pair indices [cursor, cursor + cnt).
    // Bracket work per candidate: one complex d x d product (8 d^3 flops), since
    // [a,b] = ab - (ab)^H for anti-Hermitian a, b; bytes: two operands read, one result written.
    lie_status step_fp64(int cnt, int64_t n_lo, int64_t n_hi)
    {
        const double c = cnt, Dd = (double)D, dd = d;
        timer.begin(stream);
        HIP_TRY(lie::launch_comm_f64(V64, d, cursor, nullptr, nullptr, cnt, st, H64, stream));
        timer.end(LIE_K_COMM, stream, 8.0 * dd * dd * dd * c, 3.0 * c * Dd * sizeof(double));
        lie_status s;
        if ((s = project(nullptr, nullptr, cand_a2, cand_n2, cnt, n_lo, n_hi, LIE_K_DOT, LIE_K_SUB, LIE_K_REDUCE)) !=
            LIE_OK)
            return s;
        if ((s = classify(cnt, cursor, lie::POL_ABS, tol)) != LIE_OK)
            return s;
        // re-orthogonalisation pass for the survivors only (twice is enough)
        if ((s = project(surv_rows, nsurv, rho2, h2b, cnt, 0, n_hi, LIE_K_VERIFY, LIE_K_VERIFY, LIE_K_VERIFY)) !=
            LIE_OK)
            return s;
        return accept(cnt, 1, false, surv_rows, nullptr, LIE_K_ACCEPT);
    }

    // Screened block step: FP32 bracket and projection on MFMA, classification,
    // then FP64 recomputation (bracket + two projection passes) of the survivors.
    lie_status step_screen(int cnt, int64_t n_lo, int64_t n_hi)
    {
        const double c = cnt, Dd = (double)D, dd = d, N = (double)n_lo, w = sizeof(float);
        const int64_t nh = std::min(std::max<int64_t>(n_hi, 1), cap);
        timer.begin(stream);
        HIP_TRY(lie::launch_comm_f32(Vs, d, cursor, cnt, st, Hs, cand_n2, stream));
        timer.end(LIE_K_COMM, stream, 8.0 * dd * dd * dd * c, 3.0 * c * Dd * w);
        const int tile_dot = lie::gemm_tile_f32(cnt, nh), tile_sub = lie::gemm_tile_f32(cnt, D);
        timer.begin(stream);
        HIP_TRY(lie::launch_gemm_dot_f32(Vs, st, Hs, cnt, D, nh, Cs, tile_dot, stream));
        timer.end(LIE_K_DOT, stream, 2.0 * N * Dd * c, (N * Dd + c * Dd + c * N) * w);
        timer.begin(stream);
        HIP_TRY(lie::launch_gemm_sub_f32(Vs, st, Hs, Cs, nh, cnt, D, normpart_s, tile_sub, stream));
        timer.end(LIE_K_SUB, stream, 2.0 * N * Dd * c, (N * Dd + c * N + c * Dd) * w);
        timer.begin(stream);
        HIP_TRY(lie::launch_norm_final(normpart_s, nullptr, cnt, lie::gemm_sub_tiles_f32(D, tile_sub), st, cand_a2,
                                       nullptr, stream));
        timer.end(LIE_K_REDUCE, stream, 0, 0);
        lie_status s;
        if ((s = classify(cnt, cursor, policy, policy_thr)) != LIE_OK)
            return s;
        timer.begin(stream);
        HIP_TRY(lie::launch_comm_f64(V64, d, 0, surv_pairs, nsurv, cnt, st, H64, stream));
        timer.end(LIE_K_VERIFY, stream, 0, 0);
        if ((s = project(nullptr, nsurv, rho2, h2, cnt, 0, n_hi, LIE_K_VERIFY, LIE_K_VERIFY, LIE_K_VERIFY)) != LIE_OK)
            return s;
        if ((s = project(nullptr, nsurv, rho2, h2b, cnt, 0, n_hi, LIE_K_VERIFY, LIE_K_VERIFY, LIE_K_VERIFY)) != LIE_OK)
            return s;
        return accept(cnt, 1, policy != lie::POL_ALL, nullptr, h2, LIE_K_ACCEPT);
    }

    lie_status run(int64_t budget)
    {
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
            if (cursor >= avail || queued >= kMaxQueued || over_budget) {
                if ((s = sync_state()) != LIE_OK || (s = check_state()) != LIE_OK)
                    break;
                queued = 0;
                queued_rows = 0;
                n_lo = hs.N;
                if (block == 0) {
                    // adaptive block: small while candidates are mostly accepted, large otherwise
                    const int64_t dc = hs.n_cand - last_cand, da = hs.n_acc - last_acc;
                    if (dc > 0)
                        cur = 8 * da > dc ? block_growth : block_sat;
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
            s = screened ? step_screen(cnt, n_lo, n_hi) : step_fp64(cnt, n_lo, n_hi);
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
    for (int r : out->reserved)
        if (r != 0)
            return fail(LIE_ERR_ARG, "config.reserved must be zero");
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
        h->block_sat = 1024;
    }
    h->timer.on = cfg.profile != 0;
    h->screened = cfg.precision != LIE_PREC_FP64;
    if (cfg.precision == LIE_PREC_BF16X3) {
        delete h;
        return fail(LIE_ERR_ARG, "LIE_PREC_BF16X3 is not available in this build");
    }
    if (h->screened) {
        switch (cfg.decide) {
        case LIE_DECIDE_FP64:
            h->policy = lie::POL_ALL;
            break;
        case LIE_DECIDE_STRICT:
            h->policy = lie::POL_ABS;
            h->policy_thr = tol / 100.0;
            break;
        default:
            h->policy = lie::POL_GE;
            h->policy_thr = cfg.tau_rej > 0 ? cfg.tau_rej : kDefaultTauFp32;
            break;
        }
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
    const int b = h->block > 0 ? h->block : std::max(h->block_growth, h->block_sat);
    h->bmax = b;
    auto alloc = [&](auto **p, size_t n) -> lie_status {
        using T = std::remove_pointer_t<std::remove_reference_t<decltype(*p)>>;
        hipError_t e = hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T));
        if (e != hipSuccess)
            return fail(e == hipErrorOutOfMemory ? LIE_ERR_OOM : LIE_ERR_DEVICE, "hipMalloc of %zu elements failed: %s",
                        n, hipGetErrorString(e));
        return LIE_OK;
    };
    const int bmax = std::max(b, 1);
    const size_t capr = (size_t)lie::coef_ld(h->cap);
    if ((s = alloc(&h->V64, (size_t)h->cap * D)) != LIE_OK || (s = alloc(&h->H64, (size_t)bmax * D)) != LIE_OK ||
        (s = alloc(&h->C, (size_t)bmax * capr)) != LIE_OK ||
        (s = alloc(&h->part, std::max(lie::proj_scratch_doubles(D, std::min(bmax, 64), h->cap),
                                       (size_t)bmax * lie::gemm_sub_tiles_f64(D) * 2))) != LIE_OK ||
        (s = alloc(&h->cand_a2, bmax)) != LIE_OK || (s = alloc(&h->cand_n2, bmax)) != LIE_OK ||
        (s = alloc(&h->rho2, bmax)) != LIE_OK || (s = alloc(&h->h2, bmax)) != LIE_OK ||
        (s = alloc(&h->h2b, bmax)) != LIE_OK || (s = alloc(&h->surv_rows, bmax)) != LIE_OK ||
        (s = alloc(&h->surv_pairs, bmax)) != LIE_OK || (s = alloc(&h->slot, bmax)) != LIE_OK ||
        (s = alloc(&h->nsurv, 1)) != LIE_OK || (s = alloc(&h->scalar, 1)) != LIE_OK ||
        (s = alloc(&h->st, 1)) != LIE_OK)
        return bail(s);
    if (h->screened) {
        if ((s = alloc(&h->Vs, (size_t)h->cap * D)) != LIE_OK || (s = alloc(&h->Hs, (size_t)bmax * D)) != LIE_OK ||
            (s = alloc(&h->Cs, (size_t)bmax * capr)) != LIE_OK ||
            (s = alloc(&h->normpart_s, (size_t)bmax * lie::gemm_sub_tiles_f32(D, 1) * 2)) != LIE_OK)
            return bail(s);
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
    const int64_t n = h->hs.N;
    *written = n;
    if (capacity < n)
        return fail(LIE_ERR_CAPACITY, "output holds %lld elements, basis has %lld", (long long)capacity,
                    (long long)n);
    if (n == 0)
        return LIE_OK;
    HIP_TRY(hipSetDevice(h->device));
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

lie_status lie_closure_orthogonality(lie_closure *h, double *loss)
{
    if (!h || !loss)
        return fail(LIE_ERR_ARG, "NULL argument");
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
    for (int k = 0; k < LIE_K_COUNT; ++k) {
        out->kernel_launches[k] = h->timer.n[k];
        out->kernel_ms[k] = h->timer.ms[k];
        out->kernel_flops[k] = h->timer.flops[k];
        out->kernel_bytes[k] = h->timer.bytes[k];
    }
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

struct lie_closure_batch {
    std::vector<lie_closure *> probs;
    ~lie_closure_batch()
    {
        for (auto *p : probs)
            delete p;
    }
};

extern "C" {

lie_status lie_closure_batch_init(lie_closure_batch **out, int32_t n_problems, const double *const *generators,
                                  const int32_t *n_gen, const int32_t *d, const double *tol,
                                  const lie_closure_config *cfg)
{
    if (!out || !generators || !n_gen || !d || !tol)
        return fail(LIE_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (n_problems < 1)
        return fail(LIE_ERR_ARG, "n_problems must be >= 1");
    auto *b = new (std::nothrow) lie_closure_batch();
    if (!b)
        return fail(LIE_ERR_OOM, "host allocation failed");
    for (int32_t i = 0; i < n_problems; ++i) {
        lie_closure *h = nullptr;
        lie_status s = lie_closure_init(&h, generators[i], n_gen[i], d[i], tol[i], cfg);
        if (s != LIE_OK) {
            std::string msg = g_last_error;
            delete b;
            return fail(s, "problem %d: %s", i, msg.c_str());
        }
        b->probs.push_back(h);
    }
    *out = b;
    return LIE_OK;
}

lie_status lie_closure_batch_run(lie_closure_batch *b)
{
    if (!b)
        return fail(LIE_ERR_ARG, "batch is NULL");
    for (size_t i = 0; i < b->probs.size(); ++i) {
        lie_status s = b->probs[i]->run(-1);
        if (s != LIE_OK)
            return s;
    }
    return LIE_OK;
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
    if (!b || i < 0 || i >= (int32_t)b->probs.size())
        return fail(LIE_ERR_ARG, "bad batch index");
    return lie_closure_stats_get(b->probs[i], out);
}

void lie_closure_batch_free(lie_closure_batch *b) { delete b; }

}  // extern "C"

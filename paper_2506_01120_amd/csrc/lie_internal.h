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
    double scr_max_dep;      // largest screened residual of a candidate found dependent in FP64
    double scr_min_indep;    // smallest screened residual of a candidate found independent in FP64
    int32_t numeric_error;   // 1: non-finite residual; 2: |V| would pass the ambient bound
    int32_t full;            // 1: an append was refused because the capacity is reached
    int32_t done;            // 1: early-exit bound reached
    int32_t pad;
    int64_t n_bqr;           // appended by the block Cholesky-QR prefix of the acceptance kernel
    int64_t n_rows;          // survivor residual rows read by the acceptance kernel's in-block decisions
    int64_t raw_lo;          // Algorithm 3: |V| when the last acceptance launch started (raw rows from here on)
    double vfy_flops;        // algorithmic flops of the FP64 verification of survivors (bracket + passes)
    double vfy_bytes;        // algorithmic bytes of the same
    int64_t n_reorth;        // in-block decisions that took a further pass against the whole basis
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

// ------------------------------------------------------------- grouped (batched) launches
// One launch serves several problems: workgroup b belongs to problem p with
// start[p] <= b < start[p+1]; its local index b - start[p] is split into
// (b_local % gx[p], b_local / gx[p]) for two-dimensional stage grids.  `args`
// points at nprob argument structs of the stage in device memory.
struct Batch {
    const void *args;
    const int *start;  // nprob + 1 prefix offsets
    const int *gx;     // per-problem grid width
    int nprob;
    int total;         // start[nprob]
};

// Workgroup barrier that orders LDS traffic only: it waits for this wave's LDS
// operations (lgkmcnt = 0) but not for outstanding global loads or stores, so a
// prefetch or a result store in flight does not stall every barrier.  Use it
// only where no thread reads global data another thread of the workgroup just wrote.
// s_waitcnt encoding (gfx9): vmcnt[3:0] | expcnt[6:4] | lgkmcnt[11:8] | vmcnt[5:4] << 14.
__device__ inline void lds_barrier()
{
    __builtin_amdgcn_s_waitcnt(0xC07F);  // vmcnt = 63, expcnt = 7, lgkmcnt = 0
    __builtin_amdgcn_s_barrier();
}

__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

// sum over z < n of p[z * stride], added in the order z = 0, 1, ... (a plain loop's
// rounding), with the loads of each group of eight issued together before any is added:
// a plain loop waits on each load before the next, one memory latency per term.
__device__ inline double ordered_strided_sum(const double *p, int64_t stride, int n)
{
    double s = 0.0;
    for (int z0 = 0; z0 < n; z0 += 8) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            v[q] = p[(int64_t)(z0 + q < n ? z0 + q : z0) * stride];  // a term past n re-reads a valid one
        __builtin_amdgcn_sched_barrier(0);  // all eight loads in flight before the first add
#pragma unroll
        for (int q = 0; q < 8; ++q)
            s += z0 + q < n ? v[q] : 0.0;  // adding +0 leaves a sum unchanged
    }
    return s;
}

__device__ inline int batch_find(const int *start, int n, int b)
{
    int lo = 0, hi = n;  // start[lo] <= b < start[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Per-stage argument structs (one problem each).
struct CommArgs {
    const void *V;             // basis rows (double or float, packed layout)
    int d;
    int64_t p0;                // pair index of candidate 0 (when pair_list and dp0 are null)
    const int64_t *pair_list;  // candidate c -> pair index (null: p0 + c)
    const int64_t *dp0;        // device pair cursor used instead of p0 (graph replays), or null
    const int *ncnt;           // device candidate count (null: cnt)
    int cnt;
    const DevState *st;
    void *H;                   // output rows (packed, row stride d*d)
    double *hs2;               // FP32 bracket: squared norms of the output rows
    __bf16 *Hp;                // FP32 bracket: when set, rows go to interleaved split-BF16 planes instead of H
    int64_t ldp;               // row stride of Hp (bf16 elements)
};

// Element e of an interleaved-plane row (groups of 8 hi values, then their 8 lo values):
// hi = bf16(v), lo = bf16(v - hi).
__device__ inline void store_plane(__bf16 *row, int64_t e, float v)
{
    const __bf16 hi = (__bf16)v;
    const __bf16 lo = (__bf16)(v - (float)hi);
    __bf16 *p = row + 16 * (e >> 3) + (e & 7);
    p[0] = hi;
    p[8] = lo;
}

struct NormArgs {
    const double *normpart;    // [rows][tiles][2]
    const int *nrows;
    int cnt;
    int tiles;
    const DevState *st;
    double *rho2;
    double *h2;                // may be null
};

struct ClassifyArgs {
    const double *a2, *n2;
    int cnt;
    int64_t p0;
    const int64_t *dp0;        // device pair cursor used instead of p0, or null
    int policy;
    double thr;
    const DevState *st;
    int *rows;
    int64_t *pairs;
    int *slot;
    int *nsurv;
    int64_t ambient;           // the ambient bound (d^2 - 1 or d^2) of the problem
    int certify;               // 1: the policy may reject only while st->N >= ambient (see classify_body)
};

struct GemmArgs {
    const void *H;        // candidate rows (row stride D)
    const int *rows;      // pass row -> H row (null: identity)
    const int *nrows;     // device row count (null: cnt)
    int cnt;
    const void *V;        // basis (row stride D)
    void *C;              // coefficients, row stride ldc
    int64_t ldc;
    int64_t D;
    const DevState *st;   // basis size N and abort flags
    int64_t N_fixed;      // used when st is null
    double *normpart;     // residual: per (row, column tile) squared norms [rows][tiles][2]
    int write_r;          // residual: write R over H
    int ksplit;           // K slices (grid.z); <= 1: no split
    int cslices;          // residual: coefficient slices to add while loading C (<= 1: one)
    int64_t cslice;       // element stride between coefficient slices
    void *P;              // residual with ksplit > 1: partial products, ksplit slices of cnt x D
    int64_t pslice;       // element stride between partial-product slices
};

// Candidate policies of the classification kernel (a2: squared residual, n2: squared norm).
enum Policy {
    POL_ALL = 0,  // every candidate survives
    POL_ABS = 1,  // survive iff n2 > 0 and sqrt(a2) > thr
    POL_REL = 2,  // survive iff n2 > 0 and sqrt(a2) > thr * sqrt(n2)
    POL_GE = 3,   // survive iff n2 > 0 and sqrt(a2) >= thr
    POL_GE_REL = 4  // survive iff n2 > 0 and sqrt(a2) >= thr * sqrt(n2)
};

// ------------------------------------------------------------- FP64 kernels
// All pointers are device pointers.  Kernels of a block step read the current
// basis size and the abort flags (done / numeric_error / full) from the
// DevState, so a host loop can enqueue several block steps without a round
// trip.  Grids are sized on the host for an upper bound `n_hi` of N;
// workgroups beyond N exit.  Row lists (`rows`, `nrows`) restrict a pass to
// the survivors of an earlier pass.

// Pack complex128 operators (interleaved re,im; d x d row-major) into the packed layout.
hipError_t launch_pack_c128(const double *src, double *dst, int count, int d, hipStream_t s);
// Unpack packed operators back to complex128 d x d.
hipError_t launch_unpack_c128(const double *src, double *dst, int64_t count, int d, hipStream_t s);

// H[c] = pack([V_l, V_m]) for the pair of index p0 + c (pair_list == nullptr)
// or pair_list[c], for c < cnt (or c < *ncnt when ncnt is given).  FP64.
hipError_t launch_comm_f64(const double *V, int d, int64_t p0, const int64_t *pair_list, const int *ncnt, int cnt,
                           const DevState *st, double *H, hipStream_t s, const int64_t *dp0 = nullptr);
// *cursor += cnt (one thread; keeps a device pair cursor in step with graph replays)
hipError_t launch_advance_cursor(int64_t *cursor, int cnt, hipStream_t s);
// *cursor = value (the value travels as a kernel argument, so no host buffer must outlive the call)
hipError_t launch_set_cursor(int64_t *cursor, int64_t value, hipStream_t s);

struct ProjShape {
    int64_t D;      // elements per operator (d*d)
    int cnt;        // rows in this call (upper bound when a row count lives on the device)
    int64_t n_hi;   // host upper bound of N (grid sizing, coefficient leading dimension)
};
size_t proj_scratch_doubles(int64_t D, int cnt_max, int64_t cap);
int project_split_k(int64_t D, int cnt, int64_t n_hi);
// Element-range slices of the coefficient pass below (1: none) that fit `ws_doubles`.
int dot_slices_f64(ProjShape sh, size_t ws_doubles);
// C[r][k] = <H_row(r), V_k>, leading dimension n_hi; with sd > 1, sd partial slices at a
// stride of cnt * n_hi elements (needs sd * cnt * n_hi doubles at C)
hipError_t launch_dot_f64(const double *V, const DevState *st, const double *H, const int *rows, const int *nrows,
                          double *C, ProjShape sh, hipStream_t s, int sd = 1);
// split-K partial products of C V into `part`; C holds `cs` slices (as written above)
hipError_t launch_sub_f64(const double *V, const DevState *st, const double *C, const int *nrows, double *part,
                          ProjShape sh, hipStream_t s, int cs = 1);
// R = H - sum(part) written over H_row(r); squared norms of R and of the input into rho2[r], h2[r]
hipError_t launch_reduce_f64(double *H, const int *rows, const int *nrows, double *part, const DevState *st,
                             double *rho2, double *h2, ProjShape sh, hipStream_t s);

// Acceptance of one block (one workgroup): see kernels_accept.hip.
struct AcceptArgs {
    double *V;
    float *Vs;               // FP32 shadow basis (may be null)
    DevState *st;
    double *H;               // FP64 residual rows of survivors
    const int *rrow;         // survivor r -> H row (null: r)
    const double *cand_a2;   // per candidate: screened (or FP64 first-pass) squared residual
    const double *cand_n2;   // per candidate: squared candidate norm (screen or FP64)
    const int *slot;         // per candidate: survivor index or -1
    const int *nsurv;
    const int *surv_cand;    // survivor r -> candidate c
    const double *h2;        // per survivor: squared FP64 candidate norm (null: cand_n2 of its candidate)
    const double *rho2;      // per survivor: squared FP64 residual against the block's basis snapshot
    int *keep;               // scratch (cnt ints): survivors left after the snapshot rejections
    const int64_t *surv_pairs;  // Algorithm 3: survivor r -> pair index (null: not recorded)
    int64_t *elem_src;       // Algorithm 3: element N -> its pair index, or -(generator + 1) (null: off)
    int64_t src0;            // Algorithm 3, generator phase: the source code of the (single) candidate
    int rel;                 // 1: brackets use the relative threshold tol * ||h|| (Algorithm 3)
    int track_new;           // 1: record st->raw_lo (first row appended by this launch) without elem_src
    int cnt;
    int64_t D, cap, ambient;
    double tol;
    int mode;                // 0: generator (relative threshold), 1: bracket
    int screened;            // 1: non-survivors were rejected by the screen
    int early_exit;
    int64_t lds_doubles;     // dynamic LDS of the launch, in doubles (accept_lds_doubles)
    int vpasses;             // FP64 projection passes the block's survivors went through before this launch
    int vbracket;            // 1: the survivors' brackets were recomputed in FP64 before those passes
    int d;                   // matrix size (bracket work of vbracket)
};
hipError_t launch_accept_f64(const AcceptArgs &args, hipStream_t s);
// Dynamic LDS (doubles) for an acceptance launch of cnt candidates of length D.
int64_t accept_lds_doubles(int cnt, int64_t D);
// Largest block whose acceptance launch fits in LDS (coefficients + one residual).
int accept_max_block(int64_t D);

// Algorithm 3: raw rows B[e] for the elements appended by the last acceptance launch
// (e in [st->raw_lo, st->N)): the packed generator G[g] for a source -(g+1), else the
// packed bracket [B_l, B_m] of the source pair; Bs (if non-null) gets the FP32 rounding.
hipError_t launch_raw_append(const double *G, double *B, float *Bs, int d, const int64_t *elem_src, const DevState *st,
                             int max_new, hipStream_t s, bool normalize = false);

// G = V V^T (n x n) then ||G - I||_F into *out (device), using `work` of n*n + 256 doubles.
hipError_t launch_orth_loss(const double *V, int64_t n, int64_t D, double *work, double *out, hipStream_t s);
// The same loss with G formed in row panels inside a fixed workspace of ws_doubles doubles
// (256 partial sums, then one panel of rows x n): panels of as many rows as fit, each reduced
// into the running partial sums in panel order.  Needs ws_doubles >= 256 + n.
hipError_t launch_orth_loss_panels(const double *V, int64_t n, int64_t D, double *ws, int64_t ws_doubles,
                                   double *out, hipStream_t s);

// ------------------------------------------------------------- fixed workspace (noalloc.hip)
// Size of the per-device file-scope workspace of the allocation-free entry points: 8 MiB.
constexpr int64_t kNoallocScratchDoubles = (int64_t)1 << 20;
// Look up the workspace's device address on `device` (which must be current); once per device.
hipError_t noalloc_setup(int device);
// The looked-up address on `device`, or nullptr before noalloc_setup succeeded there.
double *noalloc_scratch(int device);

// ------------------------------------------------------------- matrix-core projection GEMMs (kernels_gemm.hip)
// Coefficients C[m][n] = <H_row(m), V_n> and residual R = H - C V with per-tile
// squared norms (normpart[m][tile][2] = {||R||^2, ||H||^2} partial sums).
// The coefficient GEMMs stride over basis tiles up to the device value of N,
// so their grids may be sized for any bound; the coefficient leading dimension
// `ldc` must cover the capacity (the engine passes coef_ld(capacity)).
int64_t coef_ld(int64_t n_hi);
int gemm_tile_f32(int64_t rows, int64_t cols);     // 2: 128x128 workgroup tile, 1: 64x64
int gemm_sub_tiles_f32(int64_t D, int tile);
int gemm_sub_tiles_f64(int64_t D);
hipError_t launch_gemm_dot_f32(const float *Vs, const DevState *st, const float *Hs, int cnt, int64_t D, int64_t n_hi,
                               int64_t ldc, float *C, int tile, hipStream_t s);
hipError_t launch_gemm_sub_f32(const float *Vs, const DevState *st, const float *Hs, const float *C, int64_t n_hi,
                               int64_t ldc, int cnt, int64_t D, double *normpart, int tile, hipStream_t s);
// Split of a small FP64 pass over K (coefficients: kd slices of cnt x ldc; residual:
// ks slices of cnt x D partial products), sized to fit `ws_doubles` of workspace.
constexpr int kSplitRows = 128;  // passes over more rows are never split
struct SplitPlan {
    int kd, ks;
};
SplitPlan gemm_split_plan_f64(int cnt, int64_t n_hi, int64_t D, int64_t ldc, size_t ws_doubles);
size_t gemm_split_ws_doubles(int64_t D, int64_t ldc);
// With ksplit > 1, C receives ksplit slices at a stride of cnt * ldc elements.
hipError_t launch_gemm_dot_f64(const double *V, const DevState *st, const double *H, const int *rows,
                               const int *nrows, int cnt, int64_t D, int64_t n_hi, int64_t ldc, double *C,
                               hipStream_t s, int ksplit = 1);
// R written over H_row(m), per-tile norms into normpart.  C holds `cslices` slices (summed
// on load).  With ksplit > 1 the pass stores ksplit slices of partial products in P
// (stride cnt * D) instead, and launch_gemm_sub_finish_f64 completes it.
hipError_t launch_gemm_sub_f64(const double *V, const DevState *st, double *H, const int *rows, const int *nrows,
                               const double *C, int64_t n_hi, int64_t ldc, int cnt, int64_t D, double *normpart,
                               hipStream_t s, int cslices = 1, int ksplit = 1, double *P = nullptr);
// R = H - sum of the P slices written over H_row(m); rho2[m] = ||R||^2, h2[m] (if non-null) = ||H||^2
hipError_t launch_gemm_sub_finish_f64(const double *P, int ksplit, double *H, const int *rows, const int *nrows,
                                      int cnt, int64_t D, const DevState *st, double *rho2, double *h2, hipStream_t s);
// rho2[m] = sum of tile partials of ||R||^2, h2[m] (if non-null) of ||H||^2
hipError_t launch_norm_final(const double *normpart, const int *nrows, int cnt, int tiles, const DevState *st,
                             double *rho2, double *h2, hipStream_t s);
// Geometry of the grouped GEMM launches (fixed tiles: FP32 64x64, FP64 64x64).
int gemm_group_m(bool f32);   // rows per workgroup
int gemm_group_n(bool f32);   // columns per workgroup
// vec: every problem's D is a multiple of 16 bytes of elements (16-byte row loads)
hipError_t launch_gemm_dot_batched(const Batch &b, bool f32, bool vec, hipStream_t s);
hipError_t launch_gemm_sub_batched(const Batch &b, bool f32, bool vec, hipStream_t s);
hipError_t launch_norm_final_batched(const Batch &b, hipStream_t s);
// Grouped versions of the other stage kernels (one workgroup per candidate for the
// brackets, per problem for classification and acceptance).  lds_variant: every
// problem of the group has d <= 64 (largest dmax); otherwise the tile-pair kernel.
hipError_t launch_comm_f64_batched(const Batch &b, bool lds_variant, int dmax, hipStream_t s);
hipError_t launch_comm_f32_batched(const Batch &b, bool lds_variant, int dmax, hipStream_t s);
hipError_t launch_classify_batched(const Batch &b, hipStream_t s);
hipError_t launch_accept_batched(const Batch &b, int64_t lds_doubles, hipStream_t s);
// Bracket of d > 64 by 16 x 16 tile pairs on the matrix cores (kernels_comm.hip), one
// workgroup per candidate; FP32 rows also get their squared norms (a.hs2).
hipError_t launch_comm_pairs(const CommArgs &a, bool f64, hipStream_t s);
// 16 < d <= 32: consecutive candidates grouped by their shared left operand (FP64 or FP32)
hipError_t launch_comm_grouped(const CommArgs &a, bool f64, hipStream_t s);
hipError_t launch_comm_pairs_batched(const Batch &b, bool f64, hipStream_t s);
bool comm_f64_fits_lds(int d);
bool comm_f32_fits_lds(int d);
// DevState copies of several problems into one array (for one read-back).
hipError_t launch_gather_states(const DevState *const *src, int n, DevState *dst, hipStream_t s);

// ------------------------------------------------------------- split-BF16 projection GEMMs (kernels_bf16.hip)
// Same contracts as the FP32 coefficient / residual GEMMs; FP32 operands are
// split into bf16 hi + lo while staged, products are hi*hi + hi*lo + lo*hi.
// Split-BF16 GEMMs on pre-split interleaved planes (kernels_bf16p.hip): a row of K values
// is K/8 groups of 32 bytes, 8 hi values then 8 lo values; K is padded to a multiple of 64
// and rows to whole tiles, all padding zero.
struct PlaneGeom {
    int64_t Kp;        // d^2 padded to a multiple of 64 (K of the coefficient GEMM)
    int64_t ld;        // row stride of H and V row planes, in bf16 elements (2 Kp)
    int64_t cap_rows;  // rows of the V row planes (capacity padded)
    int64_t ldt_k;     // capacity padded to a multiple of 64 (K of the residual GEMM)
    int64_t ldt;       // row stride of the transposed V planes and of the C planes (2 ldt_k)
    int64_t d_rows;    // rows of the transposed V planes (d^2 padded)
    int64_t b_rows;    // rows of the H and C planes (block size padded)
};
PlaneGeom plane_geom(int64_t D, int64_t cap, int bmax);
struct PlaneGemmArgs {
    const __bf16 *A;   // rows m, K contiguous (interleaved planes)
    int64_t lda;
    const __bf16 *B;   // rows n, K contiguous (interleaved planes)
    int64_t ldb;
    int64_t K;         // coefficient GEMM: padded K (the residual GEMM takes K = N from st)
    int cnt;           // rows m
    const DevState *st;
    __bf16 *Cout;      // coefficient GEMM: C planes (row m, K index n)
    int64_t ldcout;
    const __bf16 *Hp;  // residual GEMM: candidate planes for the epilogue
    int64_t ldh;
    int64_t D;         // residual GEMM: columns j
    double *normpart;  // residual GEMM: [m][tn][2] squared norms of R and H
    int tm, tn;        // output tiles
};
int plane_sub_tiles(int64_t D, int tile);
// Basis rows [*done, st->N) into the row planes Vp and transposed planes Vt, then *done = N.
hipError_t launch_planes_refresh(const double *V64, int64_t D, const DevState *st, int64_t *done, __bf16 *Vp,
                                 __bf16 *Vt, const PlaneGeom &p, hipStream_t s);
hipError_t launch_bfp_dot(const __bf16 *Hp, const __bf16 *Vp, const DevState *st, int cnt, int64_t n_hi, __bf16 *Cp,
                          const PlaneGeom &p, hipStream_t s);
hipError_t launch_bfp_sub(const __bf16 *Cp, const __bf16 *Vt, const __bf16 *Hp, const DevState *st, int cnt,
                          int64_t D, double *normpart, const PlaneGeom &p, hipStream_t s);
int gemm_sub_tiles_bf16(int64_t D, int tile);
hipError_t launch_gemm_dot_bf16x3(const float *Vs, const DevState *st, const float *Hs, int cnt, int64_t D,
                                  int64_t n_hi, int64_t ldc, float *C, int tile, hipStream_t s);
hipError_t launch_gemm_sub_bf16x3(const float *Vs, const DevState *st, const float *Hs, const float *C, int64_t n_hi,
                                  int64_t ldc, int cnt, int64_t D, double *normpart, int tile, hipStream_t s);
hipError_t launch_gemm_dot_bf16x3_batched(const Batch &b, hipStream_t s);  // 64 x 64 tiles
hipError_t launch_gemm_sub_bf16x3_batched(const Batch &b, hipStream_t s);

// ------------------------------------------------------------- FP32 screening kernels (kernels_screen.hip)
// Hs[c] = fp32 packed [Vs_l, Vs_m] for pair p0 + c, hs2[c] = ||Hs[c]||^2.
hipError_t launch_comm_f32(const float *Vs, int d, int64_t p0, int cnt, const DevState *st, float *Hs, double *hs2,
                           hipStream_t s, const int64_t *dp0 = nullptr, __bf16 *Hp = nullptr, int64_t ldp = 0);
// Survivor compaction under a policy.  certify = 1: a candidate may be rejected by the policy
// only while the basis holds `ambient` elements (then it is dependent whatever its residual);
// below that bound every candidate survives.
hipError_t launch_classify(const double *a2, const double *n2, int cnt, int64_t p0, int policy, double thr,
                           const DevState *st, int *rows, int64_t *pairs, int *slot, int *nsurv, hipStream_t s,
                           const int64_t *dp0 = nullptr, int64_t ambient = 0, int certify = 0);

// ------------------------------------------------------------- rank-test baseline (rank_svd.hip)
// Standard algorithm (Algorithm 1): a candidate raises the rank of the raw basis iff the
// smallest singular value of [B_0 .. B_{N-1}, h] (packed rows) exceeds
// max(D, N+1) * eps * sigma_max.  Batched SVD of up to max_batch such matrices (N + 1 <= D).
struct RankTester;
hipError_t rank_tester_create(RankTester **out, int64_t D, int max_batch, hipStream_t s);
void rank_tester_destroy(RankTester *t);
// flags[c] (host) = 1 iff candidate row c of H (device, cnt x D) is independent of B (device, N x D).
// Synchronises the tester's stream.
hipError_t rank_tester_run(RankTester *t, const double *B, int64_t N, const double *H, int cnt, unsigned char *flags);

// ------------------------------------------------------------- sparse Pauli-sum representation (pauli_sparse.hip)
// Elements as sorted (key = x << 32 | z, coefficient of iP) term lists in a pool on the device.
struct SparsePauli;
hipError_t sparse_pauli_create(SparsePauli **out, int nq, int64_t cap, int64_t max_terms, int64_t scratch,
                               const int64_t *gen_off, int n_gen, const uint64_t *keys, const double *coefs,
                               hipStream_t s);
void sparse_pauli_destroy(SparsePauli *s);
// Generator g: projection passes and the relative decision (appends to the pool).
hipError_t sparse_pauli_generator(SparsePauli *sp, int g, DevState *st, double tol, int64_t ambient, hipStream_t s);
// Candidate of pair index p: sparse bracket, projection passes, decision.
hipError_t sparse_pauli_candidate(SparsePauli *sp, int64_t p, DevState *st, double tol, int early_exit,
                                  int64_t ambient, hipStream_t s);
// Terms stored by the first N elements (synchronises).
hipError_t sparse_pauli_terms(const SparsePauli *sp, int64_t N, int64_t *terms, hipStream_t s);
// Offsets (N + 1), keys and coefficients of the first N elements; nothing is copied but
// *written when it exceeds capacity (synchronises).
hipError_t sparse_pauli_basis(const SparsePauli *sp, int64_t N, int64_t *offsets, uint64_t *keys, double *coefs,
                              int64_t capacity, int64_t *written, hipStream_t s);

// ------------------------------------------------------------- matrix-inversion method (inverse_gram.hip)
// A^{-1} for the Gram matrix A = B B^T of the first N unit-norm raw rows (Algorithm 2), kept as
// the inverse of its Cholesky factor and bordered by each appended element.
struct GramInverse;
hipError_t gram_inverse_create(GramInverse **out, int64_t cap, int64_t D, int max_rows, hipStream_t s);
void gram_inverse_destroy(GramInverse *g);
// Expand the factor by the rows appended since the last call, up to N (B: device, row stride D);
// *info_host = (element index + 1) when its bordered pivot was not positive (A not numerically
// positive definite), else 0.  Synchronises the stream.
hipError_t gram_inverse_update(GramInverse *g, const double *B, int64_t N, int *info_host);
// X (cnt x N, row stride ldx) = beta (cnt x N, row stride ldb) A^{-1}.
hipError_t gram_inverse_apply(GramInverse *g, const double *beta, int64_t ldb, int64_t N, int cnt, double *X,
                              int64_t ldx);

// ------------------------------------------------------------- Pauli-sum representation (pauli.hip)
// Rows are coefficient vectors over the 4^n strings iP_s (index x * 2^n + z), D = 4^n.
// H[c] = [V_l, V_m] for pairs p0 + c (or *dp0 + c) through the sparse symplectic product.
hipError_t launch_comm_pauli(const double *V, const int *sup_cnt, const int *sup_idx, int n, int64_t p0, int cnt,
                             const DevState *st, double *H, hipStream_t s, const int64_t *dp0 = nullptr);
// Supports of the rows [st->raw_lo, st->N) (indices of coefficients above 1e-14 of the row norm).
hipError_t launch_pauli_support(const double *V, int64_t D, const DevState *st, int max_new, int *sup_cnt,
                                int *sup_idx, hipStream_t s);
// Host transforms between a dense anti-Hermitian d x d matrix (interleaved complex, row-major)
// and its 4^n real Pauli coordinates.
void pauli_from_dense(const double *g, int n, double *out);
void pauli_to_dense(const double *a, int n, double *g);

// ------------------------------------------------------------- autotuner (autotune.hip)
struct TuneChoice {
    int block_sat;            // saturated-phase block size
    int tile_dot, tile_sub;   // FP32 / split-BF16 GEMM tiles (gemm_tile_f32 codes; 0 for FP64)
    double us_per_candidate;  // timed cost of the two projection GEMMs per candidate
};
// Times the coefficient and residual GEMMs of one saturated block step (basis at the
// ambient bound) for every admissible block size (<= max_block) and tile pair on
// `device`, and returns the fastest.  Looks up (and appends to) the text cache at
// cache_path when it is non-null; *from_cache tells whether any timing was run.
hipError_t autotune_block_step(int device, int precision, int d, int64_t ambient, int max_block, const char *cache_path,
                               hipStream_t s, TuneChoice *out, bool *from_cache);

}  // namespace lie

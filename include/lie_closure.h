/*
 * lie_closure.h -- C ABI of the MI355X (gfx950) Lie-closure engine.
 *
 * The engine computes the closure c of a tuple of d x d anti-Hermitian
 * generators G -- the smallest Lie algebra containing G -- as an orthonormal
 * basis V built in the order of the dimension-only orthonormalization
 * algorithm of arXiv 2506.01120 (Algorithm 4, Section 3.2):
 *
 *   generator phase:  for g in G: g_perp = g - proj_V g; if g_perp != 0, append g_perp/||g_perp||
 *   bracket loop:     for each unordered pair (l, m), m < l, rows l in order:
 *                       h = [V_l, V_m];  h_perp = h - proj_V h;  if h_perp != 0, append h_perp/||h_perp||
 *
 * with the bracket [a,b] = ab - ba, the inner product <a,b> = tr(a^H b)/d and
 * the norm ||a|| = sqrt(<a,a>) of Section 2.2, and proj_V h = sum_k <V_k,h> V_k
 * (the Corollary of Theorem 1).  The returned basis satisfies
 * <V_i, V_j> = delta_ij, i.e. ||V_k||_F = sqrt(d).
 *
 * Decision rule ("h_perp != 0", which the paper leaves without a threshold):
 * a generator is kept iff ||g_perp|| > tol * ||g||; a bracket of two unit-norm
 * basis elements is kept iff ||h_perp|| > tol.  Exactly zero brackets are
 * rejected.
 *
 * The orthonormalization method (the default; Algorithms 3 and 4) and the
 * matrix-inversion method (Algorithm 2) run all of their device work in the
 * library's own HIP kernels on one GPU.  Only the comparison method
 * LIE_METHOD_RANK_SVD calls a vendor library: it takes its singular values from
 * rocSOLVER (that library SVD is what the baseline is).  Host pointers are plain CPU memory;
 * device pointers are HIP device memory of the handle's device.  No function throws; every failure returns a negative
 * lie_status and records a message readable with lie_last_error().
 *
 * Threading: a handle is not thread-safe; distinct handles are independent.
 */
#ifndef LIE_CLOSURE_H
#define LIE_CLOSURE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lie_closure lie_closure;             /* opaque; owned by the caller until lie_closure_free */
typedef struct lie_closure_batch lie_closure_batch; /* opaque; owned by the caller until lie_closure_batch_free */

typedef enum lie_status {
    LIE_OK = 0,
    LIE_INCOMPLETE = 1,            /* a budgeted run stopped early; call again to resume */
    LIE_ERR_ARG = -1,              /* invalid argument (null pointer, bad size, bad tolerance, bad config) */
    LIE_ERR_NOT_ANTIHERMITIAN = -2,/* a generator violates ||g + g^H||_F <= 1e-12 * max(1, ||g||_F) */
    LIE_ERR_NONFINITE = -3,        /* NaN or Inf in the input */
    LIE_ERR_OOM = -4,              /* device or host allocation failed */
    LIE_ERR_DEVICE = -5,           /* a HIP runtime call failed */
    LIE_ERR_STATE = -6,            /* call not allowed in the handle's state (e.g. after a failed run) */
    LIE_ERR_CAPACITY = -7,         /* the basis reached max_dim, or an output buffer is too small */
    LIE_ERR_NUMERIC = -8           /* non-finite norm, or |V| exceeded the ambient bound (spurious element) */
} lie_status;

/* Arithmetic of the screening pass (the commutator and the first projection). */
typedef enum lie_precision {
    LIE_PREC_FP64 = 0,    /* everything in FP64 */
    LIE_PREC_FP32 = 1,    /* screen in FP32 (MFMA, FP32 accumulate); FP64 verification */
    LIE_PREC_BF16X3 = 2   /* screen in split BF16 (hi*hi + hi*lo + lo*hi on MFMA, FP32 accumulate); FP64 verification */
} lie_precision;

/* Independence test.  ORTHONORMALIZATION is the paper's method (Algorithms 3 and 4: residual
 * against an orthonormal basis).  RANK_SVD is the standard algorithm it is compared with
 * (Algorithm 1 with the rank computed by an SVD, Section 3): a bracket of raw basis elements
 * is kept iff the rank of [B; h] exceeds that of B, the rank being the number of singular
 * values above max(d^2, |B|+1) * eps * sigma_max.  RANK_SVD keeps only the raw basis B
 * (lie_closure_raw_basis); it runs in FP64, one problem at a time, for d <= 16.
 * MATRIX_INVERSION is the paper's other method (Algorithm 2, Section 3.1): unit-norm raw elements
 * B, the inverse of their Gram matrix A, and the explicit residual h - B A^{-1} beta of a unit-norm
 * candidate (beta_k = <B_k, h>), kept iff its norm exceeds tol; each appended element expands A
 * (new row and column <B_i, b>, diagonal 1), and A^{-1} = L^{-T} L^{-1} follows by bordering the
 * inverse Cholesky factor; a bordered pivot that is not positive is reported as LIE_ERR_NUMERIC.
 * FP64, single problems,
 * raw basis only (unit-norm elements). */
typedef enum lie_method {
    LIE_METHOD_ORTHONORMALIZATION = 0,
    LIE_METHOD_RANK_SVD = 1,
    LIE_METHOD_MATRIX_INVERSION = 2
} lie_method;

/* Operator representation on the device.  DENSE: packed d x d matrices, brackets by one complex
 * matrix product (8 d^3 flops).  PAULI (the sparse Pauli-sum representation, Sections 3 and 4.2;
 * d = 2^n, n <= 7): real coordinates over the 4^n strings iP_s, which are orthonormal in the paper's
 * inner product, brackets by the symplectic product rule over the support of the sparser operand
 * (cost nnz * 4^n; far below 8 d^3 for sparse elements such as nested brackets of Pauli strings).
 * Inputs and outputs stay dense d x d matrices.  PAULI: FP64, single problems, method
 * ORTHONORMALIZATION without raw_basis. */
typedef enum lie_representation {
    LIE_REP_DENSE = 0,
    LIE_REP_PAULI = 1
} lie_representation;

/* How a screened candidate is decided (ignored for LIE_PREC_FP64).
 *
 * A screened residual carries rounding of about 1e-7 (FP32) to 1e-5 (split BF16) of the candidate's
 * scale, far above a threshold such as tol = 1e-8, so a small screened residual never proves that
 * the FP64 residual is at most tol (a weakly coupled direction of the closure screens as small as
 * noise).  Dependence is proved instead by the basis size: once |V| equals the ambient bound
 * (d^2 - 1 for traceless generators, else d^2) V spans every operator a bracket can produce and
 * every candidate is dependent.  STRICT and SCREEN therefore reject from the screen only at the
 * ambient bound ("certified"); below it every candidate is decided from its FP64 residual (those
 * blocks run the FP64 step directly).  Decisions then equal those of the FP64 path. */
typedef enum lie_decide {
    LIE_DECIDE_FP64 = 0,   /* every candidate is decided from its FP64 residual; the screen is computed on
                              saturated blocks and only recorded (screen_max_dependent / _min_independent) */
    LIE_DECIDE_STRICT = 1, /* certified; at the ambient bound a screened residual below 100 * tol rejects,
                              every other candidate is decided in FP64 */
    LIE_DECIDE_SCREEN = 2  /* certified; at the ambient bound a screened residual below the precision's
                              threshold (1e-4 FP32, 1e-2 split BF16) rejects, the rest are decided in FP64.
                              With config.tau_rej > 0 that threshold rejects at every basis size: an
                              approximate, uncertified screen (a candidate whose FP64 residual exceeds tol
                              but screens below tau_rej is lost) */
} lie_decide;

typedef struct lie_closure_config {
    uint32_t struct_size;  /* must be sizeof(lie_closure_config) */
    int32_t precision;     /* lie_precision, default LIE_PREC_FP64 */
    int32_t decide;        /* lie_decide, default LIE_DECIDE_SCREEN for screened precisions */
    int32_t block;         /* candidates per block: 1 = plain one-at-a-time form, 2..16384 fixed (bounded by
                              the acceptance kernel's LDS: about 18000 - d^2), 0 = adaptive
                              (small FP64-decided blocks while most candidates are accepted, large
                              screened blocks after) */
    int32_t early_exit;    /* 1: stop once |V| equals the ambient bound (exact; d^2-1 for traceless inputs) */
    int32_t device;        /* HIP device ordinal; -1 = the calling thread's current device */
    double tau_rej;        /* SCREEN: 0 = certified screen with the precision's threshold; > 0 = this threshold,
                              applied at every basis size (approximate; see lie_decide) */
    int64_t max_dim;       /* basis capacity; 0 = ambient bound */
    void *stream;          /* hipStream_t the handle runs on; NULL = a stream the library creates */
    int32_t use_graphs;    /* 1: replay block steps from captured hipGraphs (default 1) */
    int32_t profile;       /* 1: time every kernel launch with HIP events on the handle's stream */
    int32_t autotune;      /* 1 (adaptive blocks only): pick the saturated block size and the screening GEMM
                              tiles by timing them on the device at init (about 0.1-1 s once per device,
                              precision, d and ambient bound; remembered for the process); 0: heuristics */
    int32_t reserved0;     /* must be zero */
    const char *tune_cache;/* autotune: text file of earlier choices, read at init and appended to after a
                              timing run (NULL: no file); the library does not keep the pointer */
    int32_t raw_basis;     /* 1: Algorithm 3 -- also keep the raw basis B (accepted generators and nested
                              brackets, unnormalised) and bracket raw elements [B_l, B_m] instead of
                              [V_l, V_m]; raw brackets are accepted iff their residual exceeds tol * ||h||
                              (single problems only; doubles the basis memory) */
    int32_t method;        /* lie_method: LIE_METHOD_ORTHONORMALIZATION (default) or the comparison
                              baseline LIE_METHOD_RANK_SVD */
    int32_t representation;/* lie_representation: LIE_REP_DENSE (default) or LIE_REP_PAULI */
    int32_t gemm_tile;     /* screened precisions, adaptive blocks, single problems: workgroup tile of both
                              screening GEMMs of full saturated blocks; 0 = the autotuner's choice
                              (autotune = 1) or the shape heuristic, 1 = 64 x 64, 2 = 128 x 128.  Any
                              other value, or a nonzero value in FP64, fails with LIE_ERR_ARG */
    int32_t reserved[2];   /* must be zero */
} lie_closure_config;

/* Kernel classes reported by the per-kernel counters of lie_closure_stats. */
typedef enum lie_kernel_id {
    LIE_K_COMM = 0,      /* screening (or FP64) bracket of a candidate block */
    LIE_K_DOT = 1,       /* screening (or FP64) coefficients C = H V^T */
    LIE_K_SUB = 2,       /* screening (or FP64) subtraction R = H - C V (+ norm partials) */
    LIE_K_REDUCE = 3,    /* split-K reduction, residual norms, classification */
    LIE_K_ACCEPT = 4,    /* sequential in-block acceptance and append (FP64) */
    LIE_K_VERIFY = 5,    /* FP64 recomputation of screen survivors (bracket + CGS2 passes) */
    LIE_K_OTHER = 6,     /* everything else (packing, shadow copies, bookkeeping) */
    LIE_K_GROWTH = 7,    /* FP64 bracket and projections of the unscreened blocks of a screened run
                            (growth phase); FP64 runs account these as COMM / DOT / SUB */
    LIE_K_COUNT = 8
} lie_kernel_id;

typedef struct lie_closure_stats {
    uint32_t struct_size;         /* must be sizeof(lie_closure_stats) */
    int32_t done;                 /* 1 when the closure is complete (all pairs bracketed, or early exit) */
    int64_t dim;                  /* |V| */
    int64_t ambient;              /* d^2 - 1 (traceless generators) or d^2 */
    int64_t candidates;           /* bracket candidates evaluated (N(N-1)/2 in full certification) */
    int64_t generator_checks;     /* generator candidates evaluated */
    int64_t zero_brackets;        /* brackets whose screened or FP64 norm was exactly zero */
    int64_t screen_rejected;      /* candidates rejected from the screened residual alone */
    int64_t fp64_decided;         /* candidates whose decision used an FP64 residual */
    int64_t accepted;             /* elements appended by the bracket loop */
    int64_t block_qr_accepted;    /* of those, appended by the block Cholesky-QR prefix of a block's survivors */
    int64_t blocks;               /* block steps executed */
    int64_t host_syncs;           /* device-to-host synchronisations of the host loop */
    double min_accepted_residual; /* smallest FP64 residual that was accepted (bracket loop) */
    double max_rejected_residual; /* largest FP64 residual that was rejected (bracket loop) */
    double max_screen_rejected;   /* largest screened residual among screen rejects */
    double screen_max_dependent;  /* largest first-pass residual of a survivor whose FP64 residual against the
                                     same basis snapshot is <= tol (the audit of the screen) */
    double screen_min_independent;/* smallest first-pass residual of a survivor whose FP64 snapshot residual is > tol */
    double run_ms;                /* wall time spent inside lie_closure_run* calls */
    int32_t precision, decide;
    int32_t block;                /* fixed block size, or -(saturated size) when adaptive */
    int32_t early_exit;
    int32_t tile_dot, tile_sub;   /* screening GEMM tiles of full saturated blocks (0: shape heuristic) */
    int32_t autotuned;            /* 1: sizes from a timing run at init, 2: from the tune cache, 0: heuristics */
    int32_t block_growth;         /* adaptive: block size of the growth phase */
    /* Per kernel class (lie_kernel_id), accumulated over the run: launches, and
     * the algorithmic floating-point operations and bytes those launches must
     * perform (formulas in the engine source).  kernel_ms is the summed
     * HIP-event duration and is filled only when config.profile = 1. */
    int64_t kernel_launches[LIE_K_COUNT];
    double kernel_ms[LIE_K_COUNT];
    double kernel_flops[LIE_K_COUNT];
    double kernel_bytes[LIE_K_COUNT];
    int64_t reorth_passes;        /* in-block decisions that took a further pass against the whole basis because
                                     the elements appended earlier in the block removed nearly all of the
                                     candidate's norm (ratio above 64) */
    int64_t pauli_terms;          /* sparse Pauli-sum handles: terms stored by the basis (16 bytes each) */
} lie_closure_stats;

/* Fill *cfg with defaults (struct_size set).  Returns LIE_ERR_ARG for NULL. */
lie_status lie_closure_config_default(lie_closure_config *cfg);

/*
 * Create a closure problem and run the generator phase (Algorithm 4, the loop
 * over G) on the device.
 *   out        -- receives the new handle (NULL on failure)
 *   generators -- host, n_gen * d * d complex128, row-major, interleaved (re, im);
 *                 copied, the caller keeps ownership
 *   n_gen      -- >= 1; d -- 1..128; tol -- 0 < tol < 1
 *   cfg        -- NULL for defaults
 * Validates every argument before any HIP call (LIE_ERR_ARG / _NONFINITE /
 * _NOT_ANTIHERMITIAN).  Zero generators are accepted and skipped.
 */
lie_status lie_closure_init(lie_closure **out, const double *generators, int32_t n_gen, int32_t d, double tol,
                            const lie_closure_config *cfg);

/* Run the bracket loop (Algorithm 4) to completion.  Blocking.  A no-op after completion. */
lie_status lie_closure_run(lie_closure *h);

/* Run at most max_candidates more bracket candidates (rounded up to whole blocks).
 * Returns LIE_INCOMPLETE if work remains; calling again resumes at the exact pair cursor. */
lie_status lie_closure_run_budget(lie_closure *h, int64_t max_candidates);

/* Current |V| (valid any time after init). */
lie_status lie_closure_dim(const lie_closure *h, int64_t *dim);

/* Copy V (in append order) into a host buffer of capacity * d * d complex128,
 * interleaved.  *written = |V|.  LIE_ERR_CAPACITY (with *written = |V|) if
 * capacity < |V|. */
lie_status lie_closure_basis(const lie_closure *h, double *out, int64_t capacity, int64_t *written);

/* Same into device memory of the handle's device (ordered on the handle's stream). */
lie_status lie_closure_basis_device(const lie_closure *h, void *dst, int64_t capacity, int64_t *written);

/* Host utilities of the Pauli-sum representation (no device work).  For d = 2^n (1 <= n <= 7):
 * coords[x * 2^n + z] = <iP_s, M> = -i tr(P_s M) / d, real for an
 * anti-Hermitian M, where P_s = i^{|x & z|} X^x Z^z, X^x flips the basis-index bits in x and Z^z
 * multiplies |j> by (-1)^{popcount(z & j)} (so P_s is the Kronecker product of I, X, Y, Z with one
 * Y per bit set in both masks).  matrix: d x d complex128 row-major, interleaved (re, im); coords:
 * 4^n doubles.  lie_pauli_matrix is the inverse (M = sum_s coords[s] iP_s).  LIE_ERR_ARG on NULL
 * or a d that is not such a power of two. */
lie_status lie_pauli_coordinates(int32_t d, const double *matrix, double *coords);
lie_status lie_pauli_matrix(int32_t d, const double *coords, double *matrix);

/* Algorithm 3 (Section 3.2): copy the raw basis B -- the accepted generators as given and the
 * accepted nested brackets [B_l, B_m], unnormalised, in append order -- into a host buffer
 * laid out like lie_closure_basis's (capacity * d * d complex128, interleaved re,im).
 * span(B) = span(V).  *written = |B| = |V|.  Returns LIE_ERR_STATE if the handle was not
 * created with config.raw_basis = 1, LIE_ERR_CAPACITY if capacity < |B| (nothing copied). */
lie_status lie_closure_raw_basis(const lie_closure *h, double *out, int64_t capacity, int64_t *written);

/* ||G - I||_F with G_ij = <V_i, V_j>, computed in FP64 on the device. */
lie_status lie_closure_orthogonality(lie_closure *h, double *loss);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): the value of lie_closure_orthogonality,
 * computed without any allocation and without synchronising.
 *   loss_dev -- device pointer (one double, HIP device memory of the handle's device);
 *               owned by the caller; receives ||G - I||_F once the handle's stream
 *               (config.stream, or the library's own) has executed the enqueued work
 * The Gram matrix is formed in row panels inside a fixed per-device workspace of 8 MiB
 * that the library holds for the life of the process (|V| <= 2^20 - 256, which every
 * closure the library accepts satisfies; LIE_ERR_CAPACITY otherwise).  Every call on a
 * GPU shares that GPU's workspace: calls whose work overlaps on one GPU (on different
 * streams, or from different threads) race and may return wrong values; serialise them.
 * The value can differ from lie_closure_orthogonality's in the last bits (summation order). */
lie_status lie_closure_orthogonality_noalloc(lie_closure *h, double *loss_dev);

/* Counters and residual-gap statistics (out->struct_size must be set). */
lie_status lie_closure_stats_get(const lie_closure *h, lie_closure_stats *out);

/*
 * Sparse Pauli-sum representation (the paper's sparse representation of operators,
 * Sections 3 and 4.2): generators and basis elements are real combinations
 * sum_s c_s iP_s of Pauli strings P_s = i^{|x & z|} X^x Z^z on n qubits, stored as term
 * lists -- memory proportional to each element's support, no d x d matrices.  Distinct
 * strings are orthonormal in the paper's inner product, so the coefficients are the
 * element's coordinates.  Runs Algorithm 4 in FP64 (brackets of term lists, inner
 * products by joining supports, two projection passes, the same decision rule as the
 * dense path), one candidate at a time; terms below 1e-14 of a candidate's norm after a
 * summation are dropped.
 *   n_qubits      -- 1..31
 *   term_offsets  -- host, n_gen + 1 non-decreasing offsets (term_offsets[0] = 0): generator g
 *                    is terms [term_offsets[g], term_offsets[g+1])
 *   strings       -- host, one 64-bit key per term: (x << 32) | z, bit q of x (z) set when
 *                    the string has X or Y (Z or Y) on the qubit of weight 2^q in the basis
 *                    index (qubit 0 of a label "P_0 P_1 ... P_{n-1}" is the most significant)
 *   coefs         -- host, real coefficient of iP_s of each term; all inputs are copied
 *   max_terms     -- capacity of the device term pool (0: 2^24 terms, 256 MiB)
 *   cfg           -- NULL or FP64 / orthonormalization settings (early_exit, max_dim, device,
 *                    stream are honoured; max_dim 0 = min(ambient bound, 2^20))
 * Lists of a bracket (|S_l| |S_m| products) or of a projection longer than 2^20 terms fail
 * with LIE_ERR_CAPACITY, as does an exhausted pool.  lie_closure_run / _run_budget / _dim /
 * _stats_get / _free work on the handle; the dense-basis calls return LIE_ERR_STATE.
 */
lie_status lie_closure_init_pauli_sparse(lie_closure **out, int32_t n_qubits, int32_t n_gen,
                                        const int64_t *term_offsets, const uint64_t *strings, const double *coefs,
                                        double tol, int64_t max_terms, const lie_closure_config *cfg);

/* Basis of a sparse Pauli-sum handle in Algorithm 4's order: element k is terms
 * [offsets[k], offsets[k+1]) of (strings, coefs), sorted by key, with sum c^2 = 1.
 *   offsets -- host, dim + 1 entries; strings, coefs -- host, capacity_terms entries each
 * *terms_written = total terms; LIE_ERR_CAPACITY (nothing else written) if it exceeds capacity_terms. */
lie_status lie_closure_basis_pauli_sparse(const lie_closure *h, int64_t *offsets, uint64_t *strings, double *coefs,
                                          int64_t capacity_terms, int64_t *terms_written);

/* Release everything the handle owns.  NULL-safe. */
void lie_closure_free(lie_closure *h);

/* Static description of a status code. */
const char *lie_status_string(lie_status s);

/* Detail message of the last failure on the calling thread ("" if none). */
const char *lie_last_error(void);

/*
 * Batched form: n_problems independent closures (uneven d and generator
 * counts) advanced together on one stream.  Each round advances every live
 * problem by one block step, and each stage of that step is ONE grouped
 * launch covering all problems of the round, so small problems fill the GPU
 * together; finished problems leave the batch.
 *   generators[i] -- host, n_gen[i] * d[i] * d[i] complex128 (copied)
 *   tol[i]        -- per-problem tolerance
 *   cfg           -- shared configuration (precision, decide, block, early_exit)
 */
lie_status lie_closure_batch_init(lie_closure_batch **out, int32_t n_problems, const double *const *generators,
                                  const int32_t *n_gen, const int32_t *d, const double *tol,
                                  const lie_closure_config *cfg);
lie_status lie_closure_batch_run(lie_closure_batch *b);
lie_status lie_closure_batch_dim(const lie_closure_batch *b, int32_t i, int64_t *dim);
lie_status lie_closure_batch_basis(const lie_closure_batch *b, int32_t i, double *out, int64_t capacity,
                                   int64_t *written);
/* i >= 0: that problem's counters; i = -1: the whole batch (counters summed over
 * problems, blocks = rounds, kernel timers of the grouped launches). */
lie_status lie_closure_batch_stats_get(const lie_closure_batch *b, int32_t i, lie_closure_stats *out);
void lie_closure_batch_free(lie_closure_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* LIE_CLOSURE_H */

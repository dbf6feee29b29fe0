/*
 * lie_oracle.c -- reference CPU implementation of the Lie-closure construction.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct checker
 * that the GPU library is compared against.  Only the test suite, the smoke
 * entry and the benchmark's CPU-baseline leg may load it.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * What it computes (arXiv 2506.01120):
 *   - the closure of a tuple of d x d complex operators G: the smallest Lie
 *     algebra containing G (Section 1; Section 2.1), as an orthonormal basis V
 *     built in the order of Algorithm 4 (dimension-only orthonormalization);
 *   - the Lie bracket [a,b] = ab - ba (Section 2.2, matrix commutator), formed
 *     from two plain matrix products;
 *   - the inner product <a,b> = tr(a^H b)/d and the norm ||a|| = sqrt(<a,a>)
 *     (Section 2.2), over the complex field, no realness shortcut;
 *   - linear independence of a candidate h from the current span by an
 *     explicit least-squares residual min_c ||W c - h|| (the quantity the
 *     proof of Theorem 1 tests against the null operator), where W holds the
 *     accepted candidates as columns.  The least-squares problem is solved with
 *     an incrementally extended complex Householder QR of W, so no Gram matrix
 *     and no Gram-Schmidt are involved.
 *
 * Readings of points the paper leaves open (each stated once):
 *   - "h_perp != 0" (Algorithm 4): a generator g is accepted iff its residual
 *     exceeds tol * ||g||; a bracket of two unit-norm basis elements is
 *     accepted iff its residual exceeds tol (absolute, in the paper's norm).
 *     An exactly zero candidate is rejected.
 *   - Loop indices of Algorithm 4: every unordered pair (l, m), m < l, is
 *     bracketed exactly once, rows l in increasing order and m = 0..l-1 inside
 *     a row.  This is the order that matches the paper's count of
 *     N(N-1)/2 brackets (Section 3, runtime discussion).
 *   - The appended element is V_N = h_perp / ||h_perp||, with h_perp the
 *     least-squares residual vector itself (Algorithm 4 and the projection of
 *     the Corollary in Section 3.2).
 *   - Optional early exit when |V| reaches the ambient bound (d^2 - 1 when every
 *     generator is traceless, d^2 otherwise): no further candidate can be
 *     independent there.  Off by default (the literal algorithm).
 *
 * Algorithm 3 (lo_enable_raw): the same loop, but the brackets are taken
 * between the raw elements B -- the accepted generators and the accepted
 * brackets themselves, not their orthonormalised versions -- while the
 * independence test still runs against the span of the accepted candidates.
 * Raw nested brackets have no fixed scale, so a raw bracket h is accepted iff
 * its residual exceeds tol * ||h|| (the generator phase's relative rule).
 * B is returned alongside V.
 *
 * Storage: operators are d x d complex, row-major, vectorised as length d*d.
 * Reflector j is H_j = I - 2 u_j u_j^H with ||u_j||_2 = 1 and u_j[k] = 0 for
 * k < j; Q = H_0 H_1 ... H_{N-1} has the accepted candidates' span in its
 * first N columns.
 *
 * Plain C99, double precision throughout, single-threaded.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

typedef struct lo_state {
    int d;
    int64_t n;        /* vector length d*d */
    int64_t cap;      /* maximum number of basis elements */
    int64_t N;        /* current |V| */
    double tol;
    cplx *U;          /* cap reflectors, each of length n */
    cplx *V;          /* cap basis elements, each of length n, paper-normalised */
    cplx *B;          /* Algorithm 3 only: cap raw elements (generators and brackets), else NULL */
    cplx *x;          /* candidate scratch, length n */
    cplx *y;          /* transformed candidate, length n */
    cplx *t1, *t2;    /* d x d product scratch */
    /* bracket-loop cursor: next pair is (row l, column m) */
    int64_t l, m;
    int done;
    int64_t n_candidates;   /* bracket candidates evaluated */
    int64_t n_zero;         /* exactly-zero brackets */
    int64_t n_gen_checks;   /* generator candidates evaluated */
    double min_acc, max_rej;  /* residual gap of bracket decisions */
    /* optional per-candidate log */
    int log_on;
    int64_t log_len, log_cap;
    int32_t *log_l, *log_m;
    double *log_r;
    int8_t *log_acc;
} lo_state;

/* ---------------------------------------------------------------- helpers */

static double vec_norm2(const cplx *v, int64_t len)
{
    double s = 0.0;
    for (int64_t k = 0; k < len; ++k) {
        double re = creal(v[k]), im = cimag(v[k]);
        s += re * re + im * im;
    }
    return sqrt(s);
}

/* v <- H_j v for reflector j (acts on entries j..n-1). */
static void apply_reflector(const lo_state *s, int64_t j, cplx *v)
{
    const cplx *u = s->U + j * s->n;
    cplx dot = 0.0;
    for (int64_t k = j; k < s->n; ++k)
        dot += conj(u[k]) * v[k];
    dot *= 2.0;
    for (int64_t k = j; k < s->n; ++k)
        v[k] -= u[k] * dot;
}

/* c = a b for d x d row-major complex matrices (plain triple loop). */
static void matmul(int d, const cplx *a, const cplx *b, cplx *c)
{
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            cplx acc = 0.0;
            for (int k = 0; k < d; ++k)
                acc += a[(int64_t)i * d + k] * b[(int64_t)k * d + j];
            c[(int64_t)i * d + j] = acc;
        }
}

static void log_push(lo_state *s, int64_t l, int64_t m, double r, int acc)
{
    if (!s->log_on)
        return;
    if (s->log_len == s->log_cap) {
        int64_t nc = s->log_cap ? 2 * s->log_cap : 1024;
        int32_t *nl = realloc(s->log_l, nc * sizeof(int32_t));
        if (nl) s->log_l = nl;
        int32_t *nm = realloc(s->log_m, nc * sizeof(int32_t));
        if (nm) s->log_m = nm;
        double *nr = realloc(s->log_r, nc * sizeof(double));
        if (nr) s->log_r = nr;
        int8_t *na = realloc(s->log_acc, nc * sizeof(int8_t));
        if (na) s->log_acc = na;
        if (!nl || !nm || !nr || !na) {
            s->log_on = 0;  /* out of memory: stop logging, keep computing */
            return;
        }
        s->log_cap = nc;
    }
    s->log_l[s->log_len] = (int32_t)l;
    s->log_m[s->log_len] = (int32_t)m;
    s->log_r[s->log_len] = r;
    s->log_acc[s->log_len] = (int8_t)acc;
    s->log_len++;
}

/*
 * Independence test of the candidate in s->x against the accepted set.
 * Returns the least-squares residual in the paper's norm, and leaves
 * y = Q^H x in s->y.
 */
static double ls_residual(lo_state *s)
{
    memcpy(s->y, s->x, (size_t)s->n * sizeof(cplx));
    for (int64_t j = 0; j < s->N; ++j)
        apply_reflector(s, j, s->y);
    return vec_norm2(s->y + s->N, s->n - s->N) / sqrt((double)s->d);
}

/*
 * Append the orthogonal component of the candidate whose y = Q^H x is in s->y.
 * h_perp = Q [0; y[N:]] is the least-squares residual vector; the new basis
 * element is h_perp / ||h_perp||.  Then reflector N is formed from y[N:] so
 * that Q keeps spanning the accepted candidates.  Returns 0, or -1 when full.
 */
static int append_residual(lo_state *s)
{
    const int64_t N = s->N, n = s->n;
    if (N >= s->cap || N >= n)
        return -1;
    if (s->B)  /* Algorithm 3: keep the raw candidate itself */
        memcpy(s->B + N * n, s->x, (size_t)n * sizeof(cplx));
    const double ynorm = vec_norm2(s->y + N, n - N);
    /* h_perp in the candidate's coordinates */
    cplx *h = s->V + N * n;
    for (int64_t k = 0; k < N; ++k)
        h[k] = 0.0;
    for (int64_t k = N; k < n; ++k)
        h[k] = s->y[k];
    for (int64_t j = N - 1; j >= 0; --j)
        apply_reflector(s, j, h);
    /* paper norm ||h||^2 = ||vec h||_2^2 / d, so unit paper norm means ||vec h||_2 = sqrt(d) */
    const double scale = sqrt((double)s->d) / ynorm;
    for (int64_t k = 0; k < n; ++k)
        h[k] *= scale;
    /* reflector N maps y[N:] onto a multiple of e_N */
    cplx *u = s->U + N * n;
    for (int64_t k = 0; k < N; ++k)
        u[k] = 0.0;
    const cplx y0 = s->y[N];
    const double ay0 = cabs(y0);
    const cplx phase = ay0 > 0.0 ? y0 / ay0 : 1.0;
    const cplx alpha = -phase * ynorm;
    for (int64_t k = N; k < n; ++k)
        u[k] = s->y[k];
    u[N] -= alpha;
    const double un = vec_norm2(u + N, n - N);
    for (int64_t k = N; k < n; ++k)
        u[k] /= un;
    s->N = N + 1;
    return 0;
}

/* ---------------------------------------------------------------- public API */

lo_state *lo_new(int d, int64_t cap, double tol, int log_on)
{
    if (d < 1 || cap < 1 || !(tol > 0.0))
        return NULL;
    lo_state *s = calloc(1, sizeof(lo_state));
    if (!s)
        return NULL;
    s->d = d;
    s->n = (int64_t)d * d;
    if (cap > s->n)
        cap = s->n;
    s->cap = cap;
    s->tol = tol;
    s->U = malloc((size_t)(cap * s->n) * sizeof(cplx));
    s->V = malloc((size_t)(cap * s->n) * sizeof(cplx));
    s->x = malloc((size_t)s->n * sizeof(cplx));
    s->y = malloc((size_t)s->n * sizeof(cplx));
    s->t1 = malloc((size_t)s->n * sizeof(cplx));
    s->t2 = malloc((size_t)s->n * sizeof(cplx));
    if (!s->U || !s->V || !s->x || !s->y || !s->t1 || !s->t2) {
        free(s->U); free(s->V); free(s->x); free(s->y); free(s->t1); free(s->t2);
        free(s);
        return NULL;
    }
    s->l = 1;
    s->m = 0;
    s->min_acc = INFINITY;
    s->max_rej = 0.0;
    s->log_on = log_on;
    return s;
}

void lo_free(lo_state *s)
{
    if (!s)
        return;
    free(s->U); free(s->V); free(s->B); free(s->x); free(s->y); free(s->t1); free(s->t2);
    free(s->log_l); free(s->log_m); free(s->log_r); free(s->log_acc);
    free(s);
}

/*
 * Switch to Algorithm 3: keep the raw elements B and bracket them instead of V.
 * Must be called before the first generator.  Returns 0, or -1 (too late, or
 * out of memory).
 */
int lo_enable_raw(lo_state *s)
{
    if (s->N != 0 || s->n_gen_checks != 0 || s->B)
        return -1;
    s->B = malloc((size_t)(s->cap * s->n) * sizeof(cplx));
    return s->B ? 0 : -1;
}

/*
 * Generator phase of Algorithm 4 for one generator g (interleaved re,im;
 * d x d row-major).  Returns 1 if appended, 0 if dependent (or zero),
 * -1 if the basis is full.  *r_out receives the residual in the paper's norm.
 */
int lo_generator(lo_state *s, const double *g, double *r_out)
{
    for (int64_t k = 0; k < s->n; ++k)
        s->x[k] = g[2 * k] + I * g[2 * k + 1];
    const double gnorm = vec_norm2(s->x, s->n) / sqrt((double)s->d);
    s->n_gen_checks++;
    if (gnorm == 0.0) {
        if (r_out) *r_out = 0.0;
        return 0;
    }
    const double r = ls_residual(s);
    if (r_out) *r_out = r;
    if (!(r > s->tol * gnorm))
        return 0;
    return append_residual(s) == 0 ? 1 : -1;
}

/*
 * Bracket loop of Algorithm 4.  Processes at most `budget` candidates
 * (budget < 0: unlimited) from the saved cursor.  With early_exit set, stops
 * as soon as |V| reaches `ambient`.  Returns the number of candidates
 * processed in this call, or -1 if an append found the basis full.
 */
int64_t lo_brackets(lo_state *s, int early_exit, int64_t ambient, int64_t budget)
{
    const int d = s->d;
    int64_t done_here = 0;
    while (!s->done) {
        if (early_exit && s->N >= ambient) {
            s->done = 1;
            break;
        }
        if (s->l >= s->N) {
            s->done = 1;
            break;
        }
        if (budget >= 0 && done_here >= budget)
            break;
        const int64_t l = s->l, m = s->m;
        const cplx *src = s->B ? s->B : s->V;  /* Algorithm 3 brackets raw elements */
        const cplx *a = src + l * s->n;
        const cplx *b = src + m * s->n;
        matmul(d, a, b, s->t1);
        matmul(d, b, a, s->t2);
        int zero = 1;
        for (int64_t k = 0; k < s->n; ++k) {
            s->x[k] = s->t1[k] - s->t2[k];
            if (s->x[k] != 0.0)
                zero = 0;
        }
        double r = 0.0;
        int acc = 0;
        if (zero) {
            s->n_zero++;
        } else {
            r = ls_residual(s);
            const double thr = s->B ? s->tol * vec_norm2(s->x, s->n) / sqrt((double)d) : s->tol;
            if (r > thr) {
                if (append_residual(s) != 0)
                    return -1;
                acc = 1;
            }
        }
        if (acc) {
            if (r < s->min_acc) s->min_acc = r;
        } else {
            if (r > s->max_rej) s->max_rej = r;
        }
        log_push(s, l, m, r, acc);
        s->n_candidates++;
        done_here++;
        /* advance the cursor: m = 0..l-1 within row l, then the next row */
        if (++s->m == s->l) {
            s->l++;
            s->m = 0;
        }
    }
    return done_here;
}

int lo_done(const lo_state *s) { return s->done; }
int64_t lo_dim(const lo_state *s) { return s->N; }
int64_t lo_candidates(const lo_state *s) { return s->n_candidates; }
int64_t lo_zero_brackets(const lo_state *s) { return s->n_zero; }
int64_t lo_generator_checks(const lo_state *s) { return s->n_gen_checks; }
double lo_min_accepted(const lo_state *s) { return s->min_acc; }
double lo_max_rejected(const lo_state *s) { return s->max_rej; }
int64_t lo_cursor_row(const lo_state *s) { return s->l; }
int64_t lo_cursor_col(const lo_state *s) { return s->m; }

/* Copy V (N x d x d complex, interleaved) into out. */
/* Raw basis B of Algorithm 3 (interleaved re,im; N x d x d); no-op without it. */
void lo_raw_basis(const lo_state *s, double *out)
{
    if (!s->B)
        return;
    for (int64_t k = 0; k < s->N * s->n; ++k) {
        out[2 * k] = creal(s->B[k]);
        out[2 * k + 1] = cimag(s->B[k]);
    }
}

void lo_basis(const lo_state *s, double *out)
{
    for (int64_t k = 0; k < s->N * s->n; ++k) {
        out[2 * k] = creal(s->V[k]);
        out[2 * k + 1] = cimag(s->V[k]);
    }
}

int64_t lo_log_len(const lo_state *s) { return s->log_on ? s->log_len : 0; }

void lo_log_copy(const lo_state *s, int32_t *l, int32_t *m, double *r, int8_t *acc)
{
    if (!s->log_on)
        return;
    memcpy(l, s->log_l, (size_t)s->log_len * sizeof(int32_t));
    memcpy(m, s->log_m, (size_t)s->log_len * sizeof(int32_t));
    memcpy(r, s->log_r, (size_t)s->log_len * sizeof(double));
    memcpy(acc, s->log_acc, (size_t)s->log_len * sizeof(int8_t));
}

/*
 * Least-squares residual of an arbitrary operator x against the current
 * accepted set, in the paper's norm (read-only: the basis is unchanged).
 */
double lo_residual_of(lo_state *s, const double *x)
{
    for (int64_t k = 0; k < s->n; ++k)
        s->x[k] = x[2 * k] + I * x[2 * k + 1];
    return ls_residual(s);
}

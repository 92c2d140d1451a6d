/*
 * qtoracle.c -- plain FP64 CPU oracle for the Lindblad / quantum-jump hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP path.
 *
 * What it computes (arXiv:2504.21440, "QuantumToolbox.jl"):
 *   - the Lindblad master equation, Sec. 3.2, eq. (eq-lindblad-master-equation)
 *       d rho/dt = -i[H, rho] + sum_k D[C_k] rho,
 *       D[C] rho = C rho C^dag - 1/2 (C^dag C rho + rho C^dag C)
 *     (the paper prints the dissipator with a minus inside the bracket; the
 *      anticommutator is the only trace-preserving reading and is the one used
 *      here -- the trace-invariant tests pin it);
 *   - the time-dependent master equation and trajectories (H(t) = H_0 + sum_i
 *     f_i(t) H_i, collapse operators g_k(t) C_k; Sec. 2 QobjEvo, Sec. 3.4);
 *   - the Monte-Carlo wave-function method, Sec. 3.3: evolution under
 *       H_eff = H - (i/2) sum_k C_k^dag C_k,
 *     a jump when the (squared) norm of the unnormalised state falls to a
 *     threshold drawn from U(0,1), the channel drawn with probability
 *     P_k = <C_k^dag C_k> / sum_j <C_j^dag C_j>;
 *   - expectation values <O> = Tr(O rho) (mesolve) and <psi|O|psi>/<psi|psi>
 *     (mcsolve) at every point of tlist (Sec. 3.1, e_ops).
 *
 * The paper never names its integrator (it delegates to DifferentialEquations.jl).
 * This oracle uses the Dormand-Prince 5(4) pair (Dormand & Prince 1980;
 * Hairer, Norsett & Wanner, "Solving ODEs I", Sec. II.5), the HNW weighted RMS
 * error norm (Sec. II.4), the HNW PI step-size controller of DOPRI5
 * (beta = 0.04, safety 0.9, factor bounds [0.2, 10]; "Solving ODEs II", IV.2),
 * the HNW starting-step heuristic (Sec. II.4), and exact landing on every
 * tlist point.  Random numbers come from Philox-4x32-10 (Salmon, Moraes, Dror,
 * Shaw, SC'11), written from that paper's definition.
 *
 * Test infrastructure only: the tests, the smoke check and the benchmark's CPU
 * baseline call it; the GPU library never does.
 *
 * Parity unpinned: the starting-step heuristic.  A mistake in it changes only
 * the first few step sizes, which the tolerance tests absorb; no closed form or
 * invariant fixes its value, so nothing independent of its formula checks it.
 *
 * Every routine here is a direct transcription of a definition: sparse
 * operator times dense matrix as plain loops, no blocking, no fusion, no
 * reordering beyond what OpenMP row-parallelism implies (each output row is
 * still summed in the natural order).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------- */
/* Sparse operator (square, CSR, values interleaved re/im).                   */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t d;
    int64_t nnz;
    const int64_t *indptr;  /* d + 1 */
    const int32_t *indices; /* nnz   */
    const double *values;   /* 2*nnz */
} or_csr;

/* An owned CSR with complex values, used for adjoints built inside the oracle. */
typedef struct {
    int32_t d;
    int64_t nnz;
    int64_t *indptr;
    int32_t *indices;
    cplx *values;
} own_csr;

static inline cplx csr_at(const or_csr *A, int64_t p)
{
    return A->values[2 * p] + I * A->values[2 * p + 1];
}

/* Copy of A as an owned CSR. */
static own_csr own_copy(const or_csr *A)
{
    own_csr B;
    B.d = A->d;
    B.nnz = A->nnz;
    B.indptr = malloc(sizeof(int64_t) * (A->d + 1));
    B.indices = malloc(sizeof(int32_t) * (A->nnz ? A->nnz : 1));
    B.values = malloc(sizeof(cplx) * (A->nnz ? A->nnz : 1));
    memcpy(B.indptr, A->indptr, sizeof(int64_t) * (A->d + 1));
    for (int64_t p = 0; p < A->nnz; ++p) {
        B.indices[p] = A->indices[p];
        B.values[p] = csr_at(A, p);
    }
    return B;
}

/* Conjugate transpose: (A^dag)_{ji} = conj(A_{ij}). */
static own_csr own_adjoint(const or_csr *A)
{
    int32_t d = A->d;
    own_csr B;
    B.d = d;
    B.nnz = A->nnz;
    B.indptr = calloc(d + 1, sizeof(int64_t));
    B.indices = malloc(sizeof(int32_t) * (A->nnz ? A->nnz : 1));
    B.values = malloc(sizeof(cplx) * (A->nnz ? A->nnz : 1));
    for (int64_t p = 0; p < A->nnz; ++p)
        B.indptr[A->indices[p] + 1]++;
    for (int32_t i = 0; i < d; ++i)
        B.indptr[i + 1] += B.indptr[i];
    int64_t *fill = malloc(sizeof(int64_t) * (d + 1));
    memcpy(fill, B.indptr, sizeof(int64_t) * (d + 1));
    for (int32_t i = 0; i < d; ++i)
        for (int64_t p = A->indptr[i]; p < A->indptr[i + 1]; ++p) {
            int32_t j = A->indices[p];
            int64_t q = fill[j]++;
            B.indices[q] = i;
            B.values[q] = conj(csr_at(A, p));
        }
    free(fill);
    return B;
}

static void own_free(own_csr *A)
{
    free(A->indptr);
    free(A->indices);
    free(A->values);
}

/* ------------------------------------------------------------------------- */
/* Dense row-major d x d matrices X[i*d + j] = X_ij; products with CSR ops.   */
/* Every routine writes whole output rows, so rows can run in parallel.       */
/* ------------------------------------------------------------------------- */

/* out += alpha * A X */
static void acc_AX(const own_csr *A, const cplx *X, cplx alpha, cplx *out)
{
    int32_t d = A->d;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < d; ++i)
        for (int64_t p = A->indptr[i]; p < A->indptr[i + 1]; ++p) {
            int32_t k = A->indices[p];
            cplx a = alpha * A->values[p];
            for (int32_t j = 0; j < d; ++j)
                out[(int64_t)i * d + j] += a * X[(int64_t)k * d + j];
        }
}

/* out += alpha * X A,  (X A)_ij = sum_l X_il A_lj */
static void acc_XA(const cplx *X, const own_csr *A, cplx alpha, cplx *out)
{
    int32_t d = A->d;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < d; ++i)
        for (int32_t l = 0; l < d; ++l) {
            cplx x = alpha * X[(int64_t)i * d + l];
            for (int64_t p = A->indptr[l]; p < A->indptr[l + 1]; ++p)
                out[(int64_t)i * d + A->indices[p]] += x * A->values[p];
        }
}

/* ------------------------------------------------------------------------- */
/* Dormand-Prince 5(4) tableau.                                               */
/* ------------------------------------------------------------------------- */
static const double DP_C[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};
static const double DP_A[7][7] = {
    {0, 0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0, 0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0, 0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0, 0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0, 0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0, 0}};
/* fifth-order weights (equal to the last row of A: first same as last) */
static const double DP_B[7] = {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0,
                               -2187.0 / 6784.0, 11.0 / 84.0, 0.0};
/* embedded fourth-order weights */
static const double DP_BH[7] = {5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0,
                                -92097.0 / 339200.0, 187.0 / 2100.0, 1.0 / 40.0};

void or_dp5_tableau(double *c, double *a, double *b, double *bhat)
{
    for (int i = 0; i < 7; ++i) {
        c[i] = DP_C[i];
        b[i] = DP_B[i];
        bhat[i] = DP_BH[i];
        for (int j = 0; j < 7; ++j)
            a[i * 7 + j] = DP_A[i][j];
    }
}

/* ------------------------------------------------------------------------- */
/* Generic adaptive DP5 stepper over complex vectors.                         */
/* ------------------------------------------------------------------------- */
typedef void (*or_rhs)(void *ctx, double t, const cplx *y, cplx *dy);

typedef struct {
    double abstol, reltol;
    int64_t max_steps;
    double h0; /* 0 = automatic */
} or_opts;

typedef struct {
    int64_t n_accept, n_reject, n_rhs, n_jumps;
    int32_t status;
} or_stats;

enum { OR_OK = 0, OR_EINVAL = 1, OR_EMAXSTEPS = 4, OR_EDTMIN = 5, OR_ENONFINITE = 6 };

typedef struct {
    int64_t n;
    or_rhs f;
    void *ctx;
    double atol, rtol;
    cplx *y, *ynew, *k[7], *ytmp;
    double t;
    int64_t *n_rhs;
} dp5;

static void dp5_init(dp5 *s, int64_t n, or_rhs f, void *ctx, double atol, double rtol, int64_t *n_rhs)
{
    s->n = n;
    s->f = f;
    s->ctx = ctx;
    s->atol = atol;
    s->rtol = rtol;
    s->y = calloc(n, sizeof(cplx));
    s->ynew = calloc(n, sizeof(cplx));
    s->ytmp = calloc(n, sizeof(cplx));
    for (int i = 0; i < 7; ++i)
        s->k[i] = calloc(n, sizeof(cplx));
    s->n_rhs = n_rhs;
}

static void dp5_free(dp5 *s)
{
    free(s->y);
    free(s->ynew);
    free(s->ytmp);
    for (int i = 0; i < 7; ++i)
        free(s->k[i]);
}

static void dp5_eval(dp5 *s, double t, const cplx *y, cplx *dy)
{
    s->f(s->ctx, t, y, dy);
    (*s->n_rhs)++;
}

/* Weighted RMS norm (HNW II.4): sqrt( (1/n) sum_i |e_i|^2 / sc_i^2 ),
 * sc_i = atol + rtol * max(|y_i|, |z_i|); each complex entry is one component. */
static double wrms(const dp5 *s, const cplx *e, const cplx *y, const cplx *z)
{
    double acc = 0.0;
    for (int64_t i = 0; i < s->n; ++i) {
        double m = cabs(y[i]);
        if (z) {
            double mz = cabs(z[i]);
            if (mz > m)
                m = mz;
        }
        double sc = s->atol + s->rtol * m;
        double r = cabs(e[i]) / sc;
        acc += r * r;
    }
    return sqrt(acc / (double)s->n);
}

/* One trial step of size h from (t, y) with k[0] = f(t, y) already present.
 * Leaves the fifth-order solution in ynew, f(t+h, ynew) in k[6], and returns
 * the error norm of e = h sum_j (b_j - bhat_j) k_j. */
static double dp5_attempt(dp5 *s, double h)
{
    int64_t n = s->n;
    for (int st = 1; st < 7; ++st) {
        cplx *dst = (st == 6) ? s->ynew : s->ytmp;
        for (int64_t i = 0; i < n; ++i) {
            cplx acc = 0.0;
            for (int j = 0; j < st; ++j)
                acc += DP_A[st][j] * s->k[j][i];
            dst[i] = s->y[i] + h * acc;
        }
        dp5_eval(s, s->t + DP_C[st] * h, dst, s->k[st]);
    }
    for (int64_t i = 0; i < n; ++i) {
        cplx acc = 0.0;
        for (int j = 0; j < 7; ++j)
            acc += (DP_B[j] - DP_BH[j]) * s->k[j][i];
        s->ytmp[i] = h * acc;
    }
    return wrms(s, s->ytmp, s->y, s->ynew);
}

/* HNW starting step (order 5 pair, error estimate of order 4), with k[0] = f(t, y). */
static double dp5_initial_h(dp5 *s)
{
    int64_t n = s->n;
    double d0 = wrms(s, s->y, s->y, NULL);
    double d1 = wrms(s, s->k[0], s->y, NULL);
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    for (int64_t i = 0; i < n; ++i)
        s->ytmp[i] = s->y[i] + h0 * s->k[0][i];
    dp5_eval(s, s->t + h0, s->ytmp, s->k[1]);
    for (int64_t i = 0; i < n; ++i)
        s->k[2][i] = (s->k[1][i] - s->k[0][i]) / h0;
    double d2 = wrms(s, s->k[2], s->y, NULL);
    double m = d1 > d2 ? d1 : d2;
    double h1 = (m <= 1e-15) ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / m, 1.0 / 5.0);
    return fmin(100.0 * h0, h1);
}

/* PI controller factor for an accepted step (HNW DOPRI5: expo 0.2 - 0.75*beta,
 * beta = 0.04, safety 0.9, bounds [0.2, 10]). */
static double pi_factor(double err, double err_prev)
{
    if (err == 0.0)
        return 10.0;
    double f = 0.9 * pow(err, -0.17) * pow(err_prev, 0.04);
    if (f < 0.2)
        f = 0.2;
    if (f > 10.0)
        f = 10.0;
    return f;
}

/* Step-size factor after a rejected step. */
static double reject_factor(double err)
{
    double f = 0.9 * pow(err, -0.17);
    return f < 0.2 ? 0.2 : f;
}

/* The step about to be tried from t towards tstop: returns the step size and
 * sets *land when the step is clipped to land exactly on tstop. */
static double clip_to_tstop(double t, double h, double tstop, int *land)
{
    double rem = tstop - t;
    double snap = 1e-12 * fmax(1.0, fabs(tstop));
    if (h >= rem - snap) {
        *land = 1;
        return rem;
    }
    *land = 0;
    return h;
}

static int check_tlist(int32_t nt, const double *tlist)
{
    if (nt < 1)
        return OR_EINVAL;
    for (int32_t i = 1; i < nt; ++i)
        if (!(tlist[i] > tlist[i - 1]))
            return OR_EINVAL;
    return OR_OK;
}

static void swap_ptr(cplx **a, cplx **b)
{
    cplx *t = *a;
    *a = *b;
    *b = t;
}

/* Drive the stepper from tlist[0] to tlist[nt-1], calling save(idx) with the
 * state in s->y at each tlist point.  Plain adaptive integration (no jumps). */
typedef void (*or_save)(void *sctx, int32_t idx, const cplx *y);

static int32_t dp5_integrate(dp5 *s, int32_t nt, const double *tlist, const or_opts *o, or_save save,
                             void *sctx, or_stats *st)
{
    s->t = tlist[0];
    save(sctx, 0, s->y);
    if (nt == 1)
        return OR_OK;
    dp5_eval(s, s->t, s->y, s->k[0]);
    double h = o->h0 > 0 ? o->h0 : dp5_initial_h(s);
    double err_prev = 1e-4;
    int last_rejected = 0;
    int32_t idx = 1;
    int64_t steps = 0;
    while (idx < nt) {
        if (steps >= o->max_steps)
            return OR_EMAXSTEPS;
        ++steps;
        int land;
        double ht = clip_to_tstop(s->t, h, tlist[idx], &land);
        double err = dp5_attempt(s, ht);
        if (!isfinite(err))
            return OR_ENONFINITE;
        if (err <= 1.0) {
            st->n_accept++;
            s->t = land ? tlist[idx] : s->t + ht;
            swap_ptr(&s->y, &s->ynew);
            swap_ptr(&s->k[0], &s->k[6]);
            double hn = ht * pi_factor(err, err_prev);
            if (last_rejected && hn > ht)
                hn = ht;
            err_prev = fmax(err, 1e-4);
            last_rejected = 0;
            h = hn;
            if (land)
                save(sctx, idx++, s->y);
        } else {
            st->n_reject++;
            h = ht * reject_factor(err);
            last_rejected = 1;
        }
        if (idx < nt && h < 1e-14 * fmax(1.0, fabs(s->t)))
            return OR_EDTMIN;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Linear test problem y' = M y (dense M), for order / convergence pins.      */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t n;
    const cplx *M;
} lin_ctx;

static void lin_rhs(void *ctx, double t, const cplx *y, cplx *dy)
{
    (void)t;
    const lin_ctx *c = ctx;
    for (int64_t i = 0; i < c->n; ++i) {
        cplx acc = 0.0;
        for (int64_t j = 0; j < c->n; ++j)
            acc += c->M[i * c->n + j] * y[j];
        dy[i] = acc;
    }
}

typedef struct {
    int64_t n;
    cplx *out; /* nt x n */
} store_ctx;

static void store_state(void *sctx, int32_t idx, const cplx *y)
{
    store_ctx *c = sctx;
    memcpy(c->out + (int64_t)idx * c->n, y, sizeof(cplx) * c->n);
}

/* Adaptive integration of y' = M y; states at every tlist point into out. */
int32_t or_linear_solve(int64_t n, const double *M, const double *y0, int32_t nt, const double *tlist,
                        const or_opts *o, double *out, or_stats *st)
{
    memset(st, 0, sizeof(*st));
    if (check_tlist(nt, tlist))
        return st->status = OR_EINVAL;
    lin_ctx c = {n, (const cplx *)M};
    dp5 s;
    dp5_init(&s, n, lin_rhs, &c, o->abstol, o->reltol, &st->n_rhs);
    memcpy(s.y, y0, sizeof(cplx) * n);
    store_ctx sc = {n, (cplx *)out};
    int32_t rc = dp5_integrate(&s, nt, tlist, o, store_state, &sc, st);
    dp5_free(&s);
    return st->status = rc;
}

/* Fixed-step DP5 (no control): nsteps steps of size h; returns the fifth-order
 * result in y_out and the last embedded error vector in e_out (both length n). */
void or_linear_fixed(int64_t n, const double *M, const double *y0, double h, int64_t nsteps, double *y_out,
                     double *e_out)
{
    lin_ctx c = {n, (const cplx *)M};
    int64_t cnt = 0;
    dp5 s;
    dp5_init(&s, n, lin_rhs, &c, 1.0, 0.0, &cnt);
    memcpy(s.y, y0, sizeof(cplx) * n);
    s.t = 0.0;
    for (int64_t k = 0; k < nsteps; ++k) {
        dp5_eval(&s, s.t, s.y, s.k[0]);
        dp5_attempt(&s, h);
        s.t += h;
        swap_ptr(&s.y, &s.ynew);
    }
    memcpy(y_out, s.y, sizeof(cplx) * n);
    memcpy(e_out, s.ytmp, sizeof(cplx) * n);
    dp5_free(&s);
}

/* ------------------------------------------------------------------------- */
/* Lindblad right-hand side, written as the definition.                       */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t d;
    own_csr H;
    int32_t nc;
    own_csr *C, *Cd; /* C_k and C_k^dag */
    cplx *X, *Y;     /* d x d scratch */
} me_ctx;

static void me_ctx_init(me_ctx *m, const or_csr *H, int32_t nc, const or_csr *c_ops)
{
    m->d = H->d;
    m->H = own_copy(H);
    m->nc = nc;
    m->C = malloc(sizeof(own_csr) * (nc ? nc : 1));
    m->Cd = malloc(sizeof(own_csr) * (nc ? nc : 1));
    for (int32_t k = 0; k < nc; ++k) {
        m->C[k] = own_copy(&c_ops[k]);
        m->Cd[k] = own_adjoint(&c_ops[k]);
    }
    m->X = malloc(sizeof(cplx) * (size_t)m->d * m->d);
    m->Y = malloc(sizeof(cplx) * (size_t)m->d * m->d);
}

static void me_ctx_free(me_ctx *m)
{
    own_free(&m->H);
    for (int32_t k = 0; k < m->nc; ++k) {
        own_free(&m->C[k]);
        own_free(&m->Cd[k]);
    }
    free(m->C);
    free(m->Cd);
    free(m->X);
    free(m->Y);
}

/* drho = -i (H rho - rho H) + sum_k [ C rho C^dag - 1/2 C^dag C rho - 1/2 rho C^dag C ] */
static void me_rhs(void *ctx, double t, const cplx *rho, cplx *drho)
{
    (void)t;
    me_ctx *m = ctx;
    size_t nn = (size_t)m->d * m->d;
    memset(drho, 0, sizeof(cplx) * nn);
    acc_AX(&m->H, rho, -I, drho);
    acc_XA(rho, &m->H, I, drho);
    for (int32_t k = 0; k < m->nc; ++k) {
        /* X = C rho */
        memset(m->X, 0, sizeof(cplx) * nn);
        acc_AX(&m->C[k], rho, 1.0, m->X);
        /* + X C^dag */
        acc_XA(m->X, &m->Cd[k], 1.0, drho);
        /* - 1/2 C^dag X */
        acc_AX(&m->Cd[k], m->X, -0.5, drho);
        /* Y = rho C^dag ;  - 1/2 Y C */
        memset(m->Y, 0, sizeof(cplx) * nn);
        acc_XA(rho, &m->Cd[k], 1.0, m->Y);
        acc_XA(m->Y, &m->C[k], -0.5, drho);
    }
}

/* Apply the Lindblad right-hand side once (for the Liouvillian cross-check). */
void or_lindblad_apply(const or_csr *H, int32_t nc, const or_csr *c_ops, const double *rho, double *drho)
{
    me_ctx m;
    me_ctx_init(&m, H, nc, c_ops);
    me_rhs(&m, 0.0, (const cplx *)rho, (cplx *)drho);
    me_ctx_free(&m);
}

/* Tr(O rho) = sum_{(i,j) in nnz(O)} O_ij rho_ji */
static cplx trace_O_rho(const or_csr *O, const cplx *rho, int32_t d)
{
    cplx acc = 0.0;
    for (int32_t i = 0; i < d; ++i)
        for (int64_t p = O->indptr[i]; p < O->indptr[i + 1]; ++p)
            acc += csr_at(O, p) * rho[(int64_t)O->indices[p] * d + i];
    return acc;
}

void or_expect_dm(const or_csr *O, const double *rho, double *out)
{
    cplx v = trace_O_rho(O, (const cplx *)rho, O->d);
    out[0] = creal(v);
    out[1] = cimag(v);
}

/* <psi|O|psi> / <psi|psi> */
static cplx expect_ket(const or_csr *O, const cplx *psi, int32_t d)
{
    cplx acc = 0.0;
    double nrm = 0.0;
    for (int32_t i = 0; i < d; ++i) {
        cplx row = 0.0;
        for (int64_t p = O->indptr[i]; p < O->indptr[i + 1]; ++p)
            row += csr_at(O, p) * psi[O->indices[p]];
        acc += conj(psi[i]) * row;
        nrm += creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
    }
    return acc / nrm;
}

void or_expect_ket(const or_csr *O, const double *psi, double *out)
{
    cplx v = expect_ket(O, (const cplx *)psi, O->d);
    out[0] = creal(v);
    out[1] = cimag(v);
}

typedef struct {
    int32_t d, ne, nt;
    const or_csr *e_ops;
    double *expect; /* [ne][nt] complex */
    double *rho_final;
} me_save_ctx;

static void me_save(void *sctx, int32_t idx, const cplx *rho)
{
    me_save_ctx *c = sctx;
    for (int32_t k = 0; k < c->ne; ++k) {
        cplx v = trace_O_rho(&c->e_ops[k], rho, c->d);
        c->expect[2 * ((int64_t)k * c->nt + idx)] = creal(v);
        c->expect[2 * ((int64_t)k * c->nt + idx) + 1] = cimag(v);
    }
    if (c->rho_final && idx == c->nt - 1)
        memcpy(c->rho_final, rho, sizeof(cplx) * (size_t)c->d * c->d);
}

/* mesolve: rho0 is a d x d row-major complex matrix (used as given). */
int32_t or_mesolve(const or_csr *H, int32_t nc, const or_csr *c_ops, const double *rho0, int32_t nt,
                   const double *tlist, int32_t ne, const or_csr *e_ops, const or_opts *o, double *expect,
                   double *rho_final, or_stats *st)
{
    memset(st, 0, sizeof(*st));
    if (check_tlist(nt, tlist))
        return st->status = OR_EINVAL;
    int32_t d = H->d;
    me_ctx m;
    me_ctx_init(&m, H, nc, c_ops);
    dp5 s;
    dp5_init(&s, (int64_t)d * d, me_rhs, &m, o->abstol, o->reltol, &st->n_rhs);
    memcpy(s.y, rho0, sizeof(cplx) * (size_t)d * d);
    me_save_ctx sc = {d, ne, nt, e_ops, expect, rho_final};
    int32_t rc = dp5_integrate(&s, nt, tlist, o, me_save, &sc, st);
    dp5_free(&s);
    me_ctx_free(&m);
    return st->status = rc;
}

/* ------------------------------------------------------------------------- */
/* Time-dependent master equation (Sec. 3.2 with time-dependent operators,    */
/* the QobjEvo of Sec. 2 and the driven example of Sec. 3.4):                 */
/*   H(t) = H_0 + sum_i f_i(t) H_i,   collapse operators g_k(t) C_k,          */
/*   d rho/dt = -i[H_0, rho] - i sum_i f_i(t) (H_i rho - rho H_i)             */
/*              + sum_k |g_k(t)|^2 D[C_k] rho.                                */
/* f_i may be complex and H_i need not be Hermitian (a drive a^dag f + a f*   */
/* is two terms); the collapse weight enters through D[g C] = |g|^2 D[C].     */
/* ------------------------------------------------------------------------- */
enum { ORC_NONE = -1, ORC_CONST = 0, ORC_COS = 1, ORC_EXP = 2, ORC_GAUSS = 3, ORC_TABLE = 4 };

typedef struct {
    int32_t kind;
    int32_t n_table;
    double a_re, a_im;
    double omega, phi, t0, sigma;
    double table_t0, table_dt;
    const double *table; /* 2 * n_table, interleaved */
} or_coef;

/* The coefficient's value at time t, written from each kind's definition. */
static cplx coef_at(const or_coef *c, double t)
{
    const cplx a = c->a_re + I * c->a_im;
    switch (c->kind) {
    case ORC_CONST:
        return a;
    case ORC_COS:
        return a * cos(c->omega * t + c->phi);
    case ORC_EXP:
        return a * cexp(I * (c->omega * t + c->phi));
    case ORC_GAUSS: {
        const double u = (t - c->t0) / c->sigma;
        return a * exp(-0.5 * u * u) * cos(c->omega * t + c->phi);
    }
    case ORC_TABLE: {
        /* linear interpolation between the samples at table_t0 + k table_dt, held at the ends */
        const int32_t n = c->n_table;
        const double u = (t - c->table_t0) / c->table_dt;
        cplx v;
        if (n == 1 || u <= 0.0) {
            v = c->table[0] + I * c->table[1];
        } else if (u >= (double)(n - 1)) {
            v = c->table[2 * (n - 1)] + I * c->table[2 * (n - 1) + 1];
        } else {
            const int32_t k = (int32_t)floor(u);
            const double f = u - (double)k;
            const cplx lo = c->table[2 * k] + I * c->table[2 * k + 1];
            const cplx hi = c->table[2 * k + 2] + I * c->table[2 * k + 3];
            v = (1.0 - f) * lo + f * hi;
        }
        return a * v;
    }
    default:
        return 1.0;
    }
}

void or_coef_eval(const or_coef *c, double t, double *out)
{
    const cplx v = coef_at(c, t);
    out[0] = creal(v);
    out[1] = cimag(v);
}

typedef struct {
    me_ctx base;      /* H_0 and every C_k */
    int32_t nh;
    own_csr *Hk;      /* H_i */
    const or_coef *fh;
    const or_coef *gc; /* per collapse operator; kind ORC_NONE: weight 1 */
} me_td_ctx;

static void me_td_rhs(void *ctx, double t, const cplx *rho, cplx *drho)
{
    me_td_ctx *m = ctx;
    me_ctx *b = &m->base;
    size_t nn = (size_t)b->d * b->d;
    memset(drho, 0, sizeof(cplx) * nn);
    acc_AX(&b->H, rho, -I, drho);
    acc_XA(rho, &b->H, I, drho);
    for (int32_t i = 0; i < m->nh; ++i) {
        const cplx f = coef_at(&m->fh[i], t);
        acc_AX(&m->Hk[i], rho, -I * f, drho);
        acc_XA(rho, &m->Hk[i], I * f, drho);
    }
    for (int32_t k = 0; k < b->nc; ++k) {
        double w = 1.0;
        if (m->gc && m->gc[k].kind != ORC_NONE) {
            const cplx g = coef_at(&m->gc[k], t);
            w = creal(g) * creal(g) + cimag(g) * cimag(g);
        }
        memset(b->X, 0, sizeof(cplx) * nn);
        acc_AX(&b->C[k], rho, 1.0, b->X);
        acc_XA(b->X, &b->Cd[k], w, drho);
        acc_AX(&b->Cd[k], b->X, -0.5 * w, drho);
        memset(b->Y, 0, sizeof(cplx) * nn);
        acc_XA(rho, &b->Cd[k], 1.0, b->Y);
        acc_XA(b->Y, &b->C[k], -0.5 * w, drho);
    }
}

/* Time-dependent mesolve; c_coefs may be NULL (every collapse operator constant). */
int32_t or_mesolve_td(const or_csr *H0, int32_t nh, const or_csr *h_terms, const or_coef *h_coefs, int32_t nc,
                      const or_csr *c_ops, const or_coef *c_coefs, const double *rho0, int32_t nt,
                      const double *tlist, int32_t ne, const or_csr *e_ops, const or_opts *o, double *expect,
                      double *rho_final, or_stats *st)
{
    memset(st, 0, sizeof(*st));
    if (check_tlist(nt, tlist))
        return st->status = OR_EINVAL;
    int32_t d = H0->d;
    me_td_ctx m;
    me_ctx_init(&m.base, H0, nc, c_ops);
    m.nh = nh;
    m.Hk = malloc(sizeof(own_csr) * (nh ? nh : 1));
    for (int32_t i = 0; i < nh; ++i)
        m.Hk[i] = own_copy(&h_terms[i]);
    m.fh = h_coefs;
    m.gc = c_coefs;
    dp5 s;
    dp5_init(&s, (int64_t)d * d, me_td_rhs, &m, o->abstol, o->reltol, &st->n_rhs);
    memcpy(s.y, rho0, sizeof(cplx) * (size_t)d * d);
    me_save_ctx sc = {d, ne, nt, e_ops, expect, rho_final};
    int32_t rc = dp5_integrate(&s, nt, tlist, o, me_save, &sc, st);
    dp5_free(&s);
    for (int32_t i = 0; i < nh; ++i)
        own_free(&m.Hk[i]);
    free(m.Hk);
    me_ctx_free(&m.base);
    return st->status = rc;
}

/* ------------------------------------------------------------------------- */
/* Philox-4x32-10 (Salmon et al., SC'11), from its published definition.     */
/* ------------------------------------------------------------------------- */
void or_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* A double in (0,1) from two 32-bit words: 27 + 26 bits, half-ulp offset. */
double or_uniform_from_words(uint32_t w0, uint32_t w1)
{
    double hi = (double)(w0 >> 5);
    double lo = (double)(w1 >> 6);
    return (hi * 67108864.0 + lo + 0.5) * (1.0 / 9007199254740992.0);
}

/* Draws of trajectory j: event 0 -> (r0, unused); event m >= 1 -> (u_m, r_m),
 * u_m choosing the channel of jump m and r_m the threshold after it. */
void or_traj_draw(uint64_t seed, uint64_t traj, uint32_t event, double *first, double *second)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)traj, (uint32_t)(traj >> 32), event, 0u};
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    *first = or_uniform_from_words(w[0], w[1]);
    *second = or_uniform_from_words(w[2], w[3]);
}

/* ------------------------------------------------------------------------- */
/* Monte-Carlo wave function.                                                 */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t d;
    const or_csr *H;
    int32_t nc;
    const or_csr *C;
    own_csr *Cd;
    cplx *tmp; /* per-trajectory scratch, length d */
    /* time-dependent terms: H(t) = H + sum_i f_i(t) H_i, collapse operators g_k(t) C_k */
    int32_t nh;
    const or_csr *Hk;
    const or_coef *fh;
    const or_coef *gc; /* NULL, or per operator (kind ORC_NONE: weight 1) */
} mc_ctx;

/* |g_k(t)|^2, the weight of collapse operator k at time t (1 without a coefficient) */
static double mc_weight(const mc_ctx *m, int32_t k, double t)
{
    if (!m->gc || m->gc[k].kind == ORC_NONE)
        return 1.0;
    const cplx g = coef_at(&m->gc[k], t);
    return creal(g) * creal(g) + cimag(g) * cimag(g);
}

static void csr_mv(const or_csr *A, const cplx *x, cplx *y)
{
    for (int32_t i = 0; i < A->d; ++i) {
        cplx acc = 0.0;
        for (int64_t p = A->indptr[i]; p < A->indptr[i + 1]; ++p)
            acc += csr_at(A, p) * x[A->indices[p]];
        y[i] = acc;
    }
}

static void own_mv_acc(const own_csr *A, const cplx *x, cplx alpha, cplx *y)
{
    for (int32_t i = 0; i < A->d; ++i) {
        cplx acc = 0.0;
        for (int64_t p = A->indptr[i]; p < A->indptr[i + 1]; ++p)
            acc += A->values[p] * x[A->indices[p]];
        y[i] += alpha * acc;
    }
}

/* dpsi = -i H_eff(t) psi = -i H(t) psi - 1/2 sum_k |g_k(t)|^2 C_k^dag (C_k psi) */
static void mc_rhs(void *ctx, double t, const cplx *psi, cplx *dpsi)
{
    mc_ctx *m = ctx;
    csr_mv(m->H, psi, dpsi);
    for (int32_t i = 0; i < m->d; ++i)
        dpsi[i] *= -I;
    for (int32_t q = 0; q < m->nh; ++q) {
        const cplx f = coef_at(&m->fh[q], t);
        csr_mv(&m->Hk[q], psi, m->tmp);
        for (int32_t i = 0; i < m->d; ++i)
            dpsi[i] += -I * f * m->tmp[i];
    }
    for (int32_t k = 0; k < m->nc; ++k) {
        csr_mv(&m->C[k], psi, m->tmp);
        own_mv_acc(&m->Cd[k], m->tmp, -0.5 * mc_weight(m, k, t), dpsi);
    }
}

static double norm2(const cplx *x, int64_t n)
{
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i)
        acc += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
    return acc;
}

/* One trajectory.  expect_tr: [ne][nt] complex; jt/jc: up to maxj jump times and channels. */
static int32_t mc_trajectory(mc_ctx *m, const cplx *psi0, int32_t nt, const double *tlist, int32_t ne,
                             const or_csr *e_ops, const or_opts *o, uint64_t seed, uint64_t traj,
                             double *expect_tr, int32_t maxj, double *jt, int32_t *jc, or_stats *st)
{
    int32_t d = m->d;
    dp5 s;
    dp5_init(&s, d, mc_rhs, m, o->abstol, o->reltol, &st->n_rhs);
    double n0 = sqrt(norm2(psi0, d));
    for (int32_t i = 0; i < d; ++i)
        s.y[i] = psi0[i] / n0;
    double r, unused;
    or_traj_draw(seed, traj, 0u, &r, &unused);
    uint32_t event = 1;
    s.t = tlist[0];
    for (int32_t k = 0; k < ne; ++k) {
        cplx v = expect_ket(&e_ops[k], s.y, d);
        expect_tr[2 * ((int64_t)k * nt)] = creal(v);
        expect_tr[2 * ((int64_t)k * nt) + 1] = cimag(v);
    }
    int32_t rc = OR_OK;
    int32_t idx = 1;
    int64_t steps = 0;
    if (nt > 1) {
        dp5_eval(&s, s.t, s.y, s.k[0]);
        double h = o->h0 > 0 ? o->h0 : dp5_initial_h(&s);
        double err_prev = 1e-4;
        int last_rejected = 0;
        cplx *cpsi = calloc(d, sizeof(cplx));
        cplx *ybest = calloc(d, sizeof(cplx));
        while (idx < nt) {
            if (steps >= o->max_steps) {
                rc = OR_EMAXSTEPS;
                break;
            }
            ++steps;
            int land;
            double ht = clip_to_tstop(s.t, h, tlist[idx], &land);
            double err = dp5_attempt(&s, ht);
            if (!isfinite(err)) {
                rc = OR_ENONFINITE;
                break;
            }
            if (err > 1.0) {
                st->n_reject++;
                h = ht * reject_factor(err);
                last_rejected = 1;
                if (h < 1e-14 * fmax(1.0, fabs(s.t))) {
                    rc = OR_EDTMIN;
                    break;
                }
                continue;
            }
            st->n_accept++;
            double hn = ht * pi_factor(err, err_prev);
            if (last_rejected && hn > ht)
                hn = ht;
            err_prev = fmax(err, 1e-4);
            last_rejected = 0;
            double nrm_new = norm2(s.ynew, d);
            if (nrm_new >= r || m->nc == 0) { /* without collapse operators there is no jump */
                /* ordinary accepted step */
                s.t = land ? tlist[idx] : s.t + ht;
                swap_ptr(&s.y, &s.ynew);
                swap_ptr(&s.k[0], &s.k[6]);
                h = hn;
                if (land) {
                    for (int32_t k = 0; k < ne; ++k) {
                        cplx v = expect_ket(&e_ops[k], s.y, d);
                        expect_tr[2 * ((int64_t)k * nt + idx)] = creal(v);
                        expect_tr[2 * ((int64_t)k * nt + idx) + 1] = cimag(v);
                    }
                    ++idx;
                }
                continue;
            }
            /* The squared norm crossed r inside [t, t+ht]: locate the crossing
             * with the Illinois variant of regula falsi on
             * g(theta) = ln |psi(t + theta ht)|^2 - ln r, theta in (0, 1],
             * each probe being a fresh DP5 step of size theta*ht from (t, y). */
            double lr = log(r);
            double a = 0.0, ga = log(norm2(s.y, d)) - lr;
            double b = 1.0, gb = log(nrm_new) - lr;
            double th = 1.0, th_prev = 1.0, gth = gb;
            memcpy(ybest, s.ynew, sizeof(cplx) * d);
            int side = 0;
            for (int it = 0; it < 64; ++it) {
                th = (a * gb - b * ga) / (gb - ga);
                if (!(th > a && th < b))
                    th = 0.5 * (a + b);
                dp5_attempt(&s, th * ht);
                gth = log(norm2(s.ynew, d)) - lr;
                memcpy(ybest, s.ynew, sizeof(cplx) * d);
                if (fabs(gth) <= 1e-12)
                    break;
                if (fabs(th - th_prev) * ht <= 1e-10 * fmax(1.0, fabs(s.t)))
                    break;
                th_prev = th;
                if (gth > 0.0) {
                    a = th;
                    ga = gth;
                    if (side == 1)
                        gb *= 0.5;
                    side = 1;
                } else {
                    b = th;
                    gb = gth;
                    if (side == -1)
                        ga *= 0.5;
                    side = -1;
                }
            }
            double tj = s.t + th * ht;
            /* channel probabilities p_k = |g_k(t*)|^2 |C_k psi|^2 */
            double u, rnext;
            or_traj_draw(seed, traj, event, &u, &rnext);
            ++event;
            double tot = 0.0;
            for (int32_t k = 0; k < m->nc; ++k) {
                csr_mv(&m->C[k], ybest, cpsi);
                tot += mc_weight(m, k, tj) * norm2(cpsi, d);
            }
            double target = u * tot, cum = 0.0;
            int32_t ch = m->nc - 1;
            for (int32_t k = 0; k < m->nc; ++k) {
                csr_mv(&m->C[k], ybest, cpsi);
                cum += mc_weight(m, k, tj) * norm2(cpsi, d);
                if (cum >= target) {
                    ch = k;
                    break;
                }
            }
            csr_mv(&m->C[ch], ybest, cpsi);
            double nc_ = sqrt(norm2(cpsi, d));
            for (int32_t i = 0; i < d; ++i)
                s.y[i] = cpsi[i] / nc_;
            if (st->n_jumps < maxj && jt) {
                jt[st->n_jumps] = tj;
                jc[st->n_jumps] = ch;
            }
            st->n_jumps++;
            r = rnext;
            int at_stop = land && th == 1.0;
            s.t = at_stop ? tlist[idx] : tj;
            dp5_eval(&s, s.t, s.y, s.k[0]);
            h = hn;
            if (at_stop) {
                for (int32_t k = 0; k < ne; ++k) {
                    cplx v = expect_ket(&e_ops[k], s.y, d);
                    expect_tr[2 * ((int64_t)k * nt + idx)] = creal(v);
                    expect_tr[2 * ((int64_t)k * nt + idx) + 1] = cimag(v);
                }
                ++idx;
            }
        }
        free(cpsi);
        free(ybest);
    }
    dp5_free(&s);
    return rc;
}

/* mcsolve over trajectories [traj0, traj0 + ntraj).
 *   expect_tr: [ntraj][ne][nt] complex per-trajectory expectations
 *   njumps:    [ntraj]
 *   jt, jc:    [ntraj][maxj] first jump times / channels (nullable when maxj == 0)
 *   status:    [ntraj] */
int32_t or_mcsolve_td(const or_csr *H, int32_t nh, const or_csr *h_terms, const or_coef *h_coefs, int32_t nc,
                      const or_csr *c_ops, const or_coef *c_coefs, const double *psi0, int32_t nt,
                      const double *tlist, int32_t ne, const or_csr *e_ops, const or_opts *o, uint64_t seed,
                      uint64_t traj0, int64_t ntraj, double *expect_tr, int64_t *njumps, int32_t maxj, double *jt,
                      int32_t *jc, int32_t *status, int64_t *n_rhs_total)
{
    if (check_tlist(nt, tlist))
        return OR_EINVAL;
    int32_t d = H->d;
    own_csr *Cd = malloc(sizeof(own_csr) * (nc ? nc : 1));
    for (int32_t k = 0; k < nc; ++k)
        Cd[k] = own_adjoint(&c_ops[k]);
    int32_t worst = OR_OK;
    int64_t tot_rhs = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : tot_rhs)
    for (int64_t j = 0; j < ntraj; ++j) {
        mc_ctx m = {d, H, nc, c_ops, Cd, calloc(d, sizeof(cplx)), nh, h_terms, h_coefs, c_coefs};
        or_stats st;
        memset(&st, 0, sizeof(st));
        int32_t rc = mc_trajectory(&m, (const cplx *)psi0, nt, tlist, ne, e_ops, o, seed, traj0 + (uint64_t)j,
                                   expect_tr + 2 * (int64_t)j * ne * nt, maxj, jt ? jt + j * maxj : NULL,
                                   jc ? jc + j * maxj : NULL, &st);
        free(m.tmp);
        njumps[j] = st.n_jumps;
        status[j] = rc;
        tot_rhs += st.n_rhs;
        if (rc != OR_OK) {
#pragma omp critical
            worst = rc;
        }
    }
    for (int32_t k = 0; k < nc; ++k)
        own_free(&Cd[k]);
    free(Cd);
    if (n_rhs_total)
        *n_rhs_total = tot_rhs;
    return worst;
}

int32_t or_mcsolve(const or_csr *H, int32_t nc, const or_csr *c_ops, const double *psi0, int32_t nt,
                   const double *tlist, int32_t ne, const or_csr *e_ops, const or_opts *o, uint64_t seed,
                   uint64_t traj0, int64_t ntraj, double *expect_tr, int64_t *njumps, int32_t maxj, double *jt,
                   int32_t *jc, int32_t *status, int64_t *n_rhs_total)
{
    return or_mcsolve_td(H, 0, NULL, NULL, nc, c_ops, NULL, psi0, nt, tlist, ne, e_ops, o, seed, traj0, ntraj,
                         expect_tr, njumps, maxj, jt, jc, status, n_rhs_total);
}

/* ------------------------------------------------------------------------- */
/* Stochastic Schrodinger and master equations under homodyne detection      */
/* (Sec. 3.5), Ito form:                                                      */
/*   SSE  d psi = -i K psi dt + sum_n M_n psi dW_n,                           */
/*        K = H + i sum_n (e_n/2 S_n - 1/2 S_n^dag S_n - e_n^2/8),            */
/*        M_n = S_n - e_n/2,  e_n = <psi|S_n + S_n^dag|psi>;                  */
/*   SME  d rho = L rho dt + sum_n H[S_n] rho dW_n,  L with c_ops and sc_ops, */
/*        H[S] rho = S rho + rho S^dag - Tr(S rho + rho S^dag) rho;           */
/*   measurement current J_n = <S_n + S_n^dag> + dW_n/dt.                     */
/* Both share one form: x' = A(x) dt + sum_n (B_n x - c mu_n(x) x) dW_n, with */
/* mu_n(x) = <S_n + S_n^dag> in the state x (c = 1/2 for the SSE, 1 for the   */
/* SME); for the SSE the drift also carries sum_n (mu_n/2 S_n x - mu_n^2/8 x).*/
/* The paper does not name its SDE scheme.  Here: fixed steps (each tlist     */
/* interval cut into ceil(length / dt) equal steps), the derivative-free      */
/* order-1.0 strong scheme of Platen (Kloeden & Platen, "Numerical Solution   */
/* of Stochastic Differential Equations", Sec. 11.1) applied to each Wiener   */
/* process with its own supporting value (the cross terms of several          */
/* processes are left out), and the state renormalised after every step      */
/* (unit norm, unit trace).  Wiener increments: dW = sqrt(dt) z, z standard   */
/* normal by the Box-Muller transform of two Philox-4x32-10 uniforms, counter */
/* (traj_lo, traj_hi, step, 1 + n/2), n even -> cos branch, n odd -> sin.     */
/* ------------------------------------------------------------------------- */
void or_wiener_normals(uint64_t seed, uint64_t traj, uint32_t step, uint32_t pair, double *z0, double *z1)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4] = {(uint32_t)traj, (uint32_t)(traj >> 32), step, 1u + pair};
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    double u1 = or_uniform_from_words(w[0], w[1]);
    double u2 = or_uniform_from_words(w[2], w[3]);
    double r = sqrt(-2.0 * log(u1));
    const double two_pi = 6.283185307179586476925286766559;
    *z0 = r * cos(two_pi * u2);
    *z1 = r * sin(two_pi * u2);
}

typedef struct {
    int32_t d, nsc, sme;
    int64_t n;          /* state length: d (SSE) or d*d (SME) */
    const or_csr *H;
    const or_csr *S;    /* sc_ops */
    own_csr *Sd;        /* S_n^dag */
    me_ctx me;          /* SME: the Lindbladian with c_ops and sc_ops */
    cplx *tmp;          /* length n */
} sde_ctx;

/* out = B_n x: S_n psi (SSE), S_n rho + rho S_n^dag (SME) */
static void sde_noise_op(sde_ctx *c, int32_t k, const cplx *x, cplx *out)
{
    if (!c->sme) {
        csr_mv(&c->S[k], x, out);
        return;
    }
    own_csr Sk = own_copy(&c->S[k]);
    memset(out, 0, sizeof(cplx) * c->n);
    acc_AX(&Sk, x, 1.0, out);
    acc_XA(x, &c->Sd[k], 1.0, out);
    own_free(&Sk);
}

/* mu_n = <S_n + S_n^dag>: 2 Re<psi|S psi>/<psi|psi> (SSE), Re Tr(S rho + rho S^dag) (SME) */
static double sde_mu(const sde_ctx *c, const cplx *x, const cplx *Bx)
{
    if (!c->sme) {
        cplx num = 0.0;
        double den = 0.0;
        for (int64_t i = 0; i < c->n; ++i) {
            num += conj(x[i]) * Bx[i];
            den += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
        }
        return 2.0 * creal(num) / den;
    }
    double tr = 0.0;
    for (int32_t i = 0; i < c->d; ++i)
        tr += creal(Bx[(int64_t)i * c->d + i]);
    return tr;
}

/* drift a(x) given B_n x and mu_n already computed at x */
static void sde_drift(sde_ctx *c, const cplx *x, cplx *const *Bx, const double *mu, cplx *a)
{
    if (c->sme) {
        me_rhs(&c->me, 0.0, x, a);
        return;
    }
    /* -i H psi - 1/2 sum S^dag S psi + sum (mu/2 S psi - mu^2/8 psi) */
    csr_mv(c->H, x, a);
    for (int64_t i = 0; i < c->n; ++i)
        a[i] *= -I;
    for (int32_t k = 0; k < c->nsc; ++k) {
        own_mv_acc(&c->Sd[k], Bx[k], -0.5, a);
        for (int64_t i = 0; i < c->n; ++i)
            a[i] += 0.5 * mu[k] * Bx[k][i] - 0.125 * mu[k] * mu[k] * x[i];
    }
}

static void sde_normalise(const sde_ctx *c, cplx *x)
{
    double s = 0.0;
    if (c->sme) {
        for (int32_t i = 0; i < c->d; ++i)
            s += creal(x[(int64_t)i * c->d + i]);
    } else {
        s = sqrt(norm2(x, c->n));
    }
    for (int64_t i = 0; i < c->n; ++i)
        x[i] /= s;
}

static void sde_record(const sde_ctx *c, const cplx *x, int32_t ne, const or_csr *e_ops, int32_t nt, int32_t idx,
                       double *expect_tr)
{
    for (int32_t k = 0; k < ne; ++k) {
        cplx v = c->sme ? trace_O_rho(&e_ops[k], x, c->d) : expect_ket(&e_ops[k], x, c->d);
        expect_tr[2 * ((int64_t)k * nt + idx)] = creal(v);
        expect_tr[2 * ((int64_t)k * nt + idx) + 1] = cimag(v);
    }
}

/* One trajectory.  meas: [nsc][nt-1], the current averaged over each tlist interval. */
static void sde_trajectory(sde_ctx *c, const cplx *x0, int32_t nt, const double *tlist, int32_t ne,
                           const or_csr *e_ops, double dt, uint64_t seed, uint64_t traj, double *expect_tr,
                           double *meas)
{
    const int64_t n = c->n;
    const int32_t m = c->nsc;
    const double cg = c->sme ? 1.0 : 0.5; /* mu multiple removed by the diffusion */
    cplx *x = calloc(n, sizeof(cplx)), *a = calloc(n, sizeof(cplx)), *xs = calloc(n, sizeof(cplx));
    cplx *xn = calloc(n, sizeof(cplx));
    cplx **Bx = malloc(sizeof(cplx *) * (m ? m : 1)), **Bs = malloc(sizeof(cplx *) * (m ? m : 1));
    for (int32_t k = 0; k < m; ++k) {
        Bx[k] = calloc(n, sizeof(cplx));
        Bs[k] = calloc(n, sizeof(cplx));
    }
    double *mu = calloc(m ? m : 1, sizeof(double)), *dW = calloc(m ? m : 1, sizeof(double));
    double *acc = calloc(m ? m : 1, sizeof(double));
    memcpy(x, x0, sizeof(cplx) * n);
    sde_normalise(c, x);
    sde_record(c, x, ne, e_ops, nt, 0, expect_tr);
    uint32_t step = 0;
    for (int32_t iv = 0; iv + 1 < nt; ++iv) {
        const double len = tlist[iv + 1] - tlist[iv];
        int64_t ns = (int64_t)ceil(len / dt * (1.0 - 1e-12));
        if (ns < 1)
            ns = 1;
        const double h = len / (double)ns, sq = sqrt(h);
        for (int32_t k = 0; k < m; ++k)
            acc[k] = 0.0;
        for (int64_t q = 0; q < ns; ++q, ++step) {
            for (int32_t k = 0; k < m; k += 2) {
                double z0, z1;
                or_wiener_normals(seed, traj, step, (uint32_t)(k / 2), &z0, &z1);
                dW[k] = sq * z0;
                if (k + 1 < m)
                    dW[k + 1] = sq * z1;
            }
            /* a(Y), b_n(Y) = B_n Y - cg mu_n Y */
            for (int32_t k = 0; k < m; ++k) {
                sde_noise_op(c, k, x, Bx[k]);
                mu[k] = sde_mu(c, x, Bx[k]);
                acc[k] += mu[k] * h + dW[k];
            }
            sde_drift(c, x, Bx, mu, a);
            /* Y' = Y + a h + sum_n b_n dW_n + sum_n (b_n(Ups_n) - b_n(Y)) (dW_n^2 - h) / (2 sqrt h),
             * Ups_n = Y + a h + b_n sqrt h */
            for (int64_t i = 0; i < n; ++i)
                xn[i] = x[i] + a[i] * h;
            for (int32_t k = 0; k < m; ++k) {
                const double w = (dW[k] * dW[k] - h) / (2.0 * sq);
                for (int64_t i = 0; i < n; ++i) {
                    const cplx b = Bx[k][i] - cg * mu[k] * x[i];
                    xs[i] = x[i] + a[i] * h + b * sq;
                }
                sde_noise_op(c, k, xs, Bs[k]);
                const double ms = sde_mu(c, xs, Bs[k]);
                for (int64_t i = 0; i < n; ++i) {
                    const cplx b = Bx[k][i] - cg * mu[k] * x[i];
                    const cplx bs = Bs[k][i] - cg * ms * xs[i];
                    xn[i] += b * dW[k] + (bs - b) * w;
                }
            }
            memcpy(x, xn, sizeof(cplx) * n);
            sde_normalise(c, x);
        }
        for (int32_t k = 0; k < m; ++k)
            meas[(int64_t)k * (nt - 1) + iv] = acc[k] / len;
        sde_record(c, x, ne, e_ops, nt, iv + 1, expect_tr);
    }
    for (int32_t k = 0; k < m; ++k) {
        free(Bx[k]);
        free(Bs[k]);
    }
    free(Bx);
    free(Bs);
    free(mu);
    free(dW);
    free(acc);
    free(x);
    free(a);
    free(xs);
    free(xn);
}

/* SSE (sme = 0, x0 = psi0 of length d, c_ops ignored) or SME (sme = 1, x0 = rho0 d x d);
 * expect_tr [ntraj][ne][nt], meas [ntraj][nsc][nt-1]. */
int32_t or_sdesolve(int32_t sme, const or_csr *H, int32_t nc, const or_csr *c_ops, int32_t nsc, const or_csr *sc_ops,
                    const double *x0, int32_t nt, const double *tlist, int32_t ne, const or_csr *e_ops, double dt,
                    uint64_t seed, uint64_t traj0, int64_t ntraj, double *expect_tr, double *meas)
{
    if (check_tlist(nt, tlist) || !(dt > 0.0))
        return OR_EINVAL;
    const int32_t d = H->d;
    const int64_t n = sme ? (int64_t)d * d : d;
    own_csr *Sd = malloc(sizeof(own_csr) * (nsc ? nsc : 1));
    for (int32_t k = 0; k < nsc; ++k)
        Sd[k] = own_adjoint(&sc_ops[k]);
    or_csr *all = malloc(sizeof(or_csr) * (nc + nsc ? nc + nsc : 1));
    for (int32_t k = 0; k < nc; ++k)
        all[k] = c_ops[k];
    for (int32_t k = 0; k < nsc; ++k)
        all[nc + k] = sc_ops[k];
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < ntraj; ++j) {
        sde_ctx c;
        c.d = d;
        c.nsc = nsc;
        c.sme = sme;
        c.n = n;
        c.H = H;
        c.S = sc_ops;
        c.Sd = Sd;
        c.tmp = NULL;
        if (sme)
            me_ctx_init(&c.me, H, nc + nsc, all);
        sde_trajectory(&c, (const cplx *)x0, nt, tlist, ne, e_ops, dt, seed, traj0 + (uint64_t)j,
                       expect_tr + 2 * j * (int64_t)ne * nt, meas + j * (int64_t)nsc * (nt > 1 ? nt - 1 : 0));
        if (sme)
            me_ctx_free(&c.me);
    }
    for (int32_t k = 0; k < nsc; ++k)
        own_free(&Sd[k]);
    free(Sd);
    free(all);
    return OR_OK;
}

/* Ensemble mean and standard error (unbiased variance of the real part). */
void or_ensemble_stats(int64_t ntraj, int32_t ne, int32_t nt, const double *expect_tr, double *mean,
                       double *se)
{
    int64_t m = (int64_t)ne * nt;
    for (int64_t q = 0; q < m; ++q) {
        double sr = 0.0, si = 0.0;
        for (int64_t j = 0; j < ntraj; ++j) {
            sr += expect_tr[2 * (j * m + q)];
            si += expect_tr[2 * (j * m + q) + 1];
        }
        double mr = sr / (double)ntraj, mi = si / (double)ntraj;
        double v = 0.0;
        for (int64_t j = 0; j < ntraj; ++j) {
            double x = expect_tr[2 * (j * m + q)] - mr;
            v += x * x;
        }
        mean[2 * q] = mr;
        mean[2 * q + 1] = mi;
        se[q] = ntraj > 1 ? sqrt(v / (double)(ntraj - 1) / (double)ntraj) : 0.0;
    }
}

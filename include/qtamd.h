/*
 * qtamd.h -- C ABI of the MI355X (gfx950) Lindblad / quantum-jump solver library (libqtamd.so).
 *
 * The library integrates the Lindblad master equation (arXiv:2504.21440, Sec. 3.2,
 * eq. eq-lindblad-master-equation, dissipator in its trace-preserving anticommutator form)
 *
 *     d rho/dt = L rho = -i[H, rho] + sum_k ( C_k rho C_k^dag - 1/2 {C_k^dag C_k, rho} )
 *
 * with an adaptive Dormand-Prince 5(4) scheme run entirely on the GPU (step control included),
 * and its Monte-Carlo wave-function counterpart (Sec. 3.3): pure states evolved under
 * H_eff = H - (i/2) sum_k C_k^dag C_k, a quantum jump when the squared norm falls to a uniform
 * threshold, the channel drawn with P_k = <C_k^dag C_k> / sum_j <C_j^dag C_j>.
 * Expectation values are taken at every point of tlist (Sec. 3.1, e_ops).
 *
 * Conventions used throughout
 *  - Complex numbers are interleaved (re, im) pairs of double on the host.
 *  - Matrices are d x d, row-major; vec(rho)[i*d + j] = rho_ij.
 *  - Operators cross the boundary as host CSR (qt_csr) with int64 row pointers, int32 column
 *    indices, complex128 values; indices in a row need not be sorted; duplicates are summed.
 *  - Ownership: the caller owns every host array it passes; the library reads them during the
 *    call only and never keeps a pointer.  Handles (qt_ctx, qt_liouv, qt_me_plan, qt_mc_plan,
 *    qt_server) own their device memory until the matching *_destroy.  Arrays the library fills
 *    into a qt_csr (qt_model_*) are released with qt_csr_free.
 *  - Errors: every function returns a qt_status; nothing throws across the ABI.  On an error the
 *    outputs are unspecified except qt_stats.status; qt_last_error() gives a message (per thread).
 *  - Threads: one thread at a time per qt_ctx; different contexts are independent.
 *  - Precision: QT_F64 computes everything in FP64.  QT_MIXED stores the Liouvillian, the states
 *    and the Runge-Kutta stages in complex FP32 and applies them in FP32, while step-size control,
 *    the error-norm reduction, trace renormalisation and expectation values stay FP64 on the GPU.
 */
#ifndef QTAMD_H
#define QTAMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qt_status;
#define QT_OK 0
#define QT_EINVAL 1      /* malformed argument (shape, CSR, tlist not strictly increasing, ...) */
#define QT_ENOMEM 2      /* device or pool memory exhausted / request larger than the pool     */
#define QT_EDEVICE 3     /* HIP runtime error                                                  */
#define QT_EMAXSTEPS 4   /* opts.max_steps reached before the last tlist point                */
#define QT_EDTMIN 5      /* step size fell below 1e-14 max(1, |t|)                             */
#define QT_ENONFINITE 6  /* non-finite error norm or state                                     */
#define QT_EBUSY 7       /* server cannot admit the request now; try again after a step        */

#define QT_F64 0
#define QT_MIXED 1

#define QT_FORM_CSR 0   /* sparse Liouvillian superoperator, applied by CSR SpMV          */
#define QT_FORM_DENSE 1 /* dense operator form L(rho) = A rho + (A rho)^dag + sum C rho C^dag */

typedef struct qt_ctx qt_ctx;
typedef struct qt_liouv qt_liouv;
typedef struct qt_me_plan qt_me_plan;
typedef struct qt_mc_plan qt_mc_plan;
typedef struct qt_server qt_server;

/* Host CSR operator (square). */
typedef struct {
    int32_t rows;
    int32_t cols;
    int64_t nnz;
    const int64_t *indptr;  /* rows + 1 */
    const int32_t *indices; /* nnz */
    const double *values;   /* 2 * nnz, interleaved re/im */
} qt_csr;

/* Integrator options.  Defaults (qt_opts_default): abstol 1e-8, reltol 1e-6, max_steps 1e6,
 * h0 = 0 (automatic starting step), precision QT_F64, form QT_FORM_CSR, steps_per_launch 0
 * (library default), autotune 0.  With autotune set, a plan whose size bucket the tuning table
 * does not hold yet measures its candidate tile shapes once at creation and records the fastest
 * (qt_me_plan_autotune). */
typedef struct {
    double abstol;
    double reltol;
    int64_t max_steps;
    double h0;
    int32_t precision;
    int32_t form;
    int32_t steps_per_launch; /* RK steps recorded per graph replay (CSR form; 0: 16).  With an even
                                 count a plan of one problem folds its step control into the
                                 next step's stage-2 launch (same results, one launch fewer) */
    int32_t autotune;         /* nonzero: tune unseen size buckets at plan creation */
} qt_opts;

typedef struct {
    int64_t n_accept;
    int64_t n_reject;
    int64_t n_rhs;     /* right-hand-side applications (per trajectory summed for mcsolve) */
    int64_t n_jumps;
    int32_t status;
    int32_t reserved;
    double device_ms;  /* wall time of the device-resident part of the call */
} qt_stats;

void qt_opts_default(qt_opts *o);
const char *qt_last_error(void);
const char *qt_version(void);

/* Context: binds a HIP device and a stream (hipStream_t, may be NULL for the null stream). */
qt_status qt_ctx_create(int32_t device, void *hip_stream, qt_ctx **out);
qt_status qt_ctx_destroy(qt_ctx *ctx);

/* Model operators (host CSR filled by the library; release each with qt_csr_free).
 * Driven Kerr cavity (Sec. 6 benchmark family), Fock cutoff N:
 *     H = delta a^dag a + (U/2) a^dag a^dag a a + F (a + a^dag),  c = sqrt(kappa) a.
 * Open transverse-field Ising chain (Secs. 4, 6), L spins, spin 0 most significant,
 * basis state 0 = up (sigma_z = +1), sigma_- = |down><up|:
 *     H = J sum_i sz_i sz_{i+1} + h sum_i sx_i,  c_i = sqrt(gamma) sm_i  (c_ops has L entries). */
qt_status qt_model_kerr(int32_t N, double delta, double U, double F, double kappa, qt_csr *H, qt_csr *c);
qt_status qt_model_ising(int32_t L, double J, double h, double gamma, qt_csr *H, qt_csr *c_ops);
void qt_csr_free(qt_csr *A);

/* Liouvillian (Sec. 3.2; the precomputed-superoperator use of Sec. 5).
 * form QT_FORM_CSR: assembles on the device, in FP64, the superoperator
 *     L = A (x) I + I (x) conj(A) + sum_k C_k (x) conj(C_k),   A = -i H - 1/2 sum_k C_k^dag C_k,
 * for the row-major vec, drops entries that are zero in the storage precision, stores values as
 * complex128 (QT_F64) or complex64 (QT_MIXED) with int32 indices (nnz < 2^31), and pads every row
 * with explicit zeros to a multiple of 4 stored entries (so the SpMV can load aligned runs of 4).
 * form QT_FORM_DENSE: stores A and the C_k as dense matrices zero-padded to a multiple of 16 for
 * the batched MFMA right-hand side (in the order the kernel's lanes read them; a C_k with no
 * imaginary part keeps its real parts only); d <= 80 (QT_MIXED) or d <= 48 (QT_F64).  Solves in
 * this form need a Hermitian initial state (their results are Hermitian by construction).
 * Errors: QT_EINVAL for mismatched sizes, malformed CSR, or a dense d above the limit. */
qt_status qt_liouvillian_build(qt_ctx *ctx, const qt_csr *H, int32_t n_c, const qt_csr *c_ops, int32_t form,
                               int32_t precision, qt_liouv **out);
/* Time-dependent Liouvillian (Sec. 2, QobjEvo; Sec. 3.2 with time-dependent operators, the driven
 * example of Sec. 3.4):
 *     H(t) = H0 + sum_i f_i(t) H_i,   collapse operators g_k(t) C_k,
 *     L(t) rho = -i[H0, rho] - i sum_i f_i(t) (H_i rho - rho H_i) + sum_k w_k(t) D[C_k] rho,
 * with w_k = |g_k(t)|^2 where c_coefs[k] has a kind other than QT_COEF_NONE and w_k = 1 otherwise.
 * H0 is Hermitian; the H_i need not be (a complex drive f a^dag + conj(f) a is two terms) and the
 * f_i may be complex.  Coefficient kinds (a = (a[0], a[1]) complex):
 *     QT_COEF_CONST   a
 *     QT_COEF_COS     a cos(omega t + phi)
 *     QT_COEF_EXP     a exp(i (omega t + phi))
 *     QT_COEF_GAUSS   a exp(-(t - t0)^2 / (2 sigma^2)) cos(omega t + phi)   (sigma > 0)
 *     QT_COEF_TABLE   a times the linear interpolation of the n_table complex samples `table`
 *                     (interleaved re/im, host) taken at table_t0 + k table_dt, held at the end
 *                     values outside [table_t0, table_t0 + (n_table - 1) table_dt]  (table_dt > 0)
 * The device evaluates each coefficient in FP64 at the time of every right-hand-side evaluation.
 * The library copies the tables; the caller's arrays may be released after the call.
 * CSR form only; at most 31 time-dependent terms (H_i plus weighted collapse operators) and
 * d*d < 2^26.  Plans mix time-dependent and constant problems freely.  Errors: QT_EINVAL for the
 * dense form, too many terms, a bad kind or table, mismatched sizes. */
#define QT_COEF_NONE (-1)
#define QT_COEF_CONST 0
#define QT_COEF_COS 1
#define QT_COEF_EXP 2
#define QT_COEF_GAUSS 3
#define QT_COEF_TABLE 4
typedef struct {
    int32_t kind;
    int32_t n_table;
    double a[2];
    double omega, phi;
    double t0, sigma;
    double table_t0, table_dt;
    const double *table;
} qt_coef;
qt_status qt_liouvillian_build_td(qt_ctx *ctx, const qt_csr *H0, int32_t n_h, const qt_csr *h_terms,
                                  const qt_coef *h_coefs, int32_t n_c, const qt_csr *c_ops, const qt_coef *c_coefs,
                                  int32_t form, int32_t precision, qt_liouv **out);
/* Number of time-dependent terms of a Liouvillian (0 for a constant one). */
qt_status qt_liouv_terms(const qt_liouv *L, int32_t *n_terms);
/* d, non-zeros of L (CSR form, padding not counted; 0 for dense), device bytes held. */
qt_status qt_liouv_info(const qt_liouv *L, int32_t *d, int64_t *nnz, int64_t *bytes);
/* Device bytes the Liouvillian holds until qt_liouv_destroy: CSR row pointers, columns and values
 * (and the coefficient tables of a time-dependent one), or the dense operators.  A served request
 * is charged this plus its own state (qt_server_footprint). */
qt_status qt_liouv_footprint(const qt_liouv *L, size_t *bytes);
/* Copies the assembled CSR back to the host (values widened to complex128, row padding left out).
 * indptr: d*d + 1, indices and values: nnz from qt_liouv_info.  CSR form only. */
qt_status qt_liouv_export(const qt_liouv *L, int64_t *indptr, int32_t *indices, double *values);
qt_status qt_liouv_destroy(qt_liouv *L);

/* One master-equation problem.  rho0 is a host d x d matrix (used as given, not normalised) or,
 * with is_ket, a length-d ket turned into |psi><psi|.  tlist is strictly increasing; tlist[0] is
 * the initial time and its expectation values are recorded.  e_ops are n_e host CSR operators. */
typedef struct {
    const qt_liouv *L;
    const double *rho0;
    int32_t is_ket;
    int32_t n_t;
    const double *tlist;
    int32_t n_e;
    const qt_csr *e_ops;
} qt_me_problem;

/* One-shot solve: expect_out [n_e][n_t] complex (host), rho_final d x d complex (host, nullable). */
qt_status qt_mesolve(qt_ctx *ctx, const qt_me_problem *prob, const qt_opts *opts, double *expect_out,
                     double *rho_final, qt_stats *stats);
/* Caller-owned device workspace.  qt_me_plan_workspace reports the device bytes a plan of these
 * problems needs (initial states, save times, e_ops, expectation values, Runge-Kutta stages, block
 * tables, control records); qt_me_plan_create_ws lays the plan out in the caller's buffer dev_ws
 * (device memory on the context's device, 256-byte aligned, at least that many bytes; a torch
 * tensor's storage will do) instead of allocating, and qt_mesolve_ws is the one-shot solve in such
 * a buffer.  The buffer must stay allocated and untouched by the caller until the plan is destroyed
 * (for qt_mesolve_ws: until the call returns, which synchronises the context's stream).  The
 * library calls no hipMalloc for such a plan, at creation or later (it still allocates small pinned
 * host mirrors of the control records, and the HIP runtime may allocate internally for the graphs
 * it instantiates); results are bitwise those of the allocating calls.  Errors: QT_EINVAL for a
 * null or misaligned buffer, QT_ENOMEM when ws_bytes is below the workspace size. */
qt_status qt_me_plan_workspace(qt_ctx *ctx, int32_t n, const qt_me_problem *probs, const qt_opts *opts,
                               size_t *bytes);
qt_status qt_me_plan_create_ws(qt_ctx *ctx, int32_t n, const qt_me_problem *probs, const qt_opts *opts, void *dev_ws,
                               size_t ws_bytes, qt_me_plan **out);
qt_status qt_mesolve_ws(qt_ctx *ctx, const qt_me_problem *prob, const qt_opts *opts, void *dev_ws, size_t ws_bytes,
                        double *expect_out, double *rho_final, qt_stats *stats);
/* Many problems advanced together in the same launches (each with its own step size, accept /
 * reject decisions and save times).  expect_out[i] is [n_e][n_t] of problem i. */
qt_status qt_mesolve_batch(qt_ctx *ctx, int32_t n, const qt_me_problem *probs, const qt_opts *opts,
                           double *const *expect_out, qt_stats *stats);

/* Device-resident plans: create uploads every input once; run integrates all problems from their
 * resident initial states to their resident expectation values with no host transfer beyond a
 * status word; result copies one problem's outputs back.  run may be called repeatedly. */
qt_status qt_me_plan_create(qt_ctx *ctx, int32_t n, const qt_me_problem *probs, const qt_opts *opts,
                            qt_me_plan **out);
qt_status qt_me_plan_run(qt_me_plan *plan);
qt_status qt_me_plan_result(qt_me_plan *plan, int32_t i, double *expect_out, double *rho_final, qt_stats *stats);
qt_status qt_me_plan_destroy(qt_me_plan *plan);
/* Steady state (Sec. 3.2, steadystate): the density matrix with L rho_ss = 0 (and the trace of
 * rho0), reached by integrating the master equation with the same adaptive integrator until
 * |L rho|_2 <= tol after an accepted step (the Frobenius norm of d rho/dt, FP64).  Near the steady
 * state the explicit steps are limited by stability, and the stiff components stay at the level the
 * error control admits (about abstol per element), so |L rho|_2 levels off near
 * |L|_2 * abstol * sqrt(d^2) (measured: about 5e3 * abstol for a driven Kerr cavity of cutoff 20):
 * take abstol well below tol / (|L|_2 d), at least 1e-4 * tol, and in mixed precision tol well
 * above the FP32 rounding of L rho.  The distance to rho_ss is at most tol divided by the
 * spectral gap of L.  A problem that converges stops, and
 * every save time not yet reached receives the expectation values of the converged state; one that
 * passes its last save time unconverged ends with QT_EMAXSTEPS.  Both forms (CSR, dense).
 * qt_steadystate integrates one problem over [0, t_max]: expect_out [n_e] complex, rho_out d x d
 * (nullable). */
qt_status qt_me_plan_create_steady(qt_ctx *ctx, int32_t n, const qt_me_problem *probs, const qt_opts *opts, double tol,
                                   qt_me_plan **out);
qt_status qt_steadystate(qt_ctx *ctx, const qt_liouv *L, const double *rho0, int32_t is_ket, double tol, double t_max,
                         int32_t n_e, const qt_csr *e_ops, const qt_opts *opts, double *expect_out, double *rho_out,
                         qt_stats *stats);
/* Measurement: average device duration (HIP events on the plan's stream) of one right-hand-side
 * launch over `reps` back-to-back launches.  CSR problems: one fused SpMV-stage kernel (the stage
 * that forms the fourth stage input) over every CSR problem of the plan, from a freshly reset
 * state.  Plans with only dense problems: one whole-solve launch of the dense kernels.  The plan's
 * results are unspecified afterwards until the next qt_me_plan_run. */
qt_status qt_me_plan_time_rhs(qt_me_plan *plan, int32_t reps, double *ms_per_launch);

/* Measurement: the achievable HBM bandwidth of the context's device, bytes read plus bytes written
 * per second of a streaming copy of `bytes` bytes (16-byte non-temporal loads and stores, four in
 * flight per lane, 64 workgroups per compute unit), repeated `reps` times and timed with HIP events
 * on the context's stream; the reference point for the bandwidth-bound SpMV beside the published
 * peak.  Allocates two buffers of `bytes` for the call.  Errors: QT_EINVAL for a null argument,
 * bytes < 16 or reps < 1; QT_EDEVICE for a HIP failure, allocation included. */
qt_status qt_measure_copy_bandwidth(qt_ctx *ctx, int64_t bytes, int32_t reps, double *gbs);

/* Measurement: as qt_measure_copy_bandwidth for a streaming read of `bytes` bytes (16-byte
 * non-temporal loads summed in registers, 32 workgroups per compute unit, nothing written back):
 * bytes read per second, the ceiling for kernels whose traffic is nearly all reads, such as the CSR
 * SpMV.  Allocates one buffer of `bytes` and 4 bytes per workgroup for the call; errors as
 * qt_measure_copy_bandwidth. */
qt_status qt_measure_read_bandwidth(qt_ctx *ctx, int64_t bytes, int32_t reps, double *gbs);

/* Autotuner.  The CSR stage kernels take a launch shape (qt_csr_shape):
 *   lanes_per_row   4, 8 or 16 lanes of a wavefront share a row;
 *   rows_per_group  1, 2 or 4 rows per lane group (at most lanes_per_row);
 *   xcd_order       1: each of the 8 XCDs (each with its own L2) works through one contiguous eighth
 *                   of the rows; 0: the hardware's round-robin order;
 *   cached_matrix   1: the matrix is read through the caches (temporal loads), so a matrix that
 *                   fits the L2s can stay there across launches; 0: it is streamed past them;
 *                   2: as 1, each lane loading runs of 4 stored entries with 16-byte loads (rows are
 *                   stored padded to multiples of 4); built for 4x1, 8x1, 8x2 and 16x1.
 * xcd_order applies to plans with one CSR problem (a plan with several uses 0).
 * The dense kernel is built with a few wave counts per workgroup for each padded size (for FP32:
 * 1-2 at 16, 2 or 4 at 32, 3, 4, 6 or 8 at 48, 4 or 8 at 64, 4, 5 or 8 at 80; for FP64: 1 at 16,
 * 2 or 4 at 32, 3 or 4 at 48); the waves split the output tiles into near-equal contiguous runs.
 * qt_me_plan_autotune times the fused SpMV-stage kernel of the plan's CSR problems for every
 * candidate shape over `reps` launches (20 if reps <= 0), and each dense size bucket for each of
 * its wave counts over a budget of 8 steps; the fastest are kept for the plan and stored in a process-wide table keyed by precision
 * and size bucket (log2 of the rows and mean row length for CSR, padded dimension for dense),
 * which every later plan consults.  The plan's results are unspecified afterwards until the next
 * qt_me_plan_run.  qt_me_plan_shape reports the shape in use (zeros for a group the plan does not
 * have); qt_me_plan_set_shape imposes a CSR shape (QT_EINVAL if the kernels do not support it).
 * One shape serves every CSR problem of a plan; the row-sum and norm reduction orders follow
 * lanes_per_row and rows_per_group only, so a problem's results are bitwise the same alone and in
 * a batch, and with either xcd_order or cached_matrix, when those two are the same.  The dense
 * kernel's norms are block reductions whose order follows the wave count. */
typedef struct {
    int32_t lanes_per_row;
    int32_t rows_per_group;
    int32_t xcd_order;
    int32_t cached_matrix;
} qt_csr_shape;
qt_status qt_me_plan_autotune(qt_me_plan *plan, int32_t reps);
qt_status qt_me_plan_set_shape(qt_me_plan *plan, const qt_csr_shape *shape);
/* dense_waves: the wave count of the largest dense size bucket (0 without dense problems) */
qt_status qt_me_plan_shape(const qt_me_plan *plan, qt_csr_shape *csr, int32_t *dense_waves);
/* Persist the tuning table as a small JSON object {"key": [shape...], ...}.  load merges the
 * entries of a file written by save, ignoring any shape the kernels do not support. */
qt_status qt_tune_save(const char *path);
qt_status qt_tune_load(const char *path);

/* Expectation value (Sec. 3.1 e_ops; App. C expect): out = Tr(O rho) for a device density
 * matrix, or <psi|O|psi>/<psi|psi> for a device ket (is_ket), state stored complex128
 * (QT_F64) or complex64 (QT_MIXED), accumulated in FP64.  out: one complex (host). */
qt_status qt_expect(qt_ctx *ctx, int32_t d, const qt_csr *O, const void *dev_state, int32_t is_ket,
                    int32_t precision, double *out);
/* The same expectation value for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): it calls no hipMalloc, hipFree or
 * other allocating routine.  The operator is staged, as the caller passes it, in a device array of
 * QT_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on until the process ends;
 * an operator that needs more (about 12 (d + 1) + 20 nnz bytes plus alignment) is rejected with
 * QT_ENOMEM.  O is read in place: its entries are summed in the order given (duplicates are two
 * terms; for a canonical CSR -- rows sorted, no duplicates or exact zeros -- the result is bitwise
 * that of qt_expect).  Every call on one GPU shares that GPU's array, so calls that overlap on one
 * GPU (two threads, or two contexts whose streams run at the same time) race; the call returns
 * after its stream is synchronised.  Errors as for qt_expect, plus QT_ENOMEM for the size limit. */
#define QT_NOALLOC_SCRATCH_BYTES (8 << 20)
qt_status qt_expect_noalloc(qt_ctx *ctx, int32_t d, const qt_csr *O, const void *dev_state, int32_t is_ket,
                            int32_t precision, double *out);

/* Monte-Carlo wave function (Sec. 3.3).  Trajectory j draws from Philox-4x32-10 keyed by seed
 * with counter (j_lo, j_hi, event, 0): event 0 gives the first threshold, event m >= 1 the channel
 * uniform of jump m and the threshold after it.  psi0 is normalised before use. */
typedef struct {
    const qt_csr *H;
    int32_t n_c;
    const qt_csr *c_ops;
    const double *psi0;
    int32_t n_t;
    const double *tlist;
    int32_t n_e;
    const qt_csr *e_ops;
    int64_t ntraj;
    uint64_t seed;
} qt_mc_problem;

/* mean_out [n_e][n_t] complex; se_out [n_e][n_t] standard error of the real part (nullable);
 * expect_tr [ntraj][n_e][n_t] complex (nullable); njumps [ntraj] (nullable); jump_times and
 * jump_channels [ntraj][max_jump_record] (nullable when max_jump_record == 0); the first
 * min(njumps[j], max_jump_record) entries of row j are trajectory j's jumps in order, the rest are
 * unspecified. */
qt_status qt_mcsolve(qt_ctx *ctx, const qt_mc_problem *prob, const qt_opts *opts, double *mean_out, double *se_out,
                     double *expect_tr, int64_t *njumps, int32_t max_jump_record, double *jump_times,
                     int32_t *jump_channels, qt_stats *stats);
qt_status qt_mc_plan_create(qt_ctx *ctx, const qt_mc_problem *prob, const qt_opts *opts, int32_t max_jump_record,
                            qt_mc_plan **out);
qt_status qt_mc_plan_run(qt_mc_plan *plan);
qt_status qt_mc_plan_result(qt_mc_plan *plan, double *mean_out, double *se_out, double *expect_tr, int64_t *njumps,
                            double *jump_times, int32_t *jump_channels, qt_stats *stats);
qt_status qt_mc_plan_destroy(qt_mc_plan *plan);

/* Trajectory plans in a caller-owned device workspace, as for qt_me_plan_create_ws: the bytes a
 * plan of this problem needs (operators, per-trajectory expectation rows, jump records, counters,
 * ensemble sums), the plan laid out in the caller's buffer, and the one-shot solve in it. */
qt_status qt_mc_plan_workspace(qt_ctx *ctx, const qt_mc_problem *prob, const qt_opts *opts, int32_t max_jump_record,
                               size_t *bytes);
qt_status qt_mc_plan_create_ws(qt_ctx *ctx, const qt_mc_problem *prob, const qt_opts *opts, int32_t max_jump_record,
                               void *dev_ws, size_t ws_bytes, qt_mc_plan **out);
qt_status qt_mcsolve_ws(qt_ctx *ctx, const qt_mc_problem *prob, const qt_opts *opts, void *dev_ws, size_t ws_bytes,
                        double *mean_out, double *se_out, double *expect_tr, int64_t *njumps, int32_t max_jump_record,
                        double *jump_times, int32_t *jump_channels, qt_stats *stats);

/* Time-dependent trajectories (Sec. 3.3 with the time-dependent operators of Sec. 2, QobjEvo):
 *     H(t) = H + sum_i f_i(t) H_i,   collapse operator k is g_k(t) C_k where c_coefs[k] has a kind
 *     other than QT_COEF_NONE (c_coefs nullable: every C_k constant),
 * so H_eff(t) = H(t) - (i/2) sum_k |g_k(t)|^2 C_k^dag C_k, and a jump at t* picks channel k with
 * probability proportional to |g_k(t*)|^2 |C_k psi|^2 and applies C_k psi / |C_k psi| (the phase of
 * g_k drops out of every expectation value).  Coefficients as for qt_liouvillian_build_td; at most
 * 31 terms (H_i plus weighted collapse operators).  With td NULL or empty these are the plain calls. */
typedef struct {
    int32_t n_h;
    const qt_csr *h_terms;
    const qt_coef *h_coefs;
    const qt_coef *c_coefs;
} qt_td_terms;
qt_status qt_mc_plan_create_td(qt_ctx *ctx, const qt_mc_problem *prob, const qt_td_terms *td, const qt_opts *opts,
                               int32_t max_jump_record, qt_mc_plan **out);
qt_status qt_mcsolve_td(qt_ctx *ctx, const qt_mc_problem *prob, const qt_td_terms *td, const qt_opts *opts,
                        double *mean_out, double *se_out, double *expect_tr, int64_t *njumps, int32_t max_jump_record,
                        double *jump_times, int32_t *jump_channels, qt_stats *stats);

/* Schrodinger equation (Sec. 3.1, sesolve): d psi/dt = -i H psi with the same adaptive
 * Dormand-Prince 5(4) integrator, save-time landing and precision modes; expect_out [n_e][n_t]
 * complex (host) holds <psi|O|psi> / <psi|psi> at every point of tlist.  psi0 (length d, host) is
 * normalised before use.  Runs as a single trajectory without collapse operators, so d <= 4096. */
qt_status qt_sesolve(qt_ctx *ctx, const qt_csr *H, const double *psi0, int32_t n_t, const double *tlist, int32_t n_e,
                     const qt_csr *e_ops, const qt_opts *opts, double *expect_out, qt_stats *stats);
/* The same with H(t) = H + sum_i f_i(t) H_i (td->c_coefs ignored). */
qt_status qt_sesolve_td(qt_ctx *ctx, const qt_csr *H, const qt_td_terms *td, const double *psi0, int32_t n_t,
                        const double *tlist, int32_t n_e, const qt_csr *e_ops, const qt_opts *opts, double *expect_out,
                        qt_stats *stats);

/* Stochastic Schrodinger (SSE) and master (SME) equations under homodyne detection (Sec. 3.5, Ito
 * form): with measured operators S_n (sc_ops) and Wiener increments dW_n,
 *   SSE  d psi = -i K psi dt + sum_n (S_n - e_n/2) psi dW_n,
 *        K = H + i sum_n (e_n/2 S_n - 1/2 S_n^dag S_n - e_n^2/8),  e_n = <psi|S_n + S_n^dag|psi>;
 *   SME  d rho = -i[H, rho] dt + sum_i D[C_i] rho dt + sum_n D[S_n] rho dt
 *               + sum_n (S_n rho + rho S_n^dag - Tr(S_n rho + rho S_n^dag) rho) dW_n;
 * measurement current J_n = <S_n + S_n^dag> + dW_n/dt (reported averaged over each tlist interval).
 * Fixed steps: each tlist interval is cut into ceil(length / dt) equal steps; each step is the
 * derivative-free order-1.0 strong scheme of Platen applied to each Wiener process (exact order 1
 * for one measured operator), followed by renormalisation (unit norm / unit trace).  dW_n =
 * sqrt(h) z, z standard normal from Philox-4x32-10 keyed by seed with counter (trajectory_lo,
 * trajectory_hi, step, 1 + n/2) through the Box-Muller transform (n even: cos, odd: sin).
 * SSE: state0 a ket (is_ket = 1), no c_ops.  SME: state0 a d x d density matrix or a ket.
 * Limits: state length (d, or d*d for the SME) <= 4096, at most 8 measured operators.
 * Outputs (host): mean_out [n_e][n_t] complex, se_out [n_e][n_t] standard error of the real part,
 * expect_tr [ntraj][n_e][n_t] complex, meas_mean [n_sc][n_t - 1] and meas_tr
 * [ntraj][n_sc][n_t - 1] currents; each nullable. */
typedef struct qt_sde_plan qt_sde_plan;
typedef struct {
    const qt_csr *H;
    int32_t n_c;
    const qt_csr *c_ops;
    int32_t n_sc;
    const qt_csr *sc_ops;
    const double *state0;
    int32_t is_ket;
    int32_t n_t;
    const double *tlist;
    int32_t n_e;
    const qt_csr *e_ops;
    int64_t ntraj;
    uint64_t seed;
    double dt;
} qt_sde_problem;
/* master: 0 SSE, 1 SME */
qt_status qt_sde_plan_create(qt_ctx *ctx, const qt_sde_problem *prob, int32_t master, const qt_opts *opts,
                             qt_sde_plan **out);
qt_status qt_sde_plan_run(qt_sde_plan *plan);
qt_status qt_sde_plan_result(qt_sde_plan *plan, double *mean_out, double *se_out, double *expect_tr,
                             double *meas_mean, double *meas_tr, qt_stats *stats);
qt_status qt_sde_plan_destroy(qt_sde_plan *plan);
qt_status qt_ssesolve(qt_ctx *ctx, const qt_sde_problem *prob, const qt_opts *opts, double *mean_out, double *se_out,
                      double *meas_mean, qt_stats *stats);
qt_status qt_smesolve(qt_ctx *ctx, const qt_sde_problem *prob, const qt_opts *opts, double *mean_out, double *se_out,
                      double *meas_mean, qt_stats *stats);

/* Continuous-batching server.  Requests are admitted while their device footprint fits in the
 * pool and a slot is free; admitted requests keep rho and solver state resident and are advanced
 * together, epoch by epoch, with requests that arrived earlier.  submit returns QT_EBUSY when the
 * request does not fit now (QT_ENOMEM if it can never fit).  step runs one epoch and retires
 * finished requests; poll reports completion and copies results.  Requests of every size share
 * the CSR launches, which use 8 lanes per row and one row per lane group and read the matrices
 * through the caches in 16-byte runs of 4 entries; a request's results are bitwise those of a plan
 * with that shape (lanes_per_row 8, rows_per_group 1, cached_matrix 2). */
typedef struct {
    int64_t pool_bytes;      /* device memory budget for resident requests */
    int32_t max_slots;       /* resident requests at most */
    int32_t steps_per_epoch; /* RK steps per request per epoch */
    qt_opts opts;
} qt_server_cfg;

qt_status qt_server_create(qt_ctx *ctx, const qt_server_cfg *cfg, qt_server **out);
/* The server's device memory is one region sized at creation: the request pool (pool_bytes), the
 * slot-indexed descriptors and control records, and the block tables of both lanes at their largest
 * admissible size, so submit, step and poll never allocate device memory.  qt_server_workspace
 * reports its bytes; qt_server_create_ws places it in the caller's buffer (256-byte aligned device
 * memory on the context's device, kept until qt_server_destroy) instead of allocating it. */
qt_status qt_server_workspace(const qt_server_cfg *cfg, size_t *bytes);
qt_status qt_server_create_ws(qt_ctx *ctx, const qt_server_cfg *cfg, void *dev_ws, size_t ws_bytes, qt_server **out);
/* The problem's L must stay alive until the request completes. */
qt_status qt_server_submit(qt_server *srv, const qt_me_problem *prob, uint64_t *ticket);
qt_status qt_server_step(qt_server *srv, int32_t *n_active, int32_t *n_finished);
qt_status qt_server_poll(qt_server *srv, uint64_t ticket, int32_t *done, double *expect_out, qt_stats *stats);
qt_status qt_server_footprint(const qt_server *srv, const qt_me_problem *prob, int64_t *bytes);
qt_status qt_server_destroy(qt_server *srv);

#ifdef __cplusplus
}
#endif
#endif

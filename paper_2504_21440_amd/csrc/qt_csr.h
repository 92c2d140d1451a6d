// qt_csr.h -- device-side descriptors of the CSR-form master-equation solver.
//
// One "instance" is one master-equation problem whose Liouvillian is a CSR superoperator
// (row-major vec, n = d*d rows).  Several instances are advanced by the same kernel launches:
// each thread block serves a fixed row range of one instance, and every instance carries its
// own time, step size, accept/reject history and save index in a CsrCtl record in device
// memory, so no host round trip is needed to control the integration.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qt {

// Time-dependent Liouvillians: L(t) = sum_k w_k(t) L_k is stored as one CSR whose rows list the
// entries of every term in turn; an entry's column index carries its term k above TD_TAG_SHIFT
// (term 0 is the constant part, w_0 = 1).
constexpr int TD_TAG_SHIFT = 26;
constexpr int32_t TD_COL_MASK = (1 << TD_TAG_SHIFT) - 1;
constexpr int TD_MAX_TERMS = 31;  // time-dependent terms (tags 1..31)
constexpr int TD_SLOTS = 8;       // coefficient rows: two starting-step evaluations, stages 2..7

struct CoefDev;

constexpr int CSR_XOPS = 8;  // expectation operators whose entry ranges the descriptor holds

// Solve status kept in device control records (errors use the public QT_E* codes 1..7).
enum : int32_t {
    ST_RUNNING = 0,
    ST_DONE = 100,
};

struct CsrInst {
    int32_t n;  // rows of the superoperator (= d*d)
    int32_t d;
    int32_t nt;
    int32_t ne;
    int32_t block0;   // first block of this instance in the plan's block table (host bookkeeping)
    int32_t nblocks;  // blocks of this instance (= its partial slots)
    int32_t renorm;   // 1: rescale the trace back to its initial value after accepted steps
    int32_t use_h0;   // 1: opts.h0 given
    double atol, rtol, h0;
    int64_t max_steps;
    const int32_t *rowptr;
    const int32_t *col;
    const void *val;  // float2 / double2 [nnz]
    const void *rho0; // resident initial state (state precision) [n]
    void *Y[2];       // y and the candidate y_new, exchanged on acceptance via CsrCtl::parity
    void *K[2];       // k1 and k7 (first same as last), exchanged on acceptance
    void *ks[5];      // k2 .. k6
    void *ys[2];      // stage inputs, alternating
    const double *tlist;
    const int32_t *eptr;  // ne * (d+1) row pointers into ecol/eval (instance-local offsets)
    const int32_t *ecol;
    const double2 *eval;
    const int32_t *evidx; // per e_op entry (i, j): index j*d + i of rho_ji in vec(rho)
    double2 *expect;      // [ne][nt]
    double *partials;     // 2 * nblocks doubles
    // entries of the first CSR_XOPS expectation operators (offsets into ecol / eval / evidx and
    // counts), so that the control kernel can request them together with its control record
    int32_t xbeg[CSR_XOPS];
    int32_t xcnt[CSR_XOPS];
    // time dependence (nterms = 0: none)
    int32_t nterms;          // time-dependent terms (column tags 1..nterms)
    int32_t pad_td;
    const CoefDev *coefs;    // [nterms]
    void *cstage;            // [TD_SLOTS][nterms + 1] coefficient values (state precision), column 0 = 1
    // steady-state mode (0: off): stop once |L y|_2^2 <= steady_tol2 after an accepted step
    double steady_tol2;
};

// Host: the entry ranges of the first CSR_XOPS of ne expectation operators, from their
// instance-local CSR row pointers (ne * (d + 1) of them).
inline void csr_set_expect_ranges(CsrInst &c, const int32_t *eptr, int ne, int d)
{
    for (int k = 0; k < CSR_XOPS; ++k) {
        c.xbeg[k] = k < ne ? eptr[(size_t)k * (d + 1)] : 0;
        c.xcnt[k] = k < ne ? eptr[(size_t)k * (d + 1) + d] - c.xbeg[k] : 0;
    }
}

struct CsrCtl {
    double t;
    double h;        // proposed step
    double h_try;    // step being tried (clipped to the next save time)
    double err_prev;
    double scale;    // trace renormalisation factor applied to y and k1
    double tr0;      // initial trace (renormalisation target)
    double h0;       // starting-step heuristic intermediate
    double last_err;
    int32_t status;
    int32_t phase;  // 1: second starting-step evaluation pending, 0: stepping
    int32_t land;
    int32_t last_rejected;
    int32_t save_idx;
    int32_t parity;
    int32_t pending;  // folded control: a stage 7 ran since this record was decided (its partials wait)
    int32_t pad;
    int64_t n_accept, n_reject, n_steps, n_rhs;
};

}  // namespace qt

// qt_dense.h -- descriptors of the dense-form (oscillator) master-equation solver.
//
// For small dense operators the right-hand side of the master equation (arXiv:2504.21440,
// Sec. 3.2) is evaluated in operator form,
//     L(rho) = A rho + (A rho)^dag + sum_k C_k rho C_k^dag,   A = -i H - 1/2 sum_k C_k^dag C_k,
// which uses rho = rho^dag and costs 1 + 2K complex matrix products per evaluation -- work for the
// matrix cores.  One workgroup owns one problem for a whole launch and runs the adaptive
// Dormand-Prince 5(4) loop itself, so problems of different size and step count never wait for
// each other.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/qtamd.h"

namespace qt {

// padded dimension limits set by LDS: three complex NP x (NP + 16 bytes) matrices must fit in 160 KB
constexpr int DENSE_MAX_NP_F32 = 80;
constexpr int DENSE_MAX_NP_F64 = 48;

struct DenseInst {
    int32_t d, np, nc, nt, ne;
    int32_t use_h0, renorm, creal;  // creal: bit k set when C_k is real
    double atol, rtol, h0;
    int64_t max_steps;
    const void *ops;   // A then C_k, np x np each, zero padded, state precision, in fragment order
    const void *rho0;  // d x d row-major, state precision
    void *vec;         // 10 vectors of np*np elements; the upper tiles' elements in tile order
    const double *tlist;
    const int32_t *eptr;
    const int32_t *ecol;
    const double2 *eval;
    double2 *expect;
    double steady_tol2;  // steady-state mode (0: off): stop once |L y|_2^2 <= steady_tol2
};

enum : int32_t { DENSE_ST_INIT = 200 };

struct DenseCtl {
    double t, h, err_prev, scale, tr0;
    int32_t status, save_idx, last_rejected, parity;
    int64_t n_accept, n_reject, n_steps, n_rhs;
};

inline int dense_np(int d) { return ((d + 15) / 16) * 16; }
inline int dense_state_vectors() { return 10; }

// Lays out the operators A, C_0, ... (nops of them, np x np row-major FP64 complex, zero padded)
// for the solver in the state precision: fragment order, real parts only for the C_k whose bit k
// is set in creal.  out receives nops * np * np complex elements' worth of bytes.
void dense_pack_ops(const double2 *rowmajor, int np, int nops, uint32_t creal, int prec, std::vector<char> &out);
// creal: bit k set when collapse operator k is real (its products then take half the work)
void dense_fill_inst(DenseInst *g, int d, int nc, uint32_t creal, int nt, int ne, const void *ops,
                     const void *rho0, void *vec, const double *tlist, const int32_t *eptr, const int32_t *ecol, const double2 *eval,
                     double2 *expect, const qt_opts &opts, int prec);
// waves per workgroup for a dimension: the autotuner's choice if it has one, else a default
int dense_choose_config(int d, int prec);
// whether the solver is built with this many waves per workgroup for padded size np
bool dense_waves_allowed(int np, int prec, int waves);
// the wave counts built for padded size np (at most max of them into out); returns their number
int dense_waves_candidates(int np, int prec, int *out, int max);
// pointer to the current state vector (tile order) of an instance, for diagnostics
const void *dense_state_ptr(const void *vec, int d, int prec);
// Launch the persistent solver for `count` instances of padded size np (order[] lists them).
// max_steps_launch < 0: run to completion.  reset: start every instance from rho0.
void dense_launch_bucket(int np, bool f64, int waves, const DenseInst *insts, DenseCtl *ctls, const int32_t *order,
                         int count, int max_steps_launch, int reset, hipStream_t s);
// Host-side conversion of a state vector (upper tiles) to a row-major d x d matrix (complex128).
void dense_unpack(const void *host_vec, int d, int prec, double scale, double *out);

}  // namespace qt

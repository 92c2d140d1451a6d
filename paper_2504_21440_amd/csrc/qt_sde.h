// qt_sde.h -- descriptors of the stochastic Schrodinger / master equation solver (homodyne
// detection, arXiv:2504.21440, Sec. 3.5).
//
// Both equations are integrated as x' = a(x) dt + sum_n (B_n x - cg mu_n(x) x) dW_n for a state
// vector x of length n: the ket (SSE, n = d) or vec(rho) (SME, n = d*d).  A is the linear part of
// the drift (SSE: -i H - 1/2 sum S^dag S; SME: the Lindbladian with c_ops and sc_ops), B_n the
// measured operator acting on x (SSE: S_n; SME: rho -> S_n rho + rho S_n^dag), and
// mu_n = <S_n + S_n^dag> in the state x; cg = 1/2 (SSE) or 1 (SME), and the SSE drift adds
// sum_n (mu_n/2 B_n x - mu_n^2/8 x).  The current J_n = mu_n + dW_n/dt is averaged over each tlist
// interval.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qt {

constexpr int SDE_THREADS = 256;
constexpr int SDE_MAX_ROWS = 16;  // n <= 4096
constexpr int SDE_MAX_SC = 8;     // measured operators

struct SdeParams {
    int32_t n, d, m, ne, nt, rows, sme;
    int32_t occ2;          // complex64 variant held to 2 waves per SIMD (set by sde_choose_variant)
    int32_t WA, WB;       // ELL widths of A and of each B_n
    double cg;
    uint64_t seed;
    int64_t ntraj;
    const int32_t *a_col;  // A in ELL, column-major: entry k of row r at k * n + r
    const void *a_val;     // state precision
    const int32_t *b_col;  // B_n: m blocks of n * WB, column-major within a block
    const void *b_val;
    const int32_t *eptr;   // e_ops CSR (d x d): ne * (d + 1)
    const int32_t *ecol;
    const double2 *eval;
    const int32_t *evidx;  // SME: per e_op entry (i, j), the vec index j*d + i of rho_ji
    const void *x0;        // normalised initial state, state precision
    const double *tlist;
    const int32_t *nsub;   // [nt - 1] steps of each tlist interval
    double2 *expect_tr;    // [ntraj][ne][nt]
    double *meas;          // [ntraj][m][nt - 1]
    int32_t *status;       // [ntraj]
    unsigned long long *queue;
};

size_t sde_lds_bytes(const SdeParams &p, bool f64);
// Sets p.occ2 from the ensemble size and the device's compute-unit count.
void sde_choose_variant(SdeParams &p, bool f64, int device);
int sde_grid(const SdeParams &p, bool f64, int device);
void sde_launch(const SdeParams &p, const SdeParams *dev_p, bool f64, int grid, hipStream_t s);

}  // namespace qt

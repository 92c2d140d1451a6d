// qt_mc.h -- descriptors of the Monte-Carlo wave-function (quantum-jump) solver.
//
// arXiv:2504.21440, Sec. 3.3: each trajectory evolves a pure state under
// H_eff = H - (i/2) sum_k C_k^dag C_k (so dpsi/dt = A psi with A = -i H - 1/2 sum_k C_k^dag C_k),
// jumps when the squared norm falls to a uniform threshold, the channel k drawn with probability
// proportional to |C_k psi|^2, then psi <- C_k psi / |C_k psi| and a new threshold is drawn.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qt {

constexpr int MC_THREADS = 256;
constexpr int MC_MAX_ROWS = 16;  // rows of the state per thread: d <= 4096
constexpr int MC_TAG_SHIFT = 26;
constexpr int MC_MAX_TERMS = 31;

struct CoefDev;

struct McParams {
    int32_t d, W, nc, ne, nt, rows;  // rows = rows per thread (power of two)
    int32_t use_h0, maxj;
    double atol, rtol, h0;
    int64_t max_steps;
    uint64_t seed;
    int64_t ntraj;
    const int32_t *ell_col;  // A in ELL, column-major: entry k of row r at k * d + r
    const void *ell_val;     // state precision
    const int32_t *cptr;     // C_k CSR: nc * (d + 1) row pointers into ccol / cval
    const int32_t *ccol;
    const void *cval;        // state precision
    const int32_t *eptr;     // e_ops CSR: ne * (d + 1)
    const int32_t *ecol;
    const double2 *eval;
    const void *psi0;        // normalised initial state, state precision
    const double *tlist;
    double2 *expect_tr;      // [ntraj][ne][nt]
    int64_t *njumps;         // [ntraj]
    double *jtimes;          // [ntraj][maxj]
    int32_t *jchan;          // [ntraj][maxj]
    int32_t *status;         // [ntraj]
    int64_t *nrhs;           // [ntraj]
    int64_t *naccept;        // [ntraj]
    int64_t *nreject;        // [ntraj]
    unsigned long long *queue;  // next trajectory to start
    // time dependence (nterms = 0: none): A(t) = A_0 + sum_i f_i(t) (-i H_i) + sum_k |g_k(t)|^2 (-1/2 C_k^dag C_k);
    // an ELL entry's column carries its term (0 = constant part) above MC_TAG_SHIFT
    int32_t nterms;
    int32_t pad_td;
    const CoefDev *coefs;     // [nterms]
    const int32_t *cweight;   // [nc]: coefficient (index into coefs) of collapse channel k, -1 for constant
};

// td: the plan has time-dependent terms (the weighted kernel)
void mc_launch(const McParams &p, const McParams *dev_p, bool f64, bool td, int grid, hipStream_t s);
int mc_grid(const McParams &p, bool f64, bool td, int device);
void mc_launch_stats(const double2 *expect_tr, int64_t ntraj, int ne, int nt, double2 *mean, double *se,
                     hipStream_t s);
void mc_launch_queue_reset(unsigned long long *q, hipStream_t s);

}  // namespace qt

// qt_host.h -- host-side runtime types of libqtamd (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qtamd.h"

namespace qt {

using cd = std::complex<double>;

// Error reporting ------------------------------------------------------------------------------
qt_status set_error(qt_status code, const std::string &msg);
#define QT_HIP(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return ::qt::set_error(QT_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Canonical host CSR: square, rows sorted, duplicates summed, exact zeros dropped.
struct HCsr {
    int32_t d = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> idx;
    std::vector<cd> val;
    int64_t nnz() const { return (int64_t)idx.size(); }
};

qt_status csr_from_abi(const qt_csr *A, int32_t d_expect, HCsr *out, const char *what);
HCsr csr_adjoint(const HCsr &A);
HCsr csr_matmul(const HCsr &A, const HCsr &B);
HCsr csr_axpby(cd a, const HCsr &A, cd b, const HCsr &B);
HCsr csr_zero(int32_t d);
// For concatenated e_op CSR rows (ne blocks of d+1 row pointers into col): the vec(rho) index
// j*d + i of rho_ji paired with each entry O_ij, so Tr(O rho) is one gather per entry.
std::vector<int32_t> expect_vec_index(const std::vector<int32_t> &eptr, const std::vector<int32_t> &ecol, int32_t d,
                                      int32_t ne);

// A device arena: one hipMalloc carved into 256-byte aligned pieces, or a caller's device buffer
// (adopt), which the arena never frees.
struct Arena {
    void *base = nullptr;
    size_t size = 0, used = 0;
    bool external = false;
    std::vector<std::pair<size_t, size_t>> plan;  // planned offsets
    size_t reserve(size_t bytes)
    {
        size_t off = (size + 255) & ~size_t(255);
        size = off + bytes;
        return off;
    }
    qt_status alloc();
    // Places the planned layout in the caller's buffer (256-byte aligned, at least `size` bytes).
    qt_status adopt(void *ws, size_t ws_bytes, const char *who);
    // alloc() without a caller buffer, adopt() with one.
    qt_status place(void *ws, size_t ws_bytes, const char *who) { return ws ? adopt(ws, ws_bytes, who) : alloc(); }
    void *at(size_t off) const { return (char *)base + off; }
    void release();
};

struct Ctx {
    int32_t device = 0;
    hipStream_t stream = nullptr;
    hipStream_t aux = nullptr;  // second stream for overlapping independent work
    static constexpr int NPOOL = 4;
    hipStream_t pool[NPOOL] = {};  // streams for concurrent dense-size buckets
    bool own_stream = false;
    int refs = 0;  // live Liouvillians, plans and servers created on this context
};

struct Liouv {
    Ctx *ctx = nullptr;
    int32_t form = QT_FORM_CSR;
    int32_t precision = QT_F64;
    int32_t d = 0;
    int64_t nnz = 0;         // entries of L (CSR form)
    int64_t nnz_stored = 0;  // stored entries: every row padded to a multiple of 4 with zeros
    int64_t bytes = 0;
    int32_t nc = 0;
    // CSR form
    int32_t *rowptr = nullptr;
    int32_t *col = nullptr;
    void *val = nullptr;
    // dense form: A then C_k, each d x d row-major, in the solve precision; bit k of dense_creal
    // set when C_k is real
    void *dense = nullptr;
    uint32_t dense_creal = 0;
    // time dependence (CSR form): column tags 1..nterms select the coefficient of each entry
    int32_t nterms = 0;
    void *coefs = nullptr;  // device: CoefDev[nterms] followed by their sample tables
    // host copies needed by the Monte-Carlo path and by the server footprint estimate
};

// Time-dependent coefficients: validation of a qt_coef (QT_COEF_NONE accepted when allow_none) and
// its device descriptor (table pointer left null for the caller to place).
struct CoefDev;
qt_status check_coef(const qt_coef &c, bool allow_none, const char *what);
CoefDev coef_from_abi(const qt_coef &c, int modsq);

// Kernel launchers (defined in the .hip files)
struct CsrInst;
struct CsrCtl;
int csr_rows_per_block(int lpr, int rg);
bool csr_shape_supported(int lpr, int rg);
// A tile shape with a matrix load kind: keep 0 streamed, 1 through the caches, 2 through the caches
// with 16-byte loads of 4-entry runs (built for 4x1, 8x1, 8x2 and 16x1).
bool csr_shape_supported(int lpr, int rg, int keep);
// One launch configuration of the CSR step kernels.
struct CsrLaunch {
    bool f64 = false;
    int lpr = 8, rg = 1, xcd = 0;  // tile shape and block order
    int keep = 0;                  // matrix loads: 0 streamed, 1 through the caches, 2 as 1 with 16-byte loads
    int nblk = 0, ninst = 0;       // workgroups, problems
    const CsrInst *insts = nullptr;
    CsrCtl *ctls = nullptr;
    const int32_t *bi = nullptr, *br = nullptr;  // block table: problem, first row
    const int32_t *ilist = nullptr;              // problems the control launch visits (null: 0..ninst-1)
    // Device-side fill of a table sized for a capacity (null: nblk / ninst are exact): blocks at or
    // past bound[0] and control workgroups at or past ibound[0] return at once, so a graph captured
    // for the capacity stays valid while the table contents change.
    const int32_t *bound = nullptr, *ibound = nullptr;
    const CsrInst *one_host = nullptr;           // host copy of the descriptor when ninst == 1
    bool td = false;  // some problem has a time-dependent Liouvillian: the SpMV kernels weight its terms
    // One problem with runs of 4 stored entries and no steady-state test: the step control
    // is folded into the next step's stage-2 launch (csr_launch_step).
    bool fused = false;
};
// Resets the control records (and the coefficient rows of problems that have them).
void csr_launch_reset(const CsrInst *insts, CsrCtl *ctls, int ninst, bool f64, hipStream_t s);
void csr_launch_init(int which, const CsrLaunch &L, hipStream_t s);
// One DP5 step: stages 2..7 and the control launch, or, with L.fused and the step's index j within
// its graph (j >= 0), stage 2 with the previous step's control folded in and stages 3..7 (the
// control record double-buffered in L.ctls[0..1]; an even number of steps ends in L.ctls[0]).
void csr_launch_step(const CsrLaunch &L, hipStream_t s, int j = -1);
void csr_launch_stage3(const CsrLaunch &L, hipStream_t s);
constexpr int CSR_MIN_ROWS_PER_BLOCK = 16;  // smallest tile (16 lanes per row, one row per group)
// Looks up the device address of the allocation-free scratch array on `device` (current).
qt_status noalloc_init_device(int32_t device);
void launch_expect(bool f64, int d, const int32_t *rp, const int32_t *ci, const double2 *v, const void *state,
                   int is_ket, double2 *out, hipStream_t s);


}  // namespace qt

struct qt_ctx : qt::Ctx {};
struct qt_liouv : qt::Liouv {};

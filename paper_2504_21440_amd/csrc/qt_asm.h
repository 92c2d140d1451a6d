// qt_asm.h -- operand descriptor of the device Liouvillian assembly (kernels_assembly.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qt {

// Operands of  L = A (x) I + I (x) conj(B) + sum_k C_k (x) conj(C_k), i.e. L rho = A rho + rho B^dag
// + sum_k C_k rho C_k^dag, as int32 CSR on the device.  The master-equation generator takes
// B = A = -i H - 1/2 sum_k C_k^dag C_k; a Hamiltonian term -i(H rho - rho H) of a time-dependent
// problem takes A = -i H, B = -i H^dag and no C_k.
struct AsmOps {
    int d;
    int nc;
    const int32_t *arp;  // A row pointers, d + 1
    const int32_t *aci;
    const double2 *av;
    const int32_t *crp;  // C_k row pointers, nc * (d + 1), offsets into cci / cv
    const int32_t *cci;
    const double2 *cv;
    const int32_t *brp;  // B (null: B = A)
    const int32_t *bci;
    const double2 *bv;
};

// One term of a time-dependent Liouvillian, already assembled (solve precision values).
struct TdTerm {
    const int32_t *rp;
    const int32_t *ci;
    const void *v;
};

// counts[r]: stored entries of row r, padded to a multiple of 4; *real (device) accumulates the
// entries that are not padding.
void asm_launch_count(const AsmOps &op, int32_t *counts, int *flags, unsigned long long *real, bool f64,
                      hipStream_t s);
void asm_launch_scan(const int32_t *counts, int64_t n, int64_t *bsum, int32_t *rowptr, int *flags, hipStream_t s);
void asm_launch_fill(const AsmOps &op, const int32_t *rowptr, int32_t *col, void *val, bool f64, hipStream_t s);
// Concatenate the rows of nt assembled terms (device array `terms`) into one CSR whose column
// indices carry the term number above TD_TAG_SHIFT.  rowptr[r] is the sum of the terms' row
// pointers; rowptr[n] is written from the terms' totals.
void asm_launch_td_merge(const TdTerm *terms, int nt, int64_t n, int32_t *rowptr, int32_t *col, void *val,
                         bool f64, hipStream_t s);

}  // namespace qt

// qt_asm.h -- operand descriptor of the device Liouvillian assembly (kernels_assembly.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qt {

// A = -i H - 1/2 sum_k C_k^dag C_k and the collapse operators C_k, as int32 CSR on the device.
struct AsmOps {
    int d;
    int nc;
    const int32_t *arp;  // A row pointers, d + 1
    const int32_t *aci;
    const double2 *av;
    const int32_t *crp;  // C_k row pointers, nc * (d + 1), offsets into cci / cv
    const int32_t *cci;
    const double2 *cv;
};

void asm_launch_count(const AsmOps &op, int32_t *counts, int *flags, hipStream_t s);
void asm_launch_scan(const int32_t *counts, int64_t n, int64_t *bsum, int32_t *rowptr, int *flags, hipStream_t s);
void asm_launch_fill(const AsmOps &op, const int32_t *rowptr, int32_t *col, void *val, bool f64, hipStream_t s);

}  // namespace qt

// kernels_assembly.hip -- device assembly of the CSR Liouvillian superoperator.
//
// For the row-major vectorisation vec(rho)[i*d + j] = rho_ij one has vec(X rho Y) = (X kron Y^T)
// vec(rho), so the master-equation generator (arXiv:2504.21440, Sec. 3.2) is
//     L = A kron I + I kron conj(A) + sum_k C_k kron conj(C_k),   A = -i H - 1/2 sum_k C_k^dag C_k.
// Row (i, j) of L therefore collects
//     A_ik at column (k, j),  conj(A_jl) at column (i, l),  C_ip conj(C_jq) at column (p, q).
// (A Hamiltonian term of a time-dependent problem uses a second operator B in the place of the
// right-hand A; see qt_asm.h.)
// Each thread builds one row: it gathers these candidates, sorts them by column, sums duplicates
// and drops entries that are zero in the storage precision.  A count pass, a three-kernel scan and
// a fill pass produce CSR directly in device memory, values computed in FP64 and stored in the
// solve precision.  Every row is padded to a multiple of 4 stored entries with explicit zeros
// (column = the row itself), so each row starts 16-byte aligned in the column array and the SpMV
// can load runs of 4 entries at once; every stored zero is padding.
#include "qt_common.h"
#include "qt_asm.h"
#include "qt_csr.h"

namespace qt {

constexpr int ASM_MAXC = 128;  // candidates per Liouvillian row handled by the device builder


// Insert (c, v) into the sorted candidate list, summing a duplicate column.
__device__ __forceinline__ void cand_insert(int *cols, double2 *vals, int &n, int c, double2 v, int *overflow)
{
    int pos = n;
    while (pos > 0 && cols[pos - 1] > c) --pos;
    if (pos > 0 && cols[pos - 1] == c) {
        vals[pos - 1].x += v.x;
        vals[pos - 1].y += v.y;
        return;
    }
    if (n >= ASM_MAXC) {
        *overflow = 1;
        return;
    }
    for (int m = n; m > pos; --m) {
        cols[m] = cols[m - 1];
        vals[m] = vals[m - 1];
    }
    cols[pos] = c;
    vals[pos] = v;
    ++n;
}

__device__ int build_row(const AsmOps &op, int64_t r, int *cols, double2 *vals, int *overflow)
{
    const int d = op.d;
    const int i = (int)(r / d), j = (int)(r % d);
    int n = 0;
    for (int p = op.arp[i]; p < op.arp[i + 1]; ++p) cand_insert(cols, vals, n, op.aci[p] * d + j, op.av[p], overflow);
    const int32_t *brp = op.brp ? op.brp : op.arp, *bci = op.brp ? op.bci : op.aci;
    const double2 *bv = op.brp ? op.bv : op.av;
    for (int p = brp[j]; p < brp[j + 1]; ++p) {
        const double2 b = bv[p];
        cand_insert(cols, vals, n, i * d + bci[p], make_double2(b.x, -b.y), overflow);
    }
    for (int k = 0; k < op.nc; ++k) {
        const int32_t *rp = op.crp + (size_t)k * (d + 1);
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const double2 ci = op.cv[p];
            for (int q = rp[j]; q < rp[j + 1]; ++q) {
                const double2 cj = op.cv[q];
                // C_ip * conj(C_jq)
                const double2 v = make_double2(ci.x * cj.x + ci.y * cj.y, ci.y * cj.x - ci.x * cj.y);
                cand_insert(cols, vals, n, op.cci[p] * d + op.cci[q], v, overflow);
            }
        }
    }
    return n;
}

// A candidate value survives when it is nonzero in the storage precision.
__device__ __forceinline__ bool stored_nonzero(double2 v, bool f64)
{
    return f64 ? (v.x != 0.0 || v.y != 0.0) : ((float)v.x != 0.0f || (float)v.y != 0.0f);
}

// counts[r]: stored entries of row r (padded to a multiple of 4); real[0] += the entries that are
// not padding.
__global__ __launch_bounds__(128) void k_asm_count(AsmOps op, int32_t *counts, int *flags,
                                                   unsigned long long *real, int f64)
{
    const int64_t n = (int64_t)op.d * op.d;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int cnt = 0;
    if (r < n) {
        int cols[ASM_MAXC];
        double2 vals[ASM_MAXC];
        int ovf = 0;
        const int m = build_row(op, r, cols, vals, &ovf);
        for (int k = 0; k < m; ++k) cnt += stored_nonzero(vals[k], f64 != 0);
        counts[r] = (cnt + 3) & ~3;
        if (ovf) atomicOr(&flags[0], 1);
    }
    const int tot = wave_sum(cnt);
    if ((threadIdx.x & 63) == 0 && tot) atomicAdd(real, (unsigned long long)tot);
}

template <typename V>
__global__ __launch_bounds__(128) void k_asm_fill(AsmOps op, const int32_t *rowptr, int32_t *col, V *val)
{
    const int64_t n = (int64_t)op.d * op.d;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int cols[ASM_MAXC];
    double2 vals[ASM_MAXC];
    int ovf = 0;
    const int m = build_row(op, r, cols, vals, &ovf);
    int o = rowptr[r];
    for (int k = 0; k < m; ++k) {
        if (!stored_nonzero(vals[k], sizeof(V) == 16)) continue;
        col[o] = cols[k];
        val[o] = from_d2<V>(vals[k]);
        ++o;
    }
    for (const int e = rowptr[r + 1]; o < e; ++o) {  // padding: explicit zeros in this row's own column
        col[o] = (int32_t)r;
        val[o] = from_d2<V>(make_double2(0.0, 0.0));
    }
}

// ---- time-dependent terms: one CSR with the term number in the column's high bits ----
template <typename V>
__global__ __launch_bounds__(128) void k_td_merge(const TdTerm *__restrict__ terms, int nt, int64_t n,
                                                  int32_t *__restrict__ rowptr, int32_t *__restrict__ col,
                                                  V *__restrict__ val)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > n) return;
    int32_t o = 0;
    for (int k = 0; k < nt; ++k) o += terms[k].rp[r];
    rowptr[r] = o;
    if (r == n) return;
    for (int k = 0; k < nt; ++k) {
        const TdTerm t = terms[k];
        const V *tv = (const V *)t.v;
        for (int32_t p = t.rp[r]; p < t.rp[r + 1]; ++p) {
            col[o] = t.ci[p] | (k << TD_TAG_SHIFT);
            val[o] = tv[p];
            ++o;
        }
    }
}

void asm_launch_td_merge(const TdTerm *terms, int nt, int64_t n, int32_t *rowptr, int32_t *col, void *val,
                         bool f64, hipStream_t s)
{
    const dim3 g((unsigned)((n + 1 + 127) / 128)), t(128);
    if (f64) hipLaunchKernelGGL(k_td_merge<double2>, g, t, 0, s, terms, nt, n, rowptr, col, (double2 *)val);
    else hipLaunchKernelGGL(k_td_merge<float2>, g, t, 0, s, terms, nt, n, rowptr, col, (float2 *)val);
}

// ---- exclusive scan of int32 counts into int32 row pointers (total checked against 2^31) ----
constexpr int SCAN_B = 1024;

__global__ __launch_bounds__(SCAN_B) void k_scan_sums(const int32_t *counts, int64_t n, int64_t *bsum)
{
    __shared__ double scr[16];
    const int64_t i = (int64_t)blockIdx.x * SCAN_B + threadIdx.x;
    const double v = (i < n) ? (double)counts[i] : 0.0;  // exact: partial sums < 2^53
    const double s = block_sum(v, scr);
    if (threadIdx.x == 0) bsum[blockIdx.x] = (int64_t)s;
}

__global__ __launch_bounds__(SCAN_B) void k_scan_top(int64_t *bsum, int64_t nb, int32_t *rowptr, int64_t n,
                                                     int *flags)
{
    __shared__ int64_t sh[SCAN_B];
    int64_t carry = 0;
    for (int64_t base = 0; base < nb; base += SCAN_B) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = (i < nb) ? bsum[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < SCAN_B; off <<= 1) {
            const int64_t t = (threadIdx.x >= off) ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb) bsum[i] = carry + sh[threadIdx.x] - v;  // exclusive
        const int64_t tot = sh[SCAN_B - 1];
        __syncthreads();
        carry += tot;
    }
    if (threadIdx.x == 0) {
        if (carry >= 2147483647LL) flags[1] = 1;
        rowptr[n] = (int32_t)carry;
    }
}

__global__ __launch_bounds__(SCAN_B) void k_scan_apply(const int32_t *counts, int64_t n, const int64_t *boff,
                                                       int32_t *rowptr)
{
    __shared__ int32_t sh[SCAN_B];
    const int64_t i = (int64_t)blockIdx.x * SCAN_B + threadIdx.x;
    const int32_t v = (i < n) ? counts[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_B; off <<= 1) {
        const int32_t t = (threadIdx.x >= off) ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) rowptr[i] = (int32_t)(boff[blockIdx.x] + sh[threadIdx.x] - v);
}

// Host launchers ------------------------------------------------------------------------------
void asm_launch_count(const AsmOps &op, int32_t *counts, int *flags, unsigned long long *real, bool f64,
                      hipStream_t s)
{
    const int64_t n = (int64_t)op.d * op.d;
    hipLaunchKernelGGL(k_asm_count, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, op, counts, flags, real,
                       (int)f64);
}

void asm_launch_scan(const int32_t *counts, int64_t n, int64_t *bsum, int32_t *rowptr, int *flags, hipStream_t s)
{
    const int64_t nb = (n + SCAN_B - 1) / SCAN_B;
    hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(SCAN_B), 0, s, counts, n, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_B), 0, s, bsum, nb, rowptr, n, flags);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SCAN_B), 0, s, counts, n, bsum, rowptr);
}

void asm_launch_fill(const AsmOps &op, const int32_t *rowptr, int32_t *col, void *val, bool f64, hipStream_t s)
{
    const int64_t n = (int64_t)op.d * op.d;
    const dim3 g((unsigned)((n + 127) / 128)), t(128);
    if (f64) hipLaunchKernelGGL(k_asm_fill<double2>, g, t, 0, s, op, rowptr, col, (double2 *)val);
    else hipLaunchKernelGGL(k_asm_fill<float2>, g, t, 0, s, op, rowptr, col, (float2 *)val);
}

}  // namespace qt

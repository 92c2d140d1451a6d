// csr_kernels.h -- device code of the CSR-form solver and its launch plumbing, shared by the
// constant-Liouvillian kernels (kernels_csr.hip) and the time-dependent ones (kernels_csr_td.hip),
// which are compiled as separate translation units.  What the kernels do is described at the top
// of kernels_csr.hip.
#pragma once
#include <cstring>

#include "qt_coef.h"
#include "qt_common.h"
#include "qt_csr.h"
#include "qt_host.h"

namespace qt {


constexpr int CSR_THREADS = 256;
constexpr int CTL_THREADS = 512;  // 8 waves: one expectation operator per wave for up to 8 e_ops
constexpr int CTL_MAX_EOPS = 64;  // operators whose sums the control kernel holds in LDS
enum : int32_t { PH_STEP = 0, PH_INIT1 = 1, PH_INIT0 = 2 };

template <int LPR, int RG> struct CsrGeom {
    static constexpr int RPW = 64 / LPR;                  // lane groups per wave
    static constexpr int GPB = (CSR_THREADS / 64) * RPW;  // lane groups per block
    static constexpr int RPB = GPB * RG;                  // rows per block
    static constexpr int U = (LPR >= 8) ? 4 : (LPR == 4 ? 6 : 8);  // non-zeros per row in flight per lane
};

template <typename V> __device__ __forceinline__ V shfl_xor_c(V v, int m)
{
    v.x = __shfl_xor(v.x, m, 64);
    v.y = __shfl_xor(v.y, m, 64);
    return v;
}

typedef float nf2 __attribute__((ext_vector_type(2)));
typedef double nd2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld_stream(const float2 *p)
{
    const nf2 v = __builtin_nontemporal_load((const nf2 *)p);
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ double2 ld_stream(const double2 *p)
{
    const nd2 v = __builtin_nontemporal_load((const nd2 *)p);
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ int32_t ld_stream(const int32_t *p) { return __builtin_nontemporal_load(p); }

// Logical block index of this workgroup (see "Block order" above).
__device__ __forceinline__ int csr_block(int xcd)
{
    const int b = blockIdx.x;
    if (!xcd) return b;
    const int n = gridDim.x, q = n >> 3, r = n & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

// Row bounds of the RG rows r0 + g * stride (g < RG) of this lane's group.
template <int RG> struct RowBounds {
    int s[RG], e[RG];
};
template <int RG>
__device__ __forceinline__ RowBounds<RG> csr_bounds(const int32_t *__restrict__ rowptr, int r0, int stride, int n)
{
    RowBounds<RG> b;
#pragma unroll
    for (int g = 0; g < RG; ++g) {
        const int r = r0 + g * stride;
        const bool ok = r < n;
        b.s[g] = ok ? rowptr[r] : 0;
        b.e[g] = ok ? rowptr[r + 1] : 0;
    }
    return b;
}

// Row sums  sum_k val[k] * x(col[k])  over the bounds from csr_bounds; every lane of the group
// returns all RG sums.  X returns the (stage) input at a column.  TD: the Liouvillian is a sum of
// terms whose column indices carry the term number above TD_TAG_SHIFT; entry k is weighted by the
// term's coefficient cw[term] at this evaluation's time (cw[0] = 1 for the constant part).
template <typename V, int LPR, int RG, bool KEEP, bool TD, typename X>
__device__ __forceinline__ void csr_rows(const RowBounds<RG> &b, const int32_t *__restrict__ col,
                                         const V *__restrict__ val, int q, X x, V (&acc)[RG],
                                         const V *__restrict__ cw = nullptr)
{
    constexpr int U = CsrGeom<LPR, RG>::U;
#pragma unroll
    for (int g = 0; g < RG; ++g) {
        acc[g].x = 0;
        acc[g].y = 0;
    }
    for (int base = q;; base += LPR * U) {
        int cc[RG][U];
        V vv[RG][U];
        bool any = false;
#pragma unroll
        for (int g = 0; g < RG; ++g)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = b.s[g] + base + u * LPR;
                if (k < b.e[g]) {
                    cc[g][u] = KEEP ? col[k] : ld_stream(col + k);
                    vv[g][u] = KEEP ? val[k] : ld_stream(val + k);
                    any = true;
                } else {
                    cc[g][u] = -1;
                }
            }
        if (!any) break;
#pragma unroll
        for (int g = 0; g < RG; ++g)
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (cc[g][u] >= 0) {
                    if constexpr (TD) {
                        const int c = cc[g][u] & TD_COL_MASK;
                        cfma(acc[g], cmul(vv[g][u], cw[cc[g][u] >> TD_TAG_SHIFT]), x(c));
                    } else {
                        cfma(acc[g], vv[g][u], x(cc[g][u]));
                    }
                }
    }
#pragma unroll
    for (int g = 0; g < RG; ++g)
#pragma unroll
        for (int m = LPR / 2; m >= 1; m >>= 1) acc[g] = cadd(acc[g], shfl_xor_c(acc[g], m));
}

// Tile shapes built with 16-byte matrix loads (cached_matrix = 2).
template <int LPR, int RG> constexpr bool csr_wide_shape()
{
    return (LPR == 4 && RG == 1) || (LPR == 8 && (RG == 1 || RG == 2)) || (LPR == 16 && RG == 1);
}

typedef int32_t ci4 __attribute__((ext_vector_type(4)));
typedef float cf4 __attribute__((ext_vector_type(4)));
// Four consecutive stored values (k a multiple of 4: 32- / 64-byte aligned).
__device__ __forceinline__ void ld_quad(const float2 *__restrict__ p, float2 (&v)[4])
{
    const cf4 a = *(const cf4 *)p, b = *(const cf4 *)(p + 2);
    v[0] = make_float2(a.x, a.y);
    v[1] = make_float2(a.z, a.w);
    v[2] = make_float2(b.x, b.y);
    v[3] = make_float2(b.z, b.w);
}
__device__ __forceinline__ void ld_quad(const double2 *__restrict__ p, double2 (&v)[4])
{
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = p[j];
}

// Row sums as csr_rows, with each lane taking runs of 4 consecutive stored entries: one 16-byte
// load of the column indices and 16-byte loads of the values.  Needs rows padded to multiples of 4
// stored entries (every CSR Liouvillian is).  Matrix loads go through the caches.
template <typename V, int LPR, int RG, bool TD, typename X>
__device__ __forceinline__ void csr_rows4(const RowBounds<RG> &b, const int32_t *__restrict__ col,
                                          const V *__restrict__ val, int q, X x, V (&acc)[RG],
                                          const V *__restrict__ cw = nullptr)
{
    constexpr int U = LPR >= 8 ? 1 : 2;  // runs of 4 per row in flight per lane
#pragma unroll
    for (int g = 0; g < RG; ++g) {
        acc[g].x = 0;
        acc[g].y = 0;
    }
    for (int base = 4 * q;; base += 4 * LPR * U) {
        ci4 cc[RG][U];
        V vv[RG][U][4];
        bool ok[RG][U];
        bool any = false;
#pragma unroll
        for (int g = 0; g < RG; ++g)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = b.s[g] + base + u * 4 * LPR;
                ok[g][u] = k < b.e[g];
                if (ok[g][u]) {
                    cc[g][u] = *(const ci4 *)(col + k);
                    ld_quad(val + k, vv[g][u]);
                    any = true;
                }
            }
        if (!any) break;
#pragma unroll
        for (int g = 0; g < RG; ++g)
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (ok[g][u]) {
                    const int cs[4] = {cc[g][u].x, cc[g][u].y, cc[g][u].z, cc[g][u].w};
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        if constexpr (TD)
                            cfma(acc[g], cmul(vv[g][u][j], cw[cs[j] >> TD_TAG_SHIFT]), x(cs[j] & TD_COL_MASK));
                        else
                            cfma(acc[g], vv[g][u][j], x(cs[j]));
                    }
                }
    }
#pragma unroll
    for (int g = 0; g < RG; ++g)
#pragma unroll
        for (int m = LPR / 2; m >= 1; m >>= 1) acc[g] = cadd(acc[g], shfl_xor_c(acc[g], m));
}

// Row sums with the kernel's matrix load kind.
template <typename V, int LPR, int RG, bool KEEP, bool WIDE, bool TD, typename X>
__device__ __forceinline__ void csr_rows_k(const RowBounds<RG> &b, const int32_t *__restrict__ col,
                                           const V *__restrict__ val, int q, X x, V (&acc)[RG],
                                           const V *__restrict__ cw = nullptr)
{
    if constexpr (WIDE) csr_rows4<V, LPR, RG, TD>(b, col, val, q, x, acc, cw);
    else csr_rows<V, LPR, RG, KEEP, TD>(b, col, val, q, x, acc, cw);
}

// acc[q] without dynamic register indexing
template <typename V, int RG> __device__ __forceinline__ V pick(const V (&a)[RG], int q)
{
    V r = a[0];
#pragma unroll
    for (int g = 1; g < RG; ++g)
        if (q == g) r = a[g];
    return r;
}

// Tr(O_k Y) for operator k, accumulated in FP64 by one wave: Tr(O rho) = sum_{(i,j) in nnz(O)}
// O_ij rho_ji, one gather per entry through evidx, reduced with shuffles in a fixed order.
template <typename V>
__device__ __forceinline__ double2 csr_expect_range(const CsrInst &I, const V *__restrict__ Y, int b, int e)
{
    const int lane = threadIdx.x & 63;
    double sr = 0.0, si = 0.0;
#pragma unroll 4
    for (int p = b + lane; p < e; p += 64) {
        const double2 o = I.eval[p];
        const double2 r = to_d2(Y[I.evidx[p]]);
        sr += o.x * r.x - o.y * r.y;
        si += o.x * r.y + o.y * r.x;
    }
    return make_double2(wave_sum(sr), wave_sum(si));
}

template <typename V>
__device__ __forceinline__ double2 csr_expect_one(const CsrInst &I, const V *__restrict__ Y, int k)
{
    const int32_t *ep = I.eptr + (size_t)k * (I.d + 1);
    return csr_expect_range(I, Y, ep[0], ep[I.d]);
}

// Expectation values of the state Y (times `scale`) into expect[k][idx]: one wave per operator,
// the waves of the block taking the operators in turn, so no block barrier sits between them.
template <typename V>
__device__ void csr_record_expect(const CsrInst &I, const V *__restrict__ Y, double scale, int idx)
{
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int k = threadIdx.x >> 6; k < I.ne; k += nw) {
        const double2 s = csr_expect_one(I, Y, k);
        if (lane == 0) I.expect[(size_t)k * I.nt + idx] = make_double2(s.x * scale, s.y * scale);
    }
}

// This thread's share of Tr(Y) (real part), to be block-summed.
template <typename V> __device__ __forceinline__ double csr_trace_part(const CsrInst &I, const V *__restrict__ Y)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < I.d; i += blockDim.x) s += (double)Y[(size_t)i * I.d + i].x;
    return s;
}

template <typename V> __device__ double csr_trace(const CsrInst &I, const V *__restrict__ Y, double *scr)
{
    return block_sum(csr_trace_part(I, Y), scr);
}

// Thread v's share of one partial column over the instance's blocks, as a block of T threads forms
// it, in a fixed order: eight loads in flight per thread, then the strided tail.
__device__ __forceinline__ double partials_part_at(const CsrInst &I, int col, int v, int T)
{
    const int nb = I.nblocks;
    const double *__restrict__ P = I.partials + col;
    double t = 0.0;
    int k = v;
    for (; k + 7 * T < nb; k += 8 * T) {
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = P[2 * (k + u * T)];
#pragma unroll
        for (int u = 0; u < 8; ++u) t += a[u];
    }
    for (; k < nb; k += T) t += P[2 * k];
    return t;
}

// This thread's share in the calling block's own order.
__device__ __forceinline__ double partials_part(const CsrInst &I, int col)
{
    return partials_part_at(I, col, threadIdx.x, blockDim.x);
}

// The step control's two FP64 sums -- the error partials (column 0) and the trace of the candidate
// y_new (when the problem renormalises) -- formed in a CSR_THREADS block exactly as a CTL_THREADS
// control block forms them with block_sum_n: each thread takes the virtual threads t and
// t + CSR_THREADS of the larger block, each virtual wave is reduced with the same butterfly by the
// physical wave holding its lanes, and the virtual waves' sums are added in order.  So a stage
// kernel that takes the decision reaches the control kernel's result bitwise.  Every thread of the
// block receives both sums; scratch: >= 32 doubles of LDS.
template <typename V>
__device__ __forceinline__ void ctl_step_sums(const CsrInst &I, const V *__restrict__ ynew, double &err_sum,
                                              double &tr_sum, double *scratch)
{
    static_assert(CTL_THREADS % CSR_THREADS == 0 && CTL_THREADS / 64 <= 16, "virtual control block");
    constexpr int NV = CTL_THREADS / CSR_THREADS, PW = CSR_THREADS / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double e[NV], t[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const int v = threadIdx.x + j * CSR_THREADS;
        e[j] = partials_part_at(I, 0, v, CTL_THREADS);
        double trp = 0.0;
        if (I.renorm) {
            if (v < I.d) trp += (double)ynew[(size_t)v * (I.d + 1)].x;
            for (int i = v + CTL_THREADS; i < I.d; i += CTL_THREADS) trp += (double)ynew[(size_t)i * I.d + i].x;
        }
        t[j] = wave_sum(trp);
        e[j] = wave_sum(e[j]);
    }
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            scratch[w + j * PW] = e[j];
            scratch[16 + w + j * PW] = t[j];
        }
    }
    __syncthreads();
    double se = 0.0, st = 0.0;
    for (int i = 0; i < CTL_THREADS / 64; ++i) se += scratch[i];
    for (int i = 0; i < CTL_THREADS / 64; ++i) st += scratch[16 + i];
    err_sum = se;
    tr_sum = st;
    __syncthreads();
}

__device__ __forceinline__ double sum_partials(const CsrInst &I, int col, double *scr)
{
    return block_sum(partials_part(I, col), scr);
}

// Coefficient row of one evaluation of a time-dependent problem (slot 0: first starting-step
// evaluation, 1: second, S: Runge-Kutta stage S), written by the control and reset kernels.
template <typename V, bool TD> __device__ __forceinline__ const V *td_coefs(const CsrInst &I, int slot)
{
    if constexpr (TD) return (const V *)I.cstage + (size_t)slot * (I.nterms + 1);
    else return nullptr;
}

// Coefficient rows first..last of a time-dependent problem, by every thread of the block: row 1 at
// t + h (the second starting-step evaluation, h = h0), row S = 2..7 at t + c_S h (Runge-Kutta stage
// S); column 0 is the constant part.  The time of each evaluation is formed exactly as the
// integrator defines it, so the coefficients match the stage the SpMV kernel evaluates.
template <typename V>
__device__ void td_rows(const CsrInst &I, int first, int last, double t, double h, int tid, int nthr)
{
    const int nt = I.nterms, cols = nt + 1;
    const int total = (last - first + 1) * cols;
    for (int idx = tid; idx < total; idx += nthr) {
        const int slot = first + idx / cols, k = idx % cols;
        const double c = slot <= 1 ? (double)slot
                                   : slot == 2 ? DP5::c2
                                               : slot == 3 ? DP5::c3 : slot == 4 ? DP5::c4 : slot == 5 ? DP5::c5 : 1.0;
        double2 w = make_double2(1.0, 0.0);
        if (k > 0) w = coef_value(I.coefs[k - 1], t + c * h);
        ((V *)I.cstage)[(size_t)slot * cols + k] = from_d2<V>(w);
    }
}

// The step decision after stage 7: the new control record from the one the step ran with (c), its
// error norm, whether it is accepted, the trace scale of the accepted state, steady-state
// convergence, and the save times it may land on (t_save: the next one, t_after: the one after).
// Taken by one thread, in the control kernel or in a stage-2 kernel that folds the control in.
__device__ __forceinline__ CsrCtl step_record(const CsrInst &I, const CsrCtl &c, double err, bool accept,
                                              double scale_new, bool conv, bool steady, double t_save,
                                              double t_after)
{
    const double h = c.h_try;
    const int sidx = c.save_idx;
    CsrCtl n = c;
    n.n_steps += 1;
    n.n_rhs += 6;
    if (!isfinite(err)) {
        n.status = 6;  // QT_ENONFINITE
    } else if (accept) {
        n.n_accept += 1;
        n.t = c.land ? t_save : c.t + h;
        n.parity = 1 - c.parity;
        double hn = h * pi_factor(err, c.err_prev);
        if (c.last_rejected && hn > h) hn = h;
        n.h = hn;
        n.err_prev = fmax(err, 1e-4);
        n.last_rejected = 0;
        n.scale = scale_new;
        if (conv) {
            n.save_idx = I.nt;
            n.status = ST_DONE;
        } else if (c.land) {
            n.save_idx = sidx + 1;
            // in steady-state mode, passing the last save time unconverged is a failure
            if (sidx + 1 >= I.nt) n.status = steady ? 4 : ST_DONE;  // QT_EMAXSTEPS
        }
    } else {
        n.n_reject += 1;
        n.h = h * reject_factor(err);
        n.last_rejected = 1;
    }
    n.last_err = err;
    if (n.status == ST_RUNNING) {
        if (n.n_steps >= I.max_steps) {
            n.status = 4;  // QT_EMAXSTEPS
        } else if (n.h < 1e-14 * fmax(1.0, fabs(n.t))) {
            n.status = 5;  // QT_EDTMIN
        } else {
            int32_t l2;
            n.h_try = clip_step(n.t, n.h, n.save_idx == sidx ? t_save : t_after, &l2);
            n.land = l2;
        }
    }
    return n;
}

// Per-block row geometry shared by the SpMV kernels.
template <int LPR, int RG> struct RowSlot {
    int q, r0, row;
    bool valid;
    __device__ __forceinline__ RowSlot(int blk_row0, int n)
    {
        using G = CsrGeom<LPR, RG>;
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        q = lane % LPR;
        r0 = blk_row0 + w * G::RPW + lane / LPR;
        row = r0 + q * G::GPB;  // the row whose epilogue this lane runs (q < RG)
        valid = q < RG && row < n;
    }
};

// ---------------------------------------------------------------------------------------------
// Per-block bodies.  I: the problem's descriptor; C: its control record; row0: first row of the
// block; part: the block's index among the problem's blocks (its slot in I.partials).
// ---------------------------------------------------------------------------------------------

// Starting step, first evaluation: k1 = L rho0, y <- rho0, partials of |y|^2/sc^2 and |f(y)|^2/sc^2.
template <typename T, int LPR, int RG, bool KEEP, bool WIDE, bool TD>
__device__ __forceinline__ void init0_body(const CsrInst &I, const CsrCtl *C, int row0, int part)
{
    using V = typename vec2<T>::type;
    using G = CsrGeom<LPR, RG>;
    __shared__ double scr[16];
    const RowSlot<LPR, RG> rs(row0, I.n);
    const RowBounds<RG> rb = csr_bounds<RG>(I.rowptr, rs.r0, G::GPB, I.n);
    if (C->status != ST_RUNNING || C->phase != PH_INIT0) return;
    const V *__restrict__ x0 = (const V *)I.rho0;
    V acc[RG];
    csr_rows_k<V, LPR, RG, KEEP, WIDE, TD>(rb, I.col, (const V *)I.val, rs.q, [&](int c) { return x0[c]; }, acc,
                                   td_coefs<V, TD>(I, 0));
    double sa = 0.0, sb = 0.0;
    if (rs.valid) {
        const V a = pick(acc, rs.q);
        const V y = x0[rs.row];
        ((V *)I.K[0])[rs.row] = a;
        ((V *)I.Y[0])[rs.row] = y;
        const double sc = I.atol + I.rtol * sqrt(abs2d(y));
        sa = abs2d(y) / (sc * sc);
        sb = abs2d(a) / (sc * sc);
    }
    sa = block_sum(sa, scr);
    sb = block_sum(sb, scr);
    if (threadIdx.x == 0) {
        I.partials[2 * part] = sa;
        I.partials[2 * part + 1] = sb;
    }
}

// Starting step, second evaluation: partials of |f(y + h0 f(y)) - f(y)|^2 / (h0 sc)^2.
template <typename T, int LPR, int RG, bool KEEP, bool WIDE, bool TD>
__device__ __forceinline__ void init1_body(const CsrInst &I, const CsrCtl *C, int row0, int part)
{
    using V = typename vec2<T>::type;
    using G = CsrGeom<LPR, RG>;
    __shared__ double scr[16];
    const RowSlot<LPR, RG> rs(row0, I.n);
    const RowBounds<RG> rb = csr_bounds<RG>(I.rowptr, rs.r0, G::GPB, I.n);
    if (C->status != ST_RUNNING || C->phase != PH_INIT1) return;
    const double h0 = C->h0;
    const T th0 = (T)h0;
    const V *__restrict__ y = (const V *)I.Y[0];
    const V *__restrict__ k1 = (const V *)I.K[0];
    V acc[RG];
    csr_rows_k<V, LPR, RG, KEEP, WIDE, TD>(rb, I.col, (const V *)I.val, rs.q,
                                   [&](int c) {
                                       V v = y[c];
                                       caxpy(v, th0, k1[c]);
                                       return v;
                                   },
                                   acc, td_coefs<V, TD>(I, 1));
    double sa = 0.0;
    if (rs.valid) {
        const double2 yr = to_d2(y[rs.row]);
        const double2 a = to_d2(pick(acc, rs.q)), f0 = to_d2(k1[rs.row]);
        const double sc = I.atol + I.rtol * sqrt(yr.x * yr.x + yr.y * yr.y);
        const double dx = (a.x - f0.x) / h0, dy = (a.y - f0.y) / h0;
        sa = (dx * dx + dy * dy) / (sc * sc);
    }
    sa = block_sum(sa, scr);
    if (threadIdx.x == 0) I.partials[2 * part] = sa;
}

// One Runge-Kutta stage S (2..7) of a DP5 step.
template <typename T, int LPR, int RG, int S, bool KEEP, bool WIDE, bool TD>
__device__ __forceinline__ void stage_body(const CsrInst &I, const CsrCtl *C, int row0, int part,
                                           const typename vec2<T>::type *cw_row = nullptr)
{
    using V = typename vec2<T>::type;
    using G = CsrGeom<LPR, RG>;
    __shared__ double scr[16];
    const RowSlot<LPR, RG> rs(row0, I.n);
    // the row bounds do not depend on the control record: issue them before waiting on it
    const RowBounds<RG> rb = csr_bounds<RG>(I.rowptr, rs.r0, G::GPB, I.n);
    if (C->status != ST_RUNNING || C->phase != PH_STEP) return;
    const double h = C->h_try;
    const int p = C->parity;
    const T s = (T)C->scale;
    const V *__restrict__ y = (const V *)I.Y[p];
    const V *__restrict__ k1 = (const V *)I.K[p];
    V *__restrict__ ynew = (V *)I.Y[1 - p];
    V *__restrict__ const *ks = (V *__restrict__ const *)I.ks;
    const V *__restrict__ xin;
    if (S == 2) xin = nullptr;
    else if (S == 3 || S == 5) xin = (const V *)I.ys[0];
    else if (S == 4 || S == 6) xin = (const V *)I.ys[1];
    else xin = ynew;

    // The epilogue's own-row operands do not depend on the row sum: load them first, so their
    // latency overlaps the matrix stream instead of following it.
    V yr{}, k1r{}, kr[4]{}, ynr{};
    if (rs.valid) {
        const int row = rs.row;
        yr = cscale(y[row], s);
        k1r = cscale(k1[row], s);
        if (S >= 3 && S <= 5) kr[0] = ks[0][row];
        if (S >= 4) kr[1] = ks[1][row];
        if (S >= 5) kr[2] = ks[2][row];
        if (S >= 6) kr[3] = ks[3][row];
        if (S == 7) {
            kr[0] = ks[4][row];
            ynr = ynew[row];
        }
    }
    V acc[RG];
    const V *__restrict__ cw = cw_row ? cw_row : td_coefs<V, TD>(I, S);  // this evaluation's coefficients
    // For a constant L, k1 = L y (first same as last), so the second stage's right-hand side
    // L (y + a21 h k1) = k1 + a21 h (L k1): one gather per entry instead of two.  A constant problem
    // in a plan with time-dependent ones takes the same route through the weighted kernels.
    const bool lin2 = S == 2 && (!TD || I.nterms == 0);
    if (lin2) {
        csr_rows_k<V, LPR, RG, KEEP, WIDE, TD>(rb, I.col, (const V *)I.val, rs.q, [&](int cc) { return k1[cc]; }, acc, cw);
    } else if (S == 2) {
        const T c = (T)(h * DP5::a21);
        csr_rows_k<V, LPR, RG, KEEP, WIDE, TD>(rb, I.col, (const V *)I.val, rs.q,
                                       [&](int cc) {
                                           V v = y[cc];
                                           caxpy(v, c, k1[cc]);
                                           return cscale(v, s);
                                       },
                                       acc, cw);
    } else {
        csr_rows_k<V, LPR, RG, KEEP, WIDE, TD>(rb, I.col, (const V *)I.val, rs.q, [&](int cc) { return xin[cc]; }, acc,
                                       cw);
    }

    double e2 = 0.0, l2 = 0.0;  // error norm part; |L y_new|^2 part (steady-state mode)
    if (rs.valid) {
        const int row = rs.row;
        V a = pick(acc, rs.q);
        if (lin2) {
            // the lazy trace scale s applies to y and k1 alike: L (s y + a21 h s k1) = s k1 + a21 h s (L k1)
            const V lk1 = a;
            a = k1r;
            caxpy(a, (T)(h * DP5::a21) * s, lk1);
        }
        if (S == 2) {
            ks[0][row] = a;
            V o = yr;
            caxpy(o, (T)(h * DP5::a31), k1r);
            caxpy(o, (T)(h * DP5::a32), a);
            ((V *)I.ys[0])[row] = o;
        } else if (S == 3) {
            ks[1][row] = a;
            V o = yr;
            caxpy(o, (T)(h * DP5::a41), k1r);
            caxpy(o, (T)(h * DP5::a42), kr[0]);
            caxpy(o, (T)(h * DP5::a43), a);
            ((V *)I.ys[1])[row] = o;
        } else if (S == 4) {
            ks[2][row] = a;
            V o = yr;
            caxpy(o, (T)(h * DP5::a51), k1r);
            caxpy(o, (T)(h * DP5::a52), kr[0]);
            caxpy(o, (T)(h * DP5::a53), kr[1]);
            caxpy(o, (T)(h * DP5::a54), a);
            ((V *)I.ys[0])[row] = o;
        } else if (S == 5) {
            ks[3][row] = a;
            V o = yr;
            caxpy(o, (T)(h * DP5::a61), k1r);
            caxpy(o, (T)(h * DP5::a62), kr[0]);
            caxpy(o, (T)(h * DP5::a63), kr[1]);
            caxpy(o, (T)(h * DP5::a64), kr[2]);
            caxpy(o, (T)(h * DP5::a65), a);
            ((V *)I.ys[1])[row] = o;
        } else if (S == 6) {
            ks[4][row] = a;
            V o = yr;
            caxpy(o, (T)(h * DP5::b1), k1r);
            caxpy(o, (T)(h * DP5::b3), kr[1]);
            caxpy(o, (T)(h * DP5::b4), kr[2]);
            caxpy(o, (T)(h * DP5::b5), kr[3]);
            caxpy(o, (T)(h * DP5::b6), a);
            ynew[row] = o;
        } else {
            ((V *)I.K[1 - p])[row] = a;
            // error estimate e = h sum_j (b_j - bhat_j) k_j in FP64
            double2 e = make_double2(0.0, 0.0);
            caxpy(e, h * DP5::e1, to_d2(k1r));
            caxpy(e, h * DP5::e3, to_d2(kr[1]));
            caxpy(e, h * DP5::e4, to_d2(kr[2]));
            caxpy(e, h * DP5::e5, to_d2(kr[3]));
            caxpy(e, h * DP5::e6, to_d2(kr[0]));
            caxpy(e, h * DP5::e7, to_d2(a));
            const double my = sqrt(abs2d(yr)), mn = sqrt(abs2d(ynr));
            const double sc = I.atol + I.rtol * fmax(my, mn);
            e2 = (e.x * e.x + e.y * e.y) / (sc * sc);
            l2 = abs2d(a);
        }
    }
    if (S == 7) {
        e2 = block_sum(e2, scr);
        const bool steady = I.steady_tol2 > 0.0;  // the same in every thread of the block
        if (steady) l2 = block_sum(l2, scr);
        if (threadIdx.x == 0) {
            I.partials[2 * part] = e2;
            if (steady) I.partials[2 * part + 1] = l2;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Kernels: ONE = single problem with its descriptor `one` passed by value; otherwise the block
// table (bi: problem, br: first row) of the logical block selects the problem.
// ---------------------------------------------------------------------------------------------
// Logical block -> (descriptor, control record, first row, partial slot), then the body.
// FORM 0: several problems, block table.  FORM 1: one problem, descriptor by value.  FORM 2 / 3: as
// 1 / 0, with the matrix read through the caches (temporal loads) instead of streamed past them, so
// that what of the matrices fits the L2s and the MALL is still there at the next launch.  FORM 4 / 5:
// as 2 / 3 with 16-byte loads of runs of 4 stored entries.
#define QT_CSR_DISPATCH(BODY, ...)                                                                   \
    const int lb = csr_block(xcd);                                                                   \
    constexpr bool KEEP_ = FORM >= 2, WIDE_ = FORM >= 4;                                             \
    if constexpr (FORM == 1 || FORM == 2 || FORM == 4) {                                             \
        BODY<__VA_ARGS__, KEEP_, WIDE_, TD>(one, ctls, lb * CsrGeom<LPR, RG>::RPB, lb);              \
    } else {                                                                                         \
        if (bound && lb >= bound[0]) return; /* grid sized for a capacity, table filled less */     \
        const int ii = bi[lb], row0 = br[lb];                                                        \
        BODY<__VA_ARGS__, KEEP_, WIDE_, TD>(insts[ii], ctls + ii, row0, row0 / CsrGeom<LPR, RG>::RPB); \
    }

template <typename T, int LPR, int RG, int FORM, bool TD>
__global__ __launch_bounds__(CSR_THREADS) void k_csr_init0(const CsrInst *__restrict__ insts, const CsrInst one,
                                                           const CsrCtl *__restrict__ ctls,
                                                           const int32_t *__restrict__ bi,
                                                           const int32_t *__restrict__ br, int xcd,
                                                           const int32_t *__restrict__ bound)
{
    QT_CSR_DISPATCH(init0_body, T, LPR, RG)
}

template <typename T, int LPR, int RG, int FORM, bool TD>
__global__ __launch_bounds__(CSR_THREADS) void k_csr_init1(const CsrInst *__restrict__ insts, const CsrInst one,
                                                           const CsrCtl *__restrict__ ctls,
                                                           const int32_t *__restrict__ bi,
                                                           const int32_t *__restrict__ br, int xcd,
                                                           const int32_t *__restrict__ bound)
{
    QT_CSR_DISPATCH(init1_body, T, LPR, RG)
}

template <typename T, int LPR, int RG, int FORM, int S, bool TD>
__global__ __launch_bounds__(CSR_THREADS) void k_csr_stage(const CsrInst *__restrict__ insts, const CsrInst one,
                                                           const CsrCtl *__restrict__ ctls,
                                                           const int32_t *__restrict__ bi,
                                                           const int32_t *__restrict__ br, int xcd,
                                                           const int32_t *__restrict__ bound)
{
    QT_CSR_DISPATCH(stage_body, T, LPR, RG, S)
}
#undef QT_CSR_DISPATCH

// Stage 2 with the previous step's control folded in (one problem, runs of 4 stored entries, no
// steady-state test).  The step control needs only what the previous launches wrote -- stage 7's
// partials and the candidate y_new -- so every workgroup takes the decision itself, in the control
// kernel's reduction order (bitwise the same record), and workgroup 0 writes the record, the
// save-time expectations and, for a time-dependent problem, the coefficient rows of stages 2..7
// at the new step; the kernel boundary publishes them, with no device-scope fence.  Each workgroup
// forms stage 2's own coefficient row in LDS, exactly as the rows are formed.  The record is
// double-buffered: this launch reads rd and writes wr, stages 3..7 read wr, and the next step's
// launch swaps them.  rd->pending is 0 right after the starting step (no stage 7 to decide yet).
// Removes the control launch from every step.
template <typename T, int LPR, int RG, bool TD>
__global__ __launch_bounds__(CSR_THREADS) void k_csr_stage2_ctl(const CsrInst one, const CsrCtl *__restrict__ rd,
                                                                CsrCtl *__restrict__ wr)
{
    using V = typename vec2<T>::type;
    const CsrInst &I = one;
    __shared__ double scr[32];
    __shared__ CsrCtl nsh;
    __shared__ V cw2[TD ? TD_MAX_TERMS + 1 : 1];
    const CsrCtl c = *rd;
    if (c.status != ST_RUNNING || c.phase != PH_STEP) {  // finished: carry the record forward
        if (blockIdx.x == 0 && threadIdx.x == 0) *wr = c;
        return;
    }
    if (c.pending) {
        const int sidx = c.save_idx;
        const V *ynew = (const V *)I.Y[1 - c.parity];
        const double t_save = I.tlist[sidx];                               // sidx < nt while running
        const double t_after = sidx + 1 < I.nt ? I.tlist[sidx + 1] : 0.0;
        double esum, trsum;
        ctl_step_sums(I, ynew, esum, trsum, scr);
        const double err = sqrt(esum / I.n);
        const bool accept = isfinite(err) && err <= 1.0;
        double scale_new = 1.0;
        if (I.renorm && accept) scale_new = c.tr0 / trsum;
        if (blockIdx.x == 0 && accept && c.land) csr_record_expect(I, ynew, scale_new, sidx);
        if (threadIdx.x == 0) nsh = step_record(I, c, err, accept, scale_new, false, false, t_save, t_after);
    } else if (threadIdx.x == 0) {
        nsh = c;
    }
    if (threadIdx.x == 0) nsh.pending = 1;
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) *wr = nsh;
    const V *cw = nullptr;  // stage 2's coefficient row (time-dependent problems)
    if constexpr (TD) {
        if (c.pending && nsh.status == ST_RUNNING && I.nterms > 0) {
            // the rows of the new step's evaluations, as the control kernel forms them
            if (blockIdx.x == 0) td_rows<V>(I, 2, 7, nsh.t, nsh.h_try, threadIdx.x, blockDim.x);
            if ((int)threadIdx.x <= I.nterms) {
                double2 w2 = make_double2(1.0, 0.0);
                if (threadIdx.x > 0) w2 = coef_value(I.coefs[threadIdx.x - 1], nsh.t + DP5::c2 * nsh.h_try);
                cw2[threadIdx.x] = from_d2<V>(w2);
            }
            __syncthreads();
            cw = cw2;
        }
    }
    stage_body<T, LPR, RG, 2, true, true, TD>(I, &nsh, blockIdx.x * CsrGeom<LPR, RG>::RPB, blockIdx.x, cw);
}

// ---------------------------------------------------------------------------------------------
// Launch plumbing
// ---------------------------------------------------------------------------------------------

// Launch arguments shared by every CSR launch of a step.
struct CsrArgs {
    const CsrInst *insts;
    CsrInst one;  // used when ninst == 1 and the host descriptor was given
    bool use_one;
    int form;  // kernel FORM: 0 block table, 1 one problem; 2 / 3: as 1 / 0 with temporal matrix loads;
               // 4 / 5: as 2 / 3 with 16-byte matrix loads
    CsrCtl *ctls;
    const int32_t *bi, *br, *ilist, *bound, *ibound;
    int nblk, ninst, xcd;
    hipStream_t s;
};

static inline CsrArgs make_args(const CsrLaunch &L, hipStream_t s)
{
    CsrArgs a;
    a.insts = L.insts;
    a.use_one = L.ninst == 1 && L.one_host != nullptr;
    if (a.use_one) a.one = *L.one_host;
    else std::memset(&a.one, 0, sizeof(a.one));
    a.form = a.use_one ? (L.keep == 2 ? 4 : L.keep ? 2 : 1) : (L.keep == 2 ? 5 : L.keep ? 3 : 0);
    a.ctls = L.ctls;
    a.bi = L.bi;
    a.br = L.br;
    a.ilist = L.ilist;
    a.bound = L.bound;
    a.ibound = L.ibound;
    a.nblk = L.nblk;
    a.ninst = L.ninst;
    a.xcd = L.xcd;
    a.s = s;
    return a;
}

#define QT_SHAPE_DISPATCH(LPRV, RGV, CALL) \
    switch (LPRV * 16 + RGV) {             \
    case 4 * 16 + 1: CALL(4, 1); break;    \
    case 4 * 16 + 2: CALL(4, 2); break;    \
    case 4 * 16 + 4: CALL(4, 4); break;    \
    case 8 * 16 + 2: CALL(8, 2); break;    \
    case 8 * 16 + 4: CALL(8, 4); break;    \
    case 16 * 16 + 1: CALL(16, 1); break;  \
    case 16 * 16 + 2: CALL(16, 2); break;  \
    case 16 * 16 + 4: CALL(16, 4); break;  \
    default: CALL(8, 1); break;            \
    }

// One SpMV kernel of the step sequence: which = 0 / 1 the starting-step evaluations, 2..7 the stages.
template <typename T, int LPR, int RG, int FORM, bool TD>
static void launch_spmv_form(int which, const CsrArgs &a)
{
    const dim3 g(a.nblk), t(CSR_THREADS);
#define QT_ARGS a.insts, a.one, a.ctls, a.bi, a.br, a.xcd, a.bound
    switch (which) {
    case 0: hipLaunchKernelGGL((k_csr_init0<T, LPR, RG, FORM, TD>), g, t, 0, a.s, QT_ARGS); break;
    case 1: hipLaunchKernelGGL((k_csr_init1<T, LPR, RG, FORM, TD>), g, t, 0, a.s, QT_ARGS); break;
    case 2: hipLaunchKernelGGL((k_csr_stage<T, LPR, RG, FORM, 2, TD>), g, t, 0, a.s, QT_ARGS); break;
    case 3: hipLaunchKernelGGL((k_csr_stage<T, LPR, RG, FORM, 3, TD>), g, t, 0, a.s, QT_ARGS); break;
    case 4: hipLaunchKernelGGL((k_csr_stage<T, LPR, RG, FORM, 4, TD>), g, t, 0, a.s, QT_ARGS); break;
    case 5: hipLaunchKernelGGL((k_csr_stage<T, LPR, RG, FORM, 5, TD>), g, t, 0, a.s, QT_ARGS); break;
    case 6: hipLaunchKernelGGL((k_csr_stage<T, LPR, RG, FORM, 6, TD>), g, t, 0, a.s, QT_ARGS); break;
    default: hipLaunchKernelGGL((k_csr_stage<T, LPR, RG, FORM, 7, TD>), g, t, 0, a.s, QT_ARGS); break;
    }
#undef QT_ARGS
}

// The kernel FORM of a launch; the wide forms exist for the shapes csr_wide_shape admits.
template <typename T, int LP, int RR, bool TD> static void launch_spmv_t(int w, const CsrArgs &a)
{
    if constexpr (csr_wide_shape<LP, RR>()) {
        if (a.form == 5) return launch_spmv_form<T, LP, RR, 5, TD>(w, a);
        if (a.form == 4) return launch_spmv_form<T, LP, RR, 4, TD>(w, a);
    }
    if (a.form == 3) launch_spmv_form<T, LP, RR, 3, TD>(w, a);
    else if (a.form == 2) launch_spmv_form<T, LP, RR, 2, TD>(w, a);
    else if (a.form == 1) launch_spmv_form<T, LP, RR, 1, TD>(w, a);
    else launch_spmv_form<T, LP, RR, 0, TD>(w, a);
}

// SpMV kernels first..last of the step sequence (0 / 1: starting-step evaluations, 2..7: stages).
template <bool TD>
static void launch_spmv_range(const CsrLaunch &L, const CsrArgs &a, int first, int last)
{
    for (int w = first; w <= last; ++w) {
#define QT_CALL(LP, RR)                                                                        \
        {                                                                                      \
            if (L.f64) launch_spmv_t<double, LP, RR, TD>(w, a);                                \
            else launch_spmv_t<float, LP, RR, TD>(w, a);                                       \
        }
        QT_SHAPE_DISPATCH(L.lpr, L.rg, QT_CALL)
#undef QT_CALL
    }
}

// Stage 2 with the folded step control for one problem (k_csr_stage2_ctl), reading record rd and
// writing wr; false when the tile shape has no 16-byte-run kernels (then nothing is launched).
template <bool TD> static bool launch_stage2_ctl(const CsrLaunch &L, const CsrArgs &a, const CsrCtl *rd, CsrCtl *wr)
{
    const dim3 g(a.nblk), t(CSR_THREADS);
    bool launched = false;
#define QT_CALL(LP, RR)                                                                                           \
    {                                                                                                             \
        if constexpr (csr_wide_shape<LP, RR>()) {                                                                 \
            if (L.f64) hipLaunchKernelGGL((k_csr_stage2_ctl<double, LP, RR, TD>), g, t, 0, a.s, a.one, rd, wr);   \
            else hipLaunchKernelGGL((k_csr_stage2_ctl<float, LP, RR, TD>), g, t, 0, a.s, a.one, rd, wr);          \
            launched = true;                                                                                      \
        }                                                                                                         \
    }
    QT_SHAPE_DISPATCH(L.lpr, L.rg, QT_CALL)
#undef QT_CALL
    return launched;
}

// Defined in kernels_csr_td.hip: the time-dependent SpMV kernels first..last.
void csr_td_spmv(const CsrLaunch &L, const CsrArgs &a, int first, int last);
// Defined in kernels_csr_td.hip: launch_stage2_ctl<true>.
bool csr_td_stage2_ctl(const CsrLaunch &L, const CsrArgs &a, const CsrCtl *rd, CsrCtl *wr);

}  // namespace qt

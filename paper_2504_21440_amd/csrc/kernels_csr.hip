// kernels_csr.hip -- CSR-form master-equation solver kernels for gfx950.
//
// The right-hand side is the sparse Liouvillian superoperator applied to vec(rho)
// (arXiv:2504.21440, Sec. 3.2, eq. eq-lindblad-master-equation): an HBM-bound complex CSR SpMV.
// A Dormand-Prince 5(4) step is six SpMV launches (stages 2..7; stage 1 is the previous step's
// stage 7) and one control launch.  Each SpMV carries the Runge-Kutta work of its row in its
// epilogue: the next stage input (stages 2..5), the fifth-order solution (stage 6), or the weighted
// error contribution (stage 7, reduced per block).  The control kernel -- one workgroup per problem
// -- sums the block partials in a fixed order (FP64), accepts or rejects, picks the next step size,
// lands on save times, renormalises the trace (mixed precision) and records Tr(O rho), so the host
// never sits inside the step loop and no block waits on another.
//
// Tile shape (LPR, RG): a group of LPR lanes of a 64-wide wavefront serves RG rows at once.  Every
// lane first issues the column / value loads of all its rows (non-temporal: the matrix is streamed
// once per evaluation and should not evict the state vectors from L2 / MALL), then the gathers and
// complex FMAs; the group combines with xor shuffles, and lane g of the group runs the epilogue of
// row g.  More rows per group put more bytes in flight per wave, which is what a latency-bound
// SpMV needs; fewer keep small problems spread over more workgroups.
//
// Block order (xcd): the hardware hands consecutive workgroups to the 8 XCDs in turn, and each XCD
// has its own L2.  With xcd = 1 the logical block index is remapped so that each XCD works through
// one contiguous eighth of the rows; the gathers of vec(rho) then concentrate on a slice of the
// state that fits that XCD's L2 instead of every XCD pulling the whole vector through its own L2.
// The remap changes which rows run where, never how a row or a block partial is summed, so results
// are bitwise the same either way.
//
// Launch forms: with several problems a block reads its problem index and first row from a block
// table (its slot among the problem's partials is the first row over the rows per block) and the
// problem's descriptor from device memory; with one problem (ONE) the descriptor is a kernel
// argument and the first row is the block index times the rows per block, which removes two
// dependent memory round trips from every block's critical path.
//
// The shape and block order are chosen per problem size by the autotuner (qtamd_tune.cpp).
#include <cstring>

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
// returns all RG sums.  X returns the (stage) input at a column.
template <typename V, int LPR, int RG, bool KEEP, typename X>
__device__ __forceinline__ void csr_rows(const RowBounds<RG> &b, const int32_t *__restrict__ col,
                                         const V *__restrict__ val, int q, X x, V (&acc)[RG])
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
                if (cc[g][u] >= 0) cfma(acc[g], vv[g][u], x(cc[g][u]));
    }
#pragma unroll
    for (int g = 0; g < RG; ++g)
#pragma unroll
        for (int m = LPR / 2; m >= 1; m >>= 1) acc[g] = cadd(acc[g], shfl_xor_c(acc[g], m));
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
__device__ __forceinline__ double2 csr_expect_one(const CsrInst &I, const V *__restrict__ Y, int k)
{
    const int lane = threadIdx.x & 63;
    const int32_t *ep = I.eptr + (size_t)k * (I.d + 1);
    const int b = ep[0], e = ep[I.d];
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

// This thread's share of one partial column over the instance's blocks, in a fixed order: eight
// loads in flight per thread, then the strided tail.
__device__ __forceinline__ double partials_part(const CsrInst &I, int col)
{
    const int nb = I.nblocks, T = blockDim.x;
    const double *__restrict__ P = I.partials + col;
    double t = 0.0;
    int k = threadIdx.x;
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

__device__ __forceinline__ double sum_partials(const CsrInst &I, int col, double *scr)
{
    return block_sum(partials_part(I, col), scr);
}

__global__ void k_csr_reset(const CsrInst *__restrict__ insts, CsrCtl *__restrict__ ctls, int ninst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst) return;
    CsrCtl c;
    c.t = insts[i].tlist[0];
    c.h = 0.0;
    c.h_try = 0.0;
    c.err_prev = 1e-4;
    c.scale = 1.0;
    c.tr0 = 1.0;
    c.h0 = 0.0;
    c.last_err = 0.0;
    c.status = ST_RUNNING;
    c.phase = PH_INIT0;
    c.land = 0;
    c.last_rejected = 0;
    c.save_idx = 1;
    c.parity = 0;
    c.arrive = 0u;
    c.pad = 0;
    c.n_accept = c.n_reject = c.n_steps = c.n_rhs = 0;
    ctls[i] = c;
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
template <typename T, int LPR, int RG, bool KEEP>
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
    csr_rows<V, LPR, RG, KEEP>(rb, I.col, (const V *)I.val, rs.q, [&](int c) { return x0[c]; }, acc);
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
template <typename T, int LPR, int RG, bool KEEP>
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
    csr_rows<V, LPR, RG, KEEP>(rb, I.col, (const V *)I.val, rs.q,
                         [&](int c) {
                             V v = y[c];
                             caxpy(v, th0, k1[c]);
                             return v;
                         },
                         acc);
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
template <typename T, int LPR, int RG, int S, bool KEEP>
__device__ __forceinline__ void stage_body(const CsrInst &I, const CsrCtl *C, int row0, int part)
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
    if (S == 2) {
        const T c = (T)(h * DP5::a21);
        csr_rows<V, LPR, RG, KEEP>(rb, I.col, (const V *)I.val, rs.q,
                             [&](int cc) {
                                 V v = y[cc];
                                 caxpy(v, c, k1[cc]);
                                 return cscale(v, s);
                             },
                             acc);
    } else {
        csr_rows<V, LPR, RG, KEEP>(rb, I.col, (const V *)I.val, rs.q, [&](int cc) { return xin[cc]; }, acc);
    }

    double e2 = 0.0;
    if (rs.valid) {
        const int row = rs.row;
        const V a = pick(acc, rs.q);
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
        }
    }
    if (S == 7) {
        e2 = block_sum(e2, scr);
        if (threadIdx.x == 0) I.partials[2 * part] = e2;
    }
}

// ---------------------------------------------------------------------------------------------
// Kernels: ONE = single problem with its descriptor `one` passed by value; otherwise the block
// table (bi: problem, br: first row) of the logical block selects the problem.
// ---------------------------------------------------------------------------------------------
// Logical block -> (descriptor, control record, first row, partial slot), then the body.
// FORM 0: several problems, block table.  FORM 1: one problem, descriptor by value.  FORM 2 / 3: as
// 1 / 0, with the matrix read through the caches (temporal loads) instead of streamed past them, so
// that what of the matrices fits the L2s and the MALL is still there at the next launch.
#define QT_CSR_DISPATCH(BODY, ...)                                                                   \
    const int lb = csr_block(xcd);                                                                   \
    if constexpr (FORM == 1 || FORM == 2) {                                                          \
        BODY<__VA_ARGS__, FORM == 2>(one, ctls, lb * CsrGeom<LPR, RG>::RPB, lb);                     \
    } else {                                                                                         \
        if (bound && lb >= bound[0]) return; /* grid sized for a capacity, table filled less */     \
        const int ii = bi[lb], row0 = br[lb];                                                        \
        BODY<__VA_ARGS__, FORM == 3>(insts[ii], ctls + ii, row0, row0 / CsrGeom<LPR, RG>::RPB);     \
    }

template <typename T, int LPR, int RG, int FORM>
__global__ __launch_bounds__(CSR_THREADS) void k_csr_init0(const CsrInst *__restrict__ insts, const CsrInst one,
                                                           const CsrCtl *__restrict__ ctls,
                                                           const int32_t *__restrict__ bi,
                                                           const int32_t *__restrict__ br, int xcd,
                                                           const int32_t *__restrict__ bound)
{
    QT_CSR_DISPATCH(init0_body, T, LPR, RG)
}

template <typename T, int LPR, int RG, int FORM>
__global__ __launch_bounds__(CSR_THREADS) void k_csr_init1(const CsrInst *__restrict__ insts, const CsrInst one,
                                                           const CsrCtl *__restrict__ ctls,
                                                           const int32_t *__restrict__ bi,
                                                           const int32_t *__restrict__ br, int xcd,
                                                           const int32_t *__restrict__ bound)
{
    QT_CSR_DISPATCH(init1_body, T, LPR, RG)
}

template <typename T, int LPR, int RG, int FORM, int S>
__global__ __launch_bounds__(CSR_THREADS) void k_csr_stage(const CsrInst *__restrict__ insts, const CsrInst one,
                                                           const CsrCtl *__restrict__ ctls,
                                                           const int32_t *__restrict__ bi,
                                                           const int32_t *__restrict__ br, int xcd,
                                                           const int32_t *__restrict__ bound)
{
    QT_CSR_DISPATCH(stage_body, T, LPR, RG, S)
}
#undef QT_CSR_DISPATCH

// Control: one workgroup per problem.  step_mode 0 completes a pending starting-step evaluation
// (phases INIT0 / INIT1) and leaves stepping problems alone; step_mode 1 closes a Runge-Kutta step
// (phase STEP) and leaves problems still in their starting phases alone.
template <typename T>
__device__ __forceinline__ void control_body(const CsrInst &I, CsrCtl *C, int step_mode)
{
    using V = typename vec2<T>::type;
    __shared__ double scr[16];
    __shared__ double2 exs[CTL_MAX_EOPS];
    if (C->status != ST_RUNNING) return;
    const int phase = C->phase;
    if ((phase == PH_STEP) != (step_mode != 0)) return;
    if (phase == PH_INIT0) {
        const double ta = sum_partials(I, 0, scr), tb = sum_partials(I, 1, scr);
        const V *x0 = (const V *)I.rho0;
        const double tr = csr_trace(I, x0, scr);
        csr_record_expect(I, x0, 1.0, 0);
        if (threadIdx.x == 0) {
            C->tr0 = tr;
            C->n_rhs += 1;
            if (I.nt <= 1) {
                C->status = ST_DONE;
            } else {
                const double d0 = sqrt(ta / I.n), d1 = sqrt(tb / I.n);
                if (I.use_h0) {
                    C->h = I.h0;
                    C->phase = PH_STEP;
                    int32_t land;
                    C->h_try = clip_step(C->t, C->h, I.tlist[1], &land);
                    C->land = land;
                } else {
                    C->h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
                    C->last_err = d1;
                    C->phase = PH_INIT1;
                }
            }
        }
        return;
    }
    if (phase == PH_INIT1) {
        const double ta = sum_partials(I, 0, scr);
        if (threadIdx.x == 0) {
            const double h0 = C->h0;
            const double d2 = sqrt(ta / I.n), d1 = C->last_err;
            const double m = fmax(d1, d2);
            const double h1 = (m <= 1e-15) ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / m, 0.2);
            C->h = fmin(100.0 * h0, h1);
            C->phase = PH_STEP;
            C->n_rhs += 1;
            int32_t land;
            C->h_try = clip_step(C->t, C->h, I.tlist[1], &land);
            C->land = land;
        }
        return;
    }
    // ---- step control after stage 7 ----
    const double h = C->h_try;
    const int p = C->parity;
    const int land = C->land;
    const int sidx = C->save_idx;
    const V *ynew = (const V *)I.Y[1 - p];
    // Everything that only reads is issued before the decision: the error partials, the
    // candidate's trace and, at a save time, the expectation sums (wasted on a rejection).
    const bool spec = land && I.ne <= CTL_MAX_EOPS;
    if (spec) {
        for (int k = threadIdx.x >> 6; k < I.ne; k += blockDim.x >> 6) {
            const double2 sk = csr_expect_one(I, ynew, k);
            if ((threadIdx.x & 63) == 0) exs[k] = sk;
        }
    }
    const double part = partials_part(I, 0);
    const double trp = I.renorm ? csr_trace_part(I, ynew) : 0.0;
    const double tot = block_sum(part, scr);  // its barriers also publish exs
    const double err = sqrt(tot / I.n);
    const bool finite = isfinite(err);
    const bool accept = finite && err <= 1.0;
    double scale_new = 1.0;
    if (I.renorm) {
        const double tr = block_sum(trp, scr);
        if (accept) scale_new = C->tr0 / tr;
    }
    if (accept && land) {
        if (spec) {
            for (int k = threadIdx.x; k < I.ne; k += blockDim.x)
                I.expect[(size_t)k * I.nt + sidx] = make_double2(exs[k].x * scale_new, exs[k].y * scale_new);
        } else {
            csr_record_expect(I, ynew, scale_new, sidx);
        }
    }
    if (threadIdx.x == 0) {
        C->n_steps += 1;
        C->n_rhs += 6;
        if (!finite) {
            C->status = 6;  // QT_ENONFINITE
        } else if (accept) {
            C->n_accept += 1;
            C->t = land ? I.tlist[sidx] : C->t + h;
            C->parity = 1 - p;
            double hn = h * pi_factor(err, C->err_prev);
            if (C->last_rejected && hn > h) hn = h;
            C->h = hn;
            C->err_prev = fmax(err, 1e-4);
            C->last_rejected = 0;
            C->scale = scale_new;
            if (land) {
                C->save_idx = sidx + 1;
                if (sidx + 1 >= I.nt) C->status = ST_DONE;
            }
        } else {
            C->n_reject += 1;
            C->h = h * reject_factor(err);
            C->last_rejected = 1;
        }
        C->last_err = err;
        if (C->status == ST_RUNNING) {
            if (C->n_steps >= I.max_steps) {
                C->status = 4;  // QT_EMAXSTEPS
            } else if (C->h < 1e-14 * fmax(1.0, fabs(C->t))) {
                C->status = 5;  // QT_EDTMIN
            } else {
                int32_t l2;
                C->h_try = clip_step(C->t, C->h, I.tlist[C->save_idx], &l2);
                C->land = l2;
            }
        }
    }
}

// ilist: the problems to visit (one workgroup each), or null for problems 0 .. gridDim.x - 1;
// ibound: when given, only the first ibound[0] entries of ilist are live.
template <typename T, bool ONE>
__global__ __launch_bounds__(CTL_THREADS) void k_csr_control(const CsrInst *__restrict__ insts, const CsrInst one,
                                                             CsrCtl *__restrict__ ctls, int step_mode,
                                                             const int32_t *__restrict__ ilist,
                                                             const int32_t *__restrict__ ibound)
{
    if constexpr (ONE) {
        control_body<T>(one, ctls, step_mode);
    } else {
        if (ibound && (int)blockIdx.x >= ibound[0]) return;
        const int ii = ilist ? ilist[blockIdx.x] : (int)blockIdx.x;
        control_body<T>(insts[ii], ctls + ii, step_mode);
    }
}

// ---- standalone expectation value (qt_expect) ----
template <typename T>
__global__ __launch_bounds__(256) void k_expect(int d, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                const double2 *__restrict__ v, const void *state, int is_ket,
                                                double2 *out)
{
    using V = typename vec2<T>::type;
    __shared__ double scr[16];
    const V *__restrict__ st = (const V *)state;
    double sr = 0.0, si = 0.0, nn = 0.0;
    for (int i = threadIdx.x; i < d; i += blockDim.x) {
        double rr = 0.0, ri = 0.0;
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const double2 o = v[p];
            const double2 x = to_d2(is_ket ? st[ci[p]] : st[(size_t)ci[p] * d + i]);
            rr += o.x * x.x - o.y * x.y;
            ri += o.x * x.y + o.y * x.x;
        }
        if (is_ket) {
            const double2 c = to_d2(st[i]);  // conj(psi_i) * (O psi)_i
            sr += c.x * rr + c.y * ri;
            si += c.x * ri - c.y * rr;
            nn += c.x * c.x + c.y * c.y;
        } else {
            sr += rr;
            si += ri;
        }
    }
    sr = block_sum(sr, scr);
    si = block_sum(si, scr);
    nn = block_sum(nn, scr);
    if (threadIdx.x == 0) out[0] = is_ket ? make_double2(sr / nn, si / nn) : make_double2(sr, si);
}

}  // namespace qt

// ---------------------------------------------------------------------------------------------
// Host-side launchers (called from the runtime)
// ---------------------------------------------------------------------------------------------
namespace qt {

int csr_rows_per_block(int lpr, int rg) { return (CSR_THREADS / 64) * (64 / lpr) * rg; }

bool csr_shape_supported(int lpr, int rg)
{
    return (lpr == 4 || lpr == 8 || lpr == 16) && (rg == 1 || rg == 2 || rg == 4);
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

// Launch arguments shared by every CSR launch of a step.
struct CsrArgs {
    const CsrInst *insts;
    CsrInst one;  // used when ninst == 1 and the host descriptor was given
    bool use_one;
    int form;  // kernel FORM: 0 block table, 1 one problem; 2 / 3: as 1 / 0 with temporal matrix loads
    CsrCtl *ctls;
    const int32_t *bi, *br, *ilist, *bound, *ibound;
    int nblk, ninst, xcd;
    hipStream_t s;
};

static CsrArgs make_args(const CsrLaunch &L, hipStream_t s)
{
    CsrArgs a;
    a.insts = L.insts;
    a.use_one = L.ninst == 1 && L.one_host != nullptr;
    if (a.use_one) a.one = *L.one_host;
    else std::memset(&a.one, 0, sizeof(a.one));
    a.form = a.use_one ? (L.keep ? 2 : 1) : (L.keep ? 3 : 0);
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

template <typename T>
static void launch_control(const CsrArgs &a, int step_mode)
{
    if (a.use_one)
        hipLaunchKernelGGL((k_csr_control<T, true>), dim3(1), dim3(CTL_THREADS), 0, a.s, a.insts, a.one, a.ctls,
                           step_mode, (const int32_t *)nullptr, (const int32_t *)nullptr);
    else
        hipLaunchKernelGGL((k_csr_control<T, false>), dim3(a.ninst), dim3(CTL_THREADS), 0, a.s, a.insts, a.one,
                           a.ctls, step_mode, a.ilist, a.ibound);
}

#define QT_LAUNCH(KERNEL, a)                                                                                  \
    do {                                                                                                      \
        if ((a).form == 3)                                                                                    \
            hipLaunchKernelGGL((KERNEL<T, LPR, RG, 3>), dim3((a).nblk), dim3(CSR_THREADS), 0, (a).s,         \
                               (a).insts, (a).one, (a).ctls, (a).bi, (a).br, (a).xcd, (a).bound);                       \
        else if ((a).form == 2)                                                                               \
            hipLaunchKernelGGL((KERNEL<T, LPR, RG, 2>), dim3((a).nblk), dim3(CSR_THREADS), 0, (a).s,         \
                               (a).insts, (a).one, (a).ctls, (a).bi, (a).br, (a).xcd, (a).bound);                       \
        else if ((a).form == 1)                                                                               \
            hipLaunchKernelGGL((KERNEL<T, LPR, RG, 1>), dim3((a).nblk), dim3(CSR_THREADS), 0, (a).s,         \
                               (a).insts, (a).one, (a).ctls, (a).bi, (a).br, (a).xcd, (a).bound);                       \
        else                                                                                                  \
            hipLaunchKernelGGL((KERNEL<T, LPR, RG, 0>), dim3((a).nblk), dim3(CSR_THREADS), 0, (a).s,         \
                               (a).insts, (a).one, (a).ctls, (a).bi, (a).br, (a).xcd, (a).bound);                       \
    } while (0)

#define QT_LAUNCH_STAGE(SV, a)                                                                                \
    do {                                                                                                      \
        if ((a).form == 3)                                                                                    \
            hipLaunchKernelGGL((k_csr_stage<T, LPR, RG, 3, SV>), dim3((a).nblk), dim3(CSR_THREADS), 0,       \
                               (a).s, (a).insts, (a).one, (a).ctls, (a).bi, (a).br, (a).xcd, (a).bound);                \
        else if ((a).form == 2)                                                                               \
            hipLaunchKernelGGL((k_csr_stage<T, LPR, RG, 2, SV>), dim3((a).nblk), dim3(CSR_THREADS), 0,       \
                               (a).s, (a).insts, (a).one, (a).ctls, (a).bi, (a).br, (a).xcd, (a).bound);                \
        else if ((a).form == 1)                                                                               \
            hipLaunchKernelGGL((k_csr_stage<T, LPR, RG, 1, SV>), dim3((a).nblk), dim3(CSR_THREADS), 0,       \
                               (a).s, (a).insts, (a).one, (a).ctls, (a).bi, (a).br, (a).xcd, (a).bound);                \
        else                                                                                                  \
            hipLaunchKernelGGL((k_csr_stage<T, LPR, RG, 0, SV>), dim3((a).nblk), dim3(CSR_THREADS), 0,       \
                               (a).s, (a).insts, (a).one, (a).ctls, (a).bi, (a).br, (a).xcd, (a).bound);                \
    } while (0)

template <typename T, int LPR, int RG>
static void launch_init_t(int which, const CsrArgs &a)
{
    if (which == 0) QT_LAUNCH(k_csr_init0, a);
    else QT_LAUNCH(k_csr_init1, a);
    launch_control<T>(a, 0);
}

template <typename T, int LPR, int RG>
static void launch_step_t(const CsrArgs &a)
{
    QT_LAUNCH_STAGE(2, a);
    QT_LAUNCH_STAGE(3, a);
    QT_LAUNCH_STAGE(4, a);
    QT_LAUNCH_STAGE(5, a);
    QT_LAUNCH_STAGE(6, a);
    QT_LAUNCH_STAGE(7, a);
    launch_control<T>(a, 1);
}

template <typename T, int LPR, int RG>
static void launch_stage3_t(const CsrArgs &a)
{
    QT_LAUNCH_STAGE(3, a);
}

void csr_launch_reset(const CsrInst *insts, CsrCtl *ctls, int ninst, hipStream_t s)
{
    hipLaunchKernelGGL(k_csr_reset, dim3((ninst + 63) / 64), dim3(64), 0, s, insts, ctls, ninst);
}

void csr_launch_init(int which, const CsrLaunch &L, hipStream_t s)
{
    const CsrArgs a = make_args(L, s);
#define QT_CALL(LP, RR)                                  \
    if (L.f64) launch_init_t<double, LP, RR>(which, a); \
    else launch_init_t<float, LP, RR>(which, a);
    QT_SHAPE_DISPATCH(L.lpr, L.rg, QT_CALL)
#undef QT_CALL
}

void csr_launch_step(const CsrLaunch &L, hipStream_t s)
{
    const CsrArgs a = make_args(L, s);
#define QT_CALL(LP, RR)                           \
    if (L.f64) launch_step_t<double, LP, RR>(a); \
    else launch_step_t<float, LP, RR>(a);
    QT_SHAPE_DISPATCH(L.lpr, L.rg, QT_CALL)
#undef QT_CALL
}

void csr_launch_stage3(const CsrLaunch &L, hipStream_t s)
{
    const CsrArgs a = make_args(L, s);
#define QT_CALL(LP, RR)                             \
    if (L.f64) launch_stage3_t<double, LP, RR>(a); \
    else launch_stage3_t<float, LP, RR>(a);
    QT_SHAPE_DISPATCH(L.lpr, L.rg, QT_CALL)
#undef QT_CALL
}

#undef QT_LAUNCH
#undef QT_LAUNCH_STAGE

void launch_expect(bool f64, int d, const int32_t *rp, const int32_t *ci, const double2 *v, const void *state,
                   int is_ket, double2 *out, hipStream_t s)
{
    if (f64)
        hipLaunchKernelGGL(k_expect<double>, dim3(1), dim3(256), 0, s, d, rp, ci, v, state, is_ket, out);
    else
        hipLaunchKernelGGL(k_expect<float>, dim3(1), dim3(256), 0, s, d, rp, ci, v, state, is_ket, out);
}

}  // namespace qt

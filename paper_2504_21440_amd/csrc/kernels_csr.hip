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
// never sits inside the step loop and no block waits on another.  For one problem (constant or
// time-dependent) with runs of 4 stored entries and no steady-state test, that control is folded into the next step's
// stage-2 launch instead (k_csr_stage2_ctl): every workgroup takes the same decision from the
// previous launches' output, so a step is six launches.
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
#include "csr_kernels.h"

namespace qt {

template <typename T>
__global__ void k_csr_reset(const CsrInst *__restrict__ insts, CsrCtl *__restrict__ ctls, int ninst)
{
    using V = typename vec2<T>::type;
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
    c.pending = 0;
    c.pad = 0;
    c.n_accept = c.n_reject = c.n_steps = c.n_rhs = 0;
    ctls[i] = c;
    // coefficient rows: row 0 (the first evaluation) at tlist[0]; the others are rewritten before use
    if (insts[i].cstage) td_rows<V>(insts[i], 0, TD_SLOTS - 1, c.t, 0.0, 0, 1);
}

// Control: one workgroup per problem.  step_mode 0 completes a pending starting-step evaluation
// (phases INIT0 / INIT1) and leaves stepping problems alone; step_mode 1 closes a Runge-Kutta step
// (phase STEP) and leaves problems still in their starting phases alone.
// The first XP entries per lane of one expectation operator (entries b + lane + 64 u of
// ecol / eval / evidx), requested before the state they gather from is known; then the operator's
// sum formed exactly as csr_expect_range forms it (entry order per lane, the same wave sums).
template <int XP> struct ExpectPre {
    int idx[XP];
    double2 val[XP];
    __device__ __forceinline__ void load(const CsrInst &I, int b, int e)
    {
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int u = 0; u < XP; ++u) {
            const int q = b + lane + 64 * u;
            idx[u] = 0;
            val[u] = make_double2(0.0, 0.0);
            if (q < e) {
                idx[u] = I.evidx[q];
                val[u] = I.eval[q];
            }
        }
    }
    template <typename V> __device__ __forceinline__ double2 sum(const CsrInst &I, const V *__restrict__ Y, int b, int e)
    {
        const int lane = threadIdx.x & 63;
        V g[XP];
#pragma unroll
        for (int u = 0; u < XP; ++u)
            if (b + lane + 64 * u < e) g[u] = Y[idx[u]];
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int u = 0; u < XP; ++u)
            if (b + lane + 64 * u < e) {
                const double2 r = to_d2(g[u]);
                sr += val[u].x * r.x - val[u].y * r.y;
                si += val[u].x * r.y + val[u].y * r.x;
            }
        for (int q = b + lane + 64 * XP; q < e; q += 64) {
            const double2 o = I.eval[q];
            const double2 r = to_d2(Y[I.evidx[q]]);
            sr += o.x * r.x - o.y * r.y;
            si += o.x * r.y + o.y * r.x;
        }
        return make_double2(wave_sum(sr), wave_sum(si));
    }
};

template <typename T>
__device__ __forceinline__ void control_body(const CsrInst &I, CsrCtl *C, int step_mode)
{
    using V = typename vec2<T>::type;
    __shared__ double scr[48];
    __shared__ double2 exs[CTL_MAX_EOPS];
    __shared__ double td_t, td_h;  // a time-dependent problem's next evaluations: rows td_first..td_last
    __shared__ int td_first, td_last;
    // The whole control record, this thread's share of the block partials (column 0; column 1 as
    // well when a steady-state test needs it) and the first entries of this wave's expectation
    // operator (their ranges are in the descriptor) do not depend on one another: one round trip.
    const CsrCtl c = *C;
    const int status = c.status;
    const int phase = c.phase;
    const double part0 = partials_part(I, 0);
    const double part1 = I.steady_tol2 > 0.0 ? partials_part(I, 1) : 0.0;
    const int k0 = threadIdx.x >> 6;
    const bool own = k0 < I.ne && k0 < CSR_XOPS;
    const int eb0 = own ? I.xbeg[k0] : 0, ee0 = own ? I.xbeg[k0] + I.xcnt[k0] : 0;
    ExpectPre<4> pre;
    pre.load(I, eb0, ee0);
    if (status != ST_RUNNING) return;
    if ((phase == PH_STEP) != (step_mode != 0)) return;
    // after thread 0 has decided: the coefficient rows of the evaluations the next launches make
    auto td_next = [&]() {
        if (I.nterms == 0) return;
        __syncthreads();
        if (td_first <= td_last) td_rows<V>(I, td_first, td_last, td_t, td_h, threadIdx.x, blockDim.x);
    };
    if (threadIdx.x == 0) td_first = 1, td_last = 0;
    if (phase == PH_INIT0) {
        const double ta = block_sum(part0, scr), tb = sum_partials(I, 1, scr);
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
                    td_first = 2, td_last = 7, td_t = C->t, td_h = C->h_try;
                } else {
                    C->h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
                    C->last_err = d1;
                    C->phase = PH_INIT1;
                    td_first = 1, td_last = 1, td_t = C->t, td_h = C->h0;
                }
            }
        }
        td_next();
        return;
    }
    if (phase == PH_INIT1) {
        const double ta = block_sum(part0, scr);
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
            td_first = 2, td_last = 7, td_t = C->t, td_h = C->h_try;
        }
        td_next();
        return;
    }
    // ---- step control after stage 7 ----
    const double h = c.h_try;
    const int p = c.parity;
    const int land = c.land;
    const int sidx = c.save_idx;
    const V *ynew = (const V *)I.Y[1 - p];
    // Everything that only reads is issued before the decision: the error partials, the
    // candidate's trace, the save times the update may need and, at a save time, the expectation
    // sums (wasted on a rejection).  The partials and the first entries of each wave's operator
    // went out with the control record; the rest goes out together here.
    const double t_save = I.tlist[sidx];                               // sidx < nt while running
    const double t_after = sidx + 1 < I.nt ? I.tlist[sidx + 1] : 0.0;  // the next save time
    V dg{};
    if (I.renorm && (int)threadIdx.x < I.d) dg = ynew[(size_t)threadIdx.x * (I.d + 1)];
    const bool spec = land && I.ne <= CTL_MAX_EOPS;
    if (spec) {
        for (int k = threadIdx.x >> 6; k < I.ne; k += blockDim.x >> 6) {
            const double2 sk = k == k0 && own ? pre.sum(I, ynew, eb0, ee0) : csr_expect_one(I, ynew, k);
            if ((threadIdx.x & 63) == 0) exs[k] = sk;
        }
    }
    const bool steady = I.steady_tol2 > 0.0;
    // this thread's share of the trace, summed as csr_trace_part sums it
    double trp = 0.0;
    if (I.renorm) {
        if ((int)threadIdx.x < I.d) trp += (double)dg.x;
        for (int i = threadIdx.x + blockDim.x; i < I.d; i += blockDim.x) trp += (double)ynew[(size_t)i * I.d + i].x;
    }
    // one set of barriers for the error, trace and residual sums (each summed as block_sum would);
    // the barriers also publish exs
    double sums[3] = {part0, trp, part1};
    block_sum_n<3>(sums, scr);
    const double err = sqrt(sums[0] / I.n);
    const bool finite = isfinite(err);
    const bool accept = finite && err <= 1.0;
    double scale_new = 1.0;
    if (I.renorm && accept) scale_new = c.tr0 / sums[1];
    // steady-state mode: |L y_new|_2 (of the rescaled state) at or below the tolerance ends the solve
    const bool conv = steady && accept && sums[2] * scale_new * scale_new <= I.steady_tol2;
    if (conv) {
        // the state no longer changes: every remaining save time receives its expectation values
        for (int idx = sidx; idx < I.nt; ++idx) csr_record_expect(I, ynew, scale_new, idx);
    } else if (accept && land) {
        if (spec) {
            for (int k = threadIdx.x; k < I.ne; k += blockDim.x)
                I.expect[(size_t)k * I.nt + sidx] = make_double2(exs[k].x * scale_new, exs[k].y * scale_new);
        } else {
            csr_record_expect(I, ynew, scale_new, sidx);
        }
    }
    if (threadIdx.x == 0) {
        // the new record, from the copy read at the start (no other writer in between)
        const CsrCtl n = step_record(I, c, err, accept, scale_new, conv, steady, t_save, t_after);
        if (n.status == ST_RUNNING) td_first = 2, td_last = 7, td_t = n.t, td_h = n.h_try;
        *C = n;
    }
    td_next();
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

bool csr_shape_supported(int lpr, int rg, int keep)
{
    if (!csr_shape_supported(lpr, rg) || keep < 0 || keep > 2) return false;
    if (keep < 2) return true;
    return (lpr == 4 && rg == 1) || (lpr == 8 && (rg == 1 || rg == 2)) || (lpr == 16 && rg == 1);
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

static void spmv(const CsrLaunch &L, const CsrArgs &a, int first, int last)
{
    if (L.td) csr_td_spmv(L, a, first, last);
    else launch_spmv_range<false>(L, a, first, last);
}

static void control(const CsrLaunch &L, const CsrArgs &a, int step_mode)
{
    if (L.f64) launch_control<double>(a, step_mode);
    else launch_control<float>(a, step_mode);
}

void csr_launch_reset(const CsrInst *insts, CsrCtl *ctls, int ninst, bool f64, hipStream_t s)
{
    if (f64) hipLaunchKernelGGL(k_csr_reset<double>, dim3((ninst + 63) / 64), dim3(64), 0, s, insts, ctls, ninst);
    else hipLaunchKernelGGL(k_csr_reset<float>, dim3((ninst + 63) / 64), dim3(64), 0, s, insts, ctls, ninst);
}

void csr_launch_init(int which, const CsrLaunch &L, hipStream_t s)
{
    const CsrArgs a = make_args(L, s);
    spmv(L, a, which, which);
    control(L, a, 0);
}

void csr_launch_step(const CsrLaunch &L, hipStream_t s, int j)
{
    CsrArgs a = make_args(L, s);
    if (L.fused && j >= 0 && a.use_one) {
        // step j reads record j % 2 and writes the other (see k_csr_stage2_ctl)
        CsrCtl *rd = L.ctls + (j & 1), *wr = L.ctls + ((j + 1) & 1);
        const bool launched = L.td ? csr_td_stage2_ctl(L, a, rd, wr) : launch_stage2_ctl<false>(L, a, rd, wr);
        if (launched) {
            a.ctls = wr;
            spmv(L, a, 3, 7);
            return;
        }
    }
    spmv(L, a, 2, 7);
    control(L, a, 1);
}

void csr_launch_stage3(const CsrLaunch &L, hipStream_t s)
{
    const CsrArgs a = make_args(L, s);
    spmv(L, a, 3, 3);
}

void launch_expect(bool f64, int d, const int32_t *rp, const int32_t *ci, const double2 *v, const void *state,
                   int is_ket, double2 *out, hipStream_t s)
{
    if (f64)
        hipLaunchKernelGGL(k_expect<double>, dim3(1), dim3(256), 0, s, d, rp, ci, v, state, is_ket, out);
    else
        hipLaunchKernelGGL(k_expect<float>, dim3(1), dim3(256), 0, s, d, rp, ci, v, state, is_ket, out);
}

}  // namespace qt

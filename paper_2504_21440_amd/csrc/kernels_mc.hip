// kernels_mc.hip -- Monte-Carlo wave-function (quantum-jump) trajectories on gfx950.
//
// arXiv:2504.21440, Sec. 3.3.  One 256-thread workgroup integrates one trajectory at a time with
// the adaptive Dormand-Prince 5(4) scheme and then claims the next trajectory from a device-wide
// queue, so trajectories with many jumps do not hold up the others.  Each thread owns R rows of the
// state; the state and all seven stages stay in registers.  Only the stage input is shared: it is
// written to one of two LDS buffers and the right-hand side A psi (A = -i H_eff, stored in ELL
// column-major order so every load of a row slice is coalesced) gathers from it.
//
// After an accepted step the squared norm of the new state (FP64) is compared with the trajectory's
// threshold r.  Below it, the crossing time is located with the Illinois variant of regula falsi on
// g(theta) = ln |psi(t + theta h)|^2 - ln r, each probe a fresh DP5 step of size theta h from the
// step's start (no interpolant needed); the channel k is the first whose cumulative |C_k psi|^2
// reaches u * sum_k |C_k psi|^2; psi <- C_k psi / |C_k psi|; a new threshold is drawn.  Draws come
// from Philox-4x32-10 keyed by the seed with counter (trajectory, event): event 0 gives the first
// threshold, event m >= 1 the channel uniform and the next threshold of jump m.
//
// Time-dependent problems (TD): A(t) = A_0 + sum_i f_i(t) (-i H_i) + sum_k |g_k(t)|^2 (-1/2 C_k^dag C_k)
// is one ELL whose entries carry their term in the high column bits; before each right-hand side
// the workgroup evaluates the coefficients at the stage time (its own trajectory's t + c_s h) into
// LDS, and a jump weights channel k by |g_k(t*)|^2.
#include <algorithm>
#include <cstdlib>

#include "qt_coef.h"
#include "qt_common.h"
#include "qt_mc.h"
#include "qt_rng.h"

namespace qt {

constexpr int MC_MAXC = 64;  // collapse channels handled by the jump kernel

__device__ __forceinline__ void traj_draw(uint64_t seed, uint64_t traj, uint32_t event, double *a, double *b)
{
    uint32_t c[4] = {(uint32_t)traj, (uint32_t)(traj >> 32), event, 0u};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    *a = u01(c[0], c[1]);
    *b = u01(c[2], c[3]);
}

// Block sums of two / three doubles (deterministic order, result in every thread).
__device__ __forceinline__ void block_sum_n(double *v, int n, double *scr)
{
    for (int i = 0; i < n; ++i) v[i] = wave_sum(v[i]);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0)
        for (int i = 0; i < n; ++i) scr[i * 16 + w] = v[i];
    __syncthreads();
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = 0; k < nw; ++k) s += scr[i * 16 + k];
        v[i] = s;
    }
    __syncthreads();
}

// OCC: the waves per SIMD the register allocation must allow (1: no constraint).  A large ensemble
// gains from more resident trajectories even at the price of spilled registers; a single
// trajectory does not.  ELDS: the workgroup copies the ELL of A into LDS once and every right-hand
// side of every trajectory it runs reads the matrix from there instead of from L2.
template <typename T, int R, bool TD, int OCC, bool ELDS = false>
__global__ __launch_bounds__(MC_THREADS) __attribute__((amdgpu_waves_per_eu(OCC))) void k_mc(
    const McParams *__restrict__ Pp)
{
    using V = typename vec2<T>::type;
    const McParams &P = *Pp;
    extern __shared__ char smem[];
    const int d = P.d;
    V *xs0 = (V *)smem;
    V *xs1 = xs0 + d;
    __shared__ double scr[48];
    __shared__ double pk[MC_MAXC];  // channel weights |g_k(t*)|^2 |C_k psi|^2
    __shared__ double pn[MC_MAXC];  // |C_k psi|^2, for the post-jump normalisation
    __shared__ unsigned long long jsh;
    __shared__ V cwsh[MC_MAX_TERMS + 1];  // coefficients of the current right-hand side (TD)
    const int tid = threadIdx.x;
    const V *__restrict__ ev = (const V *)P.ell_val;
    const int32_t *__restrict__ ec = P.ell_col;
    const V *__restrict__ cv = (const V *)P.cval;
    V *evs = xs1 + d;                             // ELDS: values, then columns, after the state buffers
    int32_t *ecs = (int32_t *)(evs + (size_t)P.W * d);
    if constexpr (ELDS) {
        for (int i = threadIdx.x; i < P.W * d; i += MC_THREADS) {
            evs[i] = gld(ev + i);
            ecs[i] = gld(ec + i);
        }
        __syncthreads();
    }

    auto row = [&](int m) { return tid + m * MC_THREADS; };
    // out = A(ts) x for own rows.  Every call site is preceded by a barrier after the previous
    // call, so the coefficient row may be rewritten here.
    auto rhs = [&](const V *x, V(&out)[R], double ts) {
        if constexpr (TD) {
            if (tid <= P.nterms) {
                double2 w = make_double2(1.0, 0.0);
                if (tid > 0) w = coef_value(P.coefs[tid - 1], ts);
                cwsh[tid] = from_d2<V>(w);
            }
            __syncthreads();
        }
        // complex64: entry k of all R rows of this thread at once, R independent load-gather-FMA
        // chains per entry rather than one row's W entries after another (measured: the L = 10
        // ensemble 58,700 -> 69,700 trajectories/s); complex128 keeps one row at a time, whose
        // registers the wider values would otherwise spill (22,000 -> 17,800).  Each row is summed
        // in the order k = 0 .. W-1 either way.  Global-only loads of the matrix stream: generic ones
        // would be ordered against, and waited for with, the LDS gathers of the state.
        V acc[R];
#pragma unroll
        for (int m = 0; m < R; ++m) {
            acc[m].x = 0;
            acc[m].y = 0;
        }
        if constexpr (sizeof(T) == 8) {
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const int r = row(m);
                if (r < d)
                    for (int k = 0; k < P.W; ++k) {
                        const size_t at = (size_t)k * d + r;
                        const int32_t c = ELDS ? ecs[at] : gld(ec + at);
                        const V a = ELDS ? evs[at] : gld(ev + at);
                        if constexpr (TD)
                            cfma(acc[m], cmul(a, cwsh[c >> MC_TAG_SHIFT]), x[c & ((1 << MC_TAG_SHIFT) - 1)]);
                        else
                            cfma(acc[m], a, x[c]);
                    }
            }
        } else
        for (int k = 0; k < P.W; ++k) {
            int32_t c[R];
            V a[R];
#pragma unroll
            for (int m = 0; m < R; ++m)
                if (row(m) < d) {
                    const size_t at = (size_t)k * d + row(m);
                    c[m] = ELDS ? ecs[at] : gld(ec + at);
                    a[m] = ELDS ? evs[at] : gld(ev + at);
                }
#pragma unroll
            for (int m = 0; m < R; ++m)
                if (row(m) < d) {
                    if constexpr (TD)
                        cfma(acc[m], cmul(a[m], cwsh[c[m] >> MC_TAG_SHIFT]), x[c[m] & ((1 << MC_TAG_SHIFT) - 1)]);
                    else
                        cfma(acc[m], a[m], x[c[m]]);
                }
        }
#pragma unroll
        for (int m = 0; m < R; ++m) out[m] = acc[m];
    };
    // weight |g_k(t)|^2 of collapse channel k (1 when constant)
    auto cweight = [&](int k, double tt) {
        if constexpr (TD) {
            const int q = P.cweight[k];
            if (q >= 0) return coef_value(P.coefs[q], tt).x;  // stored with modsq: the squared modulus
        }
        return 1.0;
    };
    // <x|O_q|x> / <x|x> for every e_op, into expect_tr[j][q][idx]
    auto record = [&](const V *x, uint64_t j, int idx) {
        for (int q = 0; q < P.ne; ++q) {
            const int32_t *ep = P.eptr + (size_t)q * (d + 1);
            double v[3] = {0.0, 0.0, 0.0};
            for (int i = tid; i < d; i += MC_THREADS) {
                double rr = 0.0, ri = 0.0;
                for (int p = ep[i]; p < ep[i + 1]; ++p) {
                    const double2 o = P.eval[p];
                    const double2 xv = to_d2(x[P.ecol[p]]);
                    rr += o.x * xv.x - o.y * xv.y;
                    ri += o.x * xv.y + o.y * xv.x;
                }
                const double2 c = to_d2(x[i]);
                v[0] += c.x * rr + c.y * ri;
                v[1] += c.x * ri - c.y * rr;
                v[2] += c.x * c.x + c.y * c.y;
            }
            block_sum_n(v, 3, scr);
            if (tid == 0) P.expect_tr[((size_t)j * P.ne + q) * P.nt + idx] = make_double2(v[0] / v[2], v[1] / v[2]);
        }
    };

    for (;;) {
        if (tid == 0) jsh = atomicAdd(P.queue, 1ull);
        __syncthreads();
        const uint64_t j = jsh;
        __syncthreads();
        if ((int64_t)j >= P.ntraj) break;

        V y[R], k[7][R], yn[R];
        const V *p0 = (const V *)P.psi0;
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const int r = row(m);
            if (r < d) {
                y[m] = p0[r];
                xs0[r] = y[m];
            } else {
                y[m].x = 0;
                y[m].y = 0;
            }
        }
        double r_th, unused;
        traj_draw(P.seed, j, 0u, &r_th, &unused);
        uint32_t event = 1;
        int64_t njump = 0, nrhs = 0, nacc = 0, nrej = 0, steps = 0;
        int status = ST_RUNNING;
        double t = P.tlist[0];
        __syncthreads();
        record(xs0, j, 0);
        int idx = 1;

        // DP5 trial step of size hh from (t, y) with k[0] = A y: fills k[1..6], yn (also in xs1)
        // and returns the FP64 error norm; nn receives |yn|^2.
        auto attempt = [&](double hh, double &nn) -> double {
            __syncthreads();
            const T c21 = (T)(hh * DP5::a21);
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const int r = row(m);
                if (r < d) {
                    V x = y[m];
                    caxpy(x, c21, k[0][m]);
                    xs0[r] = x;
                }
            }
            __syncthreads();
            rhs(xs0, k[1], t + DP5::c2 * hh);
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const int r = row(m);
                if (r < d) {
                    V x = y[m];
                    caxpy(x, (T)(hh * DP5::a31), k[0][m]);
                    caxpy(x, (T)(hh * DP5::a32), k[1][m]);
                    xs1[r] = x;
                }
            }
            __syncthreads();
            rhs(xs1, k[2], t + DP5::c3 * hh);
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const int r = row(m);
                if (r < d) {
                    V x = y[m];
                    caxpy(x, (T)(hh * DP5::a41), k[0][m]);
                    caxpy(x, (T)(hh * DP5::a42), k[1][m]);
                    caxpy(x, (T)(hh * DP5::a43), k[2][m]);
                    xs0[r] = x;
                }
            }
            __syncthreads();
            rhs(xs0, k[3], t + DP5::c4 * hh);
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const int r = row(m);
                if (r < d) {
                    V x = y[m];
                    caxpy(x, (T)(hh * DP5::a51), k[0][m]);
                    caxpy(x, (T)(hh * DP5::a52), k[1][m]);
                    caxpy(x, (T)(hh * DP5::a53), k[2][m]);
                    caxpy(x, (T)(hh * DP5::a54), k[3][m]);
                    xs1[r] = x;
                }
            }
            __syncthreads();
            rhs(xs1, k[4], t + DP5::c5 * hh);
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const int r = row(m);
                if (r < d) {
                    V x = y[m];
                    caxpy(x, (T)(hh * DP5::a61), k[0][m]);
                    caxpy(x, (T)(hh * DP5::a62), k[1][m]);
                    caxpy(x, (T)(hh * DP5::a63), k[2][m]);
                    caxpy(x, (T)(hh * DP5::a64), k[3][m]);
                    caxpy(x, (T)(hh * DP5::a65), k[4][m]);
                    xs0[r] = x;
                }
            }
            __syncthreads();
            rhs(xs0, k[5], t + hh);
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const int r = row(m);
                V x = y[m];
                caxpy(x, (T)(hh * DP5::b1), k[0][m]);
                caxpy(x, (T)(hh * DP5::b3), k[2][m]);
                caxpy(x, (T)(hh * DP5::b4), k[3][m]);
                caxpy(x, (T)(hh * DP5::b5), k[4][m]);
                caxpy(x, (T)(hh * DP5::b6), k[5][m]);
                yn[m] = x;
                if (r < d) xs1[r] = x;
            }
            __syncthreads();
            rhs(xs1, k[6], t + hh);
            nrhs += 6;
            double v[2] = {0.0, 0.0};
#pragma unroll
            for (int m = 0; m < R; ++m) {
                if (row(m) >= d) continue;
                double2 e = make_double2(0.0, 0.0);
                caxpy(e, hh * DP5::e1, to_d2(k[0][m]));
                caxpy(e, hh * DP5::e3, to_d2(k[2][m]));
                caxpy(e, hh * DP5::e4, to_d2(k[3][m]));
                caxpy(e, hh * DP5::e5, to_d2(k[4][m]));
                caxpy(e, hh * DP5::e6, to_d2(k[5][m]));
                caxpy(e, hh * DP5::e7, to_d2(k[6][m]));
                const double sc = P.atol + P.rtol * fmax(sqrt(abs2d(y[m])), sqrt(abs2d(yn[m])));
                v[0] += (e.x * e.x + e.y * e.y) / (sc * sc);
                v[1] += abs2d(yn[m]);
            }
            block_sum_n(v, 2, scr);
            nn = v[1];
            return sqrt(v[0] / d);
        };

        double h = 0.0;
        if (P.nt > 1) {
            rhs(xs0, k[0], t);
            nrhs += 1;
            if (P.use_h0) {
                h = P.h0;
            } else {
                double v[2] = {0.0, 0.0};
#pragma unroll
                for (int m = 0; m < R; ++m) {
                    if (row(m) >= d) continue;
                    const double ya = sqrt(abs2d(y[m]));
                    const double sc = P.atol + P.rtol * ya;
                    v[0] += ya * ya / (sc * sc);
                    v[1] += abs2d(k[0][m]) / (sc * sc);
                }
                block_sum_n(v, 2, scr);
                const double d0 = sqrt(v[0] / d), d1 = sqrt(v[1] / d);
                const double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
#pragma unroll
                for (int m = 0; m < R; ++m) {
                    const int r = row(m);
                    if (r < d) {
                        V x = y[m];
                        caxpy(x, (T)h0, k[0][m]);
                        xs1[r] = x;
                    }
                }
                __syncthreads();
                rhs(xs1, k[1], t + h0);
                nrhs += 1;
                double w2 = 0.0;
#pragma unroll
                for (int m = 0; m < R; ++m) {
                    if (row(m) >= d) continue;
                    const double2 f1 = to_d2(k[1][m]), f0 = to_d2(k[0][m]);
                    const double sc = P.atol + P.rtol * sqrt(abs2d(y[m]));
                    const double dx = (f1.x - f0.x) / h0, dy = (f1.y - f0.y) / h0;
                    w2 += (dx * dx + dy * dy) / (sc * sc);
                }
                block_sum_n(&w2, 1, scr);
                const double d2 = sqrt(w2 / d);
                const double mx = fmax(d1, d2);
                const double h1 = (mx <= 1e-15) ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / mx, 0.2);
                h = fmin(100.0 * h0, h1);
            }
        }
        double err_prev = 1e-4;
        int last_rej = 0;
        while (idx < P.nt) {
            if (steps >= P.max_steps) {
                status = 4;  // QT_EMAXSTEPS
                break;
            }
            ++steps;
            int32_t land;
            const double ht = clip_step(t, h, P.tlist[idx], &land);
            double nrm;
            const double err = attempt(ht, nrm);
            if (!isfinite(err)) {
                status = 6;  // QT_ENONFINITE
                break;
            }
            if (err > 1.0) {
                ++nrej;
                h = ht * reject_factor(err);
                last_rej = 1;
                if (h < 1e-14 * fmax(1.0, fabs(t))) {
                    status = 5;  // QT_EDTMIN
                    break;
                }
                continue;
            }
            ++nacc;
            double hn = ht * pi_factor(err, err_prev);
            if (last_rej && hn > ht) hn = ht;
            err_prev = fmax(err, 1e-4);
            last_rej = 0;
            if (nrm >= r_th || P.nc == 0) {  // no collapse channel: nothing to jump into
                t = land ? P.tlist[idx] : t + ht;
#pragma unroll
                for (int m = 0; m < R; ++m) {
                    y[m] = yn[m];
                    k[0][m] = k[6][m];
                }
                h = hn;
                if (land) record(xs1, j, idx++);
                continue;
            }
            // ---- quantum jump inside [t, t + ht]: locate the crossing of |psi|^2 = r ----
            double ny[1] = {0.0};
#pragma unroll
            for (int m = 0; m < R; ++m)
                if (row(m) < d) ny[0] += abs2d(y[m]);
            block_sum_n(ny, 1, scr);
            const double lr = log(r_th);
            double a = 0.0, ga = log(ny[0]) - lr, b = 1.0, gb = log(nrm) - lr;
            double th = 1.0, thp = 1.0;
            int side = 0;
            for (int it = 0; it < 64; ++it) {
                th = (a * gb - b * ga) / (gb - ga);
                if (!(th > a && th < b)) th = 0.5 * (a + b);
                double nn;
                (void)attempt(th * ht, nn);
                const double g = log(nn) - lr;
                if (fabs(g) <= 1e-12) break;
                if (fabs(th - thp) * ht <= 1e-10 * fmax(1.0, fabs(t))) break;
                thp = th;
                if (g > 0.0) {
                    a = th;
                    ga = g;
                    if (side == 1) gb *= 0.5;
                    side = 1;
                } else {
                    b = th;
                    gb = g;
                    if (side == -1) ga *= 0.5;
                    side = -1;
                }
            }
            // xs1 (and yn) hold psi at the crossing
            const double tj = t + th * ht;
            double u, rnext;
            traj_draw(P.seed, j, event, &u, &rnext);
            ++event;
            for (int c = 0; c < P.nc; ++c) {
                const int32_t *cp = P.cptr + (size_t)c * (d + 1);
                double v[1] = {0.0};
                for (int i = tid; i < d; i += MC_THREADS) {
                    V acc;
                    acc.x = 0;
                    acc.y = 0;
                    for (int p = cp[i]; p < cp[i + 1]; ++p) cfma(acc, cv[p], xs1[P.ccol[p]]);
                    v[0] += abs2d(acc);
                }
                block_sum_n(v, 1, scr);
                if (tid == 0) {
                    pn[c] = v[0];
                    pk[c] = v[0] * cweight(c, tj);
                }
            }
            __syncthreads();
            double tot = 0.0;
            for (int c = 0; c < P.nc; ++c) tot += pk[c];
            const double target = u * tot;
            double cum = 0.0;
            int ch = P.nc - 1;
            for (int c = 0; c < P.nc; ++c) {
                cum += pk[c];
                if (cum >= target) {
                    ch = c;
                    break;
                }
            }
            const double inv = 1.0 / sqrt(pn[ch]);
            const int32_t *cp = P.cptr + (size_t)ch * (d + 1);
#pragma unroll
            for (int m = 0; m < R; ++m) {
                const int r = row(m);
                V acc;
                acc.x = 0;
                acc.y = 0;
                if (r < d)
                    for (int p = cp[r]; p < cp[r + 1]; ++p) cfma(acc, cv[p], xs1[P.ccol[p]]);
                y[m] = cscale(acc, (T)inv);
            }
            if (tid == 0 && njump < P.maxj) {
                P.jtimes[(size_t)j * P.maxj + njump] = tj;
                P.jchan[(size_t)j * P.maxj + njump] = ch;
            }
            ++njump;
            r_th = rnext;
            // the root search keeps th strictly inside (0, 1), so a jump always falls before the end
            // of the step, and the save time it was aiming at (if any) is recorded by a later step
            t = tj;
            __syncthreads();  // every thread is done reading xs1 / pk / pn
#pragma unroll
            for (int m = 0; m < R; ++m)
                if (row(m) < d) xs0[row(m)] = y[m];
            __syncthreads();
            rhs(xs0, k[0], t);
            nrhs += 1;
            h = hn;
        }
        if (tid == 0) {
            P.njumps[j] = njump;
            P.status[j] = status == ST_RUNNING ? ST_DONE : status;
            P.nrhs[j] = nrhs;
            P.naccept[j] = nacc;
            P.nreject[j] = nrej;
        }
        __syncthreads();
    }
}

// Ensemble mean and standard error (unbiased variance of the real part), one block per (e_op, t).
__global__ __launch_bounds__(256) void k_mc_stats(const double2 *__restrict__ tr, int64_t ntraj, int ne, int nt,
                                                  double2 *mean, double *se)
{
    __shared__ double scr[16];
    const int q = blockIdx.x;  // e_op * nt + time
    const size_t stride = (size_t)ne * nt;
    double sr = 0.0, si = 0.0;
    for (int64_t j = threadIdx.x; j < ntraj; j += blockDim.x) {
        const double2 v = tr[j * stride + q];
        sr += v.x;
        si += v.y;
    }
    sr = block_sum(sr, scr);
    si = block_sum(si, scr);
    const double mr = sr / (double)ntraj, mi = si / (double)ntraj;
    double vv = 0.0;
    for (int64_t j = threadIdx.x; j < ntraj; j += blockDim.x) {
        const double x = tr[j * stride + q].x - mr;
        vv += x * x;
    }
    vv = block_sum(vv, scr);
    if (threadIdx.x == 0) {
        mean[q] = make_double2(mr, mi);
        se[q] = ntraj > 1 ? sqrt(vv / (double)(ntraj - 1) / (double)ntraj) : 0.0;
    }
}

__global__ void k_mc_queue_reset(unsigned long long *q) { *q = 0ull; }

template <typename T, int R, bool TD, int OCC, bool ELDS = false> static const void *mc_fn()
{
    return (const void *)k_mc<T, R, TD, OCC, ELDS>;
}

// Ensembles of at least this many complex64 trajectories with 2, 4 or 8 rows per thread take the
// variant held to 3 waves per SIMD (2 at 8 rows): more trajectories in flight outweigh the spilled
// registers (measured on dissipative chains of L = 9, 10, 11: +34%, +20% and +61% trajectories/s
// at 2,048 trajectories); a lone trajectory runs 10-20% slower there, so it keeps the other one.
constexpr int64_t MC_DENSE_ENSEMBLE = 2048;
static bool mc_occ3(const McParams &p, bool f64)
{
    return !f64 && (p.rows == 2 || p.rows == 4 || p.rows == 8) && p.ntraj >= MC_DENSE_ENSEMBLE;
}

// Bytes of LDS beyond the state buffers that the ELL of A takes (values and columns).
static size_t mc_ell_lds(const McParams &p, bool f64) { return (size_t)p.W * p.d * ((f64 ? 16 : 8) + 4); }
static size_t mc_lds_base(const McParams &p, bool f64) { return (size_t)2 * p.d * (f64 ? 16 : 8); }
constexpr size_t MC_LDS_LIMIT = 160 * 1024 - 4096;  // gfx950 LDS per workgroup, less the static arrays

// With QTAMD_MC_ELDS=1, complex64 ensembles whose ELL fits next to the state buffers in LDS (2 or 4
// rows per thread, constant A) read the matrix from LDS.  Off by default: one such workgroup fills
// a CU's LDS, and on the L = 10 ensemble (10,000 trajectories) that ran at 39,100 trajectories/s
// against 57,800 for the L2 variant held to 3 waves per SIMD.
static bool mc_elds(const McParams &p, bool f64, bool td)
{
    static const bool on = [] {
        const char *e = std::getenv("QTAMD_MC_ELDS");
        return e && std::atoi(e) == 1;
    }();
    return on && !f64 && !td && (p.rows == 2 || p.rows == 4) &&
           mc_lds_base(p, f64) + mc_ell_lds(p, f64) <= MC_LDS_LIMIT;
}

template <typename T, bool TD> static const void *mc_pick(int rows, bool occ3)
{
    switch (rows) {
    case 1: return mc_fn<T, 1, TD, 1>();
    case 2: return occ3 ? mc_fn<T, 2, TD, 3>() : mc_fn<T, 2, TD, 1>();
    case 4: return occ3 ? mc_fn<T, 4, TD, 3>() : mc_fn<T, 4, TD, 1>();
    case 8: return occ3 ? mc_fn<T, 8, TD, 2>() : mc_fn<T, 8, TD, 1>();
    default: return mc_fn<T, 16, TD, 1>();
    }
}

template <typename T, int R, int OCC>
static void mc_launch_t(const McParams *dev_p, bool td, int grid, size_t lds, hipStream_t s)
{
    if (td) hipLaunchKernelGGL((k_mc<T, R, true, OCC>), dim3(grid), dim3(MC_THREADS), lds, s, dev_p);
    else hipLaunchKernelGGL((k_mc<T, R, false, OCC>), dim3(grid), dim3(MC_THREADS), lds, s, dev_p);
}

static size_t mc_lds(const McParams &p, bool f64, bool td)
{
    return mc_lds_base(p, f64) + (mc_elds(p, f64, td) ? mc_ell_lds(p, f64) : 0);
}

int mc_grid(const McParams &p, bool f64, bool td, int device)
{
    const bool o3 = mc_occ3(p, f64);
    const void *fn = f64 ? (td ? mc_pick<double, true>(p.rows, o3) : mc_pick<double, false>(p.rows, o3))
                         : (td ? mc_pick<float, true>(p.rows, o3) : mc_pick<float, false>(p.rows, o3));
    if (mc_elds(p, f64, td)) fn = p.rows == 2 ? mc_fn<float, 2, false, 1, true>() : mc_fn<float, 4, false, 1, true>();
    const size_t lds = mc_lds(p, f64, td);
    if (lds > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, MC_THREADS, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 256;
    const int64_t g = std::min<int64_t>(p.ntraj, (int64_t)per_cu * cus);
    return (int)std::max<int64_t>(1, g);
}

void mc_launch(const McParams &p, const McParams *dev_p, bool f64, bool td, int grid, hipStream_t s)
{
    const size_t lds = mc_lds(p, f64, td);
    if (mc_elds(p, f64, td)) {
        if (p.rows == 2) hipLaunchKernelGGL((k_mc<float, 2, false, 1, true>), dim3(grid), dim3(MC_THREADS), lds, s, dev_p);
        else hipLaunchKernelGGL((k_mc<float, 4, false, 1, true>), dim3(grid), dim3(MC_THREADS), lds, s, dev_p);
        return;
    }
    if (f64) {
        switch (p.rows) {
        case 1: mc_launch_t<double, 1, 1>(dev_p, td, grid, lds, s); break;
        case 2: mc_launch_t<double, 2, 1>(dev_p, td, grid, lds, s); break;
        case 4: mc_launch_t<double, 4, 1>(dev_p, td, grid, lds, s); break;
        case 8: mc_launch_t<double, 8, 1>(dev_p, td, grid, lds, s); break;
        default: mc_launch_t<double, 16, 1>(dev_p, td, grid, lds, s); break;
        }
    } else {
        switch (p.rows) {
        case 1: mc_launch_t<float, 1, 1>(dev_p, td, grid, lds, s); break;
        case 2:
            if (mc_occ3(p, f64)) mc_launch_t<float, 2, 3>(dev_p, td, grid, lds, s);
            else mc_launch_t<float, 2, 1>(dev_p, td, grid, lds, s);
            break;
        case 4:
            if (mc_occ3(p, f64)) mc_launch_t<float, 4, 3>(dev_p, td, grid, lds, s);
            else mc_launch_t<float, 4, 1>(dev_p, td, grid, lds, s);
            break;
        case 8:
            if (mc_occ3(p, f64)) mc_launch_t<float, 8, 2>(dev_p, td, grid, lds, s);
            else mc_launch_t<float, 8, 1>(dev_p, td, grid, lds, s);
            break;
        default: mc_launch_t<float, 16, 1>(dev_p, td, grid, lds, s); break;
        }
    }
}

void mc_launch_stats(const double2 *expect_tr, int64_t ntraj, int ne, int nt, double2 *mean, double *se, hipStream_t s)
{
    if (ne * nt > 0) hipLaunchKernelGGL(k_mc_stats, dim3(ne * nt), dim3(256), 0, s, expect_tr, ntraj, ne, nt, mean, se);
}

void mc_launch_queue_reset(unsigned long long *q, hipStream_t s)
{
    hipLaunchKernelGGL(k_mc_queue_reset, dim3(1), dim3(1), 0, s, q);
}

}  // namespace qt

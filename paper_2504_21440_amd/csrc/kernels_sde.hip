// kernels_sde.hip -- stochastic Schrodinger and master equations under homodyne detection on gfx950.
//
// arXiv:2504.21440, Sec. 3.5 (Ito form): one 256-thread workgroup integrates one trajectory at a
// time and claims the next from a device-wide queue.  Each thread owns R rows of the state vector x
// (the ket, or vec(rho)); x, the drift and the new state stay in registers, the products B_n x of
// the thread's rows in LDS, and the vector every gather reads (x, then each supporting value) in
// one LDS buffer.  The operators A and B_n are ELL, column-major, read through L2.
//
// Step: the tlist interval is cut into equal steps of at most dt.  With a = a(x) and
// b_n = B_n x - cg mu_n x,
//     x' = x + a h + sum_n b_n dW_n + sum_n (b_n(U_n) - b_n) (dW_n^2 - h) / (2 sqrt h),
//     U_n = x + a h + b_n sqrt h,
// the derivative-free order-1.0 strong scheme of Platen (Kloeden & Platen, Sec. 11.1) taken for
// each Wiener process with its own supporting value, then x' is renormalised (unit norm for the
// SSE, unit trace for the SME).  All reductions (mu_n, norms, traces, expectation values) are FP64
// in a fixed order.  dW_n = sqrt(h) z with z from Philox-4x32-10 and the Box-Muller transform,
// counter (trajectory, step, 1 + n/2).
#include <algorithm>

#include "qt_common.h"
#include "qt_rng.h"
#include "qt_sde.h"

namespace qt {

// Block sums of N doubles in a fixed order; the result in every thread.  N is a compile-time
// size so the values stay in registers.
template <int N> __device__ __forceinline__ void sde_block_sum(double (&v)[N], double *scr)
{
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = wave_sum(v[i]);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < N; ++i) scr[i * 4 + w] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = ((scr[i * 4] + scr[i * 4 + 1]) + scr[i * 4 + 2]) + scr[i * 4 + 3];
    __syncthreads();
}

// OCC: the waves per SIMD the register allocation must allow (1: no constraint).
template <typename T, int R, bool SME, int OCC>
__global__ __launch_bounds__(SDE_THREADS) __attribute__((amdgpu_waves_per_eu(OCC))) void k_sde(
    const SdeParams *__restrict__ Pp)
{
    using V = typename vec2<T>::type;
    const SdeParams &P = *Pp;
    extern __shared__ char smem[];
    const int n = P.n, m = P.m;
    V *xs = (V *)smem;  // the vector the gathers read
    V *bx = xs + n;     // B_k x at the thread's own rows, m blocks of n
    __shared__ double scr[4 * (SDE_MAX_SC + 1)];
    __shared__ unsigned long long jsh;
    const int tid = threadIdx.x;
    const V *__restrict__ av = (const V *)P.a_val;
    const V *__restrict__ bv = (const V *)P.b_val;
    auto row = [&](int q) { return tid + q * SDE_THREADS; };
    auto is_diag = [&](int r) { return r % (P.d + 1) == 0; };
    // (A xs) at own row r
    auto a_row = [&](int r) {
        V acc;
        acc.x = 0;
        acc.y = 0;
        // global-only loads of the operator streams, apart from the LDS gathers of the state
        for (int k = 0; k < P.WA; ++k) cfma(acc, gld(av + (size_t)k * n + r), xs[gld(P.a_col + (size_t)k * n + r)]);
        return acc;
    };
    // (B_j xs) at own row r
    auto b_row = [&](int j, int r) {
        V acc;
        acc.x = 0;
        acc.y = 0;
        const size_t base = (size_t)j * P.WB * n;
        for (int k = 0; k < P.WB; ++k)
            cfma(acc, gld(bv + base + (size_t)k * n + r), xs[gld(P.b_col + base + (size_t)k * n + r)]);
        return acc;
    };
    // this thread's share of mu for the state u (its own rows) and its image Bu:
    // SSE: Re sum conj(u) Bu (the caller divides by |u|^2 and doubles), SME: Re of the diagonal of Bu
    auto mu_part = [&](V u, V bu, int r) {
        if constexpr (SME) return is_diag(r) ? (double)bu.x : 0.0;
        else return (double)u.x * (double)bu.x + (double)u.y * (double)bu.y;
    };
    auto record = [&](uint64_t j, int idx) {
        // expectation values of the state in xs
        for (int q = 0; q < P.ne; ++q) {
            const int32_t *ep = P.eptr + (size_t)q * (P.d + 1);
            double v[3] = {0.0, 0.0, 0.0};
            if constexpr (SME) {
                // Tr(O rho) = sum_{(i,j) in O} O_ij rho_ji
                for (int p = ep[0] + tid; p < ep[P.d]; p += SDE_THREADS) {
                    const double2 o = P.eval[p];
                    const double2 r = to_d2(xs[P.evidx[p]]);
                    v[0] += o.x * r.x - o.y * r.y;
                    v[1] += o.x * r.y + o.y * r.x;
                }
                v[2] = 1.0;
            } else {
                for (int i = tid; i < P.d; i += SDE_THREADS) {
                    double rr = 0.0, ri = 0.0;
                    for (int p = ep[i]; p < ep[i + 1]; ++p) {
                        const double2 o = P.eval[p];
                        const double2 xv = to_d2(xs[P.ecol[p]]);
                        rr += o.x * xv.x - o.y * xv.y;
                        ri += o.x * xv.y + o.y * xv.x;
                    }
                    const double2 c = to_d2(xs[i]);
                    v[0] += c.x * rr + c.y * ri;
                    v[1] += c.x * ri - c.y * rr;
                    v[2] += c.x * c.x + c.y * c.y;
                }
            }
            sde_block_sum(v, scr);
            if (tid == 0) {
                const double nn = SME ? 1.0 : v[2];
                P.expect_tr[((size_t)j * P.ne + q) * P.nt + idx] = make_double2(v[0] / nn, v[1] / nn);
            }
        }
    };

    for (;;) {
        if (tid == 0) jsh = atomicAdd(P.queue, 1ull);
        __syncthreads();
        const uint64_t j = jsh;
        __syncthreads();
        if ((int64_t)j >= P.ntraj) break;

        V x[R], xn[R], a[R];
        const V *x0 = (const V *)P.x0;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = row(q);
            x[q].x = 0;
            x[q].y = 0;
            if (r < n) {
                x[q] = x0[r];
                xs[r] = x[q];
            }
        }
        __syncthreads();
        record(j, 0);
        int status = ST_RUNNING;
        uint32_t step = 0;
        for (int iv = 0; iv + 1 < P.nt && status == ST_RUNNING; ++iv) {
            const double len = P.tlist[iv + 1] - P.tlist[iv];
            const int ns = P.nsub[iv];
            const double h = len / (double)ns, sq = sqrt(h);
            double acc[SDE_MAX_SC];
#pragma unroll
            for (int k = 0; k < SDE_MAX_SC; ++k) acc[k] = 0.0;
            for (int s = 0; s < ns; ++s, ++step) {
                // xs holds x here (written by the previous step or the start)
                double red[SDE_MAX_SC + 1];  // mu parts, then |x|^2 (SSE)
#pragma unroll
                for (int k = 0; k <= SDE_MAX_SC; ++k) red[k] = 0.0;
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const int r = row(q);
                    if (r >= n) continue;
                    a[q] = a_row(r);
#pragma unroll
                    for (int k = 0; k < SDE_MAX_SC; ++k) {
                        if (k >= m) break;
                        const V b = b_row(k, r);
                        bx[(size_t)k * n + r] = b;
                        red[k] += mu_part(x[q], b, r);
                    }
                    red[SDE_MAX_SC] += abs2d(x[q]);
                }
                sde_block_sum(red, scr);
                double mu[SDE_MAX_SC], dW[SDE_MAX_SC];
#pragma unroll
                for (int k = 0; k < SDE_MAX_SC; ++k) {
                    mu[k] = SME ? red[k] : 2.0 * red[k] / red[SDE_MAX_SC];
                    dW[k] = 0.0;
                }
#pragma unroll
                for (int k = 0; k < SDE_MAX_SC; k += 2) {
                    if (k >= m) break;
                    double z0, z1;
                    wiener_normals(P.seed, j, step, (uint32_t)(k / 2), &z0, &z1);
                    dW[k] = sq * z0;
                    dW[k + 1] = k + 1 < m ? sq * z1 : 0.0;
                }
#pragma unroll
                for (int k = 0; k < SDE_MAX_SC; ++k) acc[k] += mu[k] * h + dW[k];
                // drift (SSE: + sum mu/2 B x - mu^2/8 x) and the Euler-Maruyama part of the update
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const int r = row(q);
                    if (r >= n) continue;
                    if constexpr (!SME) {
#pragma unroll
                        for (int k = 0; k < SDE_MAX_SC; ++k) {
                            if (k >= m) break;
                            caxpy(a[q], (T)(0.5 * mu[k]), bx[(size_t)k * n + r]);
                            caxpy(a[q], (T)(-0.125 * mu[k] * mu[k]), x[q]);
                        }
                    }
                    V y = x[q];
                    caxpy(y, (T)h, a[q]);
#pragma unroll
                    for (int k = 0; k < SDE_MAX_SC; ++k) {
                        if (k >= m) break;
                        V b = bx[(size_t)k * n + r];
                        caxpy(b, (T)(-P.cg * mu[k]), x[q]);
                        caxpy(y, (T)dW[k], b);
                    }
                    xn[q] = y;
                }
                // supporting values U_k = x + a h + b_k sqrt(h) and the correction of each process
#pragma unroll
                for (int k = 0; k < SDE_MAX_SC; ++k) {
                    if (k >= m) break;
                    __syncthreads();  // every gather of xs is done
                    V u[R];
#pragma unroll
                    for (int q = 0; q < R; ++q) {
                        const int r = row(q);
                        if (r >= n) continue;
                        V b = bx[(size_t)k * n + r];
                        caxpy(b, (T)(-P.cg * mu[k]), x[q]);
                        u[q] = x[q];
                        caxpy(u[q], (T)h, a[q]);
                        caxpy(u[q], (T)sq, b);
                        xs[r] = u[q];
                    }
                    __syncthreads();
                    double rs[2] = {0.0, 0.0};  // mu part, |U|^2
                    V bu[R];
#pragma unroll
                    for (int q = 0; q < R; ++q) {
                        const int r = row(q);
                        if (r >= n) continue;
                        bu[q] = b_row(k, r);
                        rs[0] += mu_part(u[q], bu[q], r);
                        rs[1] += abs2d(u[q]);
                    }
                    sde_block_sum(rs, scr);
                    const double mus = SME ? rs[0] : 2.0 * rs[0] / rs[1];
                    const double w = (dW[k] * dW[k] - h) / (2.0 * sq);
#pragma unroll
                    for (int q = 0; q < R; ++q) {
                        const int r = row(q);
                        if (r >= n) continue;
                        V b = bx[(size_t)k * n + r];
                        caxpy(b, (T)(-P.cg * mu[k]), x[q]);
                        V bs = bu[q];
                        caxpy(bs, (T)(-P.cg * mus), u[q]);
                        caxpy(xn[q], (T)w, bs);
                        caxpy(xn[q], (T)(-w), b);
                    }
                }
                // renormalise: unit norm (SSE) or unit trace (SME)
                double nr[1] = {0.0};
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const int r = row(q);
                    if (r >= n) continue;
                    if constexpr (SME) nr[0] += is_diag(r) ? (double)xn[q].x : 0.0;
                    else nr[0] += abs2d(xn[q]);
                }
                sde_block_sum(nr, scr);
                const double sc = SME ? nr[0] : sqrt(nr[0]);
                if (!isfinite(sc) || sc == 0.0) {
                    status = 6;  // QT_ENONFINITE
                    break;
                }
                const T inv = (T)(1.0 / sc);
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const int r = row(q);
                    if (r >= n) continue;
                    x[q] = cscale(xn[q], inv);
                    xs[r] = x[q];
                }
                __syncthreads();
            }
            if (status != ST_RUNNING) break;
            if (tid == 0) {
#pragma unroll
                for (int k = 0; k < SDE_MAX_SC; ++k)
                    if (k < m) P.meas[((size_t)j * m + k) * (P.nt - 1) + iv] = acc[k] / len;
            }
            record(j, iv + 1);
        }
        if (tid == 0) P.status[j] = status == ST_RUNNING ? ST_DONE : status;
        __syncthreads();
    }
}

size_t sde_lds_bytes(const SdeParams &p, bool f64) { return (size_t)(1 + p.m) * p.n * (f64 ? 16 : 8); }

template <typename T, int R, bool SME, int OCC> static const void *sde_fn()
{
    return (const void *)k_sde<T, R, SME, OCC>;
}

// Complex64 ensembles with 4 or 8 rows per thread and more trajectories than the device has compute
// units take the variant held to 2 waves per SIMD, so that two trajectories share a CU (measured on
// the homodyne master equation on a 256-CU device: 512 trajectories at n = 1,024 / 1,600 run 77% /
// 64% faster than two rounds of 256 in the unconstrained variant, bitwise the same; the FP64 kernel
// spills too much there and keeps the unconstrained variant).
static int device_cus(int device)
{
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 256;
    return cus;
}

void sde_choose_variant(SdeParams &p, bool f64, int device)
{
    p.occ2 = (!f64 && (p.rows == 4 || p.rows == 8) && p.ntraj > (int64_t)device_cus(device)) ? 1 : 0;
}

template <typename T, bool SME> static const void *sde_pick(int rows, bool occ2)
{
    switch (rows) {
    case 1: return sde_fn<T, 1, SME, 1>();
    case 2: return sde_fn<T, 2, SME, 1>();  // already 2 waves per SIMD
    case 4: return occ2 ? sde_fn<T, 4, SME, 2>() : sde_fn<T, 4, SME, 1>();
    case 8: return occ2 ? sde_fn<T, 8, SME, 2>() : sde_fn<T, 8, SME, 1>();
    default: return sde_fn<T, 16, SME, 1>();
    }
}

static const void *sde_kernel(const SdeParams &p, bool f64)
{
    if (f64) return p.sme ? sde_pick<double, true>(p.rows, false) : sde_pick<double, false>(p.rows, false);
    return p.sme ? sde_pick<float, true>(p.rows, p.occ2 != 0) : sde_pick<float, false>(p.rows, p.occ2 != 0);
}

int sde_grid(const SdeParams &p, bool f64, int device)
{
    const void *fn = sde_kernel(p, f64);
    const size_t lds = sde_lds_bytes(p, f64);
    if (lds > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, SDE_THREADS, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return (int)std::max<int64_t>(1, std::min<int64_t>(p.ntraj, (int64_t)per_cu * device_cus(device)));
}

void sde_launch(const SdeParams &p, const SdeParams *dev_p, bool f64, int grid, hipStream_t s)
{
    const void *fn = sde_kernel(p, f64);
    void *args[] = {(void *)&dev_p};
    (void)hipLaunchKernel(fn, dim3(grid), dim3(SDE_THREADS), args, sde_lds_bytes(p, f64), s);
}

}  // namespace qt

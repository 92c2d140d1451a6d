// kernels_dense.hip -- dense operator-form master-equation solver on the gfx950 matrix cores.
//
// L(rho) = A rho + (A rho)^dag + sum_k C_k rho C_k^dag (arXiv:2504.21440, Sec. 3.2, with
// A = -i H - 1/2 sum_k C_k^dag C_k).  For Hermitian rho, C rho C^dag = C (C rho)^dag, so every
// product takes the operator as its left factor:
//     X_k = C_k rho,   Z = sum_k C_k X_k^dag,   M = A rho,   L(rho) = Z + M + M^dag,
// i.e. 1 + 2K complex matrix products.  Complex products run on real MFMA instructions
// (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64): Re += Ar Br - Ai Bi, Im += Ar Bi + Ai Br.
//
// One workgroup owns one problem for the whole launch and runs the adaptive Dormand-Prince 5(4)
// loop itself.  Wave w owns a contiguous run of output tiles (row-major tile order, near-equal runs
// per wave); for each tile row its run touches it loads the 16 operator rows from L2 into
// registers (all loads in flight at once), so the inner MFMA loop reads only LDS.  LDS holds two NP x (NP+1) planar (re, im)
// matrices: B0 = the stage input rho_s, B1 = scratch for X_k and then M.  The odd row stride keeps
// the transposed walks conflict-free.  Runge-Kutta stages of the elements a lane owns live in a
// per-problem global buffer in tile order (contiguous per-lane accesses); the epilogue of each
// stage is applied element by element as the right-hand side is produced.  Step control, error
// norm, trace renormalisation and expectation values are FP64 and stay inside the workgroup.
#include <algorithm>
#include <vector>

#include "qt_common.h"
#include "qt_dense.h"
#include "qt_tune.h"

namespace qt {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

// Every buffer access of this file goes through the global-only loads and stores of qt_common.h
// (gld / gst and the wider ones below): the LDS traffic of the matrix products then neither
// orders against nor waits for it.
// The 4 consecutive tile-order elements a lane owns in one output tile, with 16-byte accesses.
typedef float gf4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void gld4(const float2 *p, float2 (&r)[4])
{
    const gf4 a = *(const QT_GLOBAL gf4 *)p, b = *(const QT_GLOBAL gf4 *)(p + 2);
    r[0] = make_float2(a.x, a.y);
    r[1] = make_float2(a.z, a.w);
    r[2] = make_float2(b.x, b.y);
    r[3] = make_float2(b.z, b.w);
}
__device__ __forceinline__ void gld4(const double2 *p, double2 (&r)[4])
{
#pragma unroll
    for (int v = 0; v < 4; ++v) r[v] = gld(p + v);
}
__device__ __forceinline__ void gst4(float2 *p, const float2 (&r)[4])
{
    gf4 a, b;
    a.x = r[0].x;
    a.y = r[0].y;
    a.z = r[1].x;
    a.w = r[1].y;
    b.x = r[2].x;
    b.y = r[2].y;
    b.z = r[3].x;
    b.w = r[3].y;
    *(QT_GLOBAL gf4 *)p = a;
    *(QT_GLOBAL gf4 *)(p + 2) = b;
}
__device__ __forceinline__ void gst4(double2 *p, const double2 (&r)[4])
{
#pragma unroll
    for (int v = 0; v < 4; ++v) gst(p + v, r[v]);
}
// Two consecutive elements (16 or 32 bytes).
__device__ __forceinline__ void gld2(const float2 *p, float2 (&r)[2])
{
    const gf4 a = *(const QT_GLOBAL gf4 *)p;
    r[0] = make_float2(a.x, a.y);
    r[1] = make_float2(a.z, a.w);
}
__device__ __forceinline__ void gld2(const double2 *p, double2 (&r)[2])
{
    r[0] = gld(p);
    r[1] = gld(p + 1);
}
__device__ __forceinline__ void gst2(float2 *p, const float2 &r0, const float2 &r1)
{
    gf4 a;
    a.x = r0.x;
    a.y = r0.y;
    a.z = r1.x;
    a.w = r1.y;
    *(QT_GLOBAL gf4 *)p = a;
}
__device__ __forceinline__ void gst2(double2 *p, const double2 &r0, const double2 &r1)
{
    gst(p, r0);
    gst(p + 1, r1);
}

template <typename T> struct Mfma;
template <> struct Mfma<float> {
    using acc = v4f;
    static __device__ __forceinline__ acc mma(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<double> {
    using acc = v4d;
    static __device__ __forceinline__ acc mma(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// Row of the 16x16 output tile held in accumulator slot v by a lane with k4 = lane / 16 (the
// column is lane % 16).  Measured on gfx950: the f32 16x16x4 instruction gives each lane four
// consecutive rows (4 k4 + v); the f64 one interleaves them (k4 + 4 v).
template <typename T> __device__ __forceinline__ int mrow(int k4, int v)
{
    return sizeof(T) == 8 ? k4 + 4 * v : 4 * k4 + v;
}

// Work split: the NT x NT output tiles, in row-major order, are cut into WV contiguous chunks of
// near-equal size, one per wave, so the matrix-core work spreads evenly over the 4 SIMDs of the CU
// (with one wave per 16-row tile row, NP = 80 would put 2 of its 5 waves, 40% of the work, on one
// SIMD).  A wave reloads its operator fragments only when its chunk crosses into the next tile row.
template <typename T, int NP, int WV> struct DenseGeom {
    static constexpr int S = NP + 1;                   // LDS row stride
    static constexpr int NT = NP / 16;                 // tiles per side
    static constexpr int TILES = NT * NT;
    static constexpr int WAVES = WV;
    static constexpr int MAXJ = (TILES + WV - 1) / WV;  // tiles per wave (upper bound)
    static constexpr int KF = NP / 4;                   // operator fragments per lane
    static constexpr int PLANE = NP * S;
    static constexpr size_t LDS_BYTES = (size_t)6 * PLANE * sizeof(T);  // B0, B1, B2 (re, im)
    // first tile of wave w's chunk (the chunk of w ends where that of w + 1 starts)
    static __device__ __forceinline__ int chunk0(int w) { return (w * TILES) / WV; }
};

// Element index of (tile t, lane, v) in the tile-ordered global vectors.
__device__ __forceinline__ size_t tix(int t, int lane, int v) { return ((size_t)t * 64 + lane) * 4 + v; }

// acc += a * b on the matrix cores, complex a = (ar, ai), b = (br, bi).
template <typename T>
__device__ __forceinline__ void cmma(typename Mfma<T>::acc &aR, typename Mfma<T>::acc &aI, T ar, T ai, T br, T bi)
{
    aR = Mfma<T>::mma(ar, br, aR);
    aR = Mfma<T>::mma(-ai, bi, aR);
    aI = Mfma<T>::mma(ar, bi, aI);
    aI = Mfma<T>::mma(ai, br, aI);
}

// Lane fragments of rows [I*16, I*16+16) of an np x np operator: frag[f] = Op(I*16 + lane%16, 4f + lane/16).
template <typename T, int NP>
__device__ __forceinline__ void load_frag(const typename vec2<T>::type *__restrict__ op, int I, int lane,
                                          typename vec2<T>::type (&frag)[NP / 4])
{
    const typename vec2<T>::type *row = op + (size_t)(I * 16 + (lane & 15)) * NP + (lane >> 4);
#pragma unroll
    for (int f = 0; f < NP / 4; ++f) frag[f] = gld(row + 4 * f);
}

template <typename T, int NP, int WV> struct DenseRhs {
    using G = DenseGeom<T, NP, WV>;
    using V = typename vec2<T>::type;
    using Acc = typename Mfma<T>::acc;
    static constexpr int S = G::S;

    // C = frag (rows of this wave) times the LDS matrix R (re, im planes), one 16x16 tile J.
    static __device__ __forceinline__ void tile_mm(const V (&frag)[G::KF], const T *Rre, const T *Rim, int J,
                                                   int lane, Acc &cR, Acc &cI)
    {
        const int r16 = lane & 15, k4 = lane >> 4;
#pragma unroll
        for (int f = 0; f < G::KF; ++f) {
            const int kr = (4 * f + k4) * S + J * 16 + r16;
            cmma<T>(cR, cI, frag[f].x, frag[f].y, Rre[kr], Rim[kr]);
        }
    }
    // Same with the right factor X^dag: X^dag(kk, j) = conj(X(j, kk)).
    static __device__ __forceinline__ void tile_mm_dag(const V (&frag)[G::KF], const T *Xre, const T *Xim, int J,
                                                       int lane, Acc &cR, Acc &cI)
    {
        const int r16 = lane & 15, k4 = lane >> 4;
#pragma unroll
        for (int f = 0; f < G::KF; ++f) {
            const int kr = (J * 16 + r16) * S + 4 * f + k4;
            cmma<T>(cR, cI, frag[f].x, frag[f].y, Xre[kr], -Xim[kr]);
        }
    }
    static __device__ __forceinline__ void tile_store(T *Dre, T *Dim, int I, int J, int lane, const Acc &cR,
                                                      const Acc &cI)
    {
        const int r16 = lane & 15, k4 = lane >> 4;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = I * 16 + mrow<T>(k4, v), j = J * 16 + r16;
            Dre[i * S + j] = cR[v];
            Dim[i * S + j] = cI[v];
        }
    }

    // Evaluates L(B0) and calls epi(q, value[4]) for the elements this lane owns in tile q of the
    // wave's chunk (accumulator slots 0..3, consecutive in tile order).  B1 holds C_k B0, B2 holds
    // A B0.  With several collapse channels the running sum Z is kept per element in zbuf (tile
    // order, global).
    template <typename Epi>
    static __device__ __forceinline__ void eval(const V *__restrict__ ops, int nc, T *lds, V *__restrict__ zbuf,
                                                Epi &&epi)
    {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        const int t0 = G::chunk0(w), nq = G::chunk0(w + 1) - t0;
        const int r16 = lane & 15, k4 = lane >> 4;
        T *B0re = lds, *B0im = lds + G::PLANE, *B1re = lds + 2 * G::PLANE, *B1im = lds + 3 * G::PLANE;
        T *B2re = lds + 4 * G::PLANE, *B2im = lds + 5 * G::PLANE;
        const size_t mat = (size_t)NP * NP;
        const int kmax = nc > 0 ? nc : 1;
        // Project the stage input onto its Hermitian part.  The products below are exact only for
        // Hermitian rho; without this, rounding noise in the anti-Hermitian part would evolve under a
        // generator with the dissipative terms' signs flipped and grow exponentially.  Each pair
        // (i, j), i <= j, is handled by one thread.
        for (int e = threadIdx.x; e < NP * NP; e += blockDim.x) {
            const int i = e / NP, j = e % NP;
            if (i < j) {
                const T ar = T(0.5) * (B0re[i * S + j] + B0re[j * S + i]);
                const T ai = T(0.5) * (B0im[i * S + j] - B0im[j * S + i]);
                B0re[i * S + j] = ar;
                B0im[i * S + j] = ai;
                B0re[j * S + i] = ar;
                B0im[j * S + i] = -ai;
            } else if (i == j) {
                B0im[i * S + i] = T(0);
            }
        }
        __syncthreads();
        V frag[G::KF];
        for (int k = 0; k < kmax; ++k) {
            if (k == 0) {
                // M = A B0 -> B2
                int Icur = -1;
#pragma unroll 1
                for (int q = 0; q < nq; ++q) {
                    const int t = t0 + q, I = t / G::NT, J = t % G::NT;
                    if (I != Icur) {
                        load_frag<T, NP>(ops, I, lane, frag);
                        Icur = I;
                    }
                    Acc mR = {0, 0, 0, 0}, mI = {0, 0, 0, 0};
                    tile_mm(frag, B0re, B0im, J, lane, mR, mI);
                    tile_store(B2re, B2im, I, J, lane, mR, mI);
                }
            }
            const V *Ck = ops + (1 + k) * mat;
            int Icur = -1;
            if (nc > 0) {
                // X = C_k B0 -> B1
#pragma unroll 1
                for (int q = 0; q < nq; ++q) {
                    const int t = t0 + q, I = t / G::NT, J = t % G::NT;
                    if (I != Icur) {
                        load_frag<T, NP>(Ck, I, lane, frag);
                        Icur = I;
                    }
                    Acc xR = {0, 0, 0, 0}, xI = {0, 0, 0, 0};
                    tile_mm(frag, B0re, B0im, J, lane, xR, xI);
                    tile_store(B1re, B1im, I, J, lane, xR, xI);
                }
            }
            __syncthreads();
#pragma unroll 1
            for (int q = 0; q < nq; ++q) {
                const int t = t0 + q, I = t / G::NT, J = t % G::NT;
                Acc zR = {0, 0, 0, 0}, zI = {0, 0, 0, 0};
                if (nc > 0) {
                    // fragments reloaded per tile: keeping them across the epilogue would take
                    // the registers its loads need to be in flight together
                    V fz[G::KF];
                    load_frag<T, NP>(Ck, I, lane, fz);
                    tile_mm_dag(fz, B1re, B1im, J, lane, zR, zI);  // Z_k = C_k X_k^dag
                }
                const size_t zb = tix(t, lane, 0);
                V z[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    z[v].x = zR[v];
                    z[v].y = zI[v];
                }
                if (k > 0) {
                    V zp[4];
                    gld4(zbuf + zb, zp);
#pragma unroll
                    for (int v = 0; v < 4; ++v) z[v] = cadd(z[v], zp[v]);
                }
                if (k + 1 < kmax) {
                    gst4(zbuf + zb, z);
                } else {
                    V o[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = I * 16 + mrow<T>(k4, v), j = J * 16 + r16;
                        o[v].x = z[v].x + B2re[i * S + j] + B2re[j * S + i];
                        o[v].y = z[v].y + B2im[i * S + j] - B2im[j * S + i];
                    }
                    epi(q, o);
                }
            }
            if (k + 1 < kmax) __syncthreads();  // B1 is rewritten by the next channel
        }
    }
};

template <typename T, int NP, int WV>
__global__ __launch_bounds__(WV * 64) void k_dense_solve(const DenseInst *__restrict__ insts,
                                                                      DenseCtl *__restrict__ ctls,
                                                                      const int32_t *__restrict__ order,
                                                                      int max_steps_launch, int reset)
{
    using G = DenseGeom<T, NP, WV>;
    using V = typename vec2<T>::type;
    using R = DenseRhs<T, NP, WV>;
    constexpr int S = G::S;
    extern __shared__ char smem[];
    T *lds = (T *)smem;
    __shared__ double scr[16];
    T *B0re = lds, *B0im = lds + G::PLANE;

    const int ii = order[blockIdx.x];
    const DenseInst &I = insts[ii];
    DenseCtl *C = ctls + ii;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r16 = lane & 15, k4 = lane >> 4;
    const int t0 = G::chunk0(w), nq = G::chunk0(w + 1) - t0;  // this wave's tiles: t0 .. t0 + nq - 1
    const int d = I.d;
    const size_t nvec = (size_t)NP * NP;
    V *vec = (V *)I.vec;
    V *Yb[2] = {vec, vec + nvec};
    V *Kb[2] = {vec + 2 * nvec, vec + 3 * nvec};
    V *ks[5] = {vec + 4 * nvec, vec + 5 * nvec, vec + 6 * nvec, vec + 7 * nvec, vec + 8 * nvec};
    V *zbuf = vec + 9 * nvec;  // running sum over collapse channels (used when nc > 1)
    const V *ops = (const V *)I.ops;
    const double nd = (double)d * d;

    // element (q, v) of this lane: tile-order index and (row, column)
    auto eidx = [&](int q, int v) { return tix(t0 + q, lane, v); };
    auto erow = [&](int q, int v) { return ((t0 + q) / G::NT) * 16 + mrow<T>(k4, v); };
    auto ecol = [&](int q) { return ((t0 + q) % G::NT) * 16 + r16; };
    auto record_expect = [&](int idx, double sc) {
        for (int k = 0; k < I.ne; ++k) {
            const int32_t *ep = I.eptr + (size_t)k * (d + 1);
            double sr = 0.0, si = 0.0;
            for (int i = threadIdx.x; i < d; i += blockDim.x)
                for (int p = gld(ep + i), pe = gld(ep + i + 1); p < pe; ++p) {
                    const double2 o = gld(I.eval + p);
                    const int j = gld(I.ecol + p);
                    const double rr = (double)B0re[j * S + i], ri = (double)B0im[j * S + i];
                    sr += o.x * rr - o.y * ri;
                    si += o.x * ri + o.y * rr;
                }
            sr = block_sum(sr, scr);
            si = block_sum(si, scr);
            if (threadIdx.x == 0) gst(I.expect + (size_t)k * I.nt + idx, make_double2(sr * sc, si * sc));
        }
    };
    auto trace_b0 = [&]() {
        double s = 0.0;
        for (int i = threadIdx.x; i < d; i += blockDim.x) s += (double)B0re[i * S + i];
        return block_sum(s, scr);
    };

    double t, h, err_prev, scale, tr0;
    int status, save_idx, last_rejected, parity;
    int64_t n_accept, n_reject, n_steps, n_rhs;

    if (reset || C->status == DENSE_ST_INIT) {
        // ---- initial state into B0 (planar, zero padded) and Y[0] (tile order) ----
        const V *r0 = (const V *)I.rho0;
        for (int q = 0; q < G::MAXJ; ++q) {
            if (q >= nq) break;
            for (int v = 0; v < 4; ++v) {
                const int i = erow(q, v), j = ecol(q);
                V y;
                y.x = 0;
                y.y = 0;
                if (i < d && j < d) y = gld(r0 + (size_t)i * d + j);
                gst(Yb[0] + eidx(q, v), y);
                B0re[i * S + j] = y.x;
                B0im[i * S + j] = y.y;
            }
        }
        __syncthreads();
        t = gld(I.tlist);
        err_prev = 1e-4;
        scale = 1.0;
        save_idx = 1;
        last_rejected = 0;
        parity = 0;
        n_accept = n_reject = n_steps = 0;
        n_rhs = 0;
        status = ST_RUNNING;
        tr0 = trace_b0();
        record_expect(0, 1.0);
        if (I.nt <= 1) status = ST_DONE;
        h = 0.0;
        if (status == ST_RUNNING) {
            // k1 = L(y0); starting step from d0 = |y0|, d1 = |k1|, d2 = |f(y0 + h0 k1) - k1| / h0
            double s0 = 0.0, s1 = 0.0;
            R::eval(ops, I.nc, lds, zbuf, [&](int q, const V (&a)[4]) {
                const size_t e = eidx(q, 0);
                V y0[4];
                gld4(Yb[0] + e, y0);
                gst4(Kb[0] + e, a);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const double ya = sqrt(abs2d(y0[v]));
                    const double sc = I.atol + I.rtol * ya;
                    s0 += ya * ya / (sc * sc);
                    s1 += abs2d(a[v]) / (sc * sc);
                }
            });
            n_rhs += 1;
            s0 = block_sum(s0, scr);
            s1 = block_sum(s1, scr);
            const double d0 = sqrt(s0 / nd), d1 = sqrt(s1 / nd);
            if (I.use_h0) {
                h = I.h0;
            } else {
                const double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
                for (int q = 0; q < G::MAXJ; ++q) {
                    if (q >= nq) break;
                    V y0[4], f0[4];
                    gld4(Yb[0] + eidx(q, 0), y0);
                    gld4(Kb[0] + eidx(q, 0), f0);
                    for (int v = 0; v < 4; ++v) {
                        const int i = erow(q, v), j = ecol(q);
                        V y = y0[v];
                        caxpy(y, (T)h0, f0[v]);
                        B0re[i * S + j] = y.x;
                        B0im[i * S + j] = y.y;
                    }
                }
                __syncthreads();
                double s2 = 0.0;
                R::eval(ops, I.nc, lds, zbuf, [&](int q, const V (&a)[4]) {
                    const size_t e = eidx(q, 0);
                    V y0[4], k0[4];
                    gld4(Kb[0] + e, k0);
                    gld4(Yb[0] + e, y0);
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const double2 f1 = to_d2(a[v]), f0 = to_d2(k0[v]);
                        const double sc = I.atol + I.rtol * sqrt(abs2d(y0[v]));
                        const double dx = (f1.x - f0.x) / h0, dy = (f1.y - f0.y) / h0;
                        s2 += (dx * dx + dy * dy) / (sc * sc);
                    }
                });
                n_rhs += 1;
                s2 = block_sum(s2, scr);
                const double d2 = sqrt(s2 / nd);
                const double m = fmax(d1, d2);
                const double h1 = (m <= 1e-15) ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / m, 0.2);
                h = fmin(100.0 * h0, h1);
            }
        }
    } else {
        t = C->t;
        h = C->h;
        err_prev = C->err_prev;
        scale = C->scale;
        tr0 = C->tr0;
        status = C->status;
        save_idx = C->save_idx;
        last_rejected = C->last_rejected;
        parity = C->parity;
        n_accept = C->n_accept;
        n_reject = C->n_reject;
        n_steps = C->n_steps;
        n_rhs = C->n_rhs;
    }

    int budget = max_steps_launch;
    while (status == ST_RUNNING && budget != 0) {
        if (budget > 0) --budget;
        int32_t land;
        const double ht = clip_step(t, h, gld(I.tlist + save_idx), &land);
        const T sc = (T)scale;
        V *y = Yb[parity], *ynew = Yb[1 - parity], *k1 = Kb[parity], *k7 = Kb[1 - parity];
        // stage-2 input: y + h a21 k1
        __syncthreads();
        for (int q = 0; q < G::MAXJ; ++q) {
            if (q >= nq) break;
            V yv[4], kv[4];
            gld4(y + eidx(q, 0), yv);
            gld4(k1 + eidx(q, 0), kv);
            for (int v = 0; v < 4; ++v) {
                const int i = erow(q, v), j = ecol(q);
                V x = cscale(yv[v], sc);
                caxpy(x, (T)(ht * DP5::a21), cscale(kv[v], sc));
                B0re[i * S + j] = x.x;
                B0im[i * S + j] = x.y;
            }
        }
        __syncthreads();
        double e2 = 0.0, l2 = 0.0;  // error norm; |L y_new|^2 (steady-state mode)
        for (int s = 2; s <= 7; ++s) {
            R::eval(ops, I.nc, lds, zbuf, [&](int q, const V (&a)[4]) {
                // Two elements at a time: every load of the pair first (the stores below go to
                // other vectors, which the compiler cannot tell apart), then the combination, then
                // the stores.  Pairs keep the loads in flight within the register budget.
#pragma unroll 1
                for (int p0 = 0; p0 < 4; p0 += 2) {
                    const size_t e = eidx(q, p0);
                    V yv[2], k1v[2], kv0[2], kv1[2], kv2[2], kv3[2], kv4[2], o[2];
                    gld2(y + e, yv);
                    gld2(k1 + e, k1v);
                    if (s >= 3 && s <= 5) gld2(ks[0] + e, kv0);
                    if (s >= 4) gld2(ks[1] + e, kv1);
                    if (s >= 5) gld2(ks[2] + e, kv2);
                    if (s >= 6) gld2(ks[3] + e, kv3);
                    if (s == 7) {
                        gld2(ks[4] + e, kv4);
                        gld2(ynew + e, o);  // the candidate y_new, for the error weights
                    }
                    const V ap[2] = {p0 == 0 ? a[0] : a[2], p0 == 0 ? a[1] : a[3]};
#pragma unroll
                    for (int v = 0; v < 2; ++v) {
                        const V yr = cscale(yv[v], sc), k1r = cscale(k1v[v], sc);
                        if (s == 7) {
                            double2 er = make_double2(0.0, 0.0);
                            caxpy(er, ht * DP5::e1, to_d2(k1r));
                            caxpy(er, ht * DP5::e3, to_d2(kv1[v]));
                            caxpy(er, ht * DP5::e4, to_d2(kv2[v]));
                            caxpy(er, ht * DP5::e5, to_d2(kv3[v]));
                            caxpy(er, ht * DP5::e6, to_d2(kv4[v]));
                            caxpy(er, ht * DP5::e7, to_d2(ap[v]));
                            const double scl = I.atol + I.rtol * fmax(sqrt(abs2d(yr)), sqrt(abs2d(o[v])));
                            e2 += (er.x * er.x + er.y * er.y) / (scl * scl);
                            l2 += abs2d(ap[v]);
                            continue;
                        }
                        o[v] = yr;
                        if (s == 2) {
                            caxpy(o[v], (T)(ht * DP5::a31), k1r);
                            caxpy(o[v], (T)(ht * DP5::a32), ap[v]);
                        } else if (s == 3) {
                            caxpy(o[v], (T)(ht * DP5::a41), k1r);
                            caxpy(o[v], (T)(ht * DP5::a42), kv0[v]);
                            caxpy(o[v], (T)(ht * DP5::a43), ap[v]);
                        } else if (s == 4) {
                            caxpy(o[v], (T)(ht * DP5::a51), k1r);
                            caxpy(o[v], (T)(ht * DP5::a52), kv0[v]);
                            caxpy(o[v], (T)(ht * DP5::a53), kv1[v]);
                            caxpy(o[v], (T)(ht * DP5::a54), ap[v]);
                        } else if (s == 5) {
                            caxpy(o[v], (T)(ht * DP5::a61), k1r);
                            caxpy(o[v], (T)(ht * DP5::a62), kv0[v]);
                            caxpy(o[v], (T)(ht * DP5::a63), kv1[v]);
                            caxpy(o[v], (T)(ht * DP5::a64), kv2[v]);
                            caxpy(o[v], (T)(ht * DP5::a65), ap[v]);
                        } else {
                            caxpy(o[v], (T)(ht * DP5::b1), k1r);
                            caxpy(o[v], (T)(ht * DP5::b3), kv1[v]);
                            caxpy(o[v], (T)(ht * DP5::b4), kv2[v]);
                            caxpy(o[v], (T)(ht * DP5::b5), kv3[v]);
                            caxpy(o[v], (T)(ht * DP5::b6), ap[v]);
                        }
                        const int i = erow(q, p0 + v), j = ecol(q);
                        B0re[i * S + j] = o[v].x;
                        B0im[i * S + j] = o[v].y;
                    }
                    if (s == 7) {
                        gst2(k7 + e, ap[0], ap[1]);
                    } else {
                        gst2(vec + (size_t)(2 + s) * nvec + e, ap[0], ap[1]);  // k_s (ks[s - 2])
                        if (s == 6) gst2(ynew + e, o[0], o[1]);
                    }
                }
            });
            __syncthreads();
        }
        n_rhs += 6;
        ++n_steps;
        // B0 now holds y_new (the stage-7 input)
        e2 = block_sum(e2, scr);
        const bool steady = I.steady_tol2 > 0.0;
        if (steady) l2 = block_sum(l2, scr);
        const double err = sqrt(e2 / nd);
        if (!isfinite(err)) {
            status = 6;  // QT_ENONFINITE
            break;
        }
        if (err <= 1.0) {
            ++n_accept;
            double sc_new = 1.0;
            if (I.renorm) sc_new = tr0 / trace_b0();
            // steady-state mode: |L y_new|_2 at or below the tolerance ends the solve, and every
            // remaining save time receives the expectation values of the converged state
            const bool conv = steady && l2 * sc_new * sc_new <= I.steady_tol2;
            if (conv) {
                for (int k = save_idx; k < I.nt; ++k) record_expect(k, sc_new);
            } else if (land) {
                record_expect(save_idx, sc_new);
            }
            t = land ? gld(I.tlist + save_idx) : t + ht;
            parity = 1 - parity;
            double hn = ht * pi_factor(err, err_prev);
            if (last_rejected && hn > ht) hn = ht;
            h = hn;
            err_prev = fmax(err, 1e-4);
            last_rejected = 0;
            scale = sc_new;
            if (conv) {
                save_idx = I.nt;
                status = ST_DONE;
            } else if (land) {
                ++save_idx;
                if (save_idx >= I.nt) status = steady ? 4 : ST_DONE;  // QT_EMAXSTEPS: not converged
            }
        } else {
            ++n_reject;
            h = ht * reject_factor(err);
            last_rejected = 1;
        }
        if (status == ST_RUNNING) {
            if (n_steps >= I.max_steps) status = 4;  // QT_EMAXSTEPS
            else if (h < 1e-14 * fmax(1.0, fabs(t))) status = 5;  // QT_EDTMIN
        }
    }
    if (threadIdx.x == 0) {
        C->t = t;
        C->h = h;
        C->err_prev = err_prev;
        C->scale = scale;
        C->tr0 = tr0;
        C->status = status;
        C->save_idx = save_idx;
        C->last_rejected = last_rejected;
        C->parity = parity;
        C->n_accept = n_accept;
        C->n_reject = n_reject;
        C->n_steps = n_steps;
        C->n_rhs = n_rhs;
    }
}

// ---------------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------------
void dense_fill_inst(DenseInst *g, int d, int nc, int nt, int ne, const void *ops, const void *rho0, void *vec,
                     const double *tlist, const int32_t *eptr, const int32_t *ecol, const double2 *eval,
                     double2 *expect, const qt_opts &opts, int prec)
{
    g->d = d;
    g->np = dense_np(d);
    g->nc = nc;
    g->nt = nt;
    g->ne = ne;
    g->use_h0 = opts.h0 > 0 ? 1 : 0;
    g->renorm = prec == QT_MIXED ? 1 : 0;
    g->pad = 0;
    g->atol = opts.abstol;
    g->rtol = opts.reltol;
    g->h0 = opts.h0;
    g->max_steps = opts.max_steps;
    g->ops = ops;
    g->rho0 = rho0;
    g->vec = vec;
    g->tlist = tlist;
    g->eptr = eptr;
    g->ecol = ecol;
    g->eval = eval;
    g->expect = expect;
    g->steady_tol2 = 0.0;
}

// Wave counts built per padded size.  With one wave per tile row a size whose tile-row count is not
// a multiple of 4 loads the SIMDs unevenly; the other counts split the tiles evenly (np = 48: 9
// tiles; np = 80: 25 tiles) at one or two waves per SIMD.  FP64 keeps to the small counts (its
// fragments take twice the registers).
static int waves_built(int np, int prec, const int **list)
{
    static const int f16[] = {1, 2}, f32[] = {2, 4}, f48[] = {3, 4, 6, 8}, f64s[] = {4, 8}, f80[] = {4, 5, 8};
    static const int d16[] = {1}, d32[] = {2, 4}, d48[] = {3, 4};
    const bool dbl = prec == QT_F64;
    switch (np) {
    case 16: *list = dbl ? d16 : f16; return dbl ? 1 : 2;
    case 32: *list = dbl ? d32 : f32; return 2;
    case 48: *list = dbl ? d48 : f48; return dbl ? 2 : 4;
    case 64: *list = f64s; return dbl ? 0 : 2;
    case 80: *list = f80; return dbl ? 0 : 3;
    default: *list = nullptr; return 0;
    }
}

int dense_waves_candidates(int np, int prec, int *out, int max)
{
    const int *l;
    const int n = waves_built(np, prec, &l);
    int k = 0;
    for (int i = 0; i < n && k < max; ++i) out[k++] = l[i];
    return k;
}

bool dense_waves_allowed(int np, int prec, int waves)
{
    const int *l;
    const int n = waves_built(np, prec, &l);
    for (int i = 0; i < n; ++i)
        if (l[i] == waves) return true;
    return false;
}

int dense_choose_config(int d, int prec)
{
    // waves per workgroup: the autotuner's measured choice for this padded size, else the default
    const int np = dense_np(d);
    int waves;
    if (tune_lookup_dense(dense_tune_key(prec, np), &waves) && dense_waves_allowed(np, prec, waves)) return waves;
    return dense_default_waves(np, prec);
}

const void *dense_state_ptr(const void *vec, int d, int prec)
{
    (void)d;
    (void)prec;
    return vec;
}

template <typename T, int NP, int WV>
static void launch_np(const DenseInst *insts, DenseCtl *ctls, const int32_t *order, int count, int msl, int reset,
                      hipStream_t s)
{
    using G = DenseGeom<T, NP, WV>;
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_dense_solve<T, NP, WV>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)G::LDS_BYTES);
        attr = true;
    }
    hipLaunchKernelGGL((k_dense_solve<T, NP, WV>), dim3(count), dim3(G::WAVES * 64), G::LDS_BYTES, s, insts, ctls,
                       order, msl, reset);
}

// waves: waves per workgroup, one of the counts waves_built lists for (np, precision); the caller
// checks it with dense_waves_allowed.
void dense_launch_bucket(int np, bool f64, int waves, const DenseInst *insts, DenseCtl *ctls, const int32_t *order,
                         int count, int msl, int reset, hipStream_t s)
{
    if (count <= 0) return;
#define QT_DW(T, NP, W)                                                                                           \
    if (np == NP && waves == W) {                                                                                  \
        launch_np<T, NP, W>(insts, ctls, order, count, msl, reset, s);                                            \
        return;                                                                                                    \
    }
    if (f64) {
        QT_DW(double, 16, 1)
        QT_DW(double, 32, 2)
        QT_DW(double, 32, 4)
        QT_DW(double, 48, 3)
        QT_DW(double, 48, 4)
    } else {
        QT_DW(float, 16, 1)
        QT_DW(float, 16, 2)
        QT_DW(float, 32, 2)
        QT_DW(float, 32, 4)
        QT_DW(float, 48, 3)
        QT_DW(float, 48, 4)
        QT_DW(float, 48, 6)
        QT_DW(float, 48, 8)
        QT_DW(float, 64, 4)
        QT_DW(float, 64, 8)
        QT_DW(float, 80, 4)
        QT_DW(float, 80, 5)
        QT_DW(float, 80, 8)
    }
#undef QT_DW
}

void dense_unpack(const void *host_vec, int d, int prec, double scale, double *out)
{
    const int np = dense_np(d), nt = np / 16;
    for (int t = 0; t < nt * nt; ++t)
        for (int lane = 0; lane < 64; ++lane)
            for (int v = 0; v < 4; ++v) {
                const int q4 = lane >> 4;
                const int i = (t / nt) * 16 + (prec == QT_F64 ? q4 + 4 * v : 4 * q4 + v);
                const int j = (t % nt) * 16 + (lane & 15);
                if (i >= d || j >= d) continue;
                const size_t e = ((size_t)t * 64 + lane) * 4 + v;
                double re, im;
                if (prec == QT_F64) {
                    re = ((const double *)host_vec)[2 * e];
                    im = ((const double *)host_vec)[2 * e + 1];
                } else {
                    re = ((const float *)host_vec)[2 * e];
                    im = ((const float *)host_vec)[2 * e + 1];
                }
                out[2 * ((size_t)i * d + j)] = re * scale;
                out[2 * ((size_t)i * d + j) + 1] = im * scale;
            }
}

}  // namespace qt

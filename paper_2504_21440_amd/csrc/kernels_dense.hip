// kernels_dense.hip -- dense operator-form master-equation solver on the gfx950 matrix cores.
//
// The master equation of arXiv:2504.21440 (Sec. 3.2) in operator form,
//     L(rho) = A rho + rho A^dag + sum_k C_k rho C_k^dag,   A = -i H - 1/2 sum_k C_k^dag C_k.
// For Hermitian rho the result is Hermitian, and with P = A rho and X_k = C_k rho
//     L(rho) = P + P^dag + sum_k C_k X_k^dag.
// P and the X_k are formed on every 16x16 tile, the sum and the result only on the tiles on and
// above the diagonal; each result element goes into the next stage input together with its mirror
// image, so every stage input is exactly Hermitian.  Every product has the shape Op R^dag: Op an
// operator (A or C_k, rows read from global memory into registers; stored in the order the lanes
// consume them, so a load of the 64 lanes reads 1 KB of contiguous memory), R a matrix in LDS (rho,
// which equals rho^dag, or X_k), read by rows:
//     Re(Op R^dag) = Re Op Re R^T + Im Op Im R^T,   Im(Op R^dag) = Im Op Re R^T - Re Op Im R^T,
// three accumulators and no negated operand.  A real collapse operator (Im C_k = 0) needs two real
// products per complex one instead of four.  The real products run on v_mfma_f32_16x16x4f32 /
// v_mfma_f64_16x16x4f64.  Lane l supplies k-slot l / 16 of each instruction, and over the NP / 4
// instructions of a tile that slot walks the contiguous range [(l / 16) NP / 4, (l / 16 + 1) NP / 4)
// of the inner index, so the lane's operator elements are contiguous in a row and its LDS operands
// come in 16-byte reads of 4 (FP32) or 2 (FP64) inner steps.
//
// One workgroup owns one problem for the whole launch and runs the adaptive Dormand-Prince 5(4)
// loop itself.  LDS holds three NP x S planar (re, im) matrices: B0 = the stage input, B1 = X_k,
// B2 = P.  The row stride S is NP plus 16 bytes, which puts the 16 rows of a 16-byte read on
// distinct banks.  One right-hand side: phase 1 (P and X_0 on every tile, split over the waves by
// matrix-core work), a barrier, phase 2 (C_k X_k^dag on the upper tiles, then the
// stage epilogue, which writes the next stage input into B0), a barrier.  The Runge-Kutta stage
// vectors live in a per-problem global buffer that holds the elements of the upper tiles in
// (tile, lane, accumulator slot) order.  Step control, the error norm (an element above the diagonal
// counts for itself and its mirror), trace renormalisation and expectation values are FP64 and stay
// inside the workgroup.
#include <algorithm>
#include <vector>

#include "qt_common.h"
#include "qt_dense.h"
#include "qt_tune.h"

namespace qt {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float lf4 __attribute__((ext_vector_type(4)));   // 16-byte LDS access, FP32
typedef double ld2 __attribute__((ext_vector_type(2)));  // 16-byte LDS access, FP64

// Every buffer access of this file goes through the global-only loads and stores of qt_common.h
// (gld / gst and the wider ones below): the LDS traffic of the matrix products then neither
// orders against nor waits for it.
// The 4 consecutive elements a lane owns in one output tile, with 16-byte accesses.
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

// Work split: phase 1 cuts the NT x NT tiles (row-major order), phase 2 the NT (NT + 1) / 2 tiles
// on and above the diagonal (row-major order), into WV contiguous runs of near-equal length, one
// per wave, so the matrix-core work spreads over the 4 SIMDs of the CU.  A wave reloads its operator
// rows only when its run enters the next tile row.
template <typename T, int NP, int WV> struct DenseGeom {
    static constexpr int S = NP + 16 / (int)sizeof(T);  // LDS row stride (elements)
    static constexpr int NT = NP / 16;                   // tiles per side
    static constexpr int TILES = NT * NT;
    static constexpr int UT = NT * (NT + 1) / 2;         // tiles with I <= J
    static constexpr int WAVES = WV;
    static constexpr int KF = NP / 4;                    // inner steps per lane per tile
    static constexpr int PLANE = NP * S;
    static constexpr size_t LDS_BYTES = (size_t)6 * PLANE * sizeof(T);  // B0, B1, B2 (re, im)
    static __device__ __forceinline__ int tile0(int w) { return (w * TILES) / WV; }
    static __device__ __forceinline__ int utile0(int w) { return (w * UT) / WV; }
};

// Upper tile u (row-major order over I <= J) of an nt x nt tiling.
__device__ __forceinline__ void upper_tile(int u, int nt, int &I, int &J)
{
    int i = 0;
    while (u >= nt - i) {
        u -= nt - i;
        ++i;
    }
    I = i;
    J = i + u;
}

// Index of (upper tile u, lane, accumulator slot v) in the stage vectors.
__device__ __forceinline__ size_t uix(int u, int lane, int v) { return ((size_t)u * 64 + lane) * 4 + v; }

// Weight of element (i, j) of upper tile (I, J) in a sum over the whole matrix: above the diagonal
// it stands for itself and its mirror, on it for itself; the elements below the diagonal inside a
// diagonal tile are represented by their mirrors.
__device__ __forceinline__ double uweight(int I, int J, int i, int j)
{
    return I < J ? 2.0 : (i < j ? 2.0 : (i == j ? 1.0 : 0.0));
}

// Stage-vector values a lane's epilogue needs for one tile, loaded before the tile's products.
template <typename V> struct StageIn {
    V y[4], k1[4], kv[5][4], yn[4];
};

template <typename T, int NP, int WV> struct DenseRhs {
    using G = DenseGeom<T, NP, WV>;
    using V = typename vec2<T>::type;
    using Acc = typename Mfma<T>::acc;
    static constexpr int S = G::S, KF = G::KF;

    // Op R^dag on one tile: Re = p, Im = q - n.
    struct Acc3 {
        Acc p, q, n;
    };
    static __device__ __forceinline__ Acc3 acc0()
    {
        Acc3 a;
        a.p = Acc{0, 0, 0, 0};
        a.q = Acc{0, 0, 0, 0};
        a.n = Acc{0, 0, 0, 0};
        return a;
    }

    // Operator rows [16 I, 16 I + 16) over the lane's inner range: f[c] = Op(16 I + lane % 16,
    // (lane / 16) KF + c); complex, or the real parts only (real operators).  The operators are
    // stored in fragment order (dense_pack_ops), so each 16-byte load of the 64 lanes reads 1 KB
    // of contiguous memory.
    static __device__ __forceinline__ void frag(const V *__restrict__ op, int I, int lane, V (&f)[KF])
    {
        constexpr int E = 16 / (int)sizeof(V);  // complex elements per 16 bytes
        const T *p = (const T *)(op + ((size_t)I * (KF / E) * 64 + lane) * E);
#pragma unroll
        for (int ch = 0; ch < KF / E; ++ch) {
            if constexpr (sizeof(T) == 4) {
                const gf4 a = *(const QT_GLOBAL gf4 *)(p + ch * 64 * 4);
                f[2 * ch] = make_float2(a.x, a.y);
                f[2 * ch + 1] = make_float2(a.z, a.w);
            } else {
                f[ch] = gld((const V *)(p + ch * 64 * 2));
            }
        }
    }
    static __device__ __forceinline__ void frag(const V *__restrict__ op, int I, int lane, T (&f)[KF])
    {
        constexpr int E = 16 / (int)sizeof(T);  // real elements per 16 bytes
        const T *p = (const T *)op + ((size_t)I * (KF / E) * 64 + lane) * E;
#pragma unroll
        for (int ch = 0; ch < KF / E; ++ch) {
            if constexpr (sizeof(T) == 4) {
                const gf4 a = *(const QT_GLOBAL gf4 *)(p + ch * 64 * 4);
                f[4 * ch] = a.x, f[4 * ch + 1] = a.y, f[4 * ch + 2] = a.z, f[4 * ch + 3] = a.w;
            } else {
                const gd2 a = *(const QT_GLOBAL gd2 *)(p + ch * 64 * 2);
                f[2 * ch] = a.x, f[2 * ch + 1] = a.y;
            }
        }
    }
    // Rows [16 J, 16 J + 16) of an LDS matrix over the lane's inner range, 16-byte reads.
    static __device__ __forceinline__ void rows(const T *Rre, const T *Rim, int J, int lane, T (&rr)[KF],
                                                T (&ri)[KF])
    {
        const int o = (J * 16 + (lane & 15)) * S + (lane >> 4) * KF;
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int c = 0; c < KF / 4; ++c) {
                const lf4 a = *(const lf4 *)(Rre + o + 4 * c), b = *(const lf4 *)(Rim + o + 4 * c);
                rr[4 * c] = a.x, rr[4 * c + 1] = a.y, rr[4 * c + 2] = a.z, rr[4 * c + 3] = a.w;
                ri[4 * c] = b.x, ri[4 * c + 1] = b.y, ri[4 * c + 2] = b.z, ri[4 * c + 3] = b.w;
            }
        } else {
#pragma unroll
            for (int c = 0; c < KF / 2; ++c) {
                const ld2 a = *(const ld2 *)(Rre + o + 2 * c), b = *(const ld2 *)(Rim + o + 2 * c);
                rr[2 * c] = a.x, rr[2 * c + 1] = a.y;
                ri[2 * c] = b.x, ri[2 * c + 1] = b.y;
            }
        }
    }
    // a += Op R^dag on one tile, complex or real operator.
    static __device__ __forceinline__ void mm(const V (&f)[KF], const T (&rr)[KF], const T (&ri)[KF], Acc3 &a)
    {
#pragma unroll
        for (int c = 0; c < KF; ++c) {
            a.p = Mfma<T>::mma(f[c].x, rr[c], a.p);
            a.q = Mfma<T>::mma(f[c].y, rr[c], a.q);
            a.n = Mfma<T>::mma(f[c].x, ri[c], a.n);
            a.p = Mfma<T>::mma(f[c].y, ri[c], a.p);
        }
    }
    static __device__ __forceinline__ void mm(const T (&f)[KF], const T (&rr)[KF], const T (&ri)[KF], Acc3 &a)
    {
#pragma unroll
        for (int c = 0; c < KF; ++c) {
            a.p = Mfma<T>::mma(f[c], rr[c], a.p);
            a.n = Mfma<T>::mma(f[c], ri[c], a.n);
        }
    }
    // One tile into an LDS matrix.
    static __device__ __forceinline__ void put(T *Dre, T *Dim, int I, int J, int lane, const Acc3 &a)
    {
        const int r16 = lane & 15, k4 = lane >> 4;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = I * 16 + mrow<T>(k4, v), j = J * 16 + r16;
            Dre[i * S + j] = a.p[v];
            Dim[i * S + j] = a.q[v] - a.n[v];
        }
    }
    // The lane's 4 elements of upper tile (I, J) into B0 with their mirror images; inside a
    // diagonal tile the elements below the diagonal are left to their mirrors and the diagonal
    // is written real.
    static __device__ __forceinline__ void put_b0(T *B0re, T *B0im, int I, int J, int lane, const V (&o)[4])
    {
        const int r16 = lane & 15, k4 = lane >> 4, j = J * 16 + r16;
        if (I < J) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = I * 16 + mrow<T>(k4, v);
                B0re[i * S + j] = o[v].x;
                B0im[i * S + j] = o[v].y;
            }
            if constexpr (sizeof(T) == 4) {
                const int m = j * S + I * 16 + 4 * k4;  // rows 4 k4 .. 4 k4 + 3 of the tile: contiguous
                lf4 a, b;
                a.x = o[0].x, a.y = o[1].x, a.z = o[2].x, a.w = o[3].x;
                b.x = -o[0].y, b.y = -o[1].y, b.z = -o[2].y, b.w = -o[3].y;
                *(lf4 *)(B0re + m) = a;
                *(lf4 *)(B0im + m) = b;
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = I * 16 + mrow<T>(k4, v);
                    B0re[j * S + i] = o[v].x;
                    B0im[j * S + i] = -o[v].y;
                }
            }
        } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = I * 16 + mrow<T>(k4, v);
                if (i < j) {
                    B0re[i * S + j] = o[v].x;
                    B0im[i * S + j] = o[v].y;
                    B0re[j * S + i] = o[v].x;
                    B0im[j * S + i] = -o[v].y;
                } else if (i == j) {
                    B0re[i * S + i] = o[v].x;
                    B0im[i * S + i] = T(0);
                }
            }
        }
    }

    // Phase 1: P = A B0 into B2 (WP) and X = C B0 into B1 (WX) on every tile; F is the fragment
    // type of C (V complex, T real).  With both, the work is a list of jobs, P then X for each tile
    // in row-major order, weighted by their matrix-core instructions (4 per inner step for the
    // complex A, 2 or 4 for C); each wave takes the jobs whose start falls in its share of the total
    // weight, and a tile whose two jobs fall to one wave has its rows of B0 read once for both.
    template <bool WP, bool WX, typename F>
    static __device__ __forceinline__ void phase1(const V *__restrict__ A, const V *__restrict__ C, T *lds)
    {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        const T *B0re = lds, *B0im = lds + G::PLANE;
        T *B1re = lds + 2 * G::PLANE, *B1im = lds + 3 * G::PLANE;
        T *B2re = lds + 4 * G::PLANE, *B2im = lds + 5 * G::PLANE;
        // jobs: 2 t (P of tile t) and 2 t + 1 (X of tile t); with one kind only, every other job
        int j0, j1;
        if constexpr (WP && WX) {
            constexpr int wp = 4, wx = sizeof(F) == sizeof(T) ? 2 : 4, wt = wp + wx;
            auto first_job = [](int ww) {
                const int b = (ww * G::TILES * wt) / WV, t = b / wt, r = b % wt;
                return 2 * t + (r == 0 ? 0 : (r <= wp ? 1 : 2));
            };
            j0 = first_job(w);
            j1 = first_job(w + 1);
        } else {
            j0 = 2 * G::tile0(w) + (WP ? 0 : 1);
            j1 = 2 * G::tile0(w + 1) + (WP ? 0 : 1);
        }
        V fa[KF];
        F fc[KF];
        int Ia = -1, Ic = -1;
#pragma unroll 1
        for (int j = j0; j < j1;) {
            const int t = j >> 1, I = t / G::NT, J = t % G::NT;
            const bool doP = WP && !(j & 1), doX = WX && ((j & 1) || j + 1 < j1);
            if (WP && doP && I != Ia) {
                frag(A, I, lane, fa);
                Ia = I;
            }
            if (WX && doX && I != Ic) {
                frag(C, I, lane, fc);
                Ic = I;
            }
            T rr[KF], ri[KF];
            rows(B0re, B0im, J, lane, rr, ri);
            Acc3 a = acc0(), x = acc0();
            if (doP && doX) {
                mm(fa, rr, ri, a);
                mm(fc, rr, ri, x);
                put(B2re, B2im, I, J, lane, a);
                put(B1re, B1im, I, J, lane, x);
                j += 2;
            } else if (doP) {
                mm(fa, rr, ri, a);
                put(B2re, B2im, I, J, lane, a);
                j += WX ? 1 : 2;
            } else {
                mm(fc, rr, ri, x);
                put(B1re, B1im, I, J, lane, x);
                j += WP ? 1 : 2;
            }
        }
    }

    // Phase 2 on the wave's run of upper tiles: Z = C X^dag (X in B1; WZ), plus the running sum of
    // the earlier channels from zbuf unless first.  Not last: the sum goes back to zbuf.  Last:
    // L = Z + P + P^dag (P in B2) goes to the epilogue, whose stage-vector loads (eload) are issued
    // before the tile's products.  (Issuing them one tile earlier, with two sets in flight, spilled
    // registers and was slower.)
    template <bool WZ, typename F, typename Ld, typename Ap>
    static __device__ __forceinline__ void phase2(const V *__restrict__ C, bool first, bool last, T *lds,
                                                  V *__restrict__ zbuf, Ld &eload, Ap &eapply)
    {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        const int r16 = lane & 15, k4 = lane >> 4;
        const T *B1re = lds + 2 * G::PLANE, *B1im = lds + 3 * G::PLANE;
        const T *B2re = lds + 4 * G::PLANE, *B2im = lds + 5 * G::PLANE;
        const int u0 = G::utile0(w), u1 = G::utile0(w + 1);
        F fc[KF];
        int Icur = -1;
        auto tile = [&](int u, const StageIn<V> &in) {
            int I, J;
            upper_tile(u, G::NT, I, J);
            Acc3 z = acc0();
            if constexpr (WZ) {
                if (I != Icur) {
                    frag(C, I, lane, fc);
                    Icur = I;
                }
                T rr[KF], ri[KF];
                rows(B1re, B1im, J, lane, rr, ri);
                mm(fc, rr, ri, z);
            }
            V o[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                o[v].x = z.p[v];
                o[v].y = z.q[v] - z.n[v];
            }
            const size_t e = uix(u, lane, 0);
            if (!first) {
                V zp[4];
                gld4(zbuf + e, zp);
#pragma unroll
                for (int v = 0; v < 4; ++v) o[v] = cadd(o[v], zp[v]);
            }
            if (!last) {
                gst4(zbuf + e, o);
                return;
            }
            // + P + P^dag: P(i, j) for the lane's elements, and P(j, i) from row j
            const int j = J * 16 + r16;
            T tr[4], ti[4];
            if constexpr (sizeof(T) == 4) {
                const int m = j * S + I * 16 + 4 * k4;
                const lf4 a = *(const lf4 *)(B2re + m), b = *(const lf4 *)(B2im + m);
                tr[0] = a.x, tr[1] = a.y, tr[2] = a.z, tr[3] = a.w;
                ti[0] = b.x, ti[1] = b.y, ti[2] = b.z, ti[3] = b.w;
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = I * 16 + mrow<T>(k4, v);
                    tr[v] = B2re[j * S + i];
                    ti[v] = B2im[j * S + i];
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = I * 16 + mrow<T>(k4, v);
                o[v].x = o[v].x + B2re[i * S + j] + tr[v];
                o[v].y = o[v].y + B2im[i * S + j] - ti[v];
            }
            eapply(u, I, J, in, o);
        };
#pragma unroll 1
        for (int u = u0; u < u1; ++u) {
            StageIn<V> in;
            if (last) eload(u, in);
            tile(u, in);
        }
    }

    // Evaluates L(B0) (B0 Hermitian) and hands the upper-tile elements to the epilogue:
    // eload(u, in) fills the stage-vector values, eapply(u, I, J, in, o) receives L.  nc collapse
    // channels; bit k of creal marks C_k real.  With several channels the running sum of
    // C_k X_k^dag is kept in zbuf (upper-tile order, global).  Ends without a barrier: the caller
    // synchronises before B0, B1 or B2 are read again.
    template <typename Ld, typename Ap>
    static __device__ __forceinline__ void eval(const V *__restrict__ ops, int nc, uint32_t creal, T *lds,
                                                V *__restrict__ zbuf, Ld &&eload, Ap &&eapply)
    {
        const size_t mat = (size_t)NP * NP;
        if (nc == 0) {
            phase1<true, false, V>(ops, nullptr, lds);
            __syncthreads();
            phase2<false, V>(nullptr, true, true, lds, zbuf, eload, eapply);
            return;
        }
        for (int k = 0; k < nc; ++k) {
            const V *Ck = ops + (1 + k) * mat;
            const bool cr = k < 32 && ((creal >> k) & 1u);
            if (k > 0) __syncthreads();  // the previous channel's X is read until here
            if (k == 0) {
                if (cr) phase1<true, true, T>(ops, Ck, lds);
                else phase1<true, true, V>(ops, Ck, lds);
            } else {
                if (cr) phase1<false, true, T>(ops, Ck, lds);
                else phase1<false, true, V>(ops, Ck, lds);
            }
            __syncthreads();
            if (cr) phase2<true, T>(Ck, k == 0, k + 1 == nc, lds, zbuf, eload, eapply);
            else phase2<true, V>(Ck, k == 0, k + 1 == nc, lds, zbuf, eload, eapply);
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
    using In = StageIn<V>;
    constexpr int S = G::S;
    extern __shared__ __align__(16) char smem[];
    T *lds = (T *)smem;
    __shared__ double scr[48];
    T *B0re = lds, *B0im = lds + G::PLANE;

    const int ii = order[blockIdx.x];
    const DenseInst &g = insts[ii];
    DenseCtl *C = ctls + ii;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r16 = lane & 15, k4 = lane >> 4;
    const int u0 = G::utile0(w), u1 = G::utile0(w + 1);  // this wave's upper tiles
    const int d = g.d;
    const uint32_t creal = (uint32_t)g.creal;
    const size_t nvec = (size_t)NP * NP;
    V *vec = (V *)g.vec;
    V *Yb[2] = {vec, vec + nvec};
    V *Kb[2] = {vec + 2 * nvec, vec + 3 * nvec};
    V *ks[5] = {vec + 4 * nvec, vec + 5 * nvec, vec + 6 * nvec, vec + 7 * nvec, vec + 8 * nvec};
    V *zbuf = vec + 9 * nvec;  // running sum over collapse channels (used when nc > 1)
    const V *ops = (const V *)g.ops;
    const double nd = (double)d * d;

    auto record_expect = [&](int idx, double sc) {
        for (int k = 0; k < g.ne; ++k) {
            const int32_t *ep = g.eptr + (size_t)k * (d + 1);
            double sr = 0.0, si = 0.0;
            for (int i = threadIdx.x; i < d; i += blockDim.x)
                for (int p = gld(ep + i), pe = gld(ep + i + 1); p < pe; ++p) {
                    const double2 o = gld(g.eval + p);
                    const int j = gld(g.ecol + p);
                    const double rr = (double)B0re[j * S + i], ri = (double)B0im[j * S + i];
                    sr += o.x * rr - o.y * ri;
                    si += o.x * ri + o.y * rr;
                }
            double v2[2] = {sr, si};
            block_sum_n<2>(v2, scr);
            if (threadIdx.x == 0) gst(g.expect + (size_t)k * g.nt + idx, make_double2(v2[0] * sc, v2[1] * sc));
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
        // ---- initial state: its Hermitian part, into Y[0] (upper tiles) and B0 ----
        const V *r0 = (const V *)g.rho0;
        for (int u = u0; u < u1; ++u) {
            int TI, TJ;
            upper_tile(u, G::NT, TI, TJ);
            V o[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = TI * 16 + mrow<T>(k4, v), j = TJ * 16 + r16;
                V a, b;
                a.x = a.y = b.x = b.y = T(0);
                if (i < d && j < d) {
                    a = gld(r0 + (size_t)i * d + j);
                    b = gld(r0 + (size_t)j * d + i);
                }
                o[v].x = T(0.5) * (a.x + b.x);
                o[v].y = T(0.5) * (a.y - b.y);
            }
            gst4(Yb[0] + uix(u, lane, 0), o);
            R::put_b0(B0re, B0im, TI, TJ, lane, o);
        }
        __syncthreads();
        t = gld(g.tlist);
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
        if (g.nt <= 1) status = ST_DONE;
        h = 0.0;
        if (status == ST_RUNNING) {
            // k1 = L(y0); starting step from d0 = |y0|, d1 = |k1|, d2 = |f(y0 + h0 k1) - k1| / h0
            double s01[2] = {0.0, 0.0};
            R::eval(
                ops, g.nc, creal, lds, zbuf, [&](int u, In &in) { gld4(Yb[0] + uix(u, lane, 0), in.y); },
                [&](int u, int TI, int TJ, const In &in, const V (&a)[4]) {
                    gst4(Kb[0] + uix(u, lane, 0), a);
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const double wt = uweight(TI, TJ, TI * 16 + mrow<T>(k4, v), TJ * 16 + r16);
                        const double ya = sqrt(abs2d(in.y[v]));
                        const double sc = g.atol + g.rtol * ya;
                        s01[0] += wt * (ya * ya / (sc * sc));
                        s01[1] += wt * (abs2d(a[v]) / (sc * sc));
                    }
                });
            n_rhs += 1;
            block_sum_n<2>(s01, scr);
            const double d0 = sqrt(s01[0] / nd), d1 = sqrt(s01[1] / nd);
            if (g.use_h0) {
                h = g.h0;
            } else {
                const double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
                for (int u = u0; u < u1; ++u) {
                    int TI, TJ;
                    upper_tile(u, G::NT, TI, TJ);
                    V y0[4], f0[4], o[4];
                    gld4(Yb[0] + uix(u, lane, 0), y0);
                    gld4(Kb[0] + uix(u, lane, 0), f0);
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        o[v] = y0[v];
                        caxpy(o[v], (T)h0, f0[v]);
                    }
                    R::put_b0(B0re, B0im, TI, TJ, lane, o);
                }
                __syncthreads();
                double s2[1] = {0.0};
                R::eval(
                    ops, g.nc, creal, lds, zbuf,
                    [&](int u, In &in) {
                        gld4(Kb[0] + uix(u, lane, 0), in.k1);
                        gld4(Yb[0] + uix(u, lane, 0), in.y);
                    },
                    [&](int u, int TI, int TJ, const In &in, const V (&a)[4]) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const double wt = uweight(TI, TJ, TI * 16 + mrow<T>(k4, v), TJ * 16 + r16);
                            const double2 f1 = to_d2(a[v]), f0 = to_d2(in.k1[v]);
                            const double sc = g.atol + g.rtol * sqrt(abs2d(in.y[v]));
                            const double dx = (f1.x - f0.x) / h0, dy = (f1.y - f0.y) / h0;
                            s2[0] += wt * ((dx * dx + dy * dy) / (sc * sc));
                        }
                    });
                n_rhs += 1;
                block_sum_n<1>(s2, scr);
                const double d2 = sqrt(s2[0] / nd);
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
        const double ht = clip_step(t, h, gld(g.tlist + save_idx), &land);
        const T sc = (T)scale;
        V *y = Yb[parity], *ynew = Yb[1 - parity], *k1 = Kb[parity], *k7 = Kb[1 - parity];
        // stage-2 input: y + h a21 k1
        __syncthreads();
        for (int u = u0; u < u1; ++u) {
            int TI, TJ;
            upper_tile(u, G::NT, TI, TJ);
            V yv[4], kv[4], o[4];
            gld4(y + uix(u, lane, 0), yv);
            gld4(k1 + uix(u, lane, 0), kv);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                o[v] = cscale(yv[v], sc);
                caxpy(o[v], (T)(ht * DP5::a21), cscale(kv[v], sc));
            }
            R::put_b0(B0re, B0im, TI, TJ, lane, o);
        }
        __syncthreads();
        // error norm; |L y_new|^2 (steady-state mode); trace of y_new (from the stage-7 input)
        double acc3[3] = {0.0, 0.0, 0.0};
        for (int s = 2; s <= 7; ++s) {
            R::eval(
                ops, g.nc, creal, lds, zbuf,
                [&](int u, In &in) {
                    const size_t e = uix(u, lane, 0);
                    gld4(y + e, in.y);
                    gld4(k1 + e, in.k1);
                    if (s >= 3 && s <= 5) gld4(ks[0] + e, in.kv[0]);
                    if (s >= 4) gld4(ks[1] + e, in.kv[1]);
                    if (s >= 5) gld4(ks[2] + e, in.kv[2]);
                    if (s >= 6) gld4(ks[3] + e, in.kv[3]);
                    if (s == 7) {
                        gld4(ks[4] + e, in.kv[4]);
                        gld4(ynew + e, in.yn);  // the candidate y_new, for the error weights
                    }
                },
                [&](int u, int TI, int TJ, const In &in, const V (&ap)[4]) {
                    const size_t e = uix(u, lane, 0);
                    V o[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const V yr = cscale(in.y[v], sc), k1r = cscale(in.k1[v], sc);
                        if (s == 7) {
                            const double wt = uweight(TI, TJ, TI * 16 + mrow<T>(k4, v), TJ * 16 + r16);
                            double2 er = make_double2(0.0, 0.0);
                            caxpy(er, ht * DP5::e1, to_d2(k1r));
                            caxpy(er, ht * DP5::e3, to_d2(in.kv[1][v]));
                            caxpy(er, ht * DP5::e4, to_d2(in.kv[2][v]));
                            caxpy(er, ht * DP5::e5, to_d2(in.kv[3][v]));
                            caxpy(er, ht * DP5::e6, to_d2(in.kv[4][v]));
                            caxpy(er, ht * DP5::e7, to_d2(ap[v]));
                            const double scl = g.atol + g.rtol * fmax(sqrt(abs2d(yr)), sqrt(abs2d(in.yn[v])));
                            acc3[0] += wt * ((er.x * er.x + er.y * er.y) / (scl * scl));
                            acc3[1] += wt * abs2d(ap[v]);
                            continue;
                        }
                        o[v] = yr;
                        if (s == 2) {
                            caxpy(o[v], (T)(ht * DP5::a31), k1r);
                            caxpy(o[v], (T)(ht * DP5::a32), ap[v]);
                        } else if (s == 3) {
                            caxpy(o[v], (T)(ht * DP5::a41), k1r);
                            caxpy(o[v], (T)(ht * DP5::a42), in.kv[0][v]);
                            caxpy(o[v], (T)(ht * DP5::a43), ap[v]);
                        } else if (s == 4) {
                            caxpy(o[v], (T)(ht * DP5::a51), k1r);
                            caxpy(o[v], (T)(ht * DP5::a52), in.kv[0][v]);
                            caxpy(o[v], (T)(ht * DP5::a53), in.kv[1][v]);
                            caxpy(o[v], (T)(ht * DP5::a54), ap[v]);
                        } else if (s == 5) {
                            caxpy(o[v], (T)(ht * DP5::a61), k1r);
                            caxpy(o[v], (T)(ht * DP5::a62), in.kv[0][v]);
                            caxpy(o[v], (T)(ht * DP5::a63), in.kv[1][v]);
                            caxpy(o[v], (T)(ht * DP5::a64), in.kv[2][v]);
                            caxpy(o[v], (T)(ht * DP5::a65), ap[v]);
                        } else {
                            caxpy(o[v], (T)(ht * DP5::b1), k1r);
                            caxpy(o[v], (T)(ht * DP5::b3), in.kv[1][v]);
                            caxpy(o[v], (T)(ht * DP5::b4), in.kv[2][v]);
                            caxpy(o[v], (T)(ht * DP5::b5), in.kv[3][v]);
                            caxpy(o[v], (T)(ht * DP5::b6), ap[v]);
                            const int i = TI * 16 + mrow<T>(k4, v), j = TJ * 16 + r16;
                            if (i == j) acc3[2] += (double)o[v].x;  // trace of y_new as B0 holds it
                        }
                    }
                    if (s == 7) {
                        gst4(k7 + e, ap);
                    } else {
                        gst4(ks[s - 2] + e, ap);
                        if (s == 6) gst4(ynew + e, o);
                        R::put_b0(B0re, B0im, TI, TJ, lane, o);
                    }
                });
            __syncthreads();
        }
        n_rhs += 6;
        ++n_steps;
        // B0 now holds y_new (the stage-7 input)
        block_sum_n<3>(acc3, scr);
        const bool steady = g.steady_tol2 > 0.0;
        const double err = sqrt(acc3[0] / nd);
        if (!isfinite(err)) {
            status = 6;  // QT_ENONFINITE
            break;
        }
        if (err <= 1.0) {
            ++n_accept;
            double sc_new = 1.0;
            if (g.renorm) sc_new = tr0 / acc3[2];
            // steady-state mode: |L y_new|_2 at or below the tolerance ends the solve, and every
            // remaining save time receives the expectation values of the converged state
            const bool conv = steady && acc3[1] * sc_new * sc_new <= g.steady_tol2;
            if (conv) {
                for (int k = save_idx; k < g.nt; ++k) record_expect(k, sc_new);
            } else if (land) {
                record_expect(save_idx, sc_new);
            }
            t = land ? gld(g.tlist + save_idx) : t + ht;
            parity = 1 - parity;
            double hn = ht * pi_factor(err, err_prev);
            if (last_rejected && hn > ht) hn = ht;
            h = hn;
            err_prev = fmax(err, 1e-4);
            last_rejected = 0;
            scale = sc_new;
            if (conv) {
                save_idx = g.nt;
                status = ST_DONE;
            } else if (land) {
                ++save_idx;
                if (save_idx >= g.nt) status = steady ? 4 : ST_DONE;  // QT_EMAXSTEPS: not converged
            }
        } else {
            ++n_reject;
            h = ht * reject_factor(err);
            last_rejected = 1;
        }
        if (status == ST_RUNNING) {
            if (n_steps >= g.max_steps) status = 4;  // QT_EMAXSTEPS
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
void dense_fill_inst(DenseInst *g, int d, int nc, uint32_t creal, int nt, int ne, const void *ops, const void *rho0, void *vec,
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
    g->creal = (int32_t)creal;
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

// Operators in fragment order: for tile row I, 16-byte chunk ch and lane l, the E elements
// Op(16 I + l % 16, (l / 16) np / 4 + ch E + e), e < E, with E = 16 bytes / element size; a real
// collapse operator C_k (bit k of creal) keeps only its real parts, packed the same way.
void dense_pack_ops(const double2 *rowmajor, int np, int nops, uint32_t creal, int prec, std::vector<char> &out)
{
    const bool f64 = prec == QT_F64;
    const size_t es = f64 ? sizeof(double2) : sizeof(float2), mat = (size_t)np * np;
    const int kf = np / 4;
    out.assign((size_t)nops * mat * es, 0);
    for (int o = 0; o < nops; ++o) {
        const double2 *M = rowmajor + (size_t)o * mat;
        char *base = out.data() + (size_t)o * mat * es;
        const bool real = o > 0 && o - 1 < 32 && ((creal >> (o - 1)) & 1u);
        const int E = real ? (f64 ? 2 : 4) : (f64 ? 1 : 2);
        for (int I = 0; I < np / 16; ++I)
            for (int ch = 0; ch < kf / E; ++ch)
                for (int l = 0; l < 64; ++l)
                    for (int e = 0; e < E; ++e) {
                        const double2 v = M[(size_t)(I * 16 + (l & 15)) * np + (l >> 4) * kf + ch * E + e];
                        const size_t idx = (((size_t)I * (kf / E) + ch) * 64 + l) * E + e;
                        if (real && f64) ((double *)base)[idx] = v.x;
                        else if (real) ((float *)base)[idx] = (float)v.x;
                        else if (f64) ((double2 *)base)[idx] = v;
                        else ((float2 *)base)[idx] = make_float2((float)v.x, (float)v.y);
                    }
    }
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
    // upper tiles in row-major order; (tile, lane, slot) -> element as the kernel's accumulators
    const int np = dense_np(d), nt = np / 16;
    int u = 0;
    for (int I = 0; I < nt; ++I)
        for (int J = I; J < nt; ++J, ++u)
            for (int lane = 0; lane < 64; ++lane)
                for (int v = 0; v < 4; ++v) {
                    const int q4 = lane >> 4;
                    const int i = I * 16 + (prec == QT_F64 ? q4 + 4 * v : 4 * q4 + v);
                    const int j = J * 16 + (lane & 15);
                    if (i > j || j >= d) continue;  // below the diagonal: the mirror of (j, i)
                    const size_t e = ((size_t)u * 64 + lane) * 4 + v;
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
                    if (i != j) {
                        out[2 * ((size_t)j * d + i)] = re * scale;
                        out[2 * ((size_t)j * d + i) + 1] = -im * scale;
                    }
                }
}

}  // namespace qt

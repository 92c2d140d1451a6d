// qt_common.h -- device-side building blocks shared by the solver kernels of libqtamd.
//
// Complex arithmetic on interleaved (re, im) vectors, the Dormand-Prince 5(4) coefficients,
// the step-size controller and the wave-level reductions.  The integrator itself is never named
// in arXiv:2504.21440 (it delegates to DifferentialEquations.jl); the library uses the DP5(4) pair
// of Dormand & Prince (1980) with the PI controller of Hairer-Norsett-Wanner's DOPRI5.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qt_csr.h"

// Global-memory (address space 1) qualifier for the pointers a kernel reads out of a descriptor in
// memory.  Such pointers are generic to the compiler, which then emits flat accesses; a flat access
// may alias LDS, so it stays ordered against the kernel's LDS traffic and is waited for together
// with LDS reads.
#define QT_GLOBAL __attribute__((address_space(1)))

namespace qt {

// Loads and stores through global-only views of generic pointers (see QT_GLOBAL).
typedef float gf2 __attribute__((ext_vector_type(2)));
typedef double gd2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 gld(const float2 *p)
{
    const gf2 v = *(const QT_GLOBAL gf2 *)p;
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ double2 gld(const double2 *p)
{
    const gd2 v = *(const QT_GLOBAL gd2 *)p;
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ double gld(const double *p) { return *(const QT_GLOBAL double *)p; }
__device__ __forceinline__ int32_t gld(const int32_t *p) { return *(const QT_GLOBAL int32_t *)p; }
__device__ __forceinline__ void gst(float2 *p, float2 a)
{
    gf2 v;
    v.x = a.x;
    v.y = a.y;
    *(QT_GLOBAL gf2 *)p = v;
}
__device__ __forceinline__ void gst(double2 *p, double2 a)
{
    gd2 v;
    v.x = a.x;
    v.y = a.y;
    *(QT_GLOBAL gd2 *)p = v;
}

template <typename T> struct vec2;
template <> struct vec2<float> { using type = float2; };
template <> struct vec2<double> { using type = double2; };

template <typename V> __device__ __forceinline__ V cmul(V a, V b)
{
    V r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
// a * conj(b)
template <typename V> __device__ __forceinline__ V cmulc(V a, V b)
{
    V r;
    r.x = a.x * b.x + a.y * b.y;
    r.y = a.y * b.x - a.x * b.y;
    return r;
}
template <typename V, typename S> __device__ __forceinline__ V cscale(V a, S s)
{
    V r;
    r.x = a.x * s;
    r.y = a.y * s;
    return r;
}
template <typename V> __device__ __forceinline__ V cadd(V a, V b)
{
    V r;
    r.x = a.x + b.x;
    r.y = a.y + b.y;
    return r;
}
// acc += s * a  (real s)
template <typename V, typename S> __device__ __forceinline__ void caxpy(V &acc, S s, V a)
{
    acc.x = fma(s, a.x, acc.x);
    acc.y = fma(s, a.y, acc.y);
}
// acc += a * b (complex)
template <typename V> __device__ __forceinline__ void cfma(V &acc, V a, V b)
{
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
}
__device__ __forceinline__ double2 to_d2(float2 a) { return make_double2((double)a.x, (double)a.y); }
__device__ __forceinline__ double2 to_d2(double2 a) { return a; }
template <typename V> __device__ __forceinline__ V from_d2(double2 a);
template <> __device__ __forceinline__ float2 from_d2<float2>(double2 a) { return make_float2((float)a.x, (float)a.y); }
template <> __device__ __forceinline__ double2 from_d2<double2>(double2 a) { return a; }
template <typename V> __device__ __forceinline__ double abs2d(V a)
{
    double x = (double)a.x, y = (double)a.y;
    return x * x + y * y;
}

// ---- Dormand-Prince 5(4) coefficients (row s of A is the combination that forms stage s+1) ----
struct DP5 {
    static constexpr double c2 = 1.0 / 5.0, c3 = 3.0 / 10.0, c4 = 4.0 / 5.0, c5 = 8.0 / 9.0;
    static constexpr double a21 = 1.0 / 5.0;
    static constexpr double a31 = 3.0 / 40.0, a32 = 9.0 / 40.0;
    static constexpr double a41 = 44.0 / 45.0, a42 = -56.0 / 15.0, a43 = 32.0 / 9.0;
    static constexpr double a51 = 19372.0 / 6561.0, a52 = -25360.0 / 2187.0, a53 = 64448.0 / 6561.0,
                            a54 = -212.0 / 729.0;
    static constexpr double a61 = 9017.0 / 3168.0, a62 = -355.0 / 33.0, a63 = 46732.0 / 5247.0, a64 = 49.0 / 176.0,
                            a65 = -5103.0 / 18656.0;
    static constexpr double b1 = 35.0 / 384.0, b3 = 500.0 / 1113.0, b4 = 125.0 / 192.0, b5 = -2187.0 / 6784.0,
                            b6 = 11.0 / 84.0;
    // e_j = b_j - bhat_j (fifth minus embedded fourth order weights)
    static constexpr double e1 = 35.0 / 384.0 - 5179.0 / 57600.0;
    static constexpr double e3 = 500.0 / 1113.0 - 7571.0 / 16695.0;
    static constexpr double e4 = 125.0 / 192.0 - 393.0 / 640.0;
    static constexpr double e5 = -2187.0 / 6784.0 + 92097.0 / 339200.0;
    static constexpr double e6 = 11.0 / 84.0 - 187.0 / 2100.0;
    static constexpr double e7 = -1.0 / 40.0;
};

// ---- step-size control (FP64) ----
// accepted step: h_new = h * clamp(0.9 err^-0.17 err_prev^0.04, 0.2, 10)
__device__ __forceinline__ double pi_factor(double err, double err_prev)
{
    if (err == 0.0) return 10.0;
    double f = 0.9 * pow(err, -0.17) * pow(err_prev, 0.04);
    return fmin(10.0, fmax(0.2, f));
}
// rejected step: h_new = h * max(0.2, 0.9 err^-0.17)
__device__ __forceinline__ double reject_factor(double err) { return fmax(0.2, 0.9 * pow(err, -0.17)); }

// Steps land exactly on every save time: a step that would reach within 1e-12 max(1,|tstop|) of
// (or pass) the next save time is clipped to end on it.
__device__ __forceinline__ double clip_step(double t, double h, double tstop, int32_t *land)
{
    double rem = tstop - t;
    double snap = 1e-12 * fmax(1.0, fabs(tstop));
    if (h >= rem - snap) {
        *land = 1;
        return rem;
    }
    *land = 0;
    return h;
}

// ---- reductions ----
template <typename S> __device__ __forceinline__ S wave_sum(S v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic block sum of one double per thread (blockDim.x multiple of 64, <= 1024).
// Every thread receives the result.  scratch: >= 16 doubles of LDS.
__device__ __forceinline__ double block_sum(double v, double *scratch)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) scratch[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += scratch[i];
    __syncthreads();
    return s;
}

// Block sums of N doubles per thread at once, each summed exactly as block_sum sums it (so the
// results are bitwise those of N separate block_sum calls) with one set of barriers.
// scratch: >= 16 * N doubles of LDS.
template <int N> __device__ __forceinline__ void block_sum_n(double (&v)[N], double *scratch)
{
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = wave_sum(v[j]);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < N; ++j) scratch[16 * j + w] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double s = 0.0;
        for (int i = 0; i < nw; ++i) s += scratch[16 * j + i];
        v[j] = s;
    }
    __syncthreads();
}

}  // namespace qt

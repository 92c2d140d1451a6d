// qt_coef.h -- time-dependent coefficients of a Liouvillian term (host and device).
//
// A time-dependent problem (arXiv:2504.21440, Sec. 2, QobjEvo; Sec. 3.4) has
//     H(t) = H_0 + sum_i f_i(t) H_i   and collapse operators g_k(t) C_k,
// so its generator is L(t) = L_0 + sum_i f_i(t) L[H_i] + sum_k |g_k(t)|^2 D[C_k] with
// L[H](rho) = -i (H rho - rho H).  The coefficient kinds are closed forms the device evaluates in
// FP64 at each Runge-Kutta stage time, plus sampled values interpolated linearly.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qtamd.h"

namespace qt {

struct CoefDev {
    int32_t kind;     // QT_COEF_*
    int32_t n_table;
    int32_t modsq;    // 1: the term takes |value|^2 (a collapse-operator coefficient)
    int32_t pad;
    double a_re, a_im, omega, phi, t0, sigma, table_t0, table_dt;
    const double2 *table;  // device copy of the samples (QT_COEF_TABLE)
};

// Value of one coefficient at time t (the squared modulus for collapse terms).
__host__ __device__ inline double2 coef_value(const CoefDev &c, double t)
{
    double re = c.a_re, im = c.a_im;  // QT_COEF_CONST
    if (c.kind == QT_COEF_COS) {
        const double f = cos(c.omega * t + c.phi);
        re *= f;
        im *= f;
    } else if (c.kind == QT_COEF_EXP) {
        const double th = c.omega * t + c.phi, cs = cos(th), sn = sin(th);
        const double r = re * cs - im * sn, i = re * sn + im * cs;
        re = r;
        im = i;
    } else if (c.kind == QT_COEF_GAUSS) {
        const double u = (t - c.t0) / c.sigma;
        const double f = exp(-0.5 * u * u) * cos(c.omega * t + c.phi);
        re *= f;
        im *= f;
    } else if (c.kind == QT_COEF_TABLE) {
        // piecewise-linear through the samples at table_t0 + k table_dt, constant beyond the ends
        const double x = (t - c.table_t0) / c.table_dt;
        double2 s;
        if (c.n_table == 1 || !(x > 0.0)) {  // also a non-finite time: never index with it
            s = c.table[0];
        } else if (x >= (double)(c.n_table - 1)) {
            s = c.table[c.n_table - 1];
        } else {
            const int k = (int)floor(x);
            const double w = x - (double)k;
            const double2 lo = c.table[k], hi = c.table[k + 1];
            s = make_double2(lo.x + w * (hi.x - lo.x), lo.y + w * (hi.y - lo.y));
        }
        const double r = re * s.x - im * s.y, i = re * s.y + im * s.x;
        re = r;
        im = i;
    }
    if (c.modsq) return make_double2(re * re + im * im, 0.0);
    return make_double2(re, im);
}

}  // namespace qt

// qtamd_sde.cpp -- stochastic Schrodinger / master equation plans under homodyne detection
// (arXiv:2504.21440, Sec. 3.5).
//
// The plan builds, on the host in FP64, the linear drift A and the measured operators B_n of the
// state space (SSE: A = -i H - 1/2 sum S^dag S, B_n = S_n on kets; SME: A = the Lindbladian with
// c_ops and sc_ops and B_n = S_n (x) I + I (x) conj(S_n) on the row-major vec(rho)), stores them in
// ELL column-major order in the solve precision, uploads them with the e_ops, the normalised initial
// state and the steps of each tlist interval, and lays out the per-trajectory outputs.  Running it
// launches the persistent trajectory kernel and the FP64 ensemble reduction.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "qt_csr.h"
#include "qt_host.h"
#include "qt_mc.h"
#include "qt_sde.h"

struct qt_sde_plan {
    qt::Ctx *ctx = nullptr;
    int32_t prec = QT_MIXED;
    qt::SdeParams p{};
    qt::Arena arena;
    size_t o_params = 0, o_mean = 0, o_se = 0;
    int grid = 1;
    int64_t steps = 0;  // steps per trajectory
    double last_ms = 0.0;
};

namespace qt {

// A (x) B for square operators (dimension A.d * B.d), row-major vec convention.
static HCsr csr_kron(const HCsr &A, const HCsr &B)
{
    HCsr K;
    K.d = A.d * B.d;
    K.ptr.assign((size_t)K.d + 1, 0);
    for (int32_t i = 0; i < A.d; ++i)
        for (int32_t k = 0; k < B.d; ++k) {
            for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p)
                for (int64_t q = B.ptr[k]; q < B.ptr[k + 1]; ++q) {
                    K.idx.push_back(A.idx[p] * B.d + B.idx[q]);
                    K.val.push_back(A.val[p] * B.val[q]);
                }
            K.ptr[(size_t)i * B.d + k + 1] = (int64_t)K.idx.size();
        }
    return K;
}

static HCsr csr_conj(const HCsr &A)
{
    HCsr C = A;
    for (auto &v : C.val) v = std::conj(v);
    return C;
}

static HCsr csr_eye(int32_t d)
{
    HCsr I;
    I.d = d;
    I.ptr.resize(d + 1);
    for (int32_t i = 0; i <= d; ++i) I.ptr[i] = i;
    for (int32_t i = 0; i < d; ++i) {
        I.idx.push_back(i);
        I.val.push_back(cd(1.0, 0.0));
    }
    return I;
}

// ELL (column-major) of one operator with width W; padding: zero value on the diagonal.
static void to_ell(const HCsr &A, int32_t W, int32_t *col, double *val)
{
    const int32_t n = A.d;
    for (int32_t r = 0; r < n; ++r) {
        int32_t k = 0;
        for (int64_t p = A.ptr[r]; p < A.ptr[r + 1]; ++p, ++k) {
            col[(size_t)k * n + r] = A.idx[p];
            val[2 * ((size_t)k * n + r)] = A.val[p].real();
            val[2 * ((size_t)k * n + r) + 1] = A.val[p].imag();
        }
        for (; k < W; ++k) {
            col[(size_t)k * n + r] = r;
            val[2 * ((size_t)k * n + r)] = 0.0;
            val[2 * ((size_t)k * n + r) + 1] = 0.0;
        }
    }
}

static int32_t ell_width(const HCsr &A)
{
    int32_t W = 1;
    for (int32_t i = 0; i < A.d; ++i) W = std::max<int32_t>(W, (int32_t)(A.ptr[i + 1] - A.ptr[i]));
    return W;
}

static qt_status sde_plan_create(Ctx *ctx, const qt_sde_problem *pr, int32_t master, const qt_opts *opts_in,
                                 qt_sde_plan **out)
{
    if (!ctx || !pr || !out || !pr->H) return set_error(QT_EINVAL, "qt_sde_plan_create: null argument");
    qt_opts o;
    if (opts_in) o = *opts_in;
    else qt_opts_default(&o);
    if (o.precision != QT_F64 && o.precision != QT_MIXED) return set_error(QT_EINVAL, "opts: bad precision");
    if (pr->ntraj < 1) return set_error(QT_EINVAL, "ntraj must be >= 1");
    if (!(pr->dt > 0.0) || !std::isfinite(pr->dt)) return set_error(QT_EINVAL, "dt must be positive");
    if (pr->n_sc < 0 || pr->n_sc > SDE_MAX_SC || (pr->n_sc > 0 && !pr->sc_ops))
        return set_error(QT_EINVAL, "between 0 and 8 measured operators are supported");
    if (pr->n_c < 0 || (pr->n_c > 0 && !pr->c_ops)) return set_error(QT_EINVAL, "bad c_ops");
    if (!master && pr->n_c > 0) return set_error(QT_EINVAL, "the stochastic Schrodinger equation takes no c_ops");
    if (pr->n_t < 1 || !pr->tlist) return set_error(QT_EINVAL, "tlist must hold at least one time");
    for (int32_t i = 0; i < pr->n_t; ++i)
        if (!std::isfinite(pr->tlist[i]) || (i > 0 && !(pr->tlist[i] > pr->tlist[i - 1])))
            return set_error(QT_EINVAL, "tlist must be finite and strictly increasing");
    if (pr->n_e < 0 || (pr->n_e > 0 && !pr->e_ops)) return set_error(QT_EINVAL, "bad e_ops");
    if (!pr->state0) return set_error(QT_EINVAL, "state0 is null");
    if (!master && !pr->is_ket) return set_error(QT_EINVAL, "the stochastic Schrodinger equation needs a ket");
    HCsr H;
    qt_status st = csr_from_abi(pr->H, 0, &H, "H");
    if (st) return st;
    const int32_t d = H.d;
    const int64_t n64 = master ? (int64_t)d * d : d;
    if (n64 > (int64_t)SDE_THREADS * SDE_MAX_ROWS) return set_error(QT_EINVAL, "state longer than 4096 entries");
    const int32_t n = (int32_t)n64;
    std::vector<HCsr> cs(pr->n_c), ss(pr->n_sc), es(pr->n_e);
    for (int k = 0; k < pr->n_c; ++k)
        if ((st = csr_from_abi(&pr->c_ops[k], d, &cs[k], "c_ops"))) return st;
    for (int k = 0; k < pr->n_sc; ++k)
        if ((st = csr_from_abi(&pr->sc_ops[k], d, &ss[k], "sc_ops"))) return st;
    for (int k = 0; k < pr->n_e; ++k)
        if ((st = csr_from_abi(&pr->e_ops[k], d, &es[k], "e_ops"))) return st;

    // initial state: unit-norm ket (SSE) or unit-trace vec(rho) (SME)
    std::vector<cd> x0(n);
    if (!master) {
        double nrm = 0.0;
        for (int32_t i = 0; i < d; ++i) {
            x0[i] = cd(pr->state0[2 * i], pr->state0[2 * i + 1]);
            nrm += std::norm(x0[i]);
        }
        if (!(nrm > 0) || !std::isfinite(nrm)) return set_error(QT_EINVAL, "state0 is zero or not finite");
        for (auto &v : x0) v /= std::sqrt(nrm);
    } else {
        if (pr->is_ket) {
            for (int32_t i = 0; i < d; ++i)
                for (int32_t j = 0; j < d; ++j)
                    x0[(size_t)i * d + j] = cd(pr->state0[2 * i], pr->state0[2 * i + 1]) *
                                            std::conj(cd(pr->state0[2 * j], pr->state0[2 * j + 1]));
        } else {
            for (int32_t i = 0; i < n; ++i) x0[i] = cd(pr->state0[2 * i], pr->state0[2 * i + 1]);
        }
        cd tr = 0.0;
        for (int32_t i = 0; i < d; ++i) tr += x0[(size_t)i * d + i];
        if (!(std::abs(tr) > 0) || !std::isfinite(std::abs(tr))) return set_error(QT_EINVAL, "rho0 has zero trace");
        for (auto &v : x0) v /= tr.real();
    }

    // operators of the state space
    HCsr A;
    std::vector<HCsr> Bs(pr->n_sc);
    if (!master) {
        A = csr_axpby(cd(0.0, -1.0), H, cd(0.0, 0.0), csr_zero(d));
        for (auto &S : ss) A = csr_axpby(cd(1.0, 0.0), A, cd(-0.5, 0.0), csr_matmul(csr_adjoint(S), S));
        for (int k = 0; k < pr->n_sc; ++k) Bs[k] = ss[k];
    } else {
        HCsr A0 = csr_axpby(cd(0.0, -1.0), H, cd(0.0, 0.0), csr_zero(d));
        std::vector<const HCsr *> all;
        for (auto &C : cs) all.push_back(&C);
        for (auto &S : ss) all.push_back(&S);
        for (auto *C : all) A0 = csr_axpby(cd(1.0, 0.0), A0, cd(-0.5, 0.0), csr_matmul(csr_adjoint(*C), *C));
        const HCsr I = csr_eye(d);
        A = csr_axpby(cd(1.0, 0.0), csr_kron(A0, I), cd(1.0, 0.0), csr_kron(I, csr_conj(A0)));
        for (auto *C : all) A = csr_axpby(cd(1.0, 0.0), A, cd(1.0, 0.0), csr_kron(*C, csr_conj(*C)));
        for (int k = 0; k < pr->n_sc; ++k)
            Bs[k] = csr_axpby(cd(1.0, 0.0), csr_kron(ss[k], I), cd(1.0, 0.0), csr_kron(I, csr_conj(ss[k])));
    }
    const int32_t WA = ell_width(A);
    int32_t WB = 1;
    for (auto &B : Bs) WB = std::max(WB, ell_width(B));
    std::vector<int32_t> a_col((size_t)WA * n), b_col((size_t)std::max(1, pr->n_sc) * WB * n, 0);
    std::vector<double> a_val((size_t)WA * n * 2), b_val((size_t)std::max(1, pr->n_sc) * WB * n * 2, 0.0);
    to_ell(A, WA, a_col.data(), a_val.data());
    for (int k = 0; k < pr->n_sc; ++k)
        to_ell(Bs[k], WB, b_col.data() + (size_t)k * WB * n, b_val.data() + (size_t)k * WB * n * 2);
    std::vector<int32_t> eptr((size_t)std::max(1, pr->n_e) * (d + 1), 0), ecol;
    std::vector<double2> eval;
    for (int k = 0; k < pr->n_e; ++k) {
        const int32_t base = (int32_t)ecol.size();
        for (int32_t i = 0; i <= d; ++i) eptr[(size_t)k * (d + 1) + i] = base + (int32_t)es[k].ptr[i];
        for (int64_t p = 0; p < es[k].nnz(); ++p) {
            ecol.push_back(es[k].idx[p]);
            eval.push_back(make_double2(es[k].val[p].real(), es[k].val[p].imag()));
        }
    }
    const std::vector<int32_t> evidx = expect_vec_index(eptr, ecol, d, pr->n_e);
    std::vector<int32_t> nsub(std::max(1, pr->n_t - 1), 1);
    int64_t steps = 0;
    for (int32_t i = 0; i + 1 < pr->n_t; ++i) {
        const double len = pr->tlist[i + 1] - pr->tlist[i];
        const double q = std::ceil(len / pr->dt * (1.0 - 1e-12));
        if (!(q < 1e9)) return set_error(QT_EINVAL, "dt too small for the tlist intervals");
        nsub[i] = std::max<int32_t>(1, (int32_t)q);
        steps += nsub[i];
    }
    if (steps >= (int64_t)UINT32_MAX) return set_error(QT_EINVAL, "more than 2^32 steps per trajectory");

    const bool f64 = o.precision == QT_F64;
    const size_t es_b = f64 ? 16 : 8;
    auto to_prec = [&](const std::vector<double> &v) {
        std::vector<char> b(v.size() / 2 * es_b);
        if (f64) std::memcpy(b.data(), v.data(), v.size() * 8);
        else {
            float *f = (float *)b.data();
            for (size_t i = 0; i < v.size(); ++i) f[i] = (float)v[i];
        }
        return b;
    };
    std::vector<double> x0d((size_t)2 * n);
    for (int32_t i = 0; i < n; ++i) {
        x0d[2 * i] = x0[i].real();
        x0d[2 * i + 1] = x0[i].imag();
    }
    const std::vector<char> av_b = to_prec(a_val), bv_b = to_prec(b_val), x0_b = to_prec(x0d);

    QT_HIP(hipSetDevice(ctx->device));
    qt_sde_plan *P = new qt_sde_plan();
    P->ctx = ctx;
    P->prec = o.precision;
    P->steps = steps;
    SdeParams &p = P->p;
    p.n = n;
    p.d = d;
    p.m = pr->n_sc;
    p.ne = pr->n_e;
    p.nt = pr->n_t;
    int rows = 1;
    while (rows * SDE_THREADS < n) rows *= 2;
    p.rows = rows;
    p.sme = master ? 1 : 0;
    p.occ2 = 0;
    sde_choose_variant(p, f64, ctx->device);
    p.WA = WA;
    p.WB = WB;
    p.cg = master ? 1.0 : 0.5;
    p.seed = pr->seed;
    p.ntraj = pr->ntraj;
    if (sde_lds_bytes(p, f64) > 160 * 1024) {
        delete P;
        return set_error(QT_EINVAL, "state and measured-operator images exceed the 160 KB of LDS");
    }
    const int64_t nj = pr->ntraj;
    const size_t nm = (size_t)std::max(1, pr->n_sc) * std::max(1, pr->n_t - 1);
    Arena &a = P->arena;
    const size_t o_ac = a.reserve(a_col.size() * 4), o_av = a.reserve(av_b.size()), o_bc = a.reserve(b_col.size() * 4),
                 o_bv = a.reserve(bv_b.size()), o_ep = a.reserve(eptr.size() * 4),
                 o_ec = a.reserve(std::max<size_t>(1, ecol.size()) * 4),
                 o_ev = a.reserve(std::max<size_t>(1, eval.size()) * 16),
                 o_ei = a.reserve(std::max<size_t>(1, evidx.size()) * 4), o_x0 = a.reserve(x0_b.size()),
                 o_tl = a.reserve((size_t)pr->n_t * 8), o_ns = a.reserve(nsub.size() * 4),
                 o_tr = a.reserve(std::max<size_t>(1, (size_t)nj * pr->n_e * pr->n_t) * 16),
                 o_me = a.reserve((size_t)nj * nm * 8), o_st = a.reserve((size_t)nj * 4), o_q = a.reserve(64);
    P->o_mean = a.reserve(std::max<size_t>(1, (size_t)pr->n_e * pr->n_t) * 16);
    P->o_se = a.reserve(std::max<size_t>(1, (size_t)pr->n_e * pr->n_t) * 8);
    P->o_params = a.reserve(sizeof(SdeParams));
    if ((st = a.alloc())) {
        delete P;
        return st;
    }
    p.a_col = (const int32_t *)a.at(o_ac);
    p.a_val = a.at(o_av);
    p.b_col = (const int32_t *)a.at(o_bc);
    p.b_val = a.at(o_bv);
    p.eptr = (const int32_t *)a.at(o_ep);
    p.ecol = (const int32_t *)a.at(o_ec);
    p.eval = (const double2 *)a.at(o_ev);
    p.evidx = (const int32_t *)a.at(o_ei);
    p.x0 = a.at(o_x0);
    p.tlist = (const double *)a.at(o_tl);
    p.nsub = (const int32_t *)a.at(o_ns);
    p.expect_tr = (double2 *)a.at(o_tr);
    p.meas = (double *)a.at(o_me);
    p.status = (int32_t *)a.at(o_st);
    p.queue = (unsigned long long *)a.at(o_q);
    hipStream_t s = ctx->stream;
    hipError_t e = hipSuccess;
    auto up = [&](size_t off, const void *src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(a.at(off), src, bytes, hipMemcpyHostToDevice, s);
    };
    up(o_ac, a_col.data(), a_col.size() * 4);
    up(o_av, av_b.data(), av_b.size());
    up(o_bc, b_col.data(), b_col.size() * 4);
    up(o_bv, bv_b.data(), bv_b.size());
    up(o_ep, eptr.data(), eptr.size() * 4);
    up(o_ec, ecol.data(), ecol.size() * 4);
    up(o_ev, eval.data(), eval.size() * 16);
    up(o_ei, evidx.data(), evidx.size() * 4);
    up(o_x0, x0_b.data(), x0_b.size());
    up(o_tl, pr->tlist, (size_t)pr->n_t * 8);
    up(o_ns, nsub.data(), nsub.size() * 4);
    up(P->o_params, &p, sizeof(SdeParams));
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        a.release();
        delete P;
        return set_error(QT_EDEVICE, std::string("sde plan upload: ") + hipGetErrorString(e));
    }
    P->grid = sde_grid(p, f64, ctx->device);
    ctx->refs++;
    *out = P;
    return QT_OK;
}

}  // namespace qt

using namespace qt;

extern "C" {

qt_status qt_sde_plan_create(qt_ctx *ctx, const qt_sde_problem *prob, int32_t master, const qt_opts *opts,
                             qt_sde_plan **out)
{
    return sde_plan_create(ctx, prob, master, opts, out);
}

qt_status qt_sde_plan_run(qt_sde_plan *P)
{
    if (!P) return set_error(QT_EINVAL, "null plan");
    QT_HIP(hipSetDevice(P->ctx->device));
    hipStream_t s = P->ctx->stream;
    hipEvent_t e0, e1;
    QT_HIP(hipEventCreate(&e0));
    QT_HIP(hipEventCreate(&e1));
    QT_HIP(hipEventRecord(e0, s));
    mc_launch_queue_reset(P->p.queue, s);
    sde_launch(P->p, (const SdeParams *)P->arena.at(P->o_params), P->prec == QT_F64, P->grid, s);
    mc_launch_stats(P->p.expect_tr, P->p.ntraj, P->p.ne, P->p.nt, (double2 *)P->arena.at(P->o_mean),
                    (double *)P->arena.at(P->o_se), s);
    QT_HIP(hipGetLastError());
    QT_HIP(hipEventRecord(e1, s));
    QT_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    QT_HIP(hipEventElapsedTime(&ms, e0, e1));
    P->last_ms = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return QT_OK;
}

qt_status qt_sde_plan_result(qt_sde_plan *P, double *mean_out, double *se_out, double *expect_tr, double *meas_mean,
                             double *meas_tr, qt_stats *stats)
{
    if (!P) return set_error(QT_EINVAL, "null plan");
    QT_HIP(hipSetDevice(P->ctx->device));
    const SdeParams &p = P->p;
    const size_t mm = (size_t)p.ne * p.nt, nj = (size_t)p.ntraj;
    const size_t nm = (size_t)p.m * std::max(0, p.nt - 1);
    if (mean_out && mm) QT_HIP(hipMemcpy(mean_out, P->arena.at(P->o_mean), mm * 16, hipMemcpyDeviceToHost));
    if (se_out && mm) QT_HIP(hipMemcpy(se_out, P->arena.at(P->o_se), mm * 8, hipMemcpyDeviceToHost));
    if (expect_tr && mm) QT_HIP(hipMemcpy(expect_tr, p.expect_tr, nj * mm * 16, hipMemcpyDeviceToHost));
    if ((meas_mean || meas_tr) && nm) {
        std::vector<double> mt(nj * nm);
        QT_HIP(hipMemcpy(mt.data(), p.meas, nj * nm * 8, hipMemcpyDeviceToHost));
        if (meas_tr) std::memcpy(meas_tr, mt.data(), nj * nm * 8);
        if (meas_mean)
            for (size_t q = 0; q < nm; ++q) {
                double s = 0.0;
                for (size_t j = 0; j < nj; ++j) s += mt[j * nm + q];
                meas_mean[q] = s / (double)nj;
            }
    }
    std::vector<int32_t> sv(nj);
    QT_HIP(hipMemcpy(sv.data(), p.status, nj * 4, hipMemcpyDeviceToHost));
    qt_stats s;
    std::memset(&s, 0, sizeof(s));
    int32_t worst = QT_OK;
    for (size_t j = 0; j < nj; ++j) {
        const int32_t code = sv[j] == ST_DONE ? QT_OK : sv[j];
        if (code != QT_OK && worst == QT_OK) worst = code;
    }
    s.n_accept = P->steps * (int64_t)nj;
    s.n_rhs = P->steps * (int64_t)nj * (1 + 2 * p.m);  // A and each B_n at x, each B_n at its supporting value
    s.status = worst;
    s.device_ms = P->last_ms;
    if (stats) *stats = s;
    if (worst != QT_OK) return set_error(worst, "a trajectory stopped with status " + std::to_string(worst));
    return QT_OK;
}

qt_status qt_sde_plan_destroy(qt_sde_plan *P)
{
    if (!P) return QT_OK;
    (void)hipSetDevice(P->ctx->device);
    P->arena.release();
    P->ctx->refs--;
    delete P;
    return QT_OK;
}

static qt_status sde_solve(qt_ctx *ctx, const qt_sde_problem *prob, int32_t master, const qt_opts *opts,
                           double *mean_out, double *se_out, double *meas_mean, qt_stats *stats)
{
    qt_sde_plan *P = nullptr;
    qt_status st = qt_sde_plan_create(ctx, prob, master, opts, &P);
    if (st) {
        if (stats) stats->status = st;
        return st;
    }
    st = qt_sde_plan_run(P);
    if (!st) st = qt_sde_plan_result(P, mean_out, se_out, nullptr, meas_mean, nullptr, stats);
    qt_sde_plan_destroy(P);
    return st;
}

qt_status qt_ssesolve(qt_ctx *ctx, const qt_sde_problem *prob, const qt_opts *opts, double *mean_out, double *se_out,
                      double *meas_mean, qt_stats *stats)
{
    return sde_solve(ctx, prob, 0, opts, mean_out, se_out, meas_mean, stats);
}

qt_status qt_smesolve(qt_ctx *ctx, const qt_sde_problem *prob, const qt_opts *opts, double *mean_out, double *se_out,
                      double *meas_mean, qt_stats *stats)
{
    return sde_solve(ctx, prob, 1, opts, mean_out, se_out, meas_mean, stats);
}

}  // extern "C"

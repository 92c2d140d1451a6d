// qtamd_mc.cpp -- Monte-Carlo wave-function plans (arXiv:2504.21440, Sec. 3.3).
//
// The plan builds A = -i H_eff = -i H - 1/2 sum_k C_k^dag C_k on the host (sparse, FP64), stores it
// in ELL column-major order in the solve precision (with time-dependent terms: every term's entries
// in turn, each column tagged with its term), uploads the jump operators, e_ops and the
// normalised initial state, and lays out the per-trajectory outputs.  Running it launches the
// persistent trajectory kernel and the FP64 ensemble reduction; nothing returns to the host until
// every trajectory has finished.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "qt_coef.h"
#include "qt_csr.h"
#include "qt_host.h"
#include "qt_mc.h"

struct qt_mc_plan {
    qt::Ctx *ctx = nullptr;
    int32_t prec = QT_MIXED;
    qt::McParams p{};
    qt::Arena arena;
    size_t o_params = 0, o_mean = 0, o_se = 0;
    int grid = 1;
    bool td = false;
    double last_ms = 0.0;
};

namespace qt {

// ws: the caller's device workspace (null: the plan allocates its arena); query: only report the
// workspace bytes and create nothing.
static qt_status mc_plan_create(Ctx *ctx, const qt_mc_problem *pr, const qt_td_terms *td, const qt_opts *opts_in,
                                int32_t maxj, qt_mc_plan **out, void *ws = nullptr, size_t ws_bytes = 0,
                                size_t *query = nullptr)
{
    if (!ctx || !pr || (!out && !query) || !pr->H) return set_error(QT_EINVAL, "qt_mc_plan_create: null argument");
    qt_opts o;
    if (opts_in) o = *opts_in;
    else qt_opts_default(&o);
    if (o.precision != QT_F64 && o.precision != QT_MIXED) return set_error(QT_EINVAL, "opts: bad precision");
    if (!(o.abstol > 0) || !(o.reltol >= 0) || o.max_steps <= 0) return set_error(QT_EINVAL, "opts: bad tolerances");
    if (pr->ntraj < 1) return set_error(QT_EINVAL, "ntraj must be >= 1");
    if (pr->n_c < 0 || pr->n_c > 64 || (pr->n_c > 0 && !pr->c_ops))
        return set_error(QT_EINVAL, "between 0 and 64 collapse operators are supported");
    if (pr->n_t < 1 || !pr->tlist) return set_error(QT_EINVAL, "tlist must hold at least one time");
    for (int32_t i = 0; i < pr->n_t; ++i)
        if (!std::isfinite(pr->tlist[i]) || (i > 0 && !(pr->tlist[i] > pr->tlist[i - 1])))
            return set_error(QT_EINVAL, "tlist must be finite and strictly increasing");
    if (pr->n_e < 0 || (pr->n_e > 0 && !pr->e_ops)) return set_error(QT_EINVAL, "bad e_ops");
    if (maxj < 0) return set_error(QT_EINVAL, "max_jump_record must be >= 0");
    HCsr H;
    qt_status st = csr_from_abi(pr->H, 0, &H, "H");
    if (st) return st;
    const int32_t d = H.d;
    if (d > MC_THREADS * MC_MAX_ROWS) return set_error(QT_EINVAL, "mcsolve supports d <= 4096");
    std::vector<HCsr> cs(pr->n_c);
    for (int k = 0; k < pr->n_c; ++k)
        if ((st = csr_from_abi(&pr->c_ops[k], d, &cs[k], "c_ops"))) return st;
    std::vector<HCsr> es(pr->n_e);
    for (int k = 0; k < pr->n_e; ++k)
        if ((st = csr_from_abi(&pr->e_ops[k], d, &es[k], "e_ops"))) return st;
    if (!pr->psi0) return set_error(QT_EINVAL, "psi0 is null");
    double nrm = 0.0;
    for (int32_t i = 0; i < d; ++i) {
        if (!std::isfinite(pr->psi0[2 * i]) || !std::isfinite(pr->psi0[2 * i + 1]))
            return set_error(QT_EINVAL, "psi0 has non-finite entries");
        nrm += pr->psi0[2 * i] * pr->psi0[2 * i] + pr->psi0[2 * i + 1] * pr->psi0[2 * i + 1];
    }
    if (!(nrm > 0)) return set_error(QT_EINVAL, "psi0 is zero");
    nrm = std::sqrt(nrm);
    // time-dependent terms
    const int32_t n_h = td ? td->n_h : 0;
    if (n_h < 0 || (n_h > 0 && (!td->h_terms || !td->h_coefs))) return set_error(QT_EINVAL, "bad time-dependent terms");
    const qt_coef *c_coefs = td ? td->c_coefs : nullptr;
    std::vector<HCsr> hs(n_h);
    for (int i = 0; i < n_h; ++i) {
        if ((st = check_coef(td->h_coefs[i], false, "h_coefs"))) return st;
        if ((st = csr_from_abi(&td->h_terms[i], d, &hs[i], "h_terms"))) return st;
    }
    auto weighted = [&](int k) { return c_coefs && c_coefs[k].kind != QT_COEF_NONE; };
    int n_w = 0;
    for (int k = 0; k < pr->n_c; ++k)
        if (c_coefs) {
            if ((st = check_coef(c_coefs[k], true, "c_coefs"))) return st;
            n_w += weighted(k);
        }
    const int nterms = n_h + n_w;
    if (nterms > MC_MAX_TERMS) return set_error(QT_EINVAL, "at most 31 time-dependent terms");

    // A = -i H - 1/2 sum_k C_k^dag C_k (constant channels), then -i H_i, then -1/2 C_k^dag C_k of each
    // weighted channel, stored in ELL (column-major) with each entry's term above MC_TAG_SHIFT
    std::vector<HCsr> terms;
    std::vector<const qt_coef *> tsrc;  // coefficient of term t (t >= 1)
    std::vector<int32_t> cweight(std::max(1, pr->n_c), -1);
    {
        HCsr A = csr_axpby(cd(0.0, -1.0), H, cd(0.0, 0.0), csr_zero(d));
        for (int k = 0; k < pr->n_c; ++k)
            if (!weighted(k))
                A = csr_axpby(cd(1.0, 0.0), A, cd(-0.5, 0.0), csr_matmul(csr_adjoint(cs[k]), cs[k]));
        terms.push_back(A);
        for (int i = 0; i < n_h; ++i) {
            terms.push_back(csr_axpby(cd(0.0, -1.0), hs[i], cd(0.0, 0.0), csr_zero(d)));
            tsrc.push_back(&td->h_coefs[i]);
        }
        for (int k = 0; k < pr->n_c; ++k)
            if (weighted(k)) {
                terms.push_back(
                    csr_axpby(cd(-0.5, 0.0), csr_matmul(csr_adjoint(cs[k]), cs[k]), cd(0.0, 0.0), csr_zero(d)));
                cweight[k] = (int32_t)tsrc.size();
                tsrc.push_back(&c_coefs[k]);
            }
    }
    int32_t W = 1;
    for (int32_t i = 0; i < d; ++i) {
        int32_t w = 0;
        for (auto &T : terms) w += (int32_t)(T.ptr[i + 1] - T.ptr[i]);
        W = std::max(W, w);
    }
    const bool f64 = o.precision == QT_F64;
    const size_t es_b = f64 ? 16 : 8;
    std::vector<int32_t> ell_col((size_t)W * d);
    std::vector<double> ell_val((size_t)W * d * 2, 0.0);
    for (int32_t r = 0; r < d; ++r) {
        int32_t k = 0;
        for (size_t t = 0; t < terms.size(); ++t) {
            const HCsr &T = terms[t];
            for (int64_t p = T.ptr[r]; p < T.ptr[r + 1]; ++p, ++k) {
                ell_col[(size_t)k * d + r] = T.idx[p] | ((int32_t)t << MC_TAG_SHIFT);
                ell_val[2 * ((size_t)k * d + r)] = T.val[p].real();
                ell_val[2 * ((size_t)k * d + r) + 1] = T.val[p].imag();
            }
        }
        for (; k < W; ++k) ell_col[(size_t)k * d + r] = r;  // padding: zero value on the diagonal
    }
    // coefficient descriptors, their sample tables after them
    std::vector<CoefDev> cdev(std::max(1, nterms));
    size_t tab_bytes = 0;
    for (int t = 0; t < nterms; ++t) {
        cdev[t] = coef_from_abi(*tsrc[t], t >= n_h ? 1 : 0);
        if (tsrc[t]->kind == QT_COEF_TABLE) tab_bytes += (size_t)tsrc[t]->n_table * sizeof(double2);
    }
    std::vector<int32_t> cptr((size_t)std::max(1, pr->n_c) * (d + 1), 0), ccol;
    std::vector<double> cval;
    for (int k = 0; k < pr->n_c; ++k) {
        const int32_t base = (int32_t)ccol.size();
        for (int32_t i = 0; i <= d; ++i) cptr[(size_t)k * (d + 1) + i] = base + (int32_t)cs[k].ptr[i];
        for (int64_t p = 0; p < cs[k].nnz(); ++p) {
            ccol.push_back(cs[k].idx[p]);
            cval.push_back(cs[k].val[p].real());
            cval.push_back(cs[k].val[p].imag());
        }
    }
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
    std::vector<double> psi((size_t)2 * d);
    for (int32_t i = 0; i < 2 * d; ++i) psi[i] = pr->psi0[i] / nrm;
    auto to_prec = [&](const std::vector<double> &v) {
        std::vector<char> b(v.size() / 2 * es_b);
        if (f64) std::memcpy(b.data(), v.data(), v.size() * 8);
        else {
            float *f = (float *)b.data();
            for (size_t i = 0; i < v.size(); ++i) f[i] = (float)v[i];
        }
        return b;
    };
    const std::vector<char> ev_b = to_prec(ell_val), cv_b = to_prec(cval), ps_b = to_prec(psi);

    QT_HIP(hipSetDevice(ctx->device));
    qt_mc_plan *P = new qt_mc_plan();
    P->ctx = ctx;
    P->prec = o.precision;
    McParams &p = P->p;
    p.d = d;
    p.W = W;
    p.nc = pr->n_c;
    p.ne = pr->n_e;
    p.nt = pr->n_t;
    int rows = 1;
    while (rows * MC_THREADS < d) rows *= 2;
    p.rows = rows;
    p.use_h0 = o.h0 > 0 ? 1 : 0;
    p.maxj = maxj;
    p.atol = o.abstol;
    p.rtol = o.reltol;
    p.h0 = o.h0;
    p.max_steps = o.max_steps;
    p.seed = pr->seed;
    p.ntraj = pr->ntraj;
    const int64_t nj = pr->ntraj;
    Arena &a = P->arena;
    const size_t o_ec = a.reserve(ell_col.size() * 4), o_ev = a.reserve(ev_b.size()),
                 o_cp = a.reserve(cptr.size() * 4), o_cc = a.reserve(std::max<size_t>(1, ccol.size()) * 4),
                 o_cv = a.reserve(std::max<size_t>(1, cv_b.size())), o_ep = a.reserve(eptr.size() * 4),
                 o_ecol = a.reserve(std::max<size_t>(1, ecol.size()) * 4),
                 o_eval = a.reserve(std::max<size_t>(1, eval.size()) * 16), o_ps = a.reserve(ps_b.size()),
                 o_tl = a.reserve((size_t)pr->n_t * 8),
                 o_tr = a.reserve(std::max<size_t>(1, (size_t)nj * pr->n_e * pr->n_t) * 16),
                 o_nj = a.reserve((size_t)nj * 8), o_jt = a.reserve(std::max<size_t>(1, (size_t)nj * maxj) * 8),
                 o_jc = a.reserve(std::max<size_t>(1, (size_t)nj * maxj) * 4), o_st = a.reserve((size_t)nj * 4),
                 o_nr = a.reserve((size_t)nj * 8), o_na = a.reserve((size_t)nj * 8), o_nx = a.reserve((size_t)nj * 8),
                 o_q = a.reserve(64), o_cf = a.reserve(sizeof(CoefDev) * cdev.size()),
                 o_tab = a.reserve(std::max<size_t>(16, tab_bytes)), o_cw = a.reserve(cweight.size() * 4);
    P->o_mean = a.reserve(std::max<size_t>(1, (size_t)pr->n_e * pr->n_t) * 16);
    P->o_se = a.reserve(std::max<size_t>(1, (size_t)pr->n_e * pr->n_t) * 8);
    P->o_params = a.reserve(sizeof(McParams));
    if (query) {
        *query = a.size;
        delete P;
        return QT_OK;
    }
    if ((st = a.place(ws, ws_bytes, "qt_mc_plan_create_ws"))) {
        delete P;
        return st;
    }
    p.ell_col = (const int32_t *)a.at(o_ec);
    p.ell_val = a.at(o_ev);
    p.cptr = (const int32_t *)a.at(o_cp);
    p.ccol = (const int32_t *)a.at(o_cc);
    p.cval = a.at(o_cv);
    p.eptr = (const int32_t *)a.at(o_ep);
    p.ecol = (const int32_t *)a.at(o_ecol);
    p.eval = (const double2 *)a.at(o_eval);
    p.psi0 = a.at(o_ps);
    p.tlist = (const double *)a.at(o_tl);
    p.expect_tr = (double2 *)a.at(o_tr);
    p.njumps = (int64_t *)a.at(o_nj);
    p.jtimes = (double *)a.at(o_jt);
    p.jchan = (int32_t *)a.at(o_jc);
    p.status = (int32_t *)a.at(o_st);
    p.nrhs = (int64_t *)a.at(o_nr);
    p.naccept = (int64_t *)a.at(o_na);
    p.nreject = (int64_t *)a.at(o_nx);
    p.queue = (unsigned long long *)a.at(o_q);
    p.nterms = nterms;
    p.pad_td = 0;
    p.coefs = (const CoefDev *)a.at(o_cf);
    p.cweight = (const int32_t *)a.at(o_cw);
    P->td = nterms > 0;
    std::vector<char> tabs(std::max<size_t>(16, tab_bytes));
    {
        size_t off = 0;
        for (int t = 0; t < nterms; ++t)
            if (tsrc[t]->kind == QT_COEF_TABLE) {
                const size_t nb = (size_t)tsrc[t]->n_table * sizeof(double2);
                std::memcpy(tabs.data() + off, tsrc[t]->table, nb);
                cdev[t].table = (const double2 *)((char *)a.at(o_tab) + off);
                off += nb;
            }
    }
    hipStream_t s = ctx->stream;
    hipError_t e = hipSuccess;
    auto up = [&](size_t off, const void *src, size_t n) {
        if (e == hipSuccess && n) e = hipMemcpyAsync(a.at(off), src, n, hipMemcpyHostToDevice, s);
    };
    up(o_ec, ell_col.data(), ell_col.size() * 4);
    up(o_ev, ev_b.data(), ev_b.size());
    up(o_cp, cptr.data(), cptr.size() * 4);
    up(o_cc, ccol.data(), ccol.size() * 4);
    up(o_cv, cv_b.data(), cv_b.size());
    up(o_ep, eptr.data(), eptr.size() * 4);
    up(o_ecol, ecol.data(), ecol.size() * 4);
    up(o_eval, eval.data(), eval.size() * 16);
    up(o_ps, ps_b.data(), ps_b.size());
    up(o_tl, pr->tlist, (size_t)pr->n_t * 8);
    up(o_cf, cdev.data(), sizeof(CoefDev) * cdev.size());
    up(o_tab, tabs.data(), tab_bytes);
    up(o_cw, cweight.data(), cweight.size() * 4);
    up(P->o_params, &p, sizeof(McParams));
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        a.release();
        delete P;
        return set_error(QT_EDEVICE, std::string("mc plan upload: ") + hipGetErrorString(e));
    }
    P->grid = mc_grid(p, f64, P->td, ctx->device);
    ctx->refs++;
    *out = P;
    return QT_OK;
}

static qt_status mc_plan_run(qt_mc_plan *P)
{
    QT_HIP(hipSetDevice(P->ctx->device));
    hipStream_t s = P->ctx->stream;
    const bool f64 = P->prec == QT_F64;
    hipEvent_t e0, e1;
    QT_HIP(hipEventCreate(&e0));
    QT_HIP(hipEventCreate(&e1));
    QT_HIP(hipEventRecord(e0, s));
    mc_launch_queue_reset(P->p.queue, s);
    mc_launch(P->p, (const McParams *)P->arena.at(P->o_params), f64, P->td, P->grid, s);
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

static qt_status mc_plan_result(qt_mc_plan *P, double *mean_out, double *se_out, double *expect_tr, int64_t *njumps,
                                double *jump_times, int32_t *jump_channels, qt_stats *stats)
{
    QT_HIP(hipSetDevice(P->ctx->device));
    const McParams &p = P->p;
    const size_t m = (size_t)p.ne * p.nt, nj = (size_t)p.ntraj;
    if (mean_out && m) QT_HIP(hipMemcpy(mean_out, P->arena.at(P->o_mean), m * 16, hipMemcpyDeviceToHost));
    if (se_out && m) QT_HIP(hipMemcpy(se_out, P->arena.at(P->o_se), m * 8, hipMemcpyDeviceToHost));
    if (expect_tr && m) QT_HIP(hipMemcpy(expect_tr, p.expect_tr, nj * m * 16, hipMemcpyDeviceToHost));
    std::vector<int64_t> jv(nj), rv(nj), av(nj), xv(nj);
    std::vector<int32_t> sv(nj);
    QT_HIP(hipMemcpy(jv.data(), p.njumps, nj * 8, hipMemcpyDeviceToHost));
    QT_HIP(hipMemcpy(rv.data(), p.nrhs, nj * 8, hipMemcpyDeviceToHost));
    QT_HIP(hipMemcpy(av.data(), p.naccept, nj * 8, hipMemcpyDeviceToHost));
    QT_HIP(hipMemcpy(xv.data(), p.nreject, nj * 8, hipMemcpyDeviceToHost));
    QT_HIP(hipMemcpy(sv.data(), p.status, nj * 4, hipMemcpyDeviceToHost));
    if (njumps) std::memcpy(njumps, jv.data(), nj * 8);
    if (p.maxj > 0) {
        if (jump_times) QT_HIP(hipMemcpy(jump_times, p.jtimes, nj * p.maxj * 8, hipMemcpyDeviceToHost));
        if (jump_channels) QT_HIP(hipMemcpy(jump_channels, p.jchan, nj * p.maxj * 4, hipMemcpyDeviceToHost));
    }
    qt_stats s;
    std::memset(&s, 0, sizeof(s));
    int32_t worst = QT_OK;
    for (size_t j = 0; j < nj; ++j) {
        s.n_jumps += jv[j];
        s.n_rhs += rv[j];
        s.n_accept += av[j];
        s.n_reject += xv[j];
        const int32_t code = sv[j] == ST_DONE ? QT_OK : sv[j];
        if (code != QT_OK && worst == QT_OK) worst = code;
    }
    s.status = worst;
    s.device_ms = P->last_ms;
    if (stats) *stats = s;
    if (worst != QT_OK) return set_error(worst, "a trajectory stopped with status " + std::to_string(worst));
    return QT_OK;
}

}  // namespace qt

using namespace qt;

extern "C" {

qt_status qt_mc_plan_create(qt_ctx *ctx, const qt_mc_problem *prob, const qt_opts *opts, int32_t max_jump_record,
                            qt_mc_plan **out)
{
    return mc_plan_create(ctx, prob, nullptr, opts, max_jump_record, out);
}

qt_status qt_mc_plan_create_td(qt_ctx *ctx, const qt_mc_problem *prob, const qt_td_terms *td, const qt_opts *opts,
                               int32_t max_jump_record, qt_mc_plan **out)
{
    return mc_plan_create(ctx, prob, td, opts, max_jump_record, out);
}

qt_status qt_mc_plan_workspace(qt_ctx *ctx, const qt_mc_problem *prob, const qt_opts *opts, int32_t max_jump_record,
                               size_t *bytes)
{
    if (!bytes) return set_error(QT_EINVAL, "qt_mc_plan_workspace: null bytes");
    return mc_plan_create(ctx, prob, nullptr, opts, max_jump_record, nullptr, nullptr, 0, bytes);
}

qt_status qt_mc_plan_create_ws(qt_ctx *ctx, const qt_mc_problem *prob, const qt_opts *opts, int32_t max_jump_record,
                               void *dev_ws, size_t ws_bytes, qt_mc_plan **out)
{
    if (!dev_ws) return set_error(QT_EINVAL, "qt_mc_plan_create_ws: null workspace");
    return mc_plan_create(ctx, prob, nullptr, opts, max_jump_record, out, dev_ws, ws_bytes, nullptr);
}

qt_status qt_mcsolve_ws(qt_ctx *ctx, const qt_mc_problem *prob, const qt_opts *opts, void *dev_ws, size_t ws_bytes,
                        double *mean_out, double *se_out, double *expect_tr, int64_t *njumps, int32_t max_jump_record,
                        double *jump_times, int32_t *jump_channels, qt_stats *stats)
{
    qt_mc_plan *P = nullptr;
    qt_status st = qt_mc_plan_create_ws(ctx, prob, opts, max_jump_record, dev_ws, ws_bytes, &P);
    if (st) {
        if (stats) stats->status = st;
        return st;
    }
    st = qt_mc_plan_run(P);
    if (!st) st = qt_mc_plan_result(P, mean_out, se_out, expect_tr, njumps, jump_times, jump_channels, stats);
    qt_mc_plan_destroy(P);
    return st;
}

qt_status qt_mc_plan_run(qt_mc_plan *plan)
{
    if (!plan) return set_error(QT_EINVAL, "null plan");
    return mc_plan_run(plan);
}

qt_status qt_mc_plan_result(qt_mc_plan *plan, double *mean_out, double *se_out, double *expect_tr, int64_t *njumps,
                            double *jump_times, int32_t *jump_channels, qt_stats *stats)
{
    if (!plan) return set_error(QT_EINVAL, "null plan");
    return mc_plan_result(plan, mean_out, se_out, expect_tr, njumps, jump_times, jump_channels, stats);
}

qt_status qt_mc_plan_destroy(qt_mc_plan *plan)
{
    if (!plan) return QT_OK;
    (void)hipSetDevice(plan->ctx->device);
    plan->arena.release();
    plan->ctx->refs--;
    delete plan;
    return QT_OK;
}

qt_status qt_mcsolve_td(qt_ctx *ctx, const qt_mc_problem *prob, const qt_td_terms *td, const qt_opts *opts,
                        double *mean_out, double *se_out, double *expect_tr, int64_t *njumps, int32_t max_jump_record,
                        double *jump_times, int32_t *jump_channels, qt_stats *stats)
{
    qt_mc_plan *P = nullptr;
    qt_status st = qt_mc_plan_create_td(ctx, prob, td, opts, max_jump_record, &P);
    if (st) {
        if (stats) stats->status = st;
        return st;
    }
    st = qt_mc_plan_run(P);
    if (!st) st = qt_mc_plan_result(P, mean_out, se_out, expect_tr, njumps, jump_times, jump_channels, stats);
    qt_mc_plan_destroy(P);
    return st;
}

qt_status qt_mcsolve(qt_ctx *ctx, const qt_mc_problem *prob, const qt_opts *opts, double *mean_out, double *se_out,
                     double *expect_tr, int64_t *njumps, int32_t max_jump_record, double *jump_times,
                     int32_t *jump_channels, qt_stats *stats)
{
    return qt_mcsolve_td(ctx, prob, nullptr, opts, mean_out, se_out, expect_tr, njumps, max_jump_record, jump_times,
                         jump_channels, stats);
}

qt_status qt_sesolve(qt_ctx *ctx, const qt_csr *H, const double *psi0, int32_t n_t, const double *tlist, int32_t n_e,
                     const qt_csr *e_ops, const qt_opts *opts, double *expect_out, qt_stats *stats)
{
    // the Schrodinger equation is the no-collapse case of the trajectory integrator: H_eff = H,
    // the norm never falls below a threshold, one trajectory is the solution
    qt_mc_problem p;
    p.H = H;
    p.n_c = 0;
    p.c_ops = nullptr;
    p.psi0 = psi0;
    p.n_t = n_t;
    p.tlist = tlist;
    p.n_e = n_e;
    p.e_ops = e_ops;
    p.ntraj = 1;
    p.seed = 0;
    return qt_mcsolve(ctx, &p, opts, expect_out, nullptr, nullptr, nullptr, 0, nullptr, nullptr, stats);
}

qt_status qt_sesolve_td(qt_ctx *ctx, const qt_csr *H, const qt_td_terms *td, const double *psi0, int32_t n_t,
                        const double *tlist, int32_t n_e, const qt_csr *e_ops, const qt_opts *opts, double *expect_out,
                        qt_stats *stats)
{
    qt_mc_problem p;
    p.H = H;
    p.n_c = 0;
    p.c_ops = nullptr;
    p.psi0 = psi0;
    p.n_t = n_t;
    p.tlist = tlist;
    p.n_e = n_e;
    p.e_ops = e_ops;
    p.ntraj = 1;
    p.seed = 0;
    qt_td_terms h;
    h.n_h = td ? td->n_h : 0;
    h.h_terms = td ? td->h_terms : nullptr;
    h.h_coefs = td ? td->h_coefs : nullptr;
    h.c_coefs = nullptr;
    return qt_mcsolve_td(ctx, &p, &h, opts, expect_out, nullptr, nullptr, nullptr, 0, nullptr, nullptr, stats);
}

}  // extern "C"

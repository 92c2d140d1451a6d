// qtamd_me.cpp -- master-equation plans: device-resident batched mesolve (Sec. 3.2 of
// arXiv:2504.21440) over CSR-form and dense-form Liouvillians.
//
// A plan uploads every input once (initial states, save times, e_ops) and lays out the solver
// state of all its problems in one device arena.  Running it resets the per-problem control
// records on the device, evaluates the starting step, then replays a captured graph of
// `steps_per_launch` Runge-Kutta steps until every problem reports done; each problem keeps its
// own step size and accept/reject history on the device, so the host only polls status words.
// The CSR tile shape comes from the autotuner's table (or is measured on the plan when asked).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "qt_csr.h"
#include "qt_dense.h"
#include "qt_host.h"
#include "qt_tune.h"
#include "qt_coef.h"

namespace qt {

struct MeProb {
    const qt_liouv *L = nullptr;
    int32_t d = 0, nt = 0, ne = 0;
    bool dense = false;
    int32_t slot = -1;  // index inside its group
    size_t o_rho0 = 0, o_tlist = 0, o_eptr = 0, o_ecol = 0, o_eval = 0, o_evidx = 0, o_expect = 0;
    size_t o_vec = 0;  // state vectors
    size_t o_part = 0;
    size_t o_cstage = 0;  // coefficient rows (plans with a time-dependent problem)
    std::vector<char> rho0;  // host copy in state precision
    std::vector<double> tlist;
    std::vector<int32_t> eptr, ecol, evidx;
    std::vector<double2> eval;
};

}  // namespace qt

struct qt_me_plan {
    qt::Ctx *ctx = nullptr;
    qt_opts opts{};
    int32_t prec = QT_F64;
    std::vector<qt::MeProb> probs;
    qt::Arena arena;
    // CSR group
    int32_t ncsr = 0, nblk = 0;
    bool td = false;  // some CSR problem is time dependent: every CSR launch weights its terms
    qt::CsrShape shape;
    std::string tune_key;
    std::vector<qt::CsrInst> h_ci;  // host copy of the descriptors (block ranges change with the shape)
    std::vector<double> csr_tend;   // last save time of each CSR problem
    size_t o_cinst = 0, o_cctl = 0, o_bi = 0, o_br = 0, o_ilist = 0;
    qt::CsrCtl *h_cctl = nullptr;  // pinned
    int32_t graph_steps = 16;
    // Lanes: the CSR problems run as one or more groups, each with its own segment of the block
    // table and of the control list, its own captured graph and its own stream.  A run starts with
    // one lane holding every problem; finished problems are dropped and far-behind ones split off
    // into a lane of their own as the run goes (see me_plan_run).
    struct Lane {
        std::vector<int32_t> members;  // CSR problem slots
        int32_t boff = 0, nblk = 0;    // block-table segment
        int32_t ioff = 0;              // control-list segment
        bool listed = false;           // false: the control launch visits problems 0 .. ncsr-1
        hipStream_t stream = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t gexec = nullptr;
        int replays = 1;               // graph replays per round
        bool done = false;
        hipEvent_t e0 = nullptr, e1 = nullptr;
    };
    std::vector<Lane> lanes;
    std::vector<hipStream_t> lane_streams;  // created on demand, destroyed with the plan
    bool split = false;                     // lanes differ from the single full lane
    // dense group
    int32_t ndense = 0;
    size_t o_dinst = 0, o_dctl = 0, o_dorder = 0;
    qt::DenseCtl *h_dctl = nullptr;  // pinned
    struct Bucket {
        int32_t np, start, count;
    };
    std::vector<Bucket> buckets;  // dense problems grouped by padded size, largest first
    double last_ms = 0.0;
    bool counted = false;  // holds a reference on ctx
};

namespace qt {

// Lanes split off a plan's CSR problems, each on its own stream: QTAMD_MAX_LANES - 1 of them (at
// most 7).  The default is no splitting: on the 512-cavity sweep a split at the first compaction
// ran 15% slower than one compacted lane, because the remaining-step estimate (t_end - t) / h
// misjudged which problems would finish last and the concurrent lanes slowed each other down.
// Finished problems are dropped either way.  QTAMD_TRACE_LANES prints each round's lanes to stderr.
static int max_extra_lanes()
{
    static const int v = [] {
        const char *e = std::getenv("QTAMD_MAX_LANES");
        const int n = e ? std::atoi(e) : 1;
        return std::max(0, std::min(8, n) - 1);
    }();
    return v;
}
static bool trace_lanes()
{
    static const bool v = std::getenv("QTAMD_TRACE_LANES") != nullptr;
    return v;
}

static size_t state_es(int32_t prec) { return prec == QT_F64 ? sizeof(double2) : sizeof(float2); }

static qt_status prep_problem(const qt_me_problem &p, int32_t prec, MeProb *m)
{
    if (!p.L) return set_error(QT_EINVAL, "problem without Liouvillian");
    if (p.L->precision != prec)
        return set_error(QT_EINVAL, "Liouvillian precision differs from opts.precision");
    const int32_t d = p.L->d;
    if (p.n_t < 1 || !p.tlist) return set_error(QT_EINVAL, "tlist must hold at least one time");
    for (int32_t i = 0; i < p.n_t; ++i)
        if (!std::isfinite(p.tlist[i]) || (i > 0 && !(p.tlist[i] > p.tlist[i - 1])))
            return set_error(QT_EINVAL, "tlist must be finite and strictly increasing");
    if (!p.rho0) return set_error(QT_EINVAL, "rho0 is null");
    if (p.n_e < 0 || (p.n_e > 0 && !p.e_ops)) return set_error(QT_EINVAL, "bad e_ops");
    m->L = p.L;
    m->d = d;
    m->nt = p.n_t;
    m->ne = p.n_e;
    m->dense = p.L->form == QT_FORM_DENSE;
    m->tlist.assign(p.tlist, p.tlist + p.n_t);
    // initial state (row-major d x d), converted to the state precision
    const size_t n = (size_t)d * d;
    std::vector<double> r(2 * n);
    if (p.is_ket) {
        for (int32_t i = 0; i < d; ++i)
            for (int32_t j = 0; j < d; ++j) {
                const cd a(p.rho0[2 * i], p.rho0[2 * i + 1]), b(p.rho0[2 * j], p.rho0[2 * j + 1]);
                const cd v = a * std::conj(b);
                r[2 * ((size_t)i * d + j)] = v.real();
                r[2 * ((size_t)i * d + j) + 1] = v.imag();
            }
    } else {
        std::memcpy(r.data(), p.rho0, sizeof(double) * 2 * n);
    }
    double amax = 0.0, asym = 0.0;
    for (size_t i = 0; i < 2 * n; ++i) {
        if (!std::isfinite(r[i])) return set_error(QT_EINVAL, "rho0 has non-finite entries");
        amax = std::max(amax, std::fabs(r[i]));
    }
    if (m->dense) {
        // the operator form evaluates L on Hermitian matrices only
        for (int32_t i = 0; i < d; ++i)
            for (int32_t j = 0; j < d; ++j) {
                const size_t a = 2 * ((size_t)i * d + j), b = 2 * ((size_t)j * d + i);
                asym = std::max(asym, std::fabs(r[a] - r[b]) + std::fabs(r[a + 1] + r[b + 1]));
            }
        if (asym > 1e-12 * std::max(1.0, amax))
            return set_error(QT_EINVAL, "the dense form needs a Hermitian rho0 (use the CSR form otherwise)");
    }
    if (prec == QT_F64) {
        m->rho0.resize(n * 16);
        std::memcpy(m->rho0.data(), r.data(), n * 16);
    } else {
        m->rho0.resize(n * 8);
        float *f = (float *)m->rho0.data();
        for (size_t i = 0; i < 2 * n; ++i) f[i] = (float)r[i];
    }
    // e_ops as concatenated int32 CSR (instance-local offsets)
    m->eptr.assign((size_t)p.n_e * (d + 1), 0);
    m->ecol.clear();
    m->eval.clear();
    for (int32_t k = 0; k < p.n_e; ++k) {
        HCsr o;
        qt_status st = csr_from_abi(&p.e_ops[k], d, &o, "e_ops");
        if (st) return st;
        const int32_t base = (int32_t)m->ecol.size();
        for (int32_t i = 0; i <= d; ++i) m->eptr[(size_t)k * (d + 1) + i] = base + (int32_t)o.ptr[i];
        for (int64_t q = 0; q < o.nnz(); ++q) {
            m->ecol.push_back(o.idx[q]);
            m->eval.push_back(make_double2(o.val[q].real(), o.val[q].imag()));
        }
    }
    m->evidx = expect_vec_index(m->eptr, m->ecol, d, p.n_e);
    return QT_OK;
}

static qt_status upload(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    if (!bytes) return QT_OK;
    QT_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    return QT_OK;
}

static void drop_graph(qt_me_plan::Lane &l)
{
    if (l.gexec) (void)hipGraphExecDestroy(l.gexec);
    if (l.graph) (void)hipGraphDestroy(l.graph);
    l.gexec = nullptr;
    l.graph = nullptr;
}

// Write the block table and control list of every live lane, back to back, and upload them.  A
// lane's blocks are those of its members at the plan's shape.  Graphs are recaptured on next use.
static qt_status layout_lanes(qt_me_plan *P)
{
    const int rpb = csr_rows_per_block(P->shape.lpr, P->shape.rg);
    std::vector<int32_t> bi, br, il;
    for (auto &l : P->lanes) {
        drop_graph(l);
        if (l.done) continue;
        l.boff = (int32_t)bi.size();
        l.ioff = (int32_t)il.size();
        for (int32_t i : l.members) {
            CsrInst &c = P->h_ci[i];
            c.block0 = (int32_t)bi.size();
            for (int32_t b = 0; b < c.nblocks; ++b) {
                bi.push_back(i);
                br.push_back(b * rpb);
            }
            il.push_back(i);
        }
        l.nblk = (int32_t)bi.size() - l.boff;
    }
    hipStream_t s = P->ctx->stream;
    qt_status st;
    if ((st = upload(P->arena.at(P->o_cinst), P->h_ci.data(), sizeof(CsrInst) * P->ncsr, s))) return st;
    if ((st = upload(P->arena.at(P->o_bi), bi.data(), 4 * bi.size(), s))) return st;
    if ((st = upload(P->arena.at(P->o_br), br.data(), 4 * br.size(), s))) return st;
    if ((st = upload(P->arena.at(P->o_ilist), il.data(), 4 * il.size(), s))) return st;
    QT_HIP(hipStreamSynchronize(s));
    P->nblk = (int32_t)bi.size();
    return QT_OK;
}

// One lane with every CSR problem, on the context's stream, control launch over all problems.
static qt_status reset_lanes(qt_me_plan *P)
{
    for (auto &l : P->lanes) drop_graph(l);
    P->lanes.assign(1, qt_me_plan::Lane{});
    auto &l = P->lanes[0];
    for (int32_t i = 0; i < P->ncsr; ++i) l.members.push_back(i);
    l.stream = P->ctx->stream;
    P->split = false;
    return layout_lanes(P);
}

// Lay the CSR problems out over the launch grid for a tile shape and upload the block tables.
static qt_status apply_shape(qt_me_plan *P, CsrShape sh)
{
    if (!csr_shape_supported(sh.lpr, sh.rg, sh.keep)) return set_error(QT_EINVAL, "unsupported CSR tile shape");
    const int rpb = csr_rows_per_block(sh.lpr, sh.rg);
    for (int32_t i = 0; i < P->ncsr; ++i) P->h_ci[i].nblocks = (P->h_ci[i].n + rpb - 1) / rpb;
    P->shape = sh;
    return reset_lanes(P);
}

// Back to the single full lane if a run left the problems split or dropped; a lane that only
// finished keeps its layout and graph.
static qt_status restore_full(qt_me_plan *P)
{
    if (P->split) return reset_lanes(P);
    for (auto &l : P->lanes) l.done = false;
    return QT_OK;
}

qt_status me_plan_autotune(qt_me_plan *P, int32_t reps);

// ws: the caller's device workspace (null: the plan allocates its arena); query: only report the
// workspace bytes the problems need and create nothing.
qt_status me_plan_create(Ctx *ctx, int32_t n, const qt_me_problem *probs, const qt_opts *opts_in, qt_me_plan **out,
                         double steady_tol, void *ws = nullptr, size_t ws_bytes = 0, size_t *query = nullptr)
{
    if (!ctx || n <= 0 || !probs || (!out && !query)) return set_error(QT_EINVAL, "qt_me_plan_create: bad arguments");
    if (!(steady_tol >= 0.0) || !std::isfinite(steady_tol)) return set_error(QT_EINVAL, "steady-state tolerance");
    qt_opts opts;
    if (opts_in) opts = *opts_in;
    else qt_opts_default(&opts);
    if (!(opts.abstol > 0) || !(opts.reltol >= 0) || opts.max_steps <= 0)
        return set_error(QT_EINVAL, "opts: abstol > 0, reltol >= 0 and max_steps > 0 required");
    if (opts.precision != QT_F64 && opts.precision != QT_MIXED) return set_error(QT_EINVAL, "opts: bad precision");
    QT_HIP(hipSetDevice(ctx->device));
    qt_me_plan *P = new qt_me_plan();
    P->ctx = ctx;
    P->opts = opts;
    P->prec = opts.precision;
    P->probs.resize(n);
    for (int32_t i = 0; i < n; ++i) {
        qt_status st = prep_problem(probs[i], P->prec, &P->probs[i]);
        if (st) {
            delete P;
            return st;
        }
    }
    const size_t es = state_es(P->prec);
    // ---- layout (block tables sized for the smallest tile, so any shape fits) ----
    Arena &A = P->arena;
    int64_t nnz_tot = 0, rows_tot = 0, max_blocks = 0;
    for (auto &m : P->probs)
        if (!m.dense) {
            m.slot = P->ncsr++;
            nnz_tot += m.L->nnz;
            rows_tot += (int64_t)m.d * m.d;
            P->td = P->td || m.L->nterms > 0;
        } else {
            m.slot = P->ndense++;
        }
    if (P->td)
        for (auto &m : P->probs)
            if (!m.dense && (int64_t)m.d * m.d > (int64_t)TD_COL_MASK) {
                delete P;
                return set_error(QT_EINVAL, "a plan with a time-dependent problem holds CSR problems with d*d < 2^26");
            }
    for (auto &m : P->probs) {
        const size_t nvec = (size_t)m.d * m.d;
        m.o_rho0 = A.reserve(nvec * es);
        m.o_tlist = A.reserve(m.tlist.size() * 8);
        m.o_eptr = A.reserve(std::max<size_t>(1, m.eptr.size()) * 4);
        m.o_ecol = A.reserve(std::max<size_t>(1, m.ecol.size()) * 4);
        m.o_eval = A.reserve(std::max<size_t>(1, m.eval.size()) * 16);
        m.o_evidx = A.reserve(std::max<size_t>(1, m.evidx.size()) * 4);
        m.o_expect = A.reserve(std::max<size_t>(1, (size_t)m.ne * m.nt) * 16);
        if (!m.dense) {
            const int64_t nb = ((int64_t)nvec + CSR_MIN_ROWS_PER_BLOCK - 1) / CSR_MIN_ROWS_PER_BLOCK;
            max_blocks += nb;
            m.o_vec = A.reserve(11 * nvec * es);  // Y[2], K[2], k2..k6, ys[2]
            m.o_part = A.reserve((size_t)nb * 16);
            if (P->td) m.o_cstage = A.reserve((size_t)TD_SLOTS * (m.L->nterms + 1) * es);
        } else {
            const size_t np = (size_t)dense_np(m.d);
            m.o_vec = A.reserve(dense_state_vectors() * np * np * es);
        }
    }
    if (P->ncsr) {
        P->o_cinst = A.reserve(sizeof(CsrInst) * P->ncsr);
        P->o_cctl = A.reserve(sizeof(CsrCtl) * (P->ncsr + 1));  // + the second record of a folded control
        P->o_bi = A.reserve(sizeof(int32_t) * max_blocks);
        P->o_br = A.reserve(sizeof(int32_t) * max_blocks);
        P->o_ilist = A.reserve(sizeof(int32_t) * P->ncsr);
    }
    if (P->ndense) {
        P->o_dinst = A.reserve(sizeof(DenseInst) * P->ndense);
        P->o_dctl = A.reserve(sizeof(DenseCtl) * P->ndense);
        P->o_dorder = A.reserve(sizeof(int32_t) * P->ndense);
    }
    if (query) {
        *query = A.size;
        delete P;
        return QT_OK;
    }
    qt_status st = A.place(ws, ws_bytes, "qt_me_plan_create_ws");
    if (st) {
        delete P;
        return st;
    }
    hipStream_t s = ctx->stream;
    // ---- uploads ----
    P->h_ci.resize(P->ncsr);
    P->csr_tend.resize(P->ncsr);
    for (auto &m : P->probs)
        if (!m.dense) P->csr_tend[m.slot] = m.tlist.back();
    std::vector<DenseInst> di(P->ndense);
    for (auto &m : P->probs) {
        if ((st = upload(A.at(m.o_rho0), m.rho0.data(), m.rho0.size(), s))) break;
        if ((st = upload(A.at(m.o_tlist), m.tlist.data(), m.tlist.size() * 8, s))) break;
        if ((st = upload(A.at(m.o_eptr), m.eptr.data(), m.eptr.size() * 4, s))) break;
        if ((st = upload(A.at(m.o_ecol), m.ecol.data(), m.ecol.size() * 4, s))) break;
        if ((st = upload(A.at(m.o_eval), m.eval.data(), m.eval.size() * 16, s))) break;
        if ((st = upload(A.at(m.o_evidx), m.evidx.data(), m.evidx.size() * 4, s))) break;
        const size_t nvec = (size_t)m.d * m.d;
        if (!m.dense) {
            CsrInst &c = P->h_ci[m.slot];
            std::memset(&c, 0, sizeof(c));
            c.n = (int32_t)nvec;
            c.d = m.d;
            c.nt = m.nt;
            c.ne = m.ne;
            c.renorm = P->prec == QT_MIXED ? 1 : 0;
            c.use_h0 = opts.h0 > 0 ? 1 : 0;
            c.atol = opts.abstol;
            c.rtol = opts.reltol;
            c.h0 = opts.h0;
            c.max_steps = opts.max_steps;
            c.rowptr = m.L->rowptr;
            c.col = m.L->col;
            c.val = m.L->val;
            c.rho0 = A.at(m.o_rho0);
            char *v = (char *)A.at(m.o_vec);
            c.Y[0] = v + 0 * nvec * es;
            c.Y[1] = v + 1 * nvec * es;
            c.K[0] = v + 2 * nvec * es;
            c.K[1] = v + 3 * nvec * es;
            for (int k = 0; k < 5; ++k) c.ks[k] = v + (4 + k) * nvec * es;
            c.ys[0] = v + 9 * nvec * es;
            c.ys[1] = v + 10 * nvec * es;
            c.tlist = (const double *)A.at(m.o_tlist);
            c.eptr = (const int32_t *)A.at(m.o_eptr);
            c.ecol = (const int32_t *)A.at(m.o_ecol);
            c.eval = (const double2 *)A.at(m.o_eval);
            c.evidx = (const int32_t *)A.at(m.o_evidx);
            c.expect = (double2 *)A.at(m.o_expect);
            c.partials = (double *)A.at(m.o_part);
            csr_set_expect_ranges(c, m.eptr.data(), m.ne, m.d);
            c.steady_tol2 = steady_tol * steady_tol;
            if (P->td) {
                // every CSR problem of the plan takes the weighted kernels; a constant one has only
                // the column of ones
                c.nterms = m.L->nterms;
                c.coefs = (const CoefDev *)m.L->coefs;
                c.cstage = A.at(m.o_cstage);
            }
        } else {
            DenseInst &g = di[m.slot];
            dense_fill_inst(&g, m.d, m.L->nc, m.L->dense_creal, m.nt, m.ne, m.L->dense, A.at(m.o_rho0),
                            A.at(m.o_vec), (const double *)A.at(m.o_tlist), (const int32_t *)A.at(m.o_eptr),
                            (const int32_t *)A.at(m.o_ecol), (const double2 *)A.at(m.o_eval),
                            (double2 *)A.at(m.o_expect), opts, P->prec);
            g.steady_tol2 = steady_tol * steady_tol;
        }
    }
    if (!st && P->ncsr) {
        const double mean_row = rows_tot ? (double)nnz_tot / rows_tot : 8.0;
        P->tune_key = csr_tune_key(P->prec, rows_tot, mean_row);
        CsrShape sh;
        if (!tune_lookup_csr(P->tune_key, &sh)) sh = csr_default_shape(rows_tot, mean_row);
        if (P->ncsr > 1) sh.xcd = 0;  // see csr_candidates: a single-problem option
        st = apply_shape(P, sh);
        if (!st) {
            hipError_t e = hipHostMalloc((void **)&P->h_cctl, sizeof(CsrCtl) * P->ncsr, hipHostMallocDefault);
            if (e) st = set_error(QT_ENOMEM, "pinned host buffer");
        }
    }
    if (!st && P->ndense) {
        // largest problems first: the hardware dispatches workgroups in this order
        std::vector<int32_t> order(P->ndense);
        for (int32_t i = 0; i < P->ndense; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return di[a].d > di[b].d; });
        for (int32_t k = 0; k < P->ndense; ++k) {
            const int32_t np = di[order[k]].np;
            if (np > (P->prec == QT_F64 ? DENSE_MAX_NP_F64 : DENSE_MAX_NP_F32)) {
                st = set_error(QT_EINVAL, "dense form: dimension too large for this precision");
                break;
            }
            if (P->buckets.empty() || P->buckets.back().np != np) P->buckets.push_back({np, k, 0});
            P->buckets.back().count++;
        }
        if (!st && (st = upload(A.at(P->o_dinst), di.data(), sizeof(DenseInst) * P->ndense, s)) == QT_OK)
            st = upload(A.at(P->o_dorder), order.data(), 4 * order.size(), s);
        if (!st) {
            hipError_t e = hipHostMalloc((void **)&P->h_dctl, sizeof(DenseCtl) * P->ndense, hipHostMallocDefault);
            if (e) st = set_error(QT_ENOMEM, "pinned host buffer");
        }
    }
    if (!st) {
        hipError_t e = hipStreamSynchronize(s);
        if (e) st = set_error(QT_EDEVICE, std::string("plan upload: ") + hipGetErrorString(e));
    }
    P->graph_steps = opts.steps_per_launch > 0 ? opts.steps_per_launch : 16;
    ctx->refs++;
    P->counted = true;
    if (!st && opts.autotune) {
        bool known = true;
        CsrShape tmp;
        if (P->ncsr && !tune_lookup_csr(P->tune_key, &tmp)) known = false;
        for (auto &bk : P->buckets) {
            int w;
            if (!tune_lookup_dense(dense_tune_key(P->prec, bk.np), &w)) known = false;
        }
        if (!known) st = me_plan_autotune(P, 20);
    }
    if (st) {
        qt_me_plan_destroy(P);
        return st;
    }
    *out = P;
    return QT_OK;
}

// Launch configuration of lane `k` of the plan's CSR problems at the current shape.
// Whether a step's control folds into the next step's stage-2 launch at matrix load kind keep: one
// problem stored in runs of 4 entries (keep 2) with no steady-state test, over an even number of
// steps per graph (the double-buffered record ends where it began).
static bool folds_control(const qt_me_plan *P, int keep)
{
    return P->ncsr == 1 && keep == 2 && P->h_ci[0].steady_tol2 <= 0.0 && P->graph_steps % 2 == 0;
}

static CsrLaunch csr_args(const qt_me_plan *P, int k = 0)
{
    const auto &l = P->lanes[k];
    CsrLaunch L;
    L.f64 = P->prec == QT_F64;
    L.lpr = P->shape.lpr;
    L.rg = P->shape.rg;
    L.xcd = P->shape.xcd;
    L.keep = P->shape.keep;
    L.nblk = l.nblk;
    L.ninst = l.listed ? (int)l.members.size() : P->ncsr;
    L.ilist = l.listed ? (const int32_t *)P->arena.at(P->o_ilist) + l.ioff : nullptr;
    L.insts = (const CsrInst *)P->arena.at(P->o_cinst);
    L.ctls = (CsrCtl *)P->arena.at(P->o_cctl);
    L.bi = (const int32_t *)P->arena.at(P->o_bi) + l.boff;
    L.br = (const int32_t *)P->arena.at(P->o_br) + l.boff;
    L.one_host = P->ncsr == 1 ? &P->h_ci[0] : nullptr;
    L.td = P->td;
    L.fused = folds_control(P, P->shape.keep);
    return L;
}

static qt_status capture_graph(qt_me_plan *P, int k = 0)
{
    auto &l = P->lanes[k];
    if (l.gexec) return QT_OK;
    const CsrLaunch L = csr_args(P, k);
    QT_HIP(hipStreamBeginCapture(l.stream, hipStreamCaptureModeThreadLocal));
    for (int j = 0; j < P->graph_steps; ++j) csr_launch_step(L, l.stream, j);
    hipError_t e = hipStreamEndCapture(l.stream, &l.graph);
    if (e) return set_error(QT_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    QT_HIP(hipGraphInstantiate(&l.gexec, l.graph, nullptr, nullptr, 0));
    return QT_OK;
}

static void launch_dense_buckets(qt_me_plan *P, int max_steps_launch, hipStream_t single)
{
    const bool f64 = P->prec == QT_F64;
    for (size_t b = 0; b < P->buckets.size(); ++b) {
        const auto &bk = P->buckets[b];
        hipStream_t bs = single ? single : P->ctx->pool[b % Ctx::NPOOL];
        dense_launch_bucket(bk.np, f64, dense_choose_config(bk.np, P->prec), (const DenseInst *)P->arena.at(P->o_dinst),
                            (DenseCtl *)P->arena.at(P->o_dctl), (const int32_t *)P->arena.at(P->o_dorder) + bk.start,
                            bk.count, max_steps_launch, /*reset=*/1, bs);
    }
}

qt_status me_plan_run(qt_me_plan *P)
{
    Ctx *ctx = P->ctx;
    QT_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const bool f64 = P->prec == QT_F64;
    auto t0 = std::chrono::steady_clock::now();
    // dense buckets run on the auxiliary streams, overlapping each other and the CSR group
    hipEvent_t ev_start = nullptr;
    if (P->ndense) {
        QT_HIP(hipEventCreateWithFlags(&ev_start, hipEventDisableTiming));
        QT_HIP(hipEventRecord(ev_start, s));
        for (int b = 0; b < Ctx::NPOOL; ++b) QT_HIP(hipStreamWaitEvent(ctx->pool[b], ev_start, 0));
        launch_dense_buckets(P, -1, nullptr);
        QT_HIP(hipGetLastError());
    }
    qt_status st = QT_OK;
    if (P->ncsr) {
        if ((st = restore_full(P))) return st;
        const CsrLaunch L = csr_args(P, 0);
        auto *cc = L.ctls;
        csr_launch_reset(L.insts, L.ctls, P->ncsr, L.f64, s);
        csr_launch_init(0, L, s);
        csr_launch_init(1, L, s);
        QT_HIP(hipGetLastError());
        if ((st = capture_graph(P, 0))) return st;
        int64_t last_steps = -1;
        std::vector<double> rem(P->ncsr, 0.0);  // steps still needed, from the current step size
        for (;;) {
            // one round: every live lane replays its graph on its own stream
            for (auto &l : P->lanes) {
                if (l.done) continue;
                if (!l.e0) QT_HIP(hipEventCreate(&l.e0));
                if (!l.e1) QT_HIP(hipEventCreate(&l.e1));
                QT_HIP(hipEventRecord(l.e0, l.stream));
                for (int r = 0; r < l.replays; ++r) QT_HIP(hipGraphLaunch(l.gexec, l.stream));
                QT_HIP(hipEventRecord(l.e1, l.stream));
            }
            for (auto &l : P->lanes)
                if (!l.done) QT_HIP(hipStreamSynchronize(l.stream));
            QT_HIP(hipMemcpyAsync(P->h_cctl, cc, sizeof(CsrCtl) * P->ncsr, hipMemcpyDeviceToHost, s));
            QT_HIP(hipStreamSynchronize(s));
            if (trace_lanes()) {
                for (size_t k = 0; k < P->lanes.size(); ++k) {
                    const auto &l = P->lanes[k];
                    float ms = 0.f;
                    if (!l.done) (void)hipEventElapsedTime(&ms, l.e0, l.e1);
                    std::fprintf(stderr, "[lanes] lane %zu: %zu problems, %d blocks, %d replays, %.3f ms%s\n", k,
                                 l.members.size(), l.nblk, l.replays, ms, l.done ? " (done)" : "");
                }
            }
            int64_t steps = 0;
            for (int32_t i = 0; i < P->ncsr; ++i) steps += P->h_cctl[i].n_steps;
            if (steps == last_steps) return set_error(QT_EDEVICE, "CSR solver made no progress in a graph replay");
            last_steps = steps;
            for (int32_t i = 0; i < P->ncsr; ++i) {
                const CsrCtl &c = P->h_cctl[i];
                rem[i] = c.status == ST_RUNNING ? (P->csr_tend[i] - c.t) / (c.h > 0 ? c.h : 1e-6) : -1.0;
            }
            bool relayout = false, any = false;
            const size_t nl = P->lanes.size();
            for (size_t k = 0; k < nl; ++k) {
                auto &l = P->lanes[k];
                if (l.done) continue;
                std::vector<int32_t> live;
                int64_t live_blocks = 0;
                for (int32_t i : l.members)
                    if (rem[i] >= 0.0) {
                        live.push_back(i);
                        live_blocks += P->h_ci[i].nblocks;
                    }
                if (live.empty()) {
                    l.done = true;
                    relayout = true;
                    continue;
                }
                any = true;
                // Drop finished problems once they hold half of the lane's workgroups; at that point
                // problems far behind the others (4x the median remaining steps) move to a lane of
                // their own, so they no longer wait on the larger group's launches every step.
                if (P->ncsr > 1 && 2 * live_blocks <= l.nblk) {
                    std::vector<double> r;
                    for (int32_t i : live) r.push_back(rem[i]);
                    std::nth_element(r.begin(), r.begin() + r.size() / 2, r.end());
                    const double med = r[r.size() / 2];
                    std::vector<int32_t> slow, rest;
                    for (int32_t i : live) (rem[i] >= 4.0 * med ? slow : rest).push_back(i);
                    if (!slow.empty() && !rest.empty() && (int)P->lanes.size() < 1 + max_extra_lanes()) {
                        const size_t j = P->lanes.size() - 1;  // streams already made
                        if (j >= P->lane_streams.size()) {
                            hipStream_t ns;
                            QT_HIP(hipStreamCreateWithFlags(&ns, hipStreamNonBlocking));
                            P->lane_streams.push_back(ns);
                        }
                        qt_me_plan::Lane nlane;
                        nlane.members = slow;
                        nlane.listed = true;
                        nlane.stream = P->lane_streams[j];
                        P->lanes[k].members = rest;  // (reference l may move with the push_back)
                        P->lanes[k].listed = true;
                        P->lanes.push_back(nlane);
                    } else {
                        l.members = live;
                        l.listed = true;
                    }
                    relayout = true;
                }
            }
            if (!any) break;
            if (relayout) {
                P->split = true;
                if ((st = layout_lanes(P))) return st;
            }
            // replays for the next round: each lane at most what it still needs; the slowest lane
            // (by measured time per replay) up to 8, the others as many as fit in that round's time
            std::vector<double> want(P->lanes.size(), 1.0), per(P->lanes.size(), 0.0);
            double round_ms = 0.0;
            for (size_t k = 0; k < P->lanes.size(); ++k) {
                auto &l = P->lanes[k];
                if (l.done) continue;
                double need = 0.0;
                for (int32_t i : l.members) need = std::max(need, rem[i]);
                want[k] = std::max(1.0, std::floor(need / P->graph_steps));
                float ms = 0.f;
                if (l.e0 && l.e1 && hipEventElapsedTime(&ms, l.e0, l.e1) == hipSuccess && ms > 0.f)
                    per[k] = (double)ms / std::max(1, l.replays);
                if (per[k] > 0.0) round_ms = std::max(round_ms, std::min(8.0, want[k]) * per[k]);
            }
            for (size_t k = 0; k < P->lanes.size(); ++k) {
                auto &l = P->lanes[k];
                if (l.done) continue;
                double r = std::min(8.0, want[k]);
                if (per[k] > 0.0 && round_ms > 0.0) r = std::min({std::floor(round_ms / per[k]), want[k], 64.0});
                l.replays = (int)std::max(1.0, r);
                if ((st = capture_graph(P, (int)k))) return st;
            }
        }
    }
    if (P->ndense) {
        for (int b = 0; b < Ctx::NPOOL; ++b) QT_HIP(hipStreamSynchronize(ctx->pool[b]));
        QT_HIP(hipMemcpy(P->h_dctl, P->arena.at(P->o_dctl), sizeof(DenseCtl) * P->ndense, hipMemcpyDeviceToHost));
        (void)hipEventDestroy(ev_start);
    }
    P->last_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return QT_OK;
}

// Average milliseconds of one fused SpMV-stage launch over the CSR group (fresh starting state).
static qt_status time_stage(qt_me_plan *P, int32_t reps, double *ms)
{
    hipStream_t s = P->ctx->stream;
    qt_status st = restore_full(P);
    if (st) return st;
    const CsrLaunch L = csr_args(P);
    hipEvent_t e0, e1;
    QT_HIP(hipEventCreate(&e0));
    QT_HIP(hipEventCreate(&e1));
    csr_launch_reset(L.insts, L.ctls, P->ncsr, L.f64, s);
    csr_launch_init(0, L, s);
    csr_launch_init(1, L, s);
    csr_launch_stage3(L, s);  // warm
    QT_HIP(hipEventRecord(e0, s));
    for (int32_t k = 0; k < reps; ++k) csr_launch_stage3(L, s);
    QT_HIP(hipEventRecord(e1, s));
    QT_HIP(hipGetLastError());
    QT_HIP(hipEventSynchronize(e1));
    float t = 0.f;
    QT_HIP(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = (double)t / reps;
    return QT_OK;
}

// Measure every candidate CSR tile shape and, per dense bucket, every built wave count; keep the
// fastest in the autotuner table and in this plan.
qt_status me_plan_autotune(qt_me_plan *P, int32_t reps)
{
    QT_HIP(hipSetDevice(P->ctx->device));
    if (reps <= 0) reps = 20;
    if (P->ncsr) {
        CsrShape cand[64];
        const int nc = csr_candidates(cand, 64, P->ncsr == 1);
        CsrShape best = P->shape;
        double best_ms = 1e300;
        // The stage timing below cannot see what folding the step control into stage 2 saves (one
        // launch per step), so a plan that can fold chooses among the shapes that fold.
        const bool fold = folds_control(P, 2);
        for (int k = 0; k < nc; ++k) {
            if (fold && !folds_control(P, cand[k].keep)) continue;
            qt_status st = apply_shape(P, cand[k]);
            if (st) return st;
            double ms;
            if ((st = time_stage(P, reps, &ms))) return st;
            if (ms < best_ms) {
                best_ms = ms;
                best = cand[k];
            }
        }
        qt_status st = apply_shape(P, best);
        if (st) return st;
        tune_store_csr(P->tune_key, best);
    }
    if (P->ndense) {
        hipStream_t s = P->ctx->stream;
        const bool f64 = P->prec == QT_F64;
        for (const auto &bk : P->buckets) {
            int cand[8];
            const int nw = dense_waves_candidates(bk.np, P->prec, cand, 8);
            int best = dense_default_waves(bk.np, P->prec);
            double best_ms = 1e300;
            const DenseInst *di = (const DenseInst *)P->arena.at(P->o_dinst);
            DenseCtl *dc = (DenseCtl *)P->arena.at(P->o_dctl);
            const int32_t *ord = (const int32_t *)P->arena.at(P->o_dorder) + bk.start;
            for (int c = 0; c < nw; ++c) {
                // one untimed launch (code load, caches), then a timed one over the same step budget;
                // both restart every instance from rho0
                dense_launch_bucket(bk.np, f64, cand[c], di, dc, ord, bk.count, 2, 1, s);
                hipEvent_t e0, e1;
                QT_HIP(hipEventCreate(&e0));
                QT_HIP(hipEventCreate(&e1));
                QT_HIP(hipEventRecord(e0, s));
                dense_launch_bucket(bk.np, f64, cand[c], di, dc, ord, bk.count, 8, 1, s);
                QT_HIP(hipEventRecord(e1, s));
                QT_HIP(hipGetLastError());
                QT_HIP(hipEventSynchronize(e1));
                float t = 0.f;
                QT_HIP(hipEventElapsedTime(&t, e0, e1));
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                if (t < best_ms) {
                    best_ms = t;
                    best = cand[c];
                }
            }
            tune_store_dense(dense_tune_key(P->prec, bk.np), best);
        }
    }
    return QT_OK;
}

static qt_status status_code(int32_t s)
{
    if (s == ST_DONE) return QT_OK;
    if (s == ST_RUNNING) return QT_EMAXSTEPS;
    return s;
}

qt_status me_plan_result(qt_me_plan *P, int32_t i, double *expect_out, double *rho_final, qt_stats *stats)
{
    if (i < 0 || i >= (int32_t)P->probs.size()) return set_error(QT_EINVAL, "problem index out of range");
    QT_HIP(hipSetDevice(P->ctx->device));
    const MeProb &m = P->probs[i];
    const size_t es = state_es(P->prec);
    const size_t nvec = (size_t)m.d * m.d;
    int32_t status;
    int32_t parity = 0;
    double scale = 1.0;
    qt_stats sst;
    std::memset(&sst, 0, sizeof(sst));
    const void *ystate = nullptr;
    if (!m.dense) {
        const CsrCtl &c = P->h_cctl[m.slot];
        status = c.status;
        parity = c.parity;
        scale = c.scale;
        sst.n_accept = c.n_accept;
        sst.n_reject = c.n_reject;
        sst.n_rhs = c.n_rhs;
        ystate = (const char *)P->arena.at(m.o_vec) + parity * nvec * es;
    } else {
        const DenseCtl &c = P->h_dctl[m.slot];
        status = c.status;
        scale = c.scale;
        parity = c.parity;
        sst.n_accept = c.n_accept;
        sst.n_reject = c.n_reject;
        sst.n_rhs = c.n_rhs;
        const size_t np = (size_t)dense_np(m.d);
        ystate = (const char *)P->arena.at(m.o_vec) + parity * np * np * es;
    }
    sst.status = status_code(status);
    sst.device_ms = P->last_ms;
    if (stats) *stats = sst;
    if (expect_out && m.ne > 0)
        QT_HIP(hipMemcpy(expect_out, P->arena.at(m.o_expect), (size_t)m.ne * m.nt * 16, hipMemcpyDeviceToHost));
    if (rho_final && m.dense) {
        const size_t np = (size_t)dense_np(m.d);
        std::vector<char> hv(np * np * es);
        QT_HIP(hipMemcpy(hv.data(), ystate, hv.size(), hipMemcpyDeviceToHost));
        dense_unpack(hv.data(), m.d, P->prec, scale, rho_final);
    } else if (rho_final) {
        if (P->prec == QT_F64) {
            QT_HIP(hipMemcpy(rho_final, ystate, nvec * 16, hipMemcpyDeviceToHost));
            for (size_t q = 0; q < 2 * nvec; ++q) rho_final[q] *= scale;
        } else {
            std::vector<float> f(2 * nvec);
            QT_HIP(hipMemcpy(f.data(), ystate, nvec * 8, hipMemcpyDeviceToHost));
            for (size_t q = 0; q < 2 * nvec; ++q) rho_final[q] = (double)f[q] * scale;
        }
    }
    return sst.status == QT_OK ? QT_OK
                               : set_error(sst.status, "integration stopped with status " + std::to_string(sst.status));
}

}  // namespace qt

using namespace qt;

extern "C" {

qt_status qt_me_plan_create(qt_ctx *ctx, int32_t n, const qt_me_problem *probs, const qt_opts *opts, qt_me_plan **out)
{
    return me_plan_create(ctx, n, probs, opts, out, 0.0);
}

qt_status qt_me_plan_workspace(qt_ctx *ctx, int32_t n, const qt_me_problem *probs, const qt_opts *opts,
                               size_t *bytes)
{
    if (!bytes) return set_error(QT_EINVAL, "qt_me_plan_workspace: null bytes");
    return me_plan_create(ctx, n, probs, opts, nullptr, 0.0, nullptr, 0, bytes);
}

qt_status qt_me_plan_create_ws(qt_ctx *ctx, int32_t n, const qt_me_problem *probs, const qt_opts *opts, void *dev_ws,
                               size_t ws_bytes, qt_me_plan **out)
{
    if (!dev_ws) return set_error(QT_EINVAL, "qt_me_plan_create_ws: null workspace");
    return me_plan_create(ctx, n, probs, opts, out, 0.0, dev_ws, ws_bytes, nullptr);
}

qt_status qt_me_plan_create_steady(qt_ctx *ctx, int32_t n, const qt_me_problem *probs, const qt_opts *opts, double tol,
                                   qt_me_plan **out)
{
    if (!(tol > 0.0)) return set_error(QT_EINVAL, "qt_me_plan_create_steady: tol must be positive");
    return me_plan_create(ctx, n, probs, opts, out, tol);
}

qt_status qt_steadystate(qt_ctx *ctx, const qt_liouv *L, const double *rho0, int32_t is_ket, double tol, double t_max,
                         int32_t n_e, const qt_csr *e_ops, const qt_opts *opts, double *expect_out, double *rho_out,
                         qt_stats *stats)
{
    if (!L || !(t_max > 0.0) || !std::isfinite(t_max)) return set_error(QT_EINVAL, "qt_steadystate: bad arguments");
    const double tl[2] = {0.0, t_max};
    qt_me_problem p;
    p.L = L;
    p.rho0 = rho0;
    p.is_ket = is_ket;
    p.n_t = 2;
    p.tlist = tl;
    p.n_e = n_e;
    p.e_ops = e_ops;
    qt_me_plan *P = nullptr;
    qt_status st = qt_me_plan_create_steady(ctx, 1, &p, opts, tol, &P);
    if (st) {
        if (stats) stats->status = st;
        return st;
    }
    st = qt_me_plan_run(P);
    std::vector<double> ex((size_t)2 * std::max(1, n_e) * 2);
    if (!st) st = qt_me_plan_result(P, 0, ex.data(), rho_out, stats);
    else if (stats) stats->status = st;
    if (!st && expect_out)
        for (int32_t k = 0; k < n_e; ++k) {  // the values at the second save time: the converged state
            expect_out[2 * k] = ex[2 * ((size_t)k * 2 + 1)];
            expect_out[2 * k + 1] = ex[2 * ((size_t)k * 2 + 1) + 1];
        }
    qt_me_plan_destroy(P);
    return st;
}

qt_status qt_me_plan_run(qt_me_plan *plan)
{
    if (!plan) return set_error(QT_EINVAL, "null plan");
    return me_plan_run(plan);
}

qt_status qt_me_plan_result(qt_me_plan *plan, int32_t i, double *expect_out, double *rho_final, qt_stats *stats)
{
    if (!plan) return set_error(QT_EINVAL, "null plan");
    return me_plan_result(plan, i, expect_out, rho_final, stats);
}

qt_status qt_me_plan_autotune(qt_me_plan *plan, int32_t reps)
{
    if (!plan) return set_error(QT_EINVAL, "null plan");
    return me_plan_autotune(plan, reps);
}

qt_status qt_me_plan_set_shape(qt_me_plan *plan, const qt_csr_shape *shape)
{
    if (!plan || !shape) return set_error(QT_EINVAL, "qt_me_plan_set_shape: null argument");
    if (!csr_shape_supported(shape->lanes_per_row, shape->rows_per_group, shape->cached_matrix) ||
        shape->xcd_order < 0 || shape->xcd_order > 1)
        return set_error(QT_EINVAL, "unsupported CSR tile shape");
    if (!plan->ncsr) return QT_OK;
    QT_HIP(hipSetDevice(plan->ctx->device));
    CsrShape sh{shape->lanes_per_row, shape->rows_per_group, shape->xcd_order, shape->cached_matrix};
    if (plan->ncsr > 1) sh.xcd = 0;
    return apply_shape(plan, sh);
}

qt_status qt_me_plan_shape(const qt_me_plan *plan, qt_csr_shape *csr, int32_t *dense_waves)
{
    if (!plan) return set_error(QT_EINVAL, "null plan");
    if (csr) {
        const bool c = plan->ncsr > 0;
        csr->lanes_per_row = c ? plan->shape.lpr : 0;
        csr->rows_per_group = c ? plan->shape.rg : 0;
        csr->xcd_order = c ? plan->shape.xcd : 0;
        csr->cached_matrix = c ? plan->shape.keep : 0;
    }
    if (dense_waves)
        *dense_waves = plan->buckets.empty() ? 0 : dense_choose_config(plan->buckets[0].np, plan->prec);
    return QT_OK;
}

qt_status qt_me_plan_time_rhs(qt_me_plan *P, int32_t reps, double *ms_per_launch)
{
    if (!P || reps <= 0 || !ms_per_launch) return set_error(QT_EINVAL, "qt_me_plan_time_rhs: bad arguments");
    QT_HIP(hipSetDevice(P->ctx->device));
    if (P->ncsr) return time_stage(P, reps, ms_per_launch);
    hipStream_t s = P->ctx->stream;
    hipEvent_t e0, e1;
    QT_HIP(hipEventCreate(&e0));
    QT_HIP(hipEventCreate(&e1));
    QT_HIP(hipEventRecord(e0, s));
    for (int32_t r = 0; r < reps; ++r) launch_dense_buckets(P, -1, s);
    QT_HIP(hipEventRecord(e1, s));
    QT_HIP(hipGetLastError());
    QT_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    QT_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_per_launch = (double)ms / reps;
    return QT_OK;
}

qt_status qt_me_plan_destroy(qt_me_plan *P)
{
    if (!P) return QT_OK;
    (void)hipSetDevice(P->ctx->device);
    for (auto &l : P->lanes) {
        drop_graph(l);
        if (l.e0) (void)hipEventDestroy(l.e0);
        if (l.e1) (void)hipEventDestroy(l.e1);
    }
    for (hipStream_t ls : P->lane_streams) (void)hipStreamDestroy(ls);
    if (P->h_cctl) (void)hipHostFree(P->h_cctl);
    if (P->h_dctl) (void)hipHostFree(P->h_dctl);
    P->arena.release();
    if (P->counted) P->ctx->refs--;
    delete P;
    return QT_OK;
}

qt_status qt_mesolve(qt_ctx *ctx, const qt_me_problem *prob, const qt_opts *opts, double *expect_out,
                     double *rho_final, qt_stats *stats)
{
    qt_me_plan *P = nullptr;
    qt_status st = qt_me_plan_create(ctx, 1, prob, opts, &P);
    if (st) {
        if (stats) stats->status = st;
        return st;
    }
    st = qt_me_plan_run(P);
    if (!st) st = qt_me_plan_result(P, 0, expect_out, rho_final, stats);
    else if (stats) stats->status = st;
    qt_me_plan_destroy(P);
    return st;
}

qt_status qt_mesolve_ws(qt_ctx *ctx, const qt_me_problem *prob, const qt_opts *opts, void *dev_ws, size_t ws_bytes,
                        double *expect_out, double *rho_final, qt_stats *stats)
{
    qt_me_plan *P = nullptr;
    qt_status st = qt_me_plan_create_ws(ctx, 1, prob, opts, dev_ws, ws_bytes, &P);
    if (st) {
        if (stats) stats->status = st;
        return st;
    }
    st = qt_me_plan_run(P);
    if (!st) st = qt_me_plan_result(P, 0, expect_out, rho_final, stats);
    else if (stats) stats->status = st;
    qt_me_plan_destroy(P);
    return st;
}

qt_status qt_mesolve_batch(qt_ctx *ctx, int32_t n, const qt_me_problem *probs, const qt_opts *opts,
                           double *const *expect_out, qt_stats *stats)
{
    qt_me_plan *P = nullptr;
    qt_status st = qt_me_plan_create(ctx, n, probs, opts, &P);
    if (st) return st;
    st = qt_me_plan_run(P);
    qt_status first = st;
    for (int32_t i = 0; i < n && !st; ++i) {
        qt_status si = qt_me_plan_result(P, i, expect_out ? expect_out[i] : nullptr, nullptr, stats ? &stats[i] : nullptr);
        if (si && !first) first = si;
    }
    qt_me_plan_destroy(P);
    return first;
}

}  // extern "C"

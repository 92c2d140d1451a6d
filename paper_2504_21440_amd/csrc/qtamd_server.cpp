// qtamd_server.cpp -- continuous-batching master-equation server.
//
// Requests (master-equation problems of any size, CSR or dense form) are admitted while their
// device footprint fits in a fixed device pool and a slot is free.  Every admitted request keeps its
// density matrix, Runge-Kutta stages and control record resident in the pool; an epoch advances
// every resident request by up to `steps_per_epoch` adaptive steps in shared launches (CSR problems
// through the fused SpMV-stage kernels over a block table of all active CSR slots, dense problems
// through the persistent MFMA kernel with a step budget, resuming from their control records).
// After each epoch finished requests are retired -- their expectation values copied to the host and
// their pool memory released -- so requests that arrived meanwhile join the next epoch: a request's
// work overlaps on the device with whatever else is resident.  A request's arithmetic does not
// depend on what else is resident: its blocks, reductions and step decisions are its own.
//
// CSR requests run in two lanes, each with its own block table, epoch graphs and stream: large
// Liouvillians on the context's stream, small ones on its auxiliary stream.  A small problem's
// step costs a few microseconds of launch latency, a large one's far more, so in one shared table
// a stiff small request would advance only at the large ones' pace.  While the large lane's epoch
// runs, the small lane replays its own epoch graph, until the large lane finishes or no small
// request is left running.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <unordered_map>

#include "qt_csr.h"
#include "qt_dense.h"
#include "qt_host.h"
#include "qt_tune.h"

namespace qt {

// First-fit allocator over offsets of the device pool (256-byte granules), coalescing on free.
struct PoolAlloc {
    size_t size = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    void init(size_t n)
    {
        size = n;
        free_.clear();
        free_[0] = n;
    }
    bool alloc(size_t n, size_t *off)
    {
        n = (n + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, o2 = it->first + n;
                free_.erase(it);
                if (rest) free_[o2] = rest;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = (n + 255) & ~size_t(255);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest() const
    {
        size_t m = 0;
        for (auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }
};

struct Request {
    uint64_t ticket = 0;
    int32_t slot = -1;
    bool dense = false;
    int32_t d = 0, nt = 0, ne = 0, np = 0;
    size_t off = 0, bytes = 0;
    size_t o_expect = 0;  // offset inside the pool
    int32_t nblocks = 0;
    int64_t fp = 0;  // budget charged while resident
    bool done = false;
    int32_t status = 0;
    std::vector<double> expect;  // [ne][nt] complex, filled at retirement
    qt_stats stats{};
};

}  // namespace qt

struct qt_server {
    qt::Ctx *ctx = nullptr;
    qt_server_cfg cfg{};
    int32_t prec = QT_MIXED;
    qt::Arena arena;  // pool, slot arrays and block tables: one allocation, or the caller's workspace
    void *pool = nullptr;
    qt::PoolAlloc alloc;
    // slot-indexed device arrays
    qt::CsrInst *d_cinst = nullptr;
    qt::CsrCtl *d_cctl = nullptr;
    qt::DenseInst *d_dinst = nullptr;
    qt::DenseCtl *d_dctl = nullptr;
    int32_t *d_order = nullptr;
    // The CSR part of an epoch (starting-step evaluations, then steps_per_epoch steps) is one graph
    // per lane, captured once per grid size: the live block count rounded up to a power of two, so
    // the workgroups past the live count that return at once never outnumber the live ones.  The
    // table contents and their counts change every epoch; the graphs stay valid until the table is
    // reallocated.
    struct EpochGraph {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    struct Lane {
        int32_t *d_bi = nullptr, *d_br = nullptr, *d_ilist = nullptr;
        int32_t *d_counts = nullptr;  // [0] live blocks of the table, [1] live entries of the control list
        int32_t h_counts[2] = {0, 0};
        size_t blk_cap = 0;           // entries of d_bi / d_br (a power of two, fixed at creation)
        std::map<int, EpochGraph> graphs;
    };
    Lane lanes[2];  // 0: large Liouvillians (context stream), 1: small ones (auxiliary stream)
    qt::CsrCtl *h_cctl = nullptr;   // pinned
    qt::DenseCtl *h_dctl = nullptr; // pinned
    std::vector<int32_t> free_slots;
    std::unordered_map<uint64_t, qt::Request> reqs;  // admitted or finished, not yet polled
    std::vector<uint64_t> active;                    // tickets resident on the device
    uint64_t next_ticket = 1;
    qt::CsrShape shape;  // CSR tile shape of every epoch launch
    bool counted = false;  // holds a reference on ctx
    int64_t accounted = 0; // footprint of the resident requests
};

namespace qt {

static size_t es_of(int32_t prec) { return prec == QT_F64 ? 16 : 8; }

struct Layout {
    size_t o_rho0, o_tlist, o_eptr, o_ecol, o_eval, o_evidx, o_expect, o_vec, o_part, total;
};

static Layout layout_of(const qt_me_problem &p, int32_t prec, qt::CsrShape sh, size_t eptr_n, size_t ecol_n, int32_t *nblocks)
{
    const int32_t d = p.L->d;
    const size_t n = (size_t)d * d, es = es_of(prec);
    const bool dense = p.L->form == QT_FORM_DENSE;
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t r = o;
        o += (std::max<size_t>(b, 1) + 255) & ~size_t(255);
        return r;
    };
    L.o_rho0 = take(n * es);
    L.o_tlist = take((size_t)p.n_t * 8);
    L.o_eptr = take(eptr_n * 4);
    L.o_ecol = take(ecol_n * 4);
    L.o_eval = take(ecol_n * 16);
    L.o_evidx = take(ecol_n * 4);
    L.o_expect = take((size_t)p.n_e * p.n_t * 16);
    if (dense) {
        const size_t np = (size_t)dense_np(d);
        L.o_vec = take(dense_state_vectors() * np * np * es);
        L.o_part = 0;
        *nblocks = 0;
    } else {
        const int rpb = csr_rows_per_block(sh.lpr, sh.rg);
        *nblocks = (int32_t)((n + rpb - 1) / rpb);
        L.o_vec = take(11 * n * es);
        L.o_part = take((size_t)*nblocks * 16);
    }
    L.total = o;
    return L;
}

static size_t eops_nnz(const qt_me_problem &p)
{
    size_t s = 0;
    for (int k = 0; k < p.n_e; ++k) s += (size_t)std::max<int64_t>(0, p.e_ops[k].nnz);
    return s;
}

static qt_status server_submit(qt_server *S, const qt_me_problem *p, uint64_t *ticket)
{
    if (!p || !p->L || !ticket) return set_error(QT_EINVAL, "qt_server_submit: null argument");
    if (p->L->precision != S->prec) return set_error(QT_EINVAL, "request precision differs from the server's");
    if (p->L->nterms > 0) return set_error(QT_EINVAL, "time-dependent Liouvillians are solved through plans");
    if (p->n_t < 1 || !p->tlist || !p->rho0 || p->n_e < 0 || (p->n_e > 0 && !p->e_ops))
        return set_error(QT_EINVAL, "malformed request");
    for (int32_t i = 0; i < p->n_t; ++i)
        if (!std::isfinite(p->tlist[i]) || (i > 0 && !(p->tlist[i] > p->tlist[i - 1])))
            return set_error(QT_EINVAL, "tlist must be finite and strictly increasing");
    const int32_t d = p->L->d;
    const bool dense = p->L->form == QT_FORM_DENSE;
    // e_ops as concatenated int32 CSR
    std::vector<int32_t> eptr((size_t)std::max(1, p->n_e) * (d + 1), 0), ecol;
    std::vector<double2> eval;
    for (int k = 0; k < p->n_e; ++k) {
        HCsr o;
        qt_status st = csr_from_abi(&p->e_ops[k], d, &o, "e_ops");
        if (st) return st;
        const int32_t base = (int32_t)ecol.size();
        for (int32_t i = 0; i <= d; ++i) eptr[(size_t)k * (d + 1) + i] = base + (int32_t)o.ptr[i];
        for (int64_t q = 0; q < o.nnz(); ++q) {
            ecol.push_back(o.idx[q]);
            eval.push_back(make_double2(o.val[q].real(), o.val[q].imag()));
        }
    }
    int32_t nblocks = 0;
    const Layout Ly = layout_of(*p, S->prec, S->shape, eptr.size(), ecol.size(), &nblocks);
    // the budget covers everything the request keeps resident: its state (carved from the pool) and
    // its Liouvillian (owned by the caller)
    const int64_t fp = (int64_t)Ly.total + p->L->bytes;
    if (fp > S->cfg.pool_bytes) return set_error(QT_ENOMEM, "request footprint exceeds the server budget");
    if (S->free_slots.empty()) return set_error(QT_EBUSY, "no free slot");
    if (S->accounted + fp > S->cfg.pool_bytes) return set_error(QT_EBUSY, "budget in use by resident requests");
    size_t off = 0;
    if (!S->alloc.alloc(Ly.total, &off)) return set_error(QT_EBUSY, "pool full");
    // initial state in the solve precision
    const size_t n = (size_t)d * d, es = es_of(S->prec);
    std::vector<double> r(2 * n);
    if (p->is_ket) {
        for (int32_t i = 0; i < d; ++i)
            for (int32_t j = 0; j < d; ++j) {
                const cd a(p->rho0[2 * i], p->rho0[2 * i + 1]), b(p->rho0[2 * j], p->rho0[2 * j + 1]);
                const cd v = a * std::conj(b);
                r[2 * ((size_t)i * d + j)] = v.real();
                r[2 * ((size_t)i * d + j) + 1] = v.imag();
            }
    } else {
        std::memcpy(r.data(), p->rho0, 16 * n);
    }
    std::vector<char> rb(n * es);
    if (S->prec == QT_F64) std::memcpy(rb.data(), r.data(), n * 16);
    else
        for (size_t i = 0; i < 2 * n; ++i) ((float *)rb.data())[i] = (float)r[i];
    const int32_t slot = S->free_slots.back();
    S->free_slots.pop_back();
    char *base = (char *)S->pool + off;
    hipStream_t s = S->ctx->stream;
    hipError_t e = hipSuccess;
    auto up = [&](size_t o, const void *src, size_t b) {
        if (e == hipSuccess && b) e = hipMemcpyAsync(base + o, src, b, hipMemcpyHostToDevice, s);
    };
    up(Ly.o_rho0, rb.data(), rb.size());
    up(Ly.o_tlist, p->tlist, (size_t)p->n_t * 8);
    up(Ly.o_eptr, eptr.data(), eptr.size() * 4);
    up(Ly.o_ecol, ecol.data(), ecol.size() * 4);
    up(Ly.o_eval, eval.data(), eval.size() * 16);
    const std::vector<int32_t> evidx = expect_vec_index(eptr, ecol, d, p->n_e);
    up(Ly.o_evidx, evidx.data(), evidx.size() * 4);
    qt_opts o = S->cfg.opts;
    if (dense) {
        DenseInst g;
        dense_fill_inst(&g, d, p->L->nc, p->L->dense_creal, p->n_t, p->n_e, p->L->dense, base + Ly.o_rho0,
                        base + Ly.o_vec,
                        (const double *)(base + Ly.o_tlist), (const int32_t *)(base + Ly.o_eptr),
                        (const int32_t *)(base + Ly.o_ecol), (const double2 *)(base + Ly.o_eval),
                        (double2 *)(base + Ly.o_expect), o, S->prec);
        DenseCtl c;
        std::memset(&c, 0, sizeof(c));
        c.status = DENSE_ST_INIT;
        S->h_dctl[slot] = c;
        if (e == hipSuccess) e = hipMemcpyAsync(S->d_dinst + slot, &g, sizeof(g), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(S->d_dctl + slot, &S->h_dctl[slot], sizeof(c), hipMemcpyHostToDevice, s);
    } else {
        CsrInst c;
        std::memset(&c, 0, sizeof(c));
        c.n = (int32_t)n;
        c.d = d;
        c.nt = p->n_t;
        c.ne = p->n_e;
        c.block0 = 0;  // not used by the kernels (a block finds its partial slot from its first row)
        c.nblocks = nblocks;
        c.renorm = S->prec == QT_MIXED ? 1 : 0;
        c.use_h0 = o.h0 > 0 ? 1 : 0;
        c.atol = o.abstol;
        c.rtol = o.reltol;
        c.h0 = o.h0;
        c.max_steps = o.max_steps;
        c.rowptr = p->L->rowptr;
        c.col = p->L->col;
        c.val = p->L->val;
        c.rho0 = base + Ly.o_rho0;
        char *v = base + Ly.o_vec;
        c.Y[0] = v;
        c.Y[1] = v + n * es;
        c.K[0] = v + 2 * n * es;
        c.K[1] = v + 3 * n * es;
        for (int k = 0; k < 5; ++k) c.ks[k] = v + (4 + k) * n * es;
        c.ys[0] = v + 9 * n * es;
        c.ys[1] = v + 10 * n * es;
        c.tlist = (const double *)(base + Ly.o_tlist);
        c.eptr = (const int32_t *)(base + Ly.o_eptr);
        c.ecol = (const int32_t *)(base + Ly.o_ecol);
        c.eval = (const double2 *)(base + Ly.o_eval);
        c.evidx = (const int32_t *)(base + Ly.o_evidx);
        c.expect = (double2 *)(base + Ly.o_expect);
        c.partials = (double *)(base + Ly.o_part);
        csr_set_expect_ranges(c, eptr.data(), p->n_e, d);
        CsrCtl t;
        std::memset(&t, 0, sizeof(t));
        t.t = p->tlist[0];
        t.err_prev = 1e-4;
        t.scale = 1.0;
        t.tr0 = 1.0;
        t.status = ST_RUNNING;
        t.phase = 2;  // first starting-step evaluation pending
        t.save_idx = 1;
        S->h_cctl[slot] = t;
        if (e == hipSuccess) e = hipMemcpyAsync(S->d_cinst + slot, &c, sizeof(c), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(S->d_cctl + slot, &S->h_cctl[slot], sizeof(t), hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // host staging buffers go out of scope
    if (e != hipSuccess) {
        S->alloc.release(off, Ly.total);
        S->free_slots.push_back(slot);
        return set_error(QT_EDEVICE, std::string("qt_server_submit: ") + hipGetErrorString(e));
    }
    Request R;
    R.ticket = S->next_ticket++;
    R.slot = slot;
    R.dense = dense;
    R.d = d;
    R.nt = p->n_t;
    R.ne = p->n_e;
    R.np = dense ? dense_np(d) : 0;
    R.off = off;
    R.bytes = Ly.total;
    R.o_expect = off + Ly.o_expect;
    R.nblocks = nblocks;
    R.fp = fp;
    S->accounted += fp;
    S->reqs[R.ticket] = R;
    S->active.push_back(R.ticket);
    *ticket = R.ticket;
    return QT_OK;
}

static void drop_graphs(qt_server::Lane &ln)
{
    for (auto &g : ln.graphs) {
        if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
        if (g.second.graph) (void)hipGraphDestroy(g.second.graph);
    }
    ln.graphs.clear();
}

// Liouville rows up to which a CSR request runs in the small lane (d <= 128)
constexpr int64_t SMALL_LANE_ROWS = 16384;

// Uploads a lane's block table and control list and launches its epoch graph (capturing it on
// first use of this grid size) on stream s.
static qt_status launch_lane(qt_server *S, qt_server::Lane &ln, const std::vector<int32_t> &bi,
                             const std::vector<int32_t> &br, const std::vector<int32_t> &slots, int K, hipStream_t s)
{
    int grid = 256;
    while ((size_t)grid < bi.size()) grid *= 2;
    // the table capacity bounds every admissible mix of requests (server_table_capacity)
    if ((size_t)grid > ln.blk_cap) return set_error(QT_EDEVICE, "server block table over its capacity");
    ln.h_counts[0] = (int32_t)bi.size();
    ln.h_counts[1] = (int32_t)slots.size();
    QT_HIP(hipMemcpyAsync(ln.d_bi, bi.data(), bi.size() * 4, hipMemcpyHostToDevice, s));
    QT_HIP(hipMemcpyAsync(ln.d_br, br.data(), br.size() * 4, hipMemcpyHostToDevice, s));
    QT_HIP(hipMemcpyAsync(ln.d_ilist, slots.data(), slots.size() * 4, hipMemcpyHostToDevice, s));
    QT_HIP(hipMemcpyAsync(ln.d_counts, ln.h_counts, sizeof(ln.h_counts), hipMemcpyHostToDevice, s));
    qt_server::EpochGraph &G = ln.graphs[grid];
    if (!G.exec) {
        CsrLaunch L;
        L.f64 = S->prec == QT_F64;
        L.lpr = S->shape.lpr;
        L.rg = S->shape.rg;
        L.xcd = 0;
        L.keep = S->shape.keep;
        L.nblk = grid;               // blocks past the live count return at once
        L.ninst = S->cfg.max_slots;  // likewise for the control list
        L.ilist = ln.d_ilist;
        L.bound = ln.d_counts;
        L.ibound = ln.d_counts + 1;
        L.insts = S->d_cinst;
        L.ctls = S->d_cctl;
        L.bi = ln.d_bi;
        L.br = ln.d_br;
        QT_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        csr_launch_init(0, L, s);
        csr_launch_init(1, L, s);
        for (int k = 0; k < K; ++k) csr_launch_step(L, s);
        hipError_t ce = hipStreamEndCapture(s, &G.graph);
        if (ce) {
            ln.graphs.erase(grid);
            return set_error(QT_EDEVICE, std::string("server graph capture: ") + hipGetErrorString(ce));
        }
        ce = hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0);
        if (ce) {
            (void)hipGraphDestroy(G.graph);
            ln.graphs.erase(grid);
            return set_error(QT_EDEVICE, std::string("server graph instantiate: ") + hipGetErrorString(ce));
        }
    }
    QT_HIP(hipGraphLaunch(G.exec, s));
    QT_HIP(hipGetLastError());
    return QT_OK;
}

static qt_status server_step(qt_server *S, int32_t *n_active, int32_t *n_finished)
{
    Ctx *ctx = S->ctx;
    QT_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const bool f64 = S->prec == QT_F64;
    const int K = std::max(1, S->cfg.steps_per_epoch);
    // ---- CSR slots: one block table per lane ----
    std::vector<int32_t> bi[2], br[2], csr_slots[2];
    const int rpb = csr_rows_per_block(S->shape.lpr, S->shape.rg);
    for (uint64_t tk : S->active) {
        Request &R = S->reqs[tk];
        if (R.dense) continue;
        const int l = (int64_t)R.d * R.d <= SMALL_LANE_ROWS ? 1 : 0;
        for (int32_t b = 0; b < R.nblocks; ++b) {
            bi[l].push_back(R.slot);
            br[l].push_back(b * rpb);
        }
        csr_slots[l].push_back(R.slot);
    }
    // ---- dense slots: one budgeted launch per padded size, on the auxiliary streams ----
    std::map<int32_t, std::vector<int32_t>> buckets;
    for (uint64_t tk : S->active) {
        Request &R = S->reqs[tk];
        if (R.dense) buckets[-R.np].push_back(R.slot);  // largest first
    }
    std::vector<int32_t> order;
    for (auto &b : buckets) order.insert(order.end(), b.second.begin(), b.second.end());
    hipEvent_t ev = nullptr;
    if (!order.empty()) {
        QT_HIP(hipMemcpyAsync(S->d_order, order.data(), order.size() * 4, hipMemcpyHostToDevice, s));
        QT_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        QT_HIP(hipEventRecord(ev, s));
        size_t start = 0;
        int bn = 0;
        for (auto &b : buckets) {
            hipStream_t bs = ctx->pool[bn++ % Ctx::NPOOL];
            QT_HIP(hipStreamWaitEvent(bs, ev, 0));
            dense_launch_bucket(-b.first, f64, dense_choose_config(-b.first, S->prec), S->d_dinst, S->d_dctl,
                                S->d_order + start, (int)b.second.size(), K, 0, bs);
            start += b.second.size();
        }
        QT_HIP(hipGetLastError());
    }
    // ---- large CSR lane (after the dense launches' start event, so those run beside it) ----
    hipEvent_t big_done = nullptr;
    if (!bi[0].empty()) {
        qt_status st = launch_lane(S, S->lanes[0], bi[0], br[0], csr_slots[0], K, s);
        if (st) {
            if (ev) (void)hipEventDestroy(ev);
            return st;
        }
        QT_HIP(hipEventCreateWithFlags(&big_done, hipEventDisableTiming));
        QT_HIP(hipEventRecord(big_done, s));
    }
    // ---- small CSR lane: replayed while the large lane runs and a small request still steps ----
    if (!bi[1].empty()) {
        hipStream_t sa = ctx->aux;
        constexpr int MAX_REPLAYS = 64;  // bounds an epoch, so that new requests are admitted
        for (int rep = 0; rep < MAX_REPLAYS; ++rep) {
            qt_status st = launch_lane(S, S->lanes[1], bi[1], br[1], csr_slots[1], K, sa);
            if (st) {
                if (big_done) (void)hipEventDestroy(big_done);
                if (ev) (void)hipEventDestroy(ev);
                return st;
            }
            QT_HIP(hipMemcpyAsync(S->h_cctl, S->d_cctl, sizeof(CsrCtl) * S->cfg.max_slots, hipMemcpyDeviceToHost,
                                  sa));
            QT_HIP(hipStreamSynchronize(sa));
            if (!big_done || hipEventQuery(big_done) != hipErrorNotReady) break;
            bool running = false;
            for (int32_t slot : csr_slots[1]) running = running || S->h_cctl[slot].status == ST_RUNNING;
            if (!running) break;
        }
    }
    // ---- wait, then retire finished requests ----
    if (big_done) (void)hipEventDestroy(big_done);
    QT_HIP(hipMemcpyAsync(S->h_cctl, S->d_cctl, sizeof(CsrCtl) * S->cfg.max_slots, hipMemcpyDeviceToHost, s));
    QT_HIP(hipStreamSynchronize(s));
    if (ev) {
        for (int b = 0; b < Ctx::NPOOL; ++b) QT_HIP(hipStreamSynchronize(ctx->pool[b]));
        (void)hipEventDestroy(ev);
        QT_HIP(hipMemcpy(S->h_dctl, S->d_dctl, sizeof(DenseCtl) * S->cfg.max_slots, hipMemcpyDeviceToHost));
    }
    int32_t fin = 0;
    std::vector<uint64_t> still;
    for (uint64_t tk : S->active) {
        Request &R = S->reqs[tk];
        int32_t status;
        qt_stats st;
        std::memset(&st, 0, sizeof(st));
        if (R.dense) {
            const DenseCtl &c = S->h_dctl[R.slot];
            status = c.status;
            st.n_accept = c.n_accept;
            st.n_reject = c.n_reject;
            st.n_rhs = c.n_rhs;
        } else {
            const CsrCtl &c = S->h_cctl[R.slot];
            status = c.status;
            st.n_accept = c.n_accept;
            st.n_reject = c.n_reject;
            st.n_rhs = c.n_rhs;
        }
        if (status == ST_RUNNING || status == DENSE_ST_INIT) {
            still.push_back(tk);
            continue;
        }
        R.status = status == ST_DONE ? QT_OK : status;
        st.status = R.status;
        R.stats = st;
        R.expect.assign((size_t)2 * R.ne * R.nt, 0.0);
        if (R.ne) QT_HIP(hipMemcpy(R.expect.data(), (char *)S->pool + R.o_expect, (size_t)R.ne * R.nt * 16,
                                   hipMemcpyDeviceToHost));
        S->alloc.release(R.off, R.bytes);
        S->accounted -= R.fp;
        S->free_slots.push_back(R.slot);
        R.slot = -1;
        R.done = true;
        ++fin;
    }
    S->active.swap(still);
    if (n_active) *n_active = (int32_t)S->active.size();
    if (n_finished) *n_finished = fin;
    return QT_OK;
}

// Workgroup-table entries one lane can need: a resident CSR request of n Liouville rows has
// ceil(n / rows_per_block) blocks and holds at least 11 n state values of the pool, so the blocks of
// everything the pool admits number at most pool_bytes / (11 es rows_per_block) + max_slots.  Epoch
// grids are powers of two of at least 256, so the capacity is the power of two at or above that.
static size_t server_table_capacity(const qt_server_cfg *cfg, const CsrShape &sh)
{
    const size_t rpb = (size_t)csr_rows_per_block(sh.lpr, sh.rg);
    const size_t bound = (size_t)cfg->pool_bytes / (11 * es_of(cfg->opts.precision) * rpb) + (size_t)cfg->max_slots;
    size_t cap = 256;
    while (cap < bound) cap *= 2;
    return cap;
}

static CsrShape server_shape()
{
    // requests of many sizes share one grid: the shape for small spin and oscillator Liouvillians
    CsrShape sh = csr_default_shape(0, 19.0);
    // matrices read through the caches (many small resident ones fit the L2s / MALL), runs of 4
    // stored entries per 16-byte load
    sh.keep = 2;
    return sh;
}

static qt_status check_cfg(const qt_server_cfg *cfg)
{
    if (cfg->pool_bytes <= 0 || cfg->max_slots <= 0 || cfg->steps_per_epoch <= 0)
        return set_error(QT_EINVAL, "server config: pool_bytes, max_slots and steps_per_epoch must be positive");
    if (cfg->opts.precision != QT_F64 && cfg->opts.precision != QT_MIXED)
        return set_error(QT_EINVAL, "server config: bad precision");
    return QT_OK;
}

// Lays out the server's device memory in S->arena and returns the offsets through the members.
struct ServerLayout {
    size_t pool, cinst, cctl, dinst, dctl, order, ilist[2], counts[2], bi[2], br[2];
};
static ServerLayout server_layout(Arena &A, const qt_server_cfg *cfg, size_t cap)
{
    const size_t ns = (size_t)cfg->max_slots;
    ServerLayout L;
    L.pool = A.reserve((size_t)cfg->pool_bytes);
    L.cinst = A.reserve(sizeof(CsrInst) * ns);
    L.cctl = A.reserve(sizeof(CsrCtl) * ns);
    L.dinst = A.reserve(sizeof(DenseInst) * ns);
    L.dctl = A.reserve(sizeof(DenseCtl) * ns);
    L.order = A.reserve(sizeof(int32_t) * ns);
    for (int k = 0; k < 2; ++k) {
        L.ilist[k] = A.reserve(sizeof(int32_t) * ns);
        L.counts[k] = A.reserve(sizeof(int32_t) * 2);
        L.bi[k] = A.reserve(4 * cap);
        L.br[k] = A.reserve(4 * cap);
    }
    return L;
}

static qt_status server_create(Ctx *ctx, const qt_server_cfg *cfg, void *ws, size_t ws_bytes, qt_server **out)
{
    if (!ctx || !cfg || !out) return set_error(QT_EINVAL, "qt_server_create: null argument");
    qt_status st = check_cfg(cfg);
    if (st) return st;
    QT_HIP(hipSetDevice(ctx->device));
    qt_server *S = new qt_server();
    S->ctx = ctx;
    S->cfg = *cfg;
    S->prec = cfg->opts.precision;
    S->shape = server_shape();
    const int ns = cfg->max_slots;
    const size_t cap = server_table_capacity(cfg, S->shape);
    const ServerLayout Ly = server_layout(S->arena, cfg, cap);
    if ((st = S->arena.place(ws, ws_bytes, "qt_server_create_ws"))) {
        delete S;
        return st;
    }
    Arena &A = S->arena;
    S->pool = A.at(Ly.pool);
    S->d_cinst = (CsrInst *)A.at(Ly.cinst);
    S->d_cctl = (CsrCtl *)A.at(Ly.cctl);
    S->d_dinst = (DenseInst *)A.at(Ly.dinst);
    S->d_dctl = (DenseCtl *)A.at(Ly.dctl);
    S->d_order = (int32_t *)A.at(Ly.order);
    for (int k = 0; k < 2; ++k) {
        auto &ln = S->lanes[k];
        ln.d_ilist = (int32_t *)A.at(Ly.ilist[k]);
        ln.d_counts = (int32_t *)A.at(Ly.counts[k]);
        ln.d_bi = (int32_t *)A.at(Ly.bi[k]);
        ln.d_br = (int32_t *)A.at(Ly.br[k]);
        ln.blk_cap = cap;
    }
    hipError_t e = hipHostMalloc((void **)&S->h_cctl, sizeof(CsrCtl) * ns, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&S->h_dctl, sizeof(DenseCtl) * ns, hipHostMallocDefault);
    if (e == hipSuccess) {
        // every slot starts finished: the kernels skip it until a request is admitted into it
        for (int i = 0; i < ns; ++i) {
            std::memset(&S->h_cctl[i], 0, sizeof(CsrCtl));
            S->h_cctl[i].status = ST_DONE;
            std::memset(&S->h_dctl[i], 0, sizeof(DenseCtl));
            S->h_dctl[i].status = ST_DONE;
        }
        e = hipMemcpyAsync(S->d_cctl, S->h_cctl, sizeof(CsrCtl) * ns, hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(S->d_dctl, S->h_dctl, sizeof(DenseCtl) * ns, hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    }
    if (e != hipSuccess) {
        qt_server_destroy(S);
        return set_error(e == hipErrorOutOfMemory ? QT_ENOMEM : QT_EDEVICE,
                         std::string("qt_server_create: ") + hipGetErrorString(e));
    }
    S->alloc.init((size_t)cfg->pool_bytes);
    for (int i = ns - 1; i >= 0; --i) S->free_slots.push_back(i);
    ctx->refs++;
    S->counted = true;
    *out = S;
    return QT_OK;
}

}  // namespace qt

using namespace qt;

extern "C" {

qt_status qt_server_create(qt_ctx *ctx, const qt_server_cfg *cfg, qt_server **out)
{
    return server_create(ctx, cfg, nullptr, 0, out);
}

qt_status qt_server_workspace(const qt_server_cfg *cfg, size_t *bytes)
{
    if (!cfg || !bytes) return set_error(QT_EINVAL, "qt_server_workspace: null argument");
    qt_status st = check_cfg(cfg);
    if (st) return st;
    Arena A;
    (void)server_layout(A, cfg, server_table_capacity(cfg, server_shape()));
    *bytes = A.size;
    return QT_OK;
}

qt_status qt_server_create_ws(qt_ctx *ctx, const qt_server_cfg *cfg, void *dev_ws, size_t ws_bytes, qt_server **out)
{
    if (!dev_ws) return set_error(QT_EINVAL, "qt_server_create_ws: null workspace");
    return server_create(ctx, cfg, dev_ws, ws_bytes, out);
}

qt_status qt_server_footprint(const qt_server *srv, const qt_me_problem *prob, int64_t *bytes)
{
    if (!srv || !prob || !prob->L || !bytes) return set_error(QT_EINVAL, "qt_server_footprint: null argument");
    const int32_t d = prob->L->d;
    int32_t nb = 0;
    const Layout L = layout_of(*prob, srv->prec, srv->shape, (size_t)std::max(1, prob->n_e) * (d + 1),
                               prob->n_e > 0 && prob->e_ops ? eops_nnz(*prob) : 0, &nb);
    *bytes = (int64_t)L.total + prob->L->bytes;
    return QT_OK;
}

qt_status qt_server_submit(qt_server *srv, const qt_me_problem *prob, uint64_t *ticket)
{
    if (!srv) return set_error(QT_EINVAL, "null server");
    QT_HIP(hipSetDevice(srv->ctx->device));
    return server_submit(srv, prob, ticket);
}

qt_status qt_server_step(qt_server *srv, int32_t *n_active, int32_t *n_finished)
{
    if (!srv) return set_error(QT_EINVAL, "null server");
    return server_step(srv, n_active, n_finished);
}

qt_status qt_server_poll(qt_server *srv, uint64_t ticket, int32_t *done, double *expect_out, qt_stats *stats)
{
    if (!srv || !done) return set_error(QT_EINVAL, "qt_server_poll: null argument");
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return set_error(QT_EINVAL, "unknown ticket");
    Request &R = it->second;
    *done = R.done ? 1 : 0;
    if (!R.done) return QT_OK;
    if (expect_out && !R.expect.empty()) std::memcpy(expect_out, R.expect.data(), R.expect.size() * 8);
    if (stats) *stats = R.stats;
    const qt_status st = R.status;
    srv->reqs.erase(it);
    return st == QT_OK ? QT_OK : set_error(st, "request stopped with status " + std::to_string(st));
}

qt_status qt_server_destroy(qt_server *S)
{
    if (!S) return QT_OK;
    (void)hipSetDevice(S->ctx->device);
    (void)hipStreamSynchronize(S->ctx->stream);
    for (int b = 0; b < Ctx::NPOOL; ++b)
        if (S->ctx->pool[b]) (void)hipStreamSynchronize(S->ctx->pool[b]);
    (void)hipStreamSynchronize(S->ctx->aux);
    for (auto &ln : S->lanes) drop_graphs(ln);
    S->arena.release();
    if (S->h_cctl) (void)hipHostFree(S->h_cctl);
    if (S->h_dctl) (void)hipHostFree(S->h_dctl);
    if (S->counted) S->ctx->refs--;
    delete S;
    return QT_OK;
}

}  // extern "C"

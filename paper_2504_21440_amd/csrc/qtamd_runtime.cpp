// qtamd_runtime.cpp -- contexts, errors, model operators, host sparse algebra, Liouvillian
// construction and the standalone expectation value of libqtamd.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>

#include "qt_asm.h"
#include "qt_coef.h"
#include "qt_csr.h"
#include "qt_dense.h"
#include "qt_host.h"

namespace qt {

static thread_local std::string g_err;

qt_status set_error(qt_status code, const std::string &msg)
{
    g_err = msg;
    return code;
}

qt_status Arena::alloc()
{
    if (size == 0) return QT_OK;
    hipError_t e = hipMalloc(&base, size);
    if (e != hipSuccess) {
        base = nullptr;
        return set_error(e == hipErrorOutOfMemory ? QT_ENOMEM : QT_EDEVICE,
                         std::string("hipMalloc(") + std::to_string(size) + "): " + hipGetErrorString(e));
    }
    return QT_OK;
}

qt_status Arena::adopt(void *ws, size_t ws_bytes, const char *who)
{
    if (((uintptr_t)ws & 255) != 0)
        return set_error(QT_EINVAL, std::string(who) + ": workspace must be 256-byte aligned");
    if (ws_bytes < size)
        return set_error(QT_ENOMEM, std::string(who) + ": workspace of " + std::to_string(ws_bytes) +
                                        " bytes, " + std::to_string(size) + " needed");
    base = ws;
    external = true;
    return QT_OK;
}

void Arena::release()
{
    if (base && !external) (void)hipFree(base);
    base = nullptr;
    external = false;
    size = used = 0;
}

// ---- host CSR -----------------------------------------------------------------------------
qt_status csr_from_abi(const qt_csr *A, int32_t d_expect, HCsr *out, const char *what)
{
    if (!A) return set_error(QT_EINVAL, std::string(what) + ": null operator");
    if (A->rows <= 0 || A->rows != A->cols)
        return set_error(QT_EINVAL, std::string(what) + ": operator must be square with rows > 0");
    if (d_expect > 0 && A->rows != d_expect)
        return set_error(QT_EINVAL, std::string(what) + ": dimension " + std::to_string(A->rows) + " != " +
                                        std::to_string(d_expect));
    if (A->nnz < 0 || !A->indptr || (A->nnz > 0 && (!A->indices || !A->values)))
        return set_error(QT_EINVAL, std::string(what) + ": malformed CSR arrays");
    const int32_t d = A->rows;
    if (A->indptr[0] != 0 || A->indptr[d] != A->nnz)
        return set_error(QT_EINVAL, std::string(what) + ": indptr[0] must be 0 and indptr[rows] == nnz");
    out->d = d;
    out->ptr.assign(d + 1, 0);
    out->idx.clear();
    out->val.clear();
    std::map<int32_t, cd> row;
    for (int32_t i = 0; i < d; ++i) {
        if (A->indptr[i + 1] < A->indptr[i]) return set_error(QT_EINVAL, std::string(what) + ": decreasing indptr");
        row.clear();
        for (int64_t p = A->indptr[i]; p < A->indptr[i + 1]; ++p) {
            const int32_t j = A->indices[p];
            if (j < 0 || j >= d) return set_error(QT_EINVAL, std::string(what) + ": column index out of range");
            const double re = A->values[2 * p], im = A->values[2 * p + 1];
            if (!std::isfinite(re) || !std::isfinite(im))
                return set_error(QT_EINVAL, std::string(what) + ": non-finite value");
            row[j] += cd(re, im);
        }
        for (auto &kv : row)
            if (kv.second != cd(0.0, 0.0)) {
                out->idx.push_back(kv.first);
                out->val.push_back(kv.second);
            }
        out->ptr[i + 1] = (int64_t)out->idx.size();
    }
    return QT_OK;
}

std::vector<int32_t> expect_vec_index(const std::vector<int32_t> &eptr, const std::vector<int32_t> &ecol, int32_t d,
                                      int32_t ne)
{
    std::vector<int32_t> v(ecol.size());
    for (int32_t k = 0; k < ne; ++k)
        for (int32_t i = 0; i < d; ++i)
            for (int32_t q = eptr[(size_t)k * (d + 1) + i]; q < eptr[(size_t)k * (d + 1) + i + 1]; ++q)
                v[q] = ecol[q] * d + i;
    return v;
}

HCsr csr_zero(int32_t d)
{
    HCsr z;
    z.d = d;
    z.ptr.assign(d + 1, 0);
    return z;
}

HCsr csr_adjoint(const HCsr &A)
{
    HCsr B;
    B.d = A.d;
    B.ptr.assign(A.d + 1, 0);
    B.idx.resize(A.idx.size());
    B.val.resize(A.val.size());
    for (int32_t j : A.idx) B.ptr[j + 1]++;
    for (int32_t i = 0; i < A.d; ++i) B.ptr[i + 1] += B.ptr[i];
    std::vector<int64_t> fill(B.ptr.begin(), B.ptr.end() - 1);
    for (int32_t i = 0; i < A.d; ++i)
        for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
            const int64_t q = fill[A.idx[p]]++;
            B.idx[q] = i;
            B.val[q] = std::conj(A.val[p]);
        }
    return B;
}

// Sparse accumulator over one output row.
struct Spa {
    std::vector<cd> v;
    std::vector<char> used;
    std::vector<int32_t> list;
    explicit Spa(int32_t d) : v(d), used(d, 0) {}
    void add(int32_t j, cd x)
    {
        if (!used[j]) {
            used[j] = 1;
            list.push_back(j);
            v[j] = x;
        } else {
            v[j] += x;
        }
    }
    void flush(HCsr &out)
    {
        std::sort(list.begin(), list.end());
        for (int32_t j : list) {
            if (v[j] != cd(0.0, 0.0)) {
                out.idx.push_back(j);
                out.val.push_back(v[j]);
            }
            used[j] = 0;
        }
        list.clear();
    }
};

HCsr csr_matmul(const HCsr &A, const HCsr &B)
{
    HCsr C;
    C.d = A.d;
    C.ptr.assign(A.d + 1, 0);
    Spa s(A.d);
    for (int32_t i = 0; i < A.d; ++i) {
        for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
            const int32_t k = A.idx[p];
            for (int64_t q = B.ptr[k]; q < B.ptr[k + 1]; ++q) s.add(B.idx[q], A.val[p] * B.val[q]);
        }
        s.flush(C);
        C.ptr[i + 1] = (int64_t)C.idx.size();
    }
    return C;
}

HCsr csr_axpby(cd a, const HCsr &A, cd b, const HCsr &B)
{
    HCsr C;
    C.d = A.d;
    C.ptr.assign(A.d + 1, 0);
    Spa s(A.d);
    for (int32_t i = 0; i < A.d; ++i) {
        for (int64_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) s.add(A.idx[p], a * A.val[p]);
        for (int64_t p = B.ptr[i]; p < B.ptr[i + 1]; ++p) s.add(B.idx[p], b * B.val[p]);
        s.flush(C);
        C.ptr[i + 1] = (int64_t)C.idx.size();
    }
    return C;
}

}  // namespace qt

using namespace qt;

// ===============================================================================================
// Public ABI
// ===============================================================================================
extern "C" {

void qt_opts_default(qt_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->abstol = 1e-8;
    o->reltol = 1e-6;
    o->max_steps = 1000000;
    o->h0 = 0.0;
    o->precision = QT_F64;
    o->form = QT_FORM_CSR;
    o->steps_per_launch = 0;
}

const char *qt_last_error(void) { return g_err.c_str(); }
const char *qt_version(void) { return "qtamd 0.1 (gfx950)"; }

qt_status qt_ctx_create(int32_t device, void *hip_stream, qt_ctx **out)
{
    if (!out) return set_error(QT_EINVAL, "qt_ctx_create: null out");
    int n = 0;
    QT_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return set_error(QT_EINVAL, "qt_ctx_create: no such device");
    QT_HIP(hipSetDevice(device));
    qt_ctx *c = new qt_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    hipError_t e = hipSuccess;
    if (!c->stream) {
        // the legacy null stream cannot be captured into a graph: use a stream of our own
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        c->own_stream = true;
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking);
    for (int k = 0; k < Ctx::NPOOL && e == hipSuccess; ++k) e = hipStreamCreateWithFlags(&c->pool[k], hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete c;
        return set_error(QT_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    }
    qt_status st = noalloc_init_device(device);
    if (st) {
        qt_ctx_destroy(c);
        return st;
    }
    *out = c;
    return QT_OK;
}

qt_status qt_ctx_destroy(qt_ctx *ctx)
{
    if (!ctx) return QT_OK;
    if (ctx->refs > 0)
        return set_error(QT_EBUSY, "qt_ctx_destroy: " + std::to_string(ctx->refs) +
                                       " Liouvillian(s), plan(s) or server(s) created on this context are still alive");
    (void)hipSetDevice(ctx->device);
    if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
    for (int k = 0; k < Ctx::NPOOL; ++k)
        if (ctx->pool[k]) (void)hipStreamDestroy(ctx->pool[k]);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return QT_OK;
}

// ---- model operators ----------------------------------------------------------------------------
static void to_abi(const HCsr &A, qt_csr *out)
{
    int64_t *ip = (int64_t *)std::malloc(sizeof(int64_t) * (A.d + 1));
    int32_t *ix = (int32_t *)std::malloc(sizeof(int32_t) * std::max<int64_t>(1, A.nnz()));
    double *v = (double *)std::malloc(sizeof(double) * 2 * std::max<int64_t>(1, A.nnz()));
    std::memcpy(ip, A.ptr.data(), sizeof(int64_t) * (A.d + 1));
    for (int64_t p = 0; p < A.nnz(); ++p) {
        ix[p] = A.idx[p];
        v[2 * p] = A.val[p].real();
        v[2 * p + 1] = A.val[p].imag();
    }
    out->rows = out->cols = A.d;
    out->nnz = A.nnz();
    out->indptr = ip;
    out->indices = ix;
    out->values = v;
}

void qt_csr_free(qt_csr *A)
{
    if (!A) return;
    std::free((void *)A->indptr);
    std::free((void *)A->indices);
    std::free((void *)A->values);
    A->indptr = nullptr;
    A->indices = nullptr;
    A->values = nullptr;
    A->nnz = 0;
}

qt_status qt_model_kerr(int32_t N, double delta, double U, double F, double kappa, qt_csr *H, qt_csr *c)
{
    if (N < 1 || !H || !c || kappa < 0) return set_error(QT_EINVAL, "qt_model_kerr: bad arguments");
    // Fock basis: a|n> = sqrt(n)|n-1>, so a_{n-1,n} = sqrt(n); a^dag a a^dag... in closed form:
    // H_nn = delta n + (U/2) n (n-1);  H_{n,n+1} = H_{n+1,n} = F sqrt(n+1).
    HCsr h;
    h.d = N;
    h.ptr.assign(N + 1, 0);
    for (int32_t n = 0; n < N; ++n) {
        if (n > 0 && F != 0.0) {
            h.idx.push_back(n - 1);
            h.val.push_back(cd(F * std::sqrt((double)n), 0.0));
        }
        const double diag = delta * n + 0.5 * U * n * (n - 1.0);
        if (diag != 0.0) {
            h.idx.push_back(n);
            h.val.push_back(cd(diag, 0.0));
        }
        if (n + 1 < N && F != 0.0) {
            h.idx.push_back(n + 1);
            h.val.push_back(cd(F * std::sqrt((double)(n + 1)), 0.0));
        }
        h.ptr[n + 1] = (int64_t)h.idx.size();
    }
    HCsr a;
    a.d = N;
    a.ptr.assign(N + 1, 0);
    const double sk = std::sqrt(kappa);
    for (int32_t n = 0; n < N; ++n) {
        if (n + 1 < N && sk != 0.0) {
            a.idx.push_back(n + 1);
            a.val.push_back(cd(sk * std::sqrt((double)(n + 1)), 0.0));
        }
        a.ptr[n + 1] = (int64_t)a.idx.size();
    }
    to_abi(h, H);
    to_abi(a, c);
    return QT_OK;
}

qt_status qt_model_ising(int32_t L, double J, double h, double gamma, qt_csr *H, qt_csr *c_ops)
{
    if (L < 1 || L > 14 || !H || !c_ops || gamma < 0) return set_error(QT_EINVAL, "qt_model_ising: bad arguments");
    const int32_t d = 1 << L;
    // basis index bit (L-1-i) holds spin i (spin 0 most significant); bit value 0 = up (sz = +1).
    auto sz = [&](int32_t s, int i) { return ((s >> (L - 1 - i)) & 1) ? -1.0 : 1.0; };
    HCsr hh;
    hh.d = d;
    hh.ptr.assign(d + 1, 0);
    for (int32_t s = 0; s < d; ++s) {
        std::vector<std::pair<int32_t, double>> row;
        double diag = 0.0;
        for (int i = 0; i + 1 < L; ++i) diag += J * sz(s, i) * sz(s, i + 1);
        if (diag != 0.0) row.push_back({s, diag});
        if (h != 0.0)
            for (int i = 0; i < L; ++i) row.push_back({s ^ (1 << (L - 1 - i)), h});
        std::sort(row.begin(), row.end());
        for (auto &e : row) {
            hh.idx.push_back(e.first);
            hh.val.push_back(cd(e.second, 0.0));
        }
        hh.ptr[s + 1] = (int64_t)hh.idx.size();
    }
    to_abi(hh, H);
    const double sg = std::sqrt(gamma);
    for (int i = 0; i < L; ++i) {
        // sigma_- on spin i: |down><up|, row = state with spin i down, column = same with spin i up
        HCsr c;
        c.d = d;
        c.ptr.assign(d + 1, 0);
        const int32_t bit = 1 << (L - 1 - i);
        for (int32_t s = 0; s < d; ++s) {
            if ((s & bit) && sg != 0.0) {
                c.idx.push_back(s ^ bit);
                c.val.push_back(cd(sg, 0.0));
            }
            c.ptr[s + 1] = (int64_t)c.idx.size();
        }
        to_abi(c, &c_ops[i]);
    }
    return QT_OK;
}

// ---- Liouvillian ----------------------------------------------------------------------------------
static qt_status upload_csr32(const HCsr &A, std::vector<int32_t> &rp, std::vector<int32_t> &ci,
                              std::vector<double2> &v)
{
    if (A.nnz() >= 2147483647LL) return set_error(QT_EINVAL, "operator has too many non-zeros");
    rp.resize(A.d + 1);
    for (int32_t i = 0; i <= A.d; ++i) rp[i] = (int32_t)A.ptr[i];
    ci.assign(A.idx.begin(), A.idx.end());
    v.resize(A.nnz());
    for (int64_t p = 0; p < A.nnz(); ++p) v[p] = make_double2(A.val[p].real(), A.val[p].imag());
    return QT_OK;
}

// Device assembly of  L = A (x) I + I (x) conj(B) + sum_k C_k (x) conj(C_k)  (B null: B = A) into
// CSR with int32 indices, values in the solve precision, every row padded with zeros to a multiple
// of 4 stored entries.  On success the caller owns the three device arrays; *nnz_out counts the
// entries of L, *stored_out the stored ones.
static qt_status assemble_csr(Ctx *ctx, const HCsr &A, const HCsr *B, const std::vector<HCsr> &cs, bool f64,
                              int32_t **rowptr_out, int32_t **col_out, void **val_out, int64_t *nnz_out,
                              int64_t *stored_out)
{
    const int32_t d = A.d, n_c = (int32_t)cs.size();
    const size_t es = f64 ? sizeof(double2) : sizeof(float2);
    qt_status st;
    std::vector<int32_t> arp, aci, brp, bci;
    std::vector<double2> av, bv;
    if ((st = upload_csr32(A, arp, aci, av))) return st;
    if (B && (st = upload_csr32(*B, brp, bci, bv))) return st;
    std::vector<int32_t> crp((size_t)n_c * (d + 1)), cci;
    std::vector<double2> cv;
    for (int k = 0; k < n_c; ++k) {
        const int32_t base = (int32_t)cci.size();
        for (int32_t i = 0; i <= d; ++i) crp[(size_t)k * (d + 1) + i] = base + (int32_t)cs[k].ptr[i];
        for (int64_t p = 0; p < cs[k].nnz(); ++p) {
            cci.push_back(cs[k].idx[p]);
            cv.push_back(make_double2(cs[k].val[p].real(), cs[k].val[p].imag()));
        }
    }
    const int64_t n = (int64_t)d * d;
    if (n >= 2147483647LL) return set_error(QT_EINVAL, "Liouvillian too large for int32 indexing");
    Arena tmp;
    const size_t o_arp = tmp.reserve(arp.size() * 4), o_aci = tmp.reserve(std::max<size_t>(1, aci.size()) * 4),
                 o_av = tmp.reserve(std::max<size_t>(1, av.size()) * 16),
                 o_brp = tmp.reserve(std::max<size_t>(1, brp.size()) * 4),
                 o_bci = tmp.reserve(std::max<size_t>(1, bci.size()) * 4),
                 o_bv = tmp.reserve(std::max<size_t>(1, bv.size()) * 16),
                 o_crp = tmp.reserve(std::max<size_t>(1, crp.size()) * 4),
                 o_cci = tmp.reserve(std::max<size_t>(1, cci.size()) * 4),
                 o_cv = tmp.reserve(std::max<size_t>(1, cv.size()) * 16), o_cnt = tmp.reserve((size_t)n * 4),
                 o_bs = tmp.reserve(((size_t)(n + 1023) / 1024 + 1) * 8), o_fl = tmp.reserve(64);
    if ((st = tmp.alloc())) return st;
    hipStream_t s = ctx->stream;
    auto cp = [&](size_t off, const void *src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync(tmp.at(off), src, bytes, hipMemcpyHostToDevice, s);
    };
    hipError_t e = hipSuccess;
    e = e ? e : cp(o_arp, arp.data(), arp.size() * 4);
    e = e ? e : cp(o_aci, aci.data(), aci.size() * 4);
    e = e ? e : cp(o_av, av.data(), av.size() * 16);
    e = e ? e : cp(o_brp, brp.data(), brp.size() * 4);
    e = e ? e : cp(o_bci, bci.data(), bci.size() * 4);
    e = e ? e : cp(o_bv, bv.data(), bv.size() * 16);
    e = e ? e : cp(o_crp, crp.data(), crp.size() * 4);
    e = e ? e : cp(o_cci, cci.data(), cci.size() * 4);
    e = e ? e : cp(o_cv, cv.data(), cv.size() * 16);
    e = e ? e : hipMemsetAsync(tmp.at(o_fl), 0, 64, s);
    AsmOps op{d,
              n_c,
              (const int32_t *)tmp.at(o_arp),
              (const int32_t *)tmp.at(o_aci),
              (const double2 *)tmp.at(o_av),
              (const int32_t *)tmp.at(o_crp),
              (const int32_t *)tmp.at(o_cci),
              (const double2 *)tmp.at(o_cv),
              B ? (const int32_t *)tmp.at(o_brp) : nullptr,
              B ? (const int32_t *)tmp.at(o_bci) : nullptr,
              B ? (const double2 *)tmp.at(o_bv) : nullptr};
    int32_t *counts = (int32_t *)tmp.at(o_cnt);
    int *flags = (int *)tmp.at(o_fl);
    int32_t *rowptr = nullptr, *col = nullptr;
    void *val = nullptr;
    e = e ? e : hipMalloc(&rowptr, (size_t)(n + 1) * 4);
    if (e == hipSuccess) {
        asm_launch_count(op, counts, flags, (unsigned long long *)(flags + 4), f64, s);
        asm_launch_scan(counts, n, (int64_t *)tmp.at(o_bs), rowptr, flags, s);
        e = hipGetLastError();
    }
    int hflags[6] = {0, 0, 0, 0, 0, 0};  // overflow, too many entries, pad, pad, real count (uint64)
    int32_t total = 0;
    e = e ? e : hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, s);
    e = e ? e : hipMemcpyAsync(&total, rowptr + n, 4, hipMemcpyDeviceToHost, s);
    e = e ? e : hipStreamSynchronize(s);
    if (e == hipSuccess && (hflags[0] || hflags[1])) {
        tmp.release();
        (void)hipFree(rowptr);
        return set_error(QT_EINVAL, hflags[0] ? "Liouvillian row has too many candidate entries for CSR assembly "
                                                "(use the dense form)"
                                              : "Liouvillian has more than 2^31 non-zeros");
    }
    if (e == hipSuccess) {
        e = hipMalloc(&col, std::max<size_t>(1, (size_t)total) * 4);
        if (e == hipSuccess) e = hipMalloc(&val, std::max<size_t>(1, (size_t)total) * es);
        if (e == hipSuccess) {
            asm_launch_fill(op, rowptr, col, val, f64, s);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    tmp.release();
    if (e != hipSuccess) {
        if (rowptr) (void)hipFree(rowptr);
        if (col) (void)hipFree(col);
        if (val) (void)hipFree(val);
        return set_error(QT_EDEVICE, std::string("Liouvillian assembly: ") + hipGetErrorString(e));
    }
    unsigned long long real = 0;
    std::memcpy(&real, hflags + 4, sizeof(real));
    *rowptr_out = rowptr;
    *col_out = col;
    *val_out = val;
    *nnz_out = (int64_t)real;
    *stored_out = total;
    return QT_OK;
}

qt_status qt_liouvillian_build(qt_ctx *ctx, const qt_csr *H, int32_t n_c, const qt_csr *c_ops, int32_t form,
                               int32_t precision, qt_liouv **out)
{
    if (!ctx || !H || !out || n_c < 0 || (n_c > 0 && !c_ops))
        return set_error(QT_EINVAL, "qt_liouvillian_build: null argument");
    if (precision != QT_F64 && precision != QT_MIXED) return set_error(QT_EINVAL, "bad precision");
    if (form != QT_FORM_CSR && form != QT_FORM_DENSE) return set_error(QT_EINVAL, "bad form");
    HCsr h;
    qt_status st = csr_from_abi(H, 0, &h, "H");
    if (st) return st;
    const int32_t d = h.d;
    std::vector<HCsr> cs(n_c);
    for (int k = 0; k < n_c; ++k)
        if ((st = csr_from_abi(&c_ops[k], d, &cs[k], "c_ops"))) return st;
    QT_HIP(hipSetDevice(ctx->device));
    // A = -i H - 1/2 sum_k C_k^dag C_k
    HCsr A = csr_axpby(cd(0.0, -1.0), h, cd(0.0, 0.0), csr_zero(d));
    for (auto &c : cs) A = csr_axpby(cd(1.0, 0.0), A, cd(-0.5, 0.0), csr_matmul(csr_adjoint(c), c));

    qt_liouv *L = new qt_liouv();
    L->ctx = ctx;
    L->form = form;
    L->precision = precision;
    L->d = d;
    L->nc = n_c;
    const size_t es = precision == QT_F64 ? sizeof(double2) : sizeof(float2);

    if (form == QT_FORM_DENSE) {
        const int32_t np = dense_np(d);
        if (np > (precision == QT_F64 ? DENSE_MAX_NP_F64 : DENSE_MAX_NP_F32)) {
            delete L;
            return set_error(QT_EINVAL, "dense form supports d <= 80 (mixed) or d <= 48 (FP64)");
        }
        // A then C_k, each zero padded to np x np (np = d rounded up to a multiple of 16)
        const size_t mat = (size_t)np * np;
        std::vector<double2> host((1 + n_c) * mat, make_double2(0.0, 0.0));
        auto put = [&](const HCsr &M, size_t base) {
            for (int32_t i = 0; i < d; ++i)
                for (int64_t p = M.ptr[i]; p < M.ptr[i + 1]; ++p)
                    host[base + (size_t)i * np + M.idx[p]] = make_double2(M.val[p].real(), M.val[p].imag());
        };
        put(A, 0);
        for (int k = 0; k < n_c; ++k) put(cs[k], (1 + k) * mat);
        L->dense_creal = 0;
        for (int k = 0; k < n_c && k < 32; ++k) {
            bool real = true;
            for (const cd &v : cs[k].val) real = real && v.imag() == 0.0;
            if (real) L->dense_creal |= 1u << k;
        }
        std::vector<char> packed;
        dense_pack_ops(host.data(), np, 1 + n_c, L->dense_creal, precision, packed);
        L->bytes = (int64_t)packed.size();
        hipError_t e = hipMalloc(&L->dense, L->bytes);
        if (e != hipSuccess) {
            delete L;
            return set_error(QT_ENOMEM, "hipMalloc dense operators");
        }
        e = hipMemcpy(L->dense, packed.data(), L->bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(L->dense);
            delete L;
            return set_error(QT_EDEVICE, "upload dense operators");
        }
        ctx->refs++, *out = L;
        return QT_OK;
    }

    // CSR form: device assembly
    if ((st = assemble_csr(ctx, A, nullptr, cs, precision == QT_F64, &L->rowptr, &L->col, &L->val, &L->nnz,
                           &L->nnz_stored))) {
        delete L;
        return st;
    }
    const int64_t n = (int64_t)d * d;
    L->bytes = (int64_t)((n + 1) * 4 + L->nnz_stored * (4 + (int64_t)es));
    ctx->refs++, *out = L;
    return QT_OK;
}

}  // extern "C"

namespace qt {

CoefDev coef_from_abi(const qt_coef &c, int modsq)
{
    CoefDev g;
    g.kind = c.kind;
    g.n_table = c.kind == QT_COEF_TABLE ? c.n_table : 0;
    g.modsq = modsq;
    g.pad = 0;
    g.a_re = c.a[0];
    g.a_im = c.a[1];
    g.omega = c.omega;
    g.phi = c.phi;
    g.t0 = c.t0;
    g.sigma = c.sigma;
    g.table_t0 = c.table_t0;
    g.table_dt = c.table_dt;
    g.table = nullptr;  // the caller places the samples in device memory
    return g;
}

qt_status check_coef(const qt_coef &c, bool allow_none, const char *what)
{
    if (allow_none && c.kind == QT_COEF_NONE) return QT_OK;
    if (c.kind < QT_COEF_CONST || c.kind > QT_COEF_TABLE)
        return set_error(QT_EINVAL, std::string(what) + ": unknown coefficient kind");
    if (c.kind == QT_COEF_GAUSS && !(c.sigma > 0.0))
        return set_error(QT_EINVAL, std::string(what) + ": Gaussian coefficient needs sigma > 0");
    if (c.kind == QT_COEF_TABLE && (c.n_table < 1 || !c.table || !(c.table_dt > 0.0)))
        return set_error(QT_EINVAL, std::string(what) + ": table coefficient needs samples and table_dt > 0");
    return QT_OK;
}

}  // namespace qt

extern "C" {

qt_status qt_liouvillian_build_td(qt_ctx *ctx, const qt_csr *H0, int32_t n_h, const qt_csr *h_terms,
                                  const qt_coef *h_coefs, int32_t n_c, const qt_csr *c_ops, const qt_coef *c_coefs,
                                  int32_t form, int32_t precision, qt_liouv **out)
{
    if (!ctx || !H0 || !out || n_h < 0 || n_c < 0 || (n_h > 0 && (!h_terms || !h_coefs)) || (n_c > 0 && !c_ops))
        return set_error(QT_EINVAL, "qt_liouvillian_build_td: null argument");
    if (precision != QT_F64 && precision != QT_MIXED) return set_error(QT_EINVAL, "bad precision");
    qt_status st;
    for (int i = 0; i < n_h; ++i)
        if ((st = check_coef(h_coefs[i], false, "h_coefs"))) return st;
    int n_w = 0;  // weighted collapse operators
    for (int k = 0; k < n_c && c_coefs; ++k) {
        if ((st = check_coef(c_coefs[k], true, "c_coefs"))) return st;
        n_w += c_coefs[k].kind != QT_COEF_NONE;
    }
    const int nterms = n_h + n_w;
    if (nterms == 0) return qt_liouvillian_build(ctx, H0, n_c, c_ops, form, precision, out);
    if (form != QT_FORM_CSR) return set_error(QT_EINVAL, "time-dependent Liouvillians need the CSR form");
    if (nterms > TD_MAX_TERMS) return set_error(QT_EINVAL, "at most 31 time-dependent terms");
    HCsr h0;
    if ((st = csr_from_abi(H0, 0, &h0, "H0"))) return st;
    const int32_t d = h0.d;
    const int64_t n = (int64_t)d * d;
    if (n > (int64_t)TD_COL_MASK) return set_error(QT_EINVAL, "time-dependent Liouvillian needs d*d < 2^26");
    std::vector<HCsr> hs(n_h), cs(n_c);
    for (int i = 0; i < n_h; ++i)
        if ((st = csr_from_abi(&h_terms[i], d, &hs[i], "h_terms"))) return st;
    for (int k = 0; k < n_c; ++k)
        if ((st = csr_from_abi(&c_ops[k], d, &cs[k], "c_ops"))) return st;
    QT_HIP(hipSetDevice(ctx->device));
    const bool f64 = precision == QT_F64;
    const size_t es = f64 ? sizeof(double2) : sizeof(float2);
    auto weighted = [&](int k) { return c_coefs && c_coefs[k].kind != QT_COEF_NONE; };

    // term 0: H0 with the constant collapse operators; then each H_i; then each weighted C_k
    struct Part {
        int32_t *rp = nullptr, *ci = nullptr;
        void *v = nullptr;
        int64_t nnz = 0, stored = 0;
    };
    std::vector<Part> parts(1 + nterms);
    auto free_parts = [&]() {
        for (auto &q : parts) {
            if (q.rp) (void)hipFree(q.rp);
            if (q.ci) (void)hipFree(q.ci);
            if (q.v) (void)hipFree(q.v);
            q = Part();
        }
    };
    {
        std::vector<HCsr> c0;
        HCsr A = csr_axpby(cd(0.0, -1.0), h0, cd(0.0, 0.0), csr_zero(d));
        for (int k = 0; k < n_c; ++k)
            if (!weighted(k)) {
                A = csr_axpby(cd(1.0, 0.0), A, cd(-0.5, 0.0), csr_matmul(csr_adjoint(cs[k]), cs[k]));
                c0.push_back(cs[k]);
            }
        st = assemble_csr(ctx, A, nullptr, c0, f64, &parts[0].rp, &parts[0].ci, &parts[0].v, &parts[0].nnz,
                          &parts[0].stored);
    }
    std::vector<CoefDev> cd_host(nterms);
    std::vector<const qt_coef *> src(nterms);
    int t = 1;
    for (int i = 0; i < n_h && !st; ++i, ++t) {
        // -i (H rho - rho H):  A = -i H,  B = -i H^dag  (rho B^dag = i rho H)
        const HCsr A = csr_axpby(cd(0.0, -1.0), hs[i], cd(0.0, 0.0), csr_zero(d));
        const HCsr B = csr_axpby(cd(0.0, -1.0), csr_adjoint(hs[i]), cd(0.0, 0.0), csr_zero(d));
        st = assemble_csr(ctx, A, &B, {}, f64, &parts[t].rp, &parts[t].ci, &parts[t].v, &parts[t].nnz,
                          &parts[t].stored);
        src[t - 1] = &h_coefs[i];
        cd_host[t - 1].modsq = 0;
    }
    for (int k = 0; k < n_c && !st; ++k) {
        if (!weighted(k)) continue;
        // D[C]:  A = -1/2 C^dag C,  C (x) conj(C)
        const HCsr A = csr_axpby(cd(-0.5, 0.0), csr_matmul(csr_adjoint(cs[k]), cs[k]), cd(0.0, 0.0), csr_zero(d));
        st = assemble_csr(ctx, A, nullptr, {cs[k]}, f64, &parts[t].rp, &parts[t].ci, &parts[t].v, &parts[t].nnz,
                          &parts[t].stored);
        src[t - 1] = &c_coefs[k];
        cd_host[t - 1].modsq = 1;
        ++t;
    }
    if (st) {
        free_parts();
        return st;
    }
    int64_t total = 0, real = 0;
    for (auto &q : parts) {
        total += q.stored;
        real += q.nnz;
    }
    if (total >= 2147483647LL) {
        free_parts();
        return set_error(QT_EINVAL, "Liouvillian has more than 2^31 non-zeros");
    }
    // coefficient descriptors and their tables, one device buffer
    size_t tab_bytes = 0;
    for (int k = 0; k < nterms; ++k)
        if (src[k]->kind == QT_COEF_TABLE) tab_bytes += (size_t)src[k]->n_table * sizeof(double2);
    const size_t head = ((sizeof(CoefDev) * nterms + 255) / 256) * 256;
    qt_liouv *L = new qt_liouv();
    L->ctx = ctx;
    L->form = form;
    L->precision = precision;
    L->d = d;
    L->nc = n_c;
    L->nterms = nterms;
    L->nnz = real;
    L->nnz_stored = total;
    hipError_t e = hipMalloc(&L->coefs, head + std::max<size_t>(tab_bytes, 16));
    std::vector<char> hostbuf(head + tab_bytes, 0);
    size_t toff = head;
    for (int k = 0; k < nterms && e == hipSuccess; ++k) {
        const qt_coef &c = *src[k];
        CoefDev &g = cd_host[k];
        g = coef_from_abi(c, g.modsq);
        if (c.kind == QT_COEF_TABLE) {
            std::memcpy(hostbuf.data() + toff, c.table, (size_t)c.n_table * sizeof(double2));
            g.table = (const double2 *)((char *)L->coefs + toff);
            toff += (size_t)c.n_table * sizeof(double2);
        }
    }
    if (e == hipSuccess) {
        std::memcpy(hostbuf.data(), cd_host.data(), sizeof(CoefDev) * nterms);
        e = hipMemcpy(L->coefs, hostbuf.data(), hostbuf.size(), hipMemcpyHostToDevice);
    }
    // merged CSR
    std::vector<TdTerm> th(parts.size());
    for (size_t k = 0; k < parts.size(); ++k) th[k] = TdTerm{parts[k].rp, parts[k].ci, parts[k].v};
    TdTerm *dterms = nullptr;
    if (e == hipSuccess) e = hipMalloc(&dterms, sizeof(TdTerm) * th.size());
    if (e == hipSuccess) e = hipMemcpy(dterms, th.data(), sizeof(TdTerm) * th.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&L->rowptr, (size_t)(n + 1) * 4);
    if (e == hipSuccess) e = hipMalloc(&L->col, std::max<size_t>(1, (size_t)total) * 4);
    if (e == hipSuccess) e = hipMalloc(&L->val, std::max<size_t>(1, (size_t)total) * es);
    if (e == hipSuccess) {
        asm_launch_td_merge(dterms, (int)th.size(), n, L->rowptr, L->col, L->val, f64, ctx->stream);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (dterms) (void)hipFree(dterms);
    free_parts();
    if (e != hipSuccess) {
        if (L->rowptr) (void)hipFree(L->rowptr);
        if (L->col) (void)hipFree(L->col);
        if (L->val) (void)hipFree(L->val);
        if (L->coefs) (void)hipFree(L->coefs);
        delete L;
        return set_error(QT_EDEVICE, std::string("time-dependent Liouvillian: ") + hipGetErrorString(e));
    }
    L->bytes = (int64_t)((n + 1) * 4 + total * (4 + (int64_t)es) + head + tab_bytes);
    ctx->refs++, *out = L;
    return QT_OK;
}

qt_status qt_liouv_terms(const qt_liouv *L, int32_t *n_terms)
{
    if (!L || !n_terms) return set_error(QT_EINVAL, "qt_liouv_terms: null argument");
    *n_terms = L->nterms;
    return QT_OK;
}

qt_status qt_liouv_info(const qt_liouv *L, int32_t *d, int64_t *nnz, int64_t *bytes)
{
    if (!L) return set_error(QT_EINVAL, "null Liouvillian");
    if (d) *d = L->d;
    if (nnz) *nnz = L->nnz;
    if (bytes) *bytes = L->bytes;
    return QT_OK;
}

qt_status qt_liouv_footprint(const qt_liouv *L, size_t *bytes)
{
    if (!L || !bytes) return set_error(QT_EINVAL, "qt_liouv_footprint: null argument");
    *bytes = (size_t)L->bytes;
    return QT_OK;
}

qt_status qt_liouv_export(const qt_liouv *L, int64_t *indptr, int32_t *indices, double *values)
{
    if (!L || L->form != QT_FORM_CSR || !indptr || !indices || !values)
        return set_error(QT_EINVAL, "qt_liouv_export: CSR Liouvillian and output arrays required");
    QT_HIP(hipSetDevice(L->ctx->device));
    const int64_t n = (int64_t)L->d * L->d, ns = L->nnz_stored;
    std::vector<int32_t> rp(n + 1), ci(ns);
    std::vector<double2> v(ns);
    QT_HIP(hipMemcpy(rp.data(), L->rowptr, (n + 1) * 4, hipMemcpyDeviceToHost));
    if (ns) QT_HIP(hipMemcpy(ci.data(), L->col, ns * 4, hipMemcpyDeviceToHost));
    if (L->precision == QT_F64) {
        if (ns) QT_HIP(hipMemcpy(v.data(), L->val, ns * 16, hipMemcpyDeviceToHost));
    } else {
        std::vector<float2> f(ns);
        if (ns) QT_HIP(hipMemcpy(f.data(), L->val, ns * 8, hipMemcpyDeviceToHost));
        for (int64_t p = 0; p < ns; ++p) v[p] = make_double2(f[p].x, f[p].y);
    }
    // the stored zeros are the row padding: leave them out
    int64_t o = 0;
    indptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
            if (v[p].x == 0.0 && v[p].y == 0.0) continue;
            if (o >= L->nnz) return set_error(QT_EDEVICE, "qt_liouv_export: more entries than counted");
            indices[o] = ci[p];
            values[2 * o] = v[p].x;
            values[2 * o + 1] = v[p].y;
            ++o;
        }
        indptr[i + 1] = o;
    }
    if (o != L->nnz) return set_error(QT_EDEVICE, "qt_liouv_export: fewer entries than counted");
    return QT_OK;
}

qt_status qt_liouv_destroy(qt_liouv *L)
{
    if (!L) return QT_OK;
    (void)hipSetDevice(L->ctx->device);
    if (L->rowptr) (void)hipFree(L->rowptr);
    if (L->col) (void)hipFree(L->col);
    if (L->val) (void)hipFree(L->val);
    if (L->dense) (void)hipFree(L->dense);
    if (L->coefs) (void)hipFree(L->coefs);
    L->ctx->refs--;
    delete L;
    return QT_OK;
}

// ---- expectation value ------------------------------------------------------------------------------
qt_status qt_expect(qt_ctx *ctx, int32_t d, const qt_csr *O, const void *dev_state, int32_t is_ket,
                    int32_t precision, double *out)
{
    if (!ctx || !O || !dev_state || !out || d <= 0) return set_error(QT_EINVAL, "qt_expect: null argument");
    if (precision != QT_F64 && precision != QT_MIXED) return set_error(QT_EINVAL, "qt_expect: bad precision");
    HCsr o;
    qt_status st = csr_from_abi(O, d, &o, "O");
    if (st) return st;
    std::vector<int32_t> rp, ci;
    std::vector<double2> v;
    if ((st = upload_csr32(o, rp, ci, v))) return st;
    QT_HIP(hipSetDevice(ctx->device));
    Arena a;
    const size_t o_rp = a.reserve(rp.size() * 4), o_ci = a.reserve(std::max<size_t>(1, ci.size()) * 4),
                 o_v = a.reserve(std::max<size_t>(1, v.size()) * 16), o_out = a.reserve(16);
    if ((st = a.alloc())) return st;
    hipStream_t s = ctx->stream;
    hipError_t e = hipMemcpyAsync(a.at(o_rp), rp.data(), rp.size() * 4, hipMemcpyHostToDevice, s);
    if (!e && !ci.empty()) e = hipMemcpyAsync(a.at(o_ci), ci.data(), ci.size() * 4, hipMemcpyHostToDevice, s);
    if (!e && !v.empty()) e = hipMemcpyAsync(a.at(o_v), v.data(), v.size() * 16, hipMemcpyHostToDevice, s);
    if (!e) {
        launch_expect(precision == QT_F64, d, (const int32_t *)a.at(o_rp), (const int32_t *)a.at(o_ci),
                      (const double2 *)a.at(o_v), dev_state, is_ket, (double2 *)a.at(o_out), s);
        e = hipGetLastError();
    }
    if (!e) e = hipMemcpyAsync(out, a.at(o_out), 16, hipMemcpyDeviceToHost, s);
    if (!e) e = hipStreamSynchronize(s);
    a.release();
    if (e) return set_error(QT_EDEVICE, std::string("qt_expect: ") + hipGetErrorString(e));
    return QT_OK;
}

}  // extern "C"

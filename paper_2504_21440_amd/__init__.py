"""Python binding of libqtamd: argument marshalling over the C ABI declared in include/qtamd.h.

Every step of the solvers runs in the HIP library; this module only converts numpy / scipy inputs
to the ABI's plain arrays and structs and raises on error statuses.  Importing it never falls back
to anything else: if libqtamd.so is missing, :func:`lib` raises.

Names follow the C ABI (arXiv:2504.21440 Sec. 3: ``mesolve``, ``mcsolve``, ``liouvillian``,
``expect``).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqtamd.so")

QT_OK, QT_EINVAL, QT_ENOMEM, QT_EDEVICE, QT_EMAXSTEPS, QT_EDTMIN, QT_ENONFINITE, QT_EBUSY = range(8)
F64, MIXED = 0, 1
FORM_CSR, FORM_DENSE = 0, 1

EXPORTED = [
    "qt_opts_default", "qt_last_error", "qt_version", "qt_ctx_create", "qt_ctx_destroy", "qt_model_kerr",
    "qt_model_ising", "qt_csr_free", "qt_liouvillian_build", "qt_liouv_info", "qt_liouv_export",
    "qt_liouv_destroy", "qt_liouvillian_build_td", "qt_liouv_terms", "qt_mesolve", "qt_mesolve_batch", "qt_me_plan_create", "qt_me_plan_run",
    "qt_me_plan_result", "qt_me_plan_destroy", "qt_me_plan_time_rhs", "qt_me_plan_autotune",
    "qt_me_plan_set_shape", "qt_me_plan_shape", "qt_me_plan_create_steady", "qt_steadystate", "qt_tune_save", "qt_tune_load", "qt_expect", "qt_expect_noalloc", "qt_mcsolve", "qt_mc_plan_create", "qt_mc_plan_run",
    "qt_mc_plan_result", "qt_mc_plan_destroy", "qt_sesolve", "qt_mc_plan_create_td", "qt_mcsolve_td",
    "qt_sesolve_td", "qt_sde_plan_create", "qt_sde_plan_run", "qt_sde_plan_result", "qt_sde_plan_destroy",
    "qt_ssesolve", "qt_smesolve", "qt_server_create", "qt_server_submit", "qt_server_step",
    "qt_server_poll", "qt_server_footprint", "qt_server_destroy",
    "qt_liouv_footprint", "qt_me_plan_workspace", "qt_me_plan_create_ws", "qt_mesolve_ws", "qt_mc_plan_workspace",
    "qt_mc_plan_create_ws", "qt_mcsolve_ws", "qt_server_workspace", "qt_server_create_ws",
    "qt_measure_copy_bandwidth",
    "qt_measure_read_bandwidth",
]


class QtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"qtamd status {code}: {msg}")
        self.code = code


class CSR(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("cols", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("indptr", ctypes.c_void_p), ("indices", ctypes.c_void_p), ("values", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("abstol", ctypes.c_double), ("reltol", ctypes.c_double), ("max_steps", ctypes.c_int64),
                ("h0", ctypes.c_double), ("precision", ctypes.c_int32), ("form", ctypes.c_int32),
                ("steps_per_launch", ctypes.c_int32), ("autotune", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("n_accept", ctypes.c_int64), ("n_reject", ctypes.c_int64), ("n_rhs", ctypes.c_int64),
                ("n_jumps", ctypes.c_int64), ("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("device_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class MeProblem(ctypes.Structure):
    _fields_ = [("L", ctypes.c_void_p), ("rho0", ctypes.c_void_p), ("is_ket", ctypes.c_int32),
                ("n_t", ctypes.c_int32), ("tlist", ctypes.c_void_p), ("n_e", ctypes.c_int32),
                ("e_ops", ctypes.c_void_p)]


class McProblem(ctypes.Structure):
    _fields_ = [("H", ctypes.c_void_p), ("n_c", ctypes.c_int32), ("c_ops", ctypes.c_void_p),
                ("psi0", ctypes.c_void_p), ("n_t", ctypes.c_int32), ("tlist", ctypes.c_void_p),
                ("n_e", ctypes.c_int32), ("e_ops", ctypes.c_void_p), ("ntraj", ctypes.c_int64),
                ("seed", ctypes.c_uint64)]


class SdeProblem(ctypes.Structure):
    _fields_ = [("H", ctypes.c_void_p), ("n_c", ctypes.c_int32), ("c_ops", ctypes.c_void_p),
                ("n_sc", ctypes.c_int32), ("sc_ops", ctypes.c_void_p), ("state0", ctypes.c_void_p),
                ("is_ket", ctypes.c_int32), ("n_t", ctypes.c_int32), ("tlist", ctypes.c_void_p),
                ("n_e", ctypes.c_int32), ("e_ops", ctypes.c_void_p), ("ntraj", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("dt", ctypes.c_double)]


class CsrShape(ctypes.Structure):
    _fields_ = [("lanes_per_row", ctypes.c_int32), ("rows_per_group", ctypes.c_int32),
                ("xcd_order", ctypes.c_int32), ("cached_matrix", ctypes.c_int32)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("pool_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32), ("steps_per_epoch", ctypes.c_int32),
                ("opts", Opts)]


_lib = None


def lib():
    """The loaded libqtamd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2504_21440_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        L.qt_last_error.restype = ctypes.c_char_p
        L.qt_version.restype = ctypes.c_char_p
        for name in EXPORTED:
            if not hasattr(L, name):
                continue
            if name not in ("qt_last_error", "qt_version", "qt_opts_default", "qt_csr_free"):
                getattr(L, name).restype = ctypes.c_int32
        _lib = L
    return _lib


def _check(code):
    if code != QT_OK:
        raise QtError(code, lib().qt_last_error().decode())
    return code


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def opts(abstol=1e-8, reltol=1e-6, max_steps=1_000_000, h0=0.0, precision=F64, form=FORM_CSR, steps_per_launch=0,
         autotune=False):
    return Opts(abstol, reltol, max_steps, h0, precision, form, steps_per_launch, int(bool(autotune)))


class _Ops:
    """Host CSR operators marshalled into a qt_csr array (buffers kept alive by this object)."""

    def __init__(self, ops):
        import scipy.sparse as sp
        self.keep = []
        self.arr = (CSR * max(1, len(ops)))()
        for k, op in enumerate(ops):
            m = sp.csr_matrix(op, dtype=np.complex128)
            ip = np.ascontiguousarray(m.indptr, dtype=np.int64)
            ix = np.ascontiguousarray(m.indices, dtype=np.int32)
            v = np.ascontiguousarray(m.data, dtype=np.complex128)
            self.keep += [ip, ix, v]
            self.arr[k] = CSR(m.shape[0], m.shape[1], m.nnz, ip.ctypes.data, ix.ctypes.data, v.ctypes.data)
        self.n = len(ops)

    @property
    def ptr(self):
        return ctypes.cast(self.arr, ctypes.c_void_p)


def _csr_to_scipy(c):
    import scipy.sparse as sp
    n, nnz = c.rows, c.nnz
    ip = np.ctypeslib.as_array(ctypes.cast(c.indptr, ctypes.POINTER(ctypes.c_int64)), (n + 1,)).copy()
    ix = (np.ctypeslib.as_array(ctypes.cast(c.indices, ctypes.POINTER(ctypes.c_int32)), (nnz,)).copy()
          if nnz else np.zeros(0, np.int32))
    v = (np.ctypeslib.as_array(ctypes.cast(c.values, ctypes.POINTER(ctypes.c_double)), (2 * nnz,)).copy()
         .view(np.complex128) if nnz else np.zeros(0, np.complex128))
    lib().qt_csr_free(ctypes.byref(c))
    return sp.csr_matrix((v, ix, ip), shape=(n, n))


def model_kerr(N, delta, U, F, kappa):
    """Driven Kerr cavity operators built by the library: (H, [c])."""
    H, c = CSR(), CSR()
    _check(lib().qt_model_kerr(N, ctypes.c_double(delta), ctypes.c_double(U), ctypes.c_double(F),
                               ctypes.c_double(kappa), ctypes.byref(H), ctypes.byref(c)))
    return _csr_to_scipy(H), [_csr_to_scipy(c)]


def model_ising(L, J, h, gamma):
    """Open transverse-field Ising chain operators built by the library: (H, [c_0..c_{L-1}])."""
    H = CSR()
    cs = (CSR * L)()
    _check(lib().qt_model_ising(L, ctypes.c_double(J), ctypes.c_double(h), ctypes.c_double(gamma),
                                ctypes.byref(H), cs))
    return _csr_to_scipy(H), [_csr_to_scipy(cs[i]) for i in range(L)]


class Context:
    """A device and stream binding (qt_ctx).  stream: a HIP stream handle (int) or None."""

    def __init__(self, device=0, stream=None):
        self.h = ctypes.c_void_p()
        _check(lib().qt_ctx_create(device, ctypes.c_void_p(stream), ctypes.byref(self.h)))

    def close(self):
        """Destroys the context unless objects created on it are still alive (then a no-op)."""
        if self.h and lib().qt_ctx_destroy(self.h) == QT_OK:
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


COEF_NONE, COEF_CONST, COEF_COS, COEF_EXP, COEF_GAUSS, COEF_TABLE = -1, 0, 1, 2, 3, 4
_COEF_KIND = {None: COEF_NONE, "const": COEF_CONST, "cos": COEF_COS, "exp": COEF_EXP, "gauss": COEF_GAUSS,
              "table": COEF_TABLE}


class Coef(ctypes.Structure):
    """qt_coef: a time-dependent coefficient (see qtamd.h for the kinds)."""
    _fields_ = [("kind", ctypes.c_int32), ("n_table", ctypes.c_int32), ("a", ctypes.c_double * 2),
                ("omega", ctypes.c_double), ("phi", ctypes.c_double), ("t0", ctypes.c_double),
                ("sigma", ctypes.c_double), ("table_t0", ctypes.c_double), ("table_dt", ctypes.c_double),
                ("table", ctypes.c_void_p)]


class _Coefs:
    """Coefficient specifications (dicts with kind, a, omega, phi, t0, sigma, table, table_t0,
    table_dt; None = no coefficient) as qt_coef structs, sample tables kept alive."""

    def __init__(self, specs):
        self.keep = []
        self.arr = (Coef * max(1, len(specs)))()
        for k, c in enumerate(specs):
            if c is None:
                self.arr[k].kind = COEF_NONE
                continue
            a = complex(c.get("a", 1.0))
            e = self.arr[k]
            e.kind = _COEF_KIND[c["kind"]]
            e.a[0], e.a[1] = a.real, a.imag
            e.omega, e.phi = float(c.get("omega", 0.0)), float(c.get("phi", 0.0))
            e.t0, e.sigma = float(c.get("t0", 0.0)), float(c.get("sigma", 1.0))
            e.table_t0, e.table_dt = float(c.get("table_t0", 0.0)), float(c.get("table_dt", 1.0))
            if c["kind"] == "table":
                t = np.ascontiguousarray(np.asarray(c["table"], dtype=np.complex128))
                self.keep.append(t)
                e.n_table, e.table = len(t), t.ctypes.data

    @property
    def ptr(self):
        return ctypes.cast(self.arr, ctypes.c_void_p)


class Liouvillian:
    """qt_liouvillian_build: device Liouvillian (CSR superoperator or dense operator form).

    With h_terms = [(H_i, coef), ...] and / or c_ops entries (C_k, coef), qt_liouvillian_build_td
    builds the time-dependent generator of H(t) = H + sum_i f_i(t) H_i with collapse operators
    g_k(t) C_k; coef is a dict {"kind": "const" | "cos" | "exp" | "gauss" | "table", "a": complex,
    "omega", "phi", "t0", "sigma", "table", "table_t0", "table_dt"}."""

    def __init__(self, ctx, H, c_ops, form=FORM_CSR, precision=F64, h_terms=None):
        self.ctx = ctx
        Hs = _Ops([H])
        cs = [c[0] if isinstance(c, tuple) else c for c in c_ops]
        gs = [c[1] if isinstance(c, tuple) else None for c in c_ops]
        Cs = _Ops(cs)
        self.h = ctypes.c_void_p()
        if h_terms or any(g is not None for g in gs):
            h_terms = h_terms or []
            Ts = _Ops([h for h, _ in h_terms])
            Fs = _Coefs([f for _, f in h_terms])
            Gs = _Coefs(gs)
            _check(lib().qt_liouvillian_build_td(ctx.h, Hs.ptr, len(h_terms), Ts.ptr, Fs.ptr, len(cs), Cs.ptr,
                                                 Gs.ptr, form, precision, ctypes.byref(self.h)))
        else:
            _check(lib().qt_liouvillian_build(ctx.h, Hs.ptr, len(cs), Cs.ptr, form, precision,
                                              ctypes.byref(self.h)))
        self.form, self.precision = form, precision

    def terms(self):
        """Number of time-dependent terms (qt_liouv_terms)."""
        n = ctypes.c_int32()
        _check(lib().qt_liouv_terms(self.h, ctypes.byref(n)))
        return n.value

    def info(self):
        d, nnz, b = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().qt_liouv_info(self.h, ctypes.byref(d), ctypes.byref(nnz), ctypes.byref(b)))
        return d.value, nnz.value, b.value

    def footprint(self):
        """Device bytes the Liouvillian holds (qt_liouv_footprint)."""
        b = ctypes.c_size_t()
        _check(lib().qt_liouv_footprint(self.h, ctypes.byref(b)))
        return b.value

    def export(self):
        import scipy.sparse as sp
        d, nnz, _ = self.info()
        n = d * d
        ip = np.zeros(n + 1, np.int64)
        ix = np.zeros(max(1, nnz), np.int32)
        v = np.zeros(max(1, nnz), np.complex128)
        _check(lib().qt_liouv_export(self.h, _p(ip), _p(ix), _p(v)))
        return sp.csr_matrix((v[:nnz], ix[:nnz], ip), shape=(n, n))

    def close(self):
        if self.h:
            lib().qt_liouv_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def steadystate(ctx, L, rho0, e_ops, tol=1e-9, t_max=1e4, options=None, want_rho=False):
    """qt_steadystate: (expect [n_e] complex, stats dict, rho_ss or None) of the state the master
    equation reaches from rho0 once |L rho|_2 <= tol."""
    r, is_ket = _rho0_array(rho0)
    E = _Ops(e_ops)
    d = L.info()[0]
    ex = np.zeros(max(1, len(e_ops)), np.complex128)
    rho = np.zeros((d, d), np.complex128) if want_rho else None
    st = Stats()
    o = options or opts(precision=L.precision)
    _check(lib().qt_steadystate(ctx.h, L.h, _p(r), is_ket, ctypes.c_double(tol), ctypes.c_double(t_max),
                                len(e_ops), E.ptr, ctypes.byref(o), _p(ex), _p(rho), ctypes.byref(st)))
    return ex[:len(e_ops)], st.as_dict(), rho


def _rho0_array(rho0):
    r = np.ascontiguousarray(rho0, dtype=np.complex128)
    return r, (1 if r.ndim == 1 else 0)


class _MeProblems:
    def __init__(self, problems):
        self.keep = []
        self.arr = (MeProblem * len(problems))()
        self.meta = []
        for i, (L, rho0, tlist, e_ops) in enumerate(problems):
            r, is_ket = _rho0_array(rho0)
            tl = np.ascontiguousarray(tlist, dtype=np.float64)
            E = _Ops(e_ops)
            self.keep += [r, tl, E]
            self.arr[i] = MeProblem(L.h, r.ctypes.data, is_ket, len(tl), tl.ctypes.data, len(e_ops), E.ptr)
            d = L.info()[0]
            self.meta.append((d, len(tl), len(e_ops)))


def _ws(workspace):
    """(device pointer, bytes) of a caller-owned workspace as ctypes arguments."""
    ptr, nbytes = workspace
    return ctypes.c_void_p(int(ptr)), ctypes.c_size_t(int(nbytes))


def mesolve(ctx, L, rho0, tlist, e_ops, options=None, want_final=False, workspace=None):
    """qt_mesolve (qt_mesolve_ws with workspace = (device pointer, bytes)): returns
    (expect [n_e][n_t] complex, stats dict, rho_final or None)."""
    P = _MeProblems([(L, rho0, tlist, e_ops)])
    d, nt, ne = P.meta[0]
    ex = np.zeros((max(ne, 1), nt), np.complex128)
    fin = np.zeros((d, d), np.complex128) if want_final else None
    st = Stats()
    o = options or opts(precision=L.precision)
    if workspace is not None:
        _check(lib().qt_mesolve_ws(ctx.h, ctypes.byref(P.arr[0]), ctypes.byref(o), *_ws(workspace), _p(ex), _p(fin),
                                   ctypes.byref(st)))
    else:
        _check(lib().qt_mesolve(ctx.h, ctypes.byref(P.arr[0]), ctypes.byref(o), _p(ex), _p(fin), ctypes.byref(st)))
    return ex[:ne], st.as_dict(), fin


def me_plan_workspace(ctx, problems, options=None):
    """Device bytes a plan of these problems needs in a caller-owned workspace (qt_me_plan_workspace)."""
    P = _MeProblems(problems)
    o = options or opts(precision=problems[0][0].precision)
    b = ctypes.c_size_t()
    _check(lib().qt_me_plan_workspace(ctx.h, len(problems), P.arr, ctypes.byref(o), ctypes.byref(b)))
    return b.value


class MePlan:
    """qt_me_plan_*: device-resident batch of master-equation problems.  steady_tol > 0: steady-state
    mode (qt_me_plan_create_steady)."""

    def __init__(self, ctx, problems, options=None, steady_tol=0.0, workspace=None):
        self.ctx = ctx  # the context must outlive the plan
        self.P = _MeProblems(problems)
        o = options or opts(precision=problems[0][0].precision)
        self.h = ctypes.c_void_p()
        if workspace is not None:  # (device pointer, bytes) owned by the caller: qt_me_plan_create_ws
            if steady_tol > 0:
                raise ValueError("steady-state plans allocate their own arena")
            _check(lib().qt_me_plan_create_ws(ctx.h, len(problems), self.P.arr, ctypes.byref(o), *_ws(workspace),
                                              ctypes.byref(self.h)))
        elif steady_tol > 0:
            _check(lib().qt_me_plan_create_steady(ctx.h, len(problems), self.P.arr, ctypes.byref(o),
                                                  ctypes.c_double(steady_tol), ctypes.byref(self.h)))
        else:
            _check(lib().qt_me_plan_create(ctx.h, len(problems), self.P.arr, ctypes.byref(o), ctypes.byref(self.h)))

    def run(self):
        _check(lib().qt_me_plan_run(self.h))

    def result(self, i, want_final=False, check=True):
        d, nt, ne = self.P.meta[i]
        ex = np.zeros((max(ne, 1), nt), np.complex128)
        fin = np.zeros((d, d), np.complex128) if want_final else None
        st = Stats()
        rc = lib().qt_me_plan_result(self.h, i, _p(ex), _p(fin), ctypes.byref(st))
        if check:
            _check(rc)
        return ex[:ne], st.as_dict(), fin

    def time_rhs(self, reps=100):
        """Average device milliseconds of one right-hand-side launch (qt_me_plan_time_rhs)."""
        ms = ctypes.c_double()
        _check(lib().qt_me_plan_time_rhs(self.h, int(reps), ctypes.byref(ms)))
        return ms.value

    def autotune(self, reps=20):
        """Measure the candidate tile shapes on this plan and keep the fastest (qt_me_plan_autotune)."""
        _check(lib().qt_me_plan_autotune(self.h, int(reps)))
        return self.shape()

    def set_shape(self, lanes_per_row, rows_per_group, xcd_order=0, cached_matrix=0):
        """Impose a CSR launch shape (qt_me_plan_set_shape)."""
        sh = CsrShape(int(lanes_per_row), int(rows_per_group), int(xcd_order), int(cached_matrix))
        _check(lib().qt_me_plan_set_shape(self.h, ctypes.byref(sh)))

    def shape(self):
        """(lanes per row, rows per lane group, XCD block order, cached matrix, dense waves per
        workgroup of the largest padded size) in use (qt_me_plan_shape)."""
        sh, w = CsrShape(), ctypes.c_int32()
        _check(lib().qt_me_plan_shape(self.h, ctypes.byref(sh), ctypes.byref(w)))
        return sh.lanes_per_row, sh.rows_per_group, sh.xcd_order, sh.cached_matrix, w.value

    def close(self):
        if self.h:
            lib().qt_me_plan_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def measure_copy_bandwidth(ctx, nbytes=2 << 30, reps=20):
    """GB/s (read + write) of the library's streaming copy kernel (qt_measure_copy_bandwidth)."""
    g = ctypes.c_double()
    _check(lib().qt_measure_copy_bandwidth(ctx.h, ctypes.c_int64(int(nbytes)), int(reps), ctypes.byref(g)))
    return g.value


def measure_read_bandwidth(ctx, nbytes=2 << 30, reps=20):
    """GB/s read by the library's streaming read kernel (qt_measure_read_bandwidth)."""
    g = ctypes.c_double()
    _check(lib().qt_measure_read_bandwidth(ctx.h, ctypes.c_int64(int(nbytes)), int(reps), ctypes.byref(g)))
    return g.value


def tune_save(path):
    """Write the process-wide tuning table to a JSON file (qt_tune_save)."""
    _check(lib().qt_tune_save(os.fsencode(path)))


def tune_load(path):
    """Merge a tuning table written by tune_save (qt_tune_load)."""
    _check(lib().qt_tune_load(os.fsencode(path)))


def mesolve_batch(ctx, problems, options=None):
    """qt_mesolve_batch over (L, rho0, tlist, e_ops) tuples: list of (expect, stats)."""
    P = _MeProblems(problems)
    outs = [np.zeros((max(ne, 1), nt), np.complex128) for (d, nt, ne) in P.meta]
    ptrs = (ctypes.c_void_p * len(outs))(*[o.ctypes.data for o in outs])
    sts = (Stats * len(outs))()
    o = options or opts(precision=problems[0][0].precision)
    _check(lib().qt_mesolve_batch(ctx.h, len(outs), P.arr, ctypes.byref(o), ptrs, sts))
    return [(outs[i][:P.meta[i][2]], sts[i].as_dict()) for i in range(len(outs))]


def expect(ctx, O, dev_state_ptr, d, is_ket=False, precision=F64):
    """qt_expect on a device state (pointer as int): Tr(O rho) or <psi|O|psi>/<psi|psi>."""
    E = _Ops([O])
    out = np.zeros(2)
    _check(lib().qt_expect(ctx.h, d, E.ptr, ctypes.c_void_p(dev_state_ptr), int(is_ket), precision, _p(out)))
    return complex(out[0], out[1])


def expect_noalloc(ctx, O, dev_state_ptr, d, is_ket=False, precision=F64):
    """qt_expect_noalloc: the same value as :func:`expect`, staged in the library's fixed device
    scratch array instead of memory allocated per call."""
    E = _Ops([O])
    out = np.zeros(2)
    _check(lib().qt_expect_noalloc(ctx.h, d, E.ptr, ctypes.c_void_p(dev_state_ptr), int(is_ket), precision,
                                   _p(out)))
    return complex(out[0], out[1])


class TdTerms(ctypes.Structure):
    _fields_ = [("n_h", ctypes.c_int32), ("h_terms", ctypes.c_void_p), ("h_coefs", ctypes.c_void_p),
                ("c_coefs", ctypes.c_void_p)]


class _McProblem:
    """c_ops entries are C_k or (C_k, coefficient spec); h_terms = [(H_i, spec)] (qt_td_terms)."""

    def __init__(self, H, c_ops, psi0, tlist, e_ops, ntraj, seed, h_terms=None):
        cs = [c[0] if isinstance(c, tuple) else c for c in c_ops]
        gs = [c[1] if isinstance(c, tuple) else None for c in c_ops]
        h_terms = h_terms or []
        self.H = _Ops([H])
        self.C = _Ops(cs)
        self.E = _Ops(e_ops)
        self.psi0 = np.ascontiguousarray(psi0, dtype=np.complex128)
        self.tl = np.ascontiguousarray(tlist, dtype=np.float64)
        self.s = McProblem(self.H.ptr.value, len(cs), self.C.ptr.value, self.psi0.ctypes.data, len(self.tl),
                           self.tl.ctypes.data, len(e_ops), self.E.ptr.value, int(ntraj), int(seed))
        self.ne, self.nt, self.ntraj = len(e_ops), len(self.tl), int(ntraj)
        self.T = _Ops([h for h, _ in h_terms])
        self.F = _Coefs([f for _, f in h_terms])
        self.G = _Coefs(gs)
        self.td = TdTerms(len(h_terms), self.T.ptr.value, self.F.ptr.value,
                          self.G.ptr.value if any(g is not None for g in gs) else None)


def _mc_outputs(p, want_traj, max_jump_record):
    mean = np.zeros((max(p.ne, 1), p.nt), np.complex128)
    se = np.zeros((max(p.ne, 1), p.nt))
    tr = np.zeros((p.ntraj, max(p.ne, 1), p.nt), np.complex128) if want_traj else None
    nj = np.zeros(p.ntraj, np.int64)
    mj = int(max_jump_record)
    jt = np.zeros((p.ntraj, max(mj, 1))) if mj else None
    jc = np.zeros((p.ntraj, max(mj, 1)), np.int32) if mj else None
    return mean, se, tr, nj, mj, jt, jc


def _mc_pack(p, mean, se, tr, nj, mj, jt, jc, st):
    out = {"mean": mean[:p.ne], "se": se[:p.ne], "njumps": nj, "stats": st.as_dict()}
    if tr is not None:
        out["expect_tr"] = tr[:, :p.ne]
    if mj:
        out["jump_times"] = jt
        out["jump_channels"] = jc
    return out


def mcsolve(ctx, H, c_ops, psi0, tlist, e_ops, ntraj, seed, options=None, want_traj=False, max_jump_record=0,
            h_terms=None):
    """qt_mcsolve (qt_mcsolve_td with h_terms or weighted c_ops): dict with mean, se, njumps, stats
    and optionally per-trajectory data."""
    p = _McProblem(H, c_ops, psi0, tlist, e_ops, ntraj, seed, h_terms)
    mean, se, tr, nj, mj, jt, jc = _mc_outputs(p, want_traj, max_jump_record)
    st = Stats()
    o = options or opts(precision=MIXED)
    if p.td.n_h or p.td.c_coefs:
        _check(lib().qt_mcsolve_td(ctx.h, ctypes.byref(p.s), ctypes.byref(p.td), ctypes.byref(o), _p(mean), _p(se),
                                   _p(tr), _p(nj), mj, _p(jt), _p(jc), ctypes.byref(st)))
    else:
        _check(lib().qt_mcsolve(ctx.h, ctypes.byref(p.s), ctypes.byref(o), _p(mean), _p(se), _p(tr), _p(nj), mj,
                                _p(jt), _p(jc), ctypes.byref(st)))
    return _mc_pack(p, mean, se, tr, nj, mj, jt, jc, st)


def sesolve(ctx, H, psi0, tlist, e_ops, options=None, h_terms=None):
    """qt_sesolve (qt_sesolve_td with h_terms): (expect [n_e][n_t], stats) of the Schrodinger
    evolution of psi0 under H (+ sum_i f_i(t) H_i)."""
    p = _McProblem(H, [], psi0, tlist, e_ops, 1, 0, h_terms)
    ne, nt = len(e_ops), len(tlist)
    ex = np.zeros((max(ne, 1), nt), np.complex128)
    st = Stats()
    o = options or opts(precision=F64)
    vp = ctypes.c_void_p
    if h_terms:
        _check(lib().qt_sesolve_td(ctx.h, vp(p.s.H), ctypes.byref(p.td), vp(p.s.psi0), ctypes.c_int32(p.s.n_t),
                                   vp(p.s.tlist), ctypes.c_int32(p.s.n_e), vp(p.s.e_ops), ctypes.byref(o), _p(ex),
                                   ctypes.byref(st)))
    else:
        _check(lib().qt_sesolve(ctx.h, vp(p.s.H), vp(p.s.psi0), ctypes.c_int32(p.s.n_t), vp(p.s.tlist),
                                ctypes.c_int32(p.s.n_e), vp(p.s.e_ops), ctypes.byref(o), _p(ex), ctypes.byref(st)))
    return ex[:ne], st.as_dict()


def mc_plan_workspace(ctx, H, c_ops, psi0, tlist, e_ops, ntraj, seed, options=None, max_jump_record=0):
    """Device bytes a trajectory plan needs in a caller-owned workspace (qt_mc_plan_workspace)."""
    p = _McProblem(H, c_ops, psi0, tlist, e_ops, ntraj, seed, None)
    o = options or opts(precision=MIXED)
    b = ctypes.c_size_t()
    _check(lib().qt_mc_plan_workspace(ctx.h, ctypes.byref(p.s), ctypes.byref(o), int(max_jump_record),
                                      ctypes.byref(b)))
    return b.value


def mcsolve_ws(ctx, workspace, H, c_ops, psi0, tlist, e_ops, ntraj, seed, options=None, want_traj=False,
               max_jump_record=0):
    """qt_mcsolve_ws: mcsolve in a caller-owned device workspace (device pointer, bytes)."""
    p = _McProblem(H, c_ops, psi0, tlist, e_ops, ntraj, seed, None)
    mean, se, tr, nj, mj, jt, jc = _mc_outputs(p, want_traj, max_jump_record)
    st = Stats()
    o = options or opts(precision=MIXED)
    _check(lib().qt_mcsolve_ws(ctx.h, ctypes.byref(p.s), ctypes.byref(o), *_ws(workspace), _p(mean), _p(se), _p(tr),
                               _p(nj), mj, _p(jt), _p(jc), ctypes.byref(st)))
    return _mc_pack(p, mean, se, tr, nj, mj, jt, jc, st)


class McPlan:
    """qt_mc_plan_*: device-resident trajectory ensemble."""

    def __init__(self, ctx, H, c_ops, psi0, tlist, e_ops, ntraj, seed, options=None, max_jump_record=0,
                 h_terms=None, workspace=None):
        self.ctx = ctx
        self.p = _McProblem(H, c_ops, psi0, tlist, e_ops, ntraj, seed, h_terms)
        o = options or opts(precision=MIXED)
        self.mj = int(max_jump_record)
        self.h = ctypes.c_void_p()
        if workspace is not None:  # (device pointer, bytes) owned by the caller: qt_mc_plan_create_ws
            if self.p.td.n_h or self.p.td.c_coefs:
                raise ValueError("time-dependent trajectory plans allocate their own arena")
            _check(lib().qt_mc_plan_create_ws(ctx.h, ctypes.byref(self.p.s), ctypes.byref(o), self.mj,
                                              *_ws(workspace), ctypes.byref(self.h)))
            return
        _check(lib().qt_mc_plan_create_td(ctx.h, ctypes.byref(self.p.s), ctypes.byref(self.p.td), ctypes.byref(o),
                                          self.mj, ctypes.byref(self.h)))

    def run(self):
        _check(lib().qt_mc_plan_run(self.h))

    def result(self, want_traj=False):
        mean, se, tr, nj, mj, jt, jc = _mc_outputs(self.p, want_traj, self.mj)
        st = Stats()
        _check(lib().qt_mc_plan_result(self.h, _p(mean), _p(se), _p(tr), _p(nj), _p(jt), _p(jc),
                                       ctypes.byref(st)))
        return _mc_pack(self.p, mean, se, tr, nj, mj, jt, jc, st)

    def close(self):
        if self.h:
            lib().qt_mc_plan_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def server_workspace(pool_bytes=16 << 30, max_slots=256, steps_per_epoch=32, options=None):
    """Device bytes of a server's memory region (qt_server_workspace)."""
    o = options or opts(precision=MIXED)
    cfg = ServerCfg(int(pool_bytes), int(max_slots), int(steps_per_epoch), o)
    b = ctypes.c_size_t()
    _check(lib().qt_server_workspace(ctypes.byref(cfg), ctypes.byref(b)))
    return b.value


class Server:
    """qt_server_*: continuous-batching master-equation server."""

    def __init__(self, ctx, pool_bytes=16 << 30, max_slots=256, steps_per_epoch=32, options=None, workspace=None):
        o = options or opts(precision=MIXED)
        self.ctx = ctx
        self.cfg = ServerCfg(int(pool_bytes), int(max_slots), int(steps_per_epoch), o)
        self.h = ctypes.c_void_p()
        if workspace is not None:  # (device pointer, bytes) owned by the caller: qt_server_create_ws
            _check(lib().qt_server_create_ws(ctx.h, ctypes.byref(self.cfg), *_ws(workspace), ctypes.byref(self.h)))
        else:
            _check(lib().qt_server_create(ctx.h, ctypes.byref(self.cfg), ctypes.byref(self.h)))
        self.pending = {}

    def footprint(self, L, rho0, tlist, e_ops):
        P = _MeProblems([(L, rho0, tlist, e_ops)])
        b = ctypes.c_int64()
        _check(lib().qt_server_footprint(self.h, ctypes.byref(P.arr[0]), ctypes.byref(b)))
        return b.value

    def submit(self, L, rho0, tlist, e_ops):
        """Returns a ticket, or None when the request cannot be admitted now (QT_EBUSY)."""
        P = _MeProblems([(L, rho0, tlist, e_ops)])
        t = ctypes.c_uint64()
        rc = lib().qt_server_submit(self.h, ctypes.byref(P.arr[0]), ctypes.byref(t))
        if rc == QT_EBUSY:
            return None
        _check(rc)
        self.pending[t.value] = P.meta[0]
        return t.value

    def step(self):
        na, nf = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().qt_server_step(self.h, ctypes.byref(na), ctypes.byref(nf)))
        return na.value, nf.value

    def poll(self, ticket):
        d, nt, ne = self.pending[ticket]
        ex = np.zeros((max(ne, 1), nt), np.complex128)
        done = ctypes.c_int32()
        st = Stats()
        _check(lib().qt_server_poll(self.h, ctypes.c_uint64(ticket), ctypes.byref(done), _p(ex), ctypes.byref(st)))
        if done.value:
            del self.pending[ticket]
            return ex[:ne], st.as_dict()
        return None

    def close(self):
        if self.h:
            lib().qt_server_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SdePlan:
    """qt_sde_plan_*: stochastic Schrodinger (master=False) or master (master=True) equation under
    homodyne detection, ntraj trajectories with a fixed step of at most dt."""

    def __init__(self, ctx, H, sc_ops, state0, tlist, e_ops, ntraj, seed, dt, c_ops=(), master=False, options=None):
        self.ctx = ctx
        self.H, self.C, self.S, self.E = _Ops([H]), _Ops(list(c_ops)), _Ops(list(sc_ops)), _Ops(list(e_ops))
        self.x0 = np.ascontiguousarray(state0, dtype=np.complex128)
        self.tl = np.ascontiguousarray(tlist, dtype=np.float64)
        self.ne, self.nt, self.m, self.ntraj = len(e_ops), len(self.tl), len(sc_ops), int(ntraj)
        self.s = SdeProblem(self.H.ptr.value, len(c_ops), self.C.ptr.value, len(sc_ops), self.S.ptr.value,
                            self.x0.ctypes.data, 1 if self.x0.ndim == 1 else 0, self.nt, self.tl.ctypes.data,
                            self.ne, self.E.ptr.value, self.ntraj, int(seed), float(dt))
        o = options or opts(precision=MIXED)
        self.h = ctypes.c_void_p()
        _check(lib().qt_sde_plan_create(ctx.h, ctypes.byref(self.s), int(bool(master)), ctypes.byref(o),
                                        ctypes.byref(self.h)))

    def run(self):
        _check(lib().qt_sde_plan_run(self.h))

    def result(self, want_traj=False):
        """dict: mean [n_e][n_t], se, measurement_mean [n_sc][n_t-1], stats, and with want_traj
        expect_tr [ntraj][n_e][n_t] and measurement [ntraj][n_sc][n_t-1]."""
        ne, nt, m, nj = self.ne, self.nt, self.m, self.ntraj
        mean = np.zeros((max(ne, 1), nt), np.complex128)
        se = np.zeros((max(ne, 1), nt))
        tr = np.zeros((nj, max(ne, 1), nt), np.complex128) if want_traj else None
        mm = np.zeros((max(m, 1), max(nt - 1, 1)))
        mt = np.zeros((nj, max(m, 1), max(nt - 1, 1))) if want_traj else None
        st = Stats()
        _check(lib().qt_sde_plan_result(self.h, _p(mean), _p(se), _p(tr), _p(mm), _p(mt), ctypes.byref(st)))
        out = {"mean": mean[:ne], "se": se[:ne], "measurement_mean": mm[:m, :nt - 1], "stats": st.as_dict()}
        if want_traj:
            out["expect_tr"] = tr[:, :ne]
            out["measurement"] = mt[:, :m, :nt - 1]
        return out

    def close(self):
        if self.h:
            lib().qt_sde_plan_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ssesolve(ctx, H, sc_ops, psi0, tlist, e_ops, ntraj, seed, dt, options=None, want_traj=False):
    """Stochastic Schrodinger equation under homodyne detection (qt_sde_plan_* with master = 0)."""
    P = SdePlan(ctx, H, sc_ops, psi0, tlist, e_ops, ntraj, seed, dt, master=False, options=options)
    try:
        P.run()
        return P.result(want_traj)
    finally:
        P.close()


def smesolve(ctx, H, c_ops, sc_ops, rho0, tlist, e_ops, ntraj, seed, dt, options=None, want_traj=False):
    """Stochastic master equation under homodyne detection (qt_sde_plan_* with master = 1)."""
    P = SdePlan(ctx, H, sc_ops, rho0, tlist, e_ops, ntraj, seed, dt, c_ops=c_ops, master=True, options=options)
    try:
        P.run()
        return P.result(want_traj)
    finally:
        P.close()

"""Plain FP64 CPU oracle for the Lindblad master equation and the Monte-Carlo wave-function method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library: the integrator,
right-hand sides, expectation values and random numbers live in ``qtoracle.c`` (plain loops,
complex double), the superoperator in ``liouvillian.py`` (scipy Kronecker products) and the model
operators in ``models.py``.  Each function names the passage of arXiv:2504.21440 it follows in
its docstring or in the C source.

Parity notes: every function here is pinned by a ``-m "not gpu"`` test in ``tests/test_oracle_*.py``
against closed forms, brute-force matrix exponentials, order conditions or invariants, with one
exception inside the integrator: its starting-step heuristic is parity unpinned (see qtoracle.c).
"""
import ctypes
import os
import subprocess

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qtoracle.c")
_LIB = os.path.join(_HERE, "libqtoracle.so")
_lib = None


def build(force=True):
    """Compile the C oracle with gcc (OpenMP over rows and trajectories)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-o", _LIB + ".tmp", _SRC, "-lm"]
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _CSR(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32),
        ("nnz", ctypes.c_int64),
        ("indptr", ctypes.c_void_p),
        ("indices", ctypes.c_void_p),
        ("values", ctypes.c_void_p),
    ]


class Opts(ctypes.Structure):
    _fields_ = [
        ("abstol", ctypes.c_double),
        ("reltol", ctypes.c_double),
        ("max_steps", ctypes.c_int64),
        ("h0", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_accept", ctypes.c_int64),
        ("n_reject", ctypes.c_int64),
        ("n_rhs", ctypes.c_int64),
        ("n_jumps", ctypes.c_int64),
        ("status", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        _lib.or_mesolve.restype = ctypes.c_int32
        _lib.or_mesolve.argtypes = [P, ctypes.c_int32, P, P, ctypes.c_int32, P, ctypes.c_int32, P, P, P, P, P]
        _lib.or_mcsolve.restype = ctypes.c_int32
        _lib.or_mcsolve.argtypes = [P, ctypes.c_int32, P, P, ctypes.c_int32, P, ctypes.c_int32, P, P,
                                    ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, P, P, ctypes.c_int32, P, P,
                                    P, P]
        _lib.or_linear_solve.restype = ctypes.c_int32
        _lib.or_linear_solve.argtypes = [ctypes.c_int64, P, P, ctypes.c_int32, P, P, P, P]
        _lib.or_linear_fixed.restype = None
        _lib.or_linear_fixed.argtypes = [ctypes.c_int64, P, P, ctypes.c_double, ctypes.c_int64, P, P]
        _lib.or_dp5_tableau.argtypes = [P, P, P, P]
        _lib.or_lindblad_apply.argtypes = [P, ctypes.c_int32, P, P, P]
        _lib.or_expect_dm.argtypes = [P, P, P]
        _lib.or_expect_ket.argtypes = [P, P, P]
        _lib.or_philox4x32_10.argtypes = [P, P, P]
        _lib.or_uniform_from_words.restype = ctypes.c_double
        _lib.or_uniform_from_words.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        _lib.or_traj_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, P, P]
        _lib.or_ensemble_stats.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P, P, P]
        _lib.or_mesolve_td.restype = ctypes.c_int32
        _lib.or_mesolve_td.argtypes = [P, ctypes.c_int32, P, P, ctypes.c_int32, P, P, P, ctypes.c_int32, P,
                                       ctypes.c_int32, P, P, P, P, P]
        _lib.or_coef_eval.argtypes = [P, ctypes.c_double, P]
        _lib.or_sdesolve.restype = ctypes.c_int32
        _lib.or_sdesolve.argtypes = [ctypes.c_int32, P, ctypes.c_int32, P, ctypes.c_int32, P, P, ctypes.c_int32, P,
                                     ctypes.c_int32, P, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                                     ctypes.c_int64, P, P]
        _lib.or_wiener_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, P, P]
        _lib.or_mcsolve_td.restype = ctypes.c_int32
        _lib.or_mcsolve_td.argtypes = [P, ctypes.c_int32, P, P, ctypes.c_int32, P, P, P, ctypes.c_int32, P,
                                       ctypes.c_int32, P, P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, P, P,
                                       ctypes.c_int32, P, P, P, P]
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class _OpPack:
    """Keeps the numpy buffers of a list of CSR operators alive while C reads them."""

    def __init__(self, ops):
        self.keep = []
        self.arr = (_CSR * max(1, len(ops)))()
        for k, op in enumerate(ops):
            op = sp.csr_matrix(op, dtype=complex)
            op.sort_indices()
            ip = np.ascontiguousarray(op.indptr, dtype=np.int64)
            ix = np.ascontiguousarray(op.indices, dtype=np.int32)
            vals = np.ascontiguousarray(op.data, dtype=np.complex128)
            self.keep += [ip, ix, vals]
            self.arr[k] = _CSR(op.shape[0], op.nnz, ip.ctypes.data, ix.ctypes.data, vals.ctypes.data)

    @property
    def ptr(self):
        return ctypes.cast(self.arr, ctypes.c_void_p)


class _Coef(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("n_table", ctypes.c_int32),
        ("a_re", ctypes.c_double),
        ("a_im", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("phi", ctypes.c_double),
        ("t0", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("table_t0", ctypes.c_double),
        ("table_dt", ctypes.c_double),
        ("table", ctypes.c_void_p),
    ]


_COEF_KINDS = {None: -1, "const": 0, "cos": 1, "exp": 2, "gauss": 3, "table": 4}


class _CoefPack:
    """Coefficient specifications (dicts: kind, a, omega, phi, t0, sigma, table, table_t0, table_dt;
    None = no coefficient) as the C structs, with their sample tables kept alive."""

    def __init__(self, specs):
        self.keep = []
        self.arr = (_Coef * max(1, len(specs)))()
        for k, c in enumerate(specs):
            if c is None:
                self.arr[k] = _Coef(kind=-1)
                continue
            a = complex(c.get("a", 1.0))
            tab, n = None, 0
            if c["kind"] == "table":
                t = np.ascontiguousarray(np.asarray(c["table"], dtype=np.complex128))
                self.keep.append(t)
                tab, n = t.ctypes.data, len(t)
            self.arr[k] = _Coef(_COEF_KINDS[c["kind"]], n, a.real, a.imag, float(c.get("omega", 0.0)),
                                float(c.get("phi", 0.0)), float(c.get("t0", 0.0)), float(c.get("sigma", 1.0)),
                                float(c.get("table_t0", 0.0)), float(c.get("table_dt", 1.0)), tab)

    @property
    def ptr(self):
        return ctypes.cast(self.arr, ctypes.c_void_p)


def coef_eval(spec, t):
    """The oracle's value of one time-dependent coefficient (Sec. 2, QobjEvo) at time t."""
    lib = _load()
    pk = _CoefPack([spec])
    out = np.zeros(2)
    lib.or_coef_eval(pk.ptr, float(t), _ptr(out))
    return complex(out[0], out[1])


def mesolve_td(H0, h_terms, c_ops, rho0, tlist, e_ops, abstol=1e-8, reltol=1e-6, max_steps=1_000_000, h0=0.0,
               want_final=False):
    """Time-dependent Lindblad master equation (Sec. 3.2 with H(t) = H_0 + sum_i f_i(t) H_i as in the
    QobjEvo of Sec. 2 and the driven example of Sec. 3.4).

    h_terms: list of (H_i, coefficient spec); c_ops: list of C_k or (C_k, spec) for a collapse
    operator g_k(t) C_k (weight |g_k(t)|^2 on its dissipator).  Returns as ``mesolve``."""
    lib = _load()
    rho0 = np.asarray(rho0, dtype=np.complex128)
    if rho0.ndim == 1:
        rho0 = np.outer(rho0, rho0.conj())
    rho0 = np.ascontiguousarray(rho0)
    d = rho0.shape[0]
    tl = np.ascontiguousarray(tlist, dtype=np.float64)
    cs = [c[0] if isinstance(c, tuple) else c for c in c_ops]
    gs = [c[1] if isinstance(c, tuple) else None for c in c_ops]
    Hp = _OpPack([H0])
    Tp = _OpPack([h for h, _ in h_terms])
    Fp = _CoefPack([f for _, f in h_terms])
    Cp = _OpPack(cs)
    Gp = _CoefPack(gs)
    Ep = _OpPack(e_ops)
    ex = np.zeros((len(e_ops), len(tl)), dtype=np.complex128)
    fin = np.zeros((d, d), dtype=np.complex128) if want_final else None
    st = Stats()
    o = opts(abstol, reltol, max_steps, h0)
    rc = lib.or_mesolve_td(Hp.ptr, len(h_terms), Tp.ptr, Fp.ptr, len(cs), Cp.ptr, Gp.ptr, _ptr(rho0), len(tl),
                           _ptr(tl), len(e_ops), Ep.ptr, ctypes.byref(o), _ptr(ex),
                           _ptr(fin) if want_final else None, ctypes.byref(st))
    return ex, st.as_dict(), rc, fin


def tableau():
    """Dormand-Prince 5(4) coefficients (c, A, b, bhat) as used by the oracle integrator."""
    lib = _load()
    c = np.zeros(7)
    a = np.zeros((7, 7))
    b = np.zeros(7)
    bh = np.zeros(7)
    lib.or_dp5_tableau(_ptr(c), _ptr(a), _ptr(b), _ptr(bh))
    return c, a, b, bh


def opts(abstol=1e-8, reltol=1e-6, max_steps=1_000_000, h0=0.0):
    return Opts(abstol, reltol, max_steps, h0)


def linear_solve(M, y0, tlist, abstol=1e-8, reltol=1e-6, max_steps=1_000_000, h0=0.0):
    """Adaptive DP5 integration of y' = M y with the oracle's controller and tstop policy."""
    lib = _load()
    M = np.ascontiguousarray(M, dtype=np.complex128)
    y0 = np.ascontiguousarray(y0, dtype=np.complex128)
    tl = np.ascontiguousarray(tlist, dtype=np.float64)
    out = np.zeros((len(tl), len(y0)), dtype=np.complex128)
    st = Stats()
    o = opts(abstol, reltol, max_steps, h0)
    rc = lib.or_linear_solve(len(y0), _ptr(M), _ptr(y0), len(tl), _ptr(tl), ctypes.byref(o), _ptr(out),
                             ctypes.byref(st))
    return out, st.as_dict(), rc


def linear_fixed(M, y0, h, nsteps):
    """Fixed-step DP5 on y' = M y: returns (y(nsteps*h), last embedded error vector)."""
    lib = _load()
    M = np.ascontiguousarray(M, dtype=np.complex128)
    y0 = np.ascontiguousarray(y0, dtype=np.complex128)
    y = np.zeros_like(y0)
    e = np.zeros_like(y0)
    lib.or_linear_fixed(len(y0), _ptr(M), _ptr(y0), float(h), int(nsteps), _ptr(y), _ptr(e))
    return y, e


def lindblad_apply(H, c_ops, rho):
    """One application of the Lindblad right-hand side (Sec. 3.2) to a dense rho."""
    lib = _load()
    Hp = _OpPack([H])
    Cp = _OpPack(c_ops)
    rho = np.ascontiguousarray(rho, dtype=np.complex128)
    out = np.zeros_like(rho)
    lib.or_lindblad_apply(Hp.ptr, len(c_ops), Cp.ptr, _ptr(rho), _ptr(out))
    return out


def expect_dm(O, rho):
    """Tr(O rho)."""
    lib = _load()
    Op = _OpPack([O])
    rho = np.ascontiguousarray(rho, dtype=np.complex128)
    out = np.zeros(2)
    lib.or_expect_dm(Op.ptr, _ptr(rho), _ptr(out))
    return complex(out[0], out[1])


def expect_ket(O, psi):
    """<psi|O|psi> / <psi|psi>."""
    lib = _load()
    Op = _OpPack([O])
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    out = np.zeros(2)
    lib.or_expect_ket(Op.ptr, _ptr(psi), _ptr(out))
    return complex(out[0], out[1])


def mesolve(H, c_ops, rho0, tlist, e_ops, abstol=1e-8, reltol=1e-6, max_steps=1_000_000, h0=0.0,
            want_final=False):
    """Lindblad master equation (Sec. 3.2) integrated by the oracle's adaptive DP5.

    rho0 may be a ket (turned into |psi><psi|) or a density matrix (used as given).
    Returns (expect [ne][nt] complex, stats dict, status, rho_final or None)."""
    lib = _load()
    rho0 = np.asarray(rho0, dtype=np.complex128)
    if rho0.ndim == 1:
        rho0 = np.outer(rho0, rho0.conj())
    rho0 = np.ascontiguousarray(rho0)
    d = rho0.shape[0]
    tl = np.ascontiguousarray(tlist, dtype=np.float64)
    Hp = _OpPack([H])
    Cp = _OpPack(c_ops)
    Ep = _OpPack(e_ops)
    ex = np.zeros((len(e_ops), len(tl)), dtype=np.complex128)
    fin = np.zeros((d, d), dtype=np.complex128) if want_final else None
    st = Stats()
    o = opts(abstol, reltol, max_steps, h0)
    rc = lib.or_mesolve(Hp.ptr, len(c_ops), Cp.ptr, _ptr(rho0), len(tl), _ptr(tl), len(e_ops), Ep.ptr,
                        ctypes.byref(o), _ptr(ex), _ptr(fin) if want_final else None, ctypes.byref(st))
    return ex, st.as_dict(), rc, fin


def mcsolve(H, c_ops, psi0, tlist, e_ops, ntraj, seed, traj0=0, abstol=1e-8, reltol=1e-6,
            max_steps=1_000_000, h0=0.0, max_jump_record=0):
    """Monte-Carlo wave function (Sec. 3.3) with Philox-4x32-10 draws.

    Returns a dict with per-trajectory expectations ``expect_tr`` [ntraj][ne][nt], ensemble ``mean``
    [ne][nt] (complex), ``se`` [ne][nt] (standard error of the real part), ``njumps``, ``status``,
    and optionally the first ``max_jump_record`` jump times and channels."""
    return mcsolve_td(H, [], c_ops, psi0, tlist, e_ops, ntraj, seed, traj0, abstol, reltol, max_steps, h0,
                      max_jump_record)


def mcsolve_td(H, h_terms, c_ops, psi0, tlist, e_ops, ntraj, seed, traj0=0, abstol=1e-8, reltol=1e-6,
               max_steps=1_000_000, h0=0.0, max_jump_record=0):
    """Monte-Carlo wave function (Sec. 3.3) with the time-dependent operators of Sec. 2 (QobjEvo):
    H(t) = H + sum_i f_i(t) H_i with h_terms = [(H_i, spec)], and c_ops entries C_k or (C_k, spec)
    for a collapse operator g_k(t) C_k: H_eff(t) = H(t) - (i/2) sum_k |g_k(t)|^2 C_k^dag C_k and a jump
    at t* picks channel k with weight |g_k(t*)|^2 |C_k psi|^2.  Returns as ``mcsolve``."""
    lib = _load()
    psi0 = np.ascontiguousarray(psi0, dtype=np.complex128)
    tl = np.ascontiguousarray(tlist, dtype=np.float64)
    cs = [c[0] if isinstance(c, tuple) else c for c in c_ops]
    gs = [c[1] if isinstance(c, tuple) else None for c in c_ops]
    Hp = _OpPack([H])
    Tp = _OpPack([h for h, _ in h_terms])
    Fp = _CoefPack([f for _, f in h_terms])
    Cp = _OpPack(cs)
    Gp = _CoefPack(gs)
    Ep = _OpPack(e_ops)
    ne, nt = len(e_ops), len(tl)
    ex = np.zeros((ntraj, ne, nt), dtype=np.complex128)
    nj = np.zeros(ntraj, dtype=np.int64)
    stt = np.zeros(ntraj, dtype=np.int32)
    mj = int(max_jump_record)
    jt = np.zeros((ntraj, max(mj, 1)))
    jc = np.zeros((ntraj, max(mj, 1)), dtype=np.int32)
    nrhs = ctypes.c_int64(0)
    o = opts(abstol, reltol, max_steps, h0)
    rc = lib.or_mcsolve_td(Hp.ptr, len(h_terms), Tp.ptr, Fp.ptr, len(cs), Cp.ptr,
                           Gp.ptr if any(g is not None for g in gs) else None, _ptr(psi0), nt, _ptr(tl), ne,
                           Ep.ptr, ctypes.byref(o), ctypes.c_uint64(seed), ctypes.c_uint64(traj0),
                           ctypes.c_int64(ntraj), _ptr(ex), _ptr(nj), mj, _ptr(jt), _ptr(jc), _ptr(stt),
                           ctypes.byref(nrhs))
    mean = np.zeros((ne, nt), dtype=np.complex128)
    se = np.zeros((ne, nt))
    lib.or_ensemble_stats(ntraj, ne, nt, _ptr(ex), _ptr(mean), _ptr(se))
    out = {"expect_tr": ex, "mean": mean, "se": se, "njumps": nj, "status": stt, "rc": rc,
           "n_rhs": nrhs.value}
    if mj:
        out["jump_times"] = jt
        out["jump_channels"] = jc
    return out


def sesolve(H, psi0, tlist, e_ops, abstol=1e-8, reltol=1e-6, max_steps=1_000_000, h0=0.0):
    """Schrodinger equation (Sec. 3.1, sesolve): d psi/dt = -i H psi, integrated by the same DP5
    stepping as mcsolve; with no collapse operators no jump can happen, so one trajectory is the
    solution.  Returns (expect [ne][nt], status)."""
    out = mcsolve(H, [], psi0, tlist, e_ops, 1, 0, abstol=abstol, reltol=reltol, max_steps=max_steps, h0=h0)
    return out["expect_tr"][0], int(out["status"][0])


def sesolve_td(H, h_terms, psi0, tlist, e_ops, abstol=1e-8, reltol=1e-6, max_steps=1_000_000, h0=0.0):
    """Schrodinger equation with H(t) = H + sum_i f_i(t) H_i: the no-collapse trajectory.
    Returns (expect [ne][nt], status)."""
    out = mcsolve_td(H, h_terms, [], psi0, tlist, e_ops, 1, 0, abstol=abstol, reltol=reltol, max_steps=max_steps,
                     h0=h0)
    return out["expect_tr"][0], int(out["status"][0])


def _sdesolve(sme, H, c_ops, sc_ops, x0, tlist, e_ops, ntraj, seed, dt, traj0):
    lib = _load()
    x0 = np.ascontiguousarray(x0, dtype=np.complex128)
    tl = np.ascontiguousarray(tlist, dtype=np.float64)
    Hp, Cp, Sp, Ep = _OpPack([H]), _OpPack(c_ops), _OpPack(sc_ops), _OpPack(e_ops)
    ne, nt, m = len(e_ops), len(tl), len(sc_ops)
    ex = np.zeros((ntraj, ne, nt), dtype=np.complex128)
    meas = np.zeros((ntraj, m, max(nt - 1, 0)))
    rc = lib.or_sdesolve(int(sme), Hp.ptr, len(c_ops), Cp.ptr, m, Sp.ptr, _ptr(x0), nt, _ptr(tl), ne, Ep.ptr,
                         float(dt), ctypes.c_uint64(seed), ctypes.c_uint64(traj0), ctypes.c_int64(ntraj), _ptr(ex),
                         _ptr(meas))
    mean = np.zeros((ne, nt), dtype=np.complex128)
    se = np.zeros((ne, nt))
    lib.or_ensemble_stats(ntraj, ne, nt, _ptr(ex), _ptr(mean), _ptr(se))
    return {"expect_tr": ex, "mean": mean, "se": se, "measurement": meas, "measurement_mean": meas.mean(axis=0),
            "rc": rc}


def ssesolve(H, sc_ops, psi0, tlist, e_ops, ntraj, seed, dt, traj0=0):
    """Stochastic Schrodinger equation under homodyne detection (Sec. 3.5, Ito form) with a fixed
    step of at most dt.  Returns expect_tr [ntraj][ne][nt], mean, se, measurement [ntraj][nsc][nt-1]
    (the current J_n = <S_n + S_n^dag> + dW_n/dt averaged over each tlist interval)."""
    psi0 = np.asarray(psi0, dtype=np.complex128)
    return _sdesolve(0, H, [], sc_ops, psi0, tlist, e_ops, ntraj, seed, dt, traj0)


def smesolve(H, c_ops, sc_ops, rho0, tlist, e_ops, ntraj, seed, dt, traj0=0):
    """Stochastic master equation under homodyne detection (Sec. 3.5, Ito form); rho0 a density
    matrix or a ket.  Returns as ``ssesolve``."""
    rho0 = np.asarray(rho0, dtype=np.complex128)
    if rho0.ndim == 1:
        rho0 = np.outer(rho0, rho0.conj())
    return _sdesolve(1, H, c_ops, sc_ops, rho0, tlist, e_ops, ntraj, seed, dt, traj0)


def wiener_normals(seed, traj, step, pair):
    """The two standard normals behind Wiener increments 2*pair and 2*pair + 1 of a step."""
    a, b = ctypes.c_double(), ctypes.c_double()
    _load().or_wiener_normals(ctypes.c_uint64(seed), ctypes.c_uint64(traj), ctypes.c_uint32(step),
                              ctypes.c_uint32(pair), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def steadystate(H, c_ops):
    """Steady state of the Lindblad master equation (Sec. 3.2, steadystate): the density matrix with
    L rho = 0 and Tr rho = 1, from its definition as a linear system -- the Kronecker Liouvillian of
    ``liouvillian.py`` with the trace condition added as an extra equation -- solved by a sparse
    direct factorisation (scipy's spsolve on the normal equations is avoided: the system is square
    because the equation of rho_00 is replaced by the trace row, which is valid when the steady state
    is unique).  Returns the d x d density matrix."""
    import scipy.sparse.linalg as spl
    from oracle import liouvillian as ol
    L = ol.liouvillian(H, c_ops).tolil()
    n = L.shape[0]
    d = int(round(np.sqrt(n)))
    L[0, :] = 0.0
    for i in range(d):
        L[0, i * d + i] = 1.0
    b = np.zeros(n, dtype=complex)
    b[0] = 1.0
    x = spl.spsolve(L.tocsc(), b)
    return x.reshape(d, d)


def ensemble_stats(expect_tr):
    lib = _load()
    ex = np.ascontiguousarray(expect_tr, dtype=np.complex128)
    ntraj, ne, nt = ex.shape
    mean = np.zeros((ne, nt), dtype=np.complex128)
    se = np.zeros((ne, nt))
    lib.or_ensemble_stats(ntraj, ne, nt, _ptr(ex), _ptr(mean), _ptr(se))
    return mean, se


def philox(ctr, key):
    """Philox-4x32-10 block: four uint32 words."""
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.or_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform_from_words(w0, w1):
    return _load().or_uniform_from_words(int(w0), int(w1))


def traj_draw(seed, traj, event):
    """The two uniforms a trajectory draws at an event (event 0: first threshold)."""
    lib = _load()
    a = ctypes.c_double()
    b = ctypes.c_double()
    lib.or_traj_draw(ctypes.c_uint64(seed), ctypes.c_uint64(traj), ctypes.c_uint32(event), ctypes.byref(a),
                     ctypes.byref(b))
    return a.value, b.value

"""GPU parity of the time-dependent master equation (H(t) = H_0 + sum_i f_i(t) H_i, collapse
operators g_k(t) C_k; the QobjEvo of Sec. 2 and the driven example of Sec. 3.4) against the FP64
oracle.  Bars: max |d<O>| <= 1e-6 in FP64 mode, <= 1e-4 in mixed FP32/FP64 mode; the assembled
terms against their Kronecker definitions to rounding; a constant problem bitwise the same inside a
plan that takes the weighted kernels."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import liouvillian as ol
from oracle import models as om
import workloads
import paper_2504_21440_amd as qt

pytestmark = pytest.mark.gpu
TAG = 26


@pytest.fixture(scope="module")
def ctx():
    print("[gpu] creating context", flush=True)
    c = qt.Context(0)
    yield c
    c.close()


def _cavity():
    p = workloads.driven_cavity_td()
    N, w = p["N"], p["omega"]
    a = om.destroy(N)
    H0 = p["omega0"] * om.number(N)
    terms = [(a.conj().T.tocsr(), {"kind": "exp", "a": p["F"], "omega": -w}),
             (a, {"kind": "exp", "a": p["F"], "omega": w})]
    return p, H0, terms, [np.sqrt(p["kappa"]) * a], [om.number(N), a]


def _commutator_super(H):
    H = sp.csr_matrix(H, dtype=complex)
    Id = sp.identity(H.shape[0], dtype=complex, format="csr")
    return -1j * (sp.kron(H, Id) - sp.kron(Id, H.T))


def test_td_assembly_terms_match_definitions(ctx):
    """The stored CSR lists, row by row, the constant part, each -i[H_i, .] and each weighted D[C_k],
    the term number above bit 26 of the column."""
    print("[gpu] TD assembly vs Kronecker definitions", flush=True)
    g = np.random.default_rng(12)
    d = 5
    X = g.normal(size=(d, d)) + 1j * g.normal(size=(d, d))
    H0 = sp.csr_matrix(X + X.conj().T)
    H1 = sp.csr_matrix(g.normal(size=(d, d)) + 1j * g.normal(size=(d, d)))  # not Hermitian
    C0 = sp.csr_matrix(g.normal(size=(d, d)))
    C1 = sp.csr_matrix(g.normal(size=(d, d)) + 1j * g.normal(size=(d, d)))
    want = [ol.liouvillian(H0, [C0]), _commutator_super(H1), ol.liouvillian(0 * H0, [C1])]
    for prec, tol in [(qt.F64, 1e-13), (qt.MIXED, 2e-6)]:
        L = qt.Liouvillian(ctx, H0, [C0, (C1, {"kind": "cos", "a": 1.0, "omega": 1.0})], qt.FORM_CSR, prec,
                           h_terms=[(H1, {"kind": "exp", "a": 0.5, "omega": 2.0})])
        assert L.terms() == 2
        got = L.export()
        tags = got.indices >> TAG
        n = d * d
        for k, ref in enumerate(want):
            sel = got.copy()
            sel.data = np.where(tags == k, got.data, 0)
            sel.indices = got.indices & ((1 << TAG) - 1)
            sel = sp.csr_matrix((sel.data, sel.indices, sel.indptr), shape=(n, n))
            sel.sum_duplicates()
            diff = abs(sel - ref).max()
            assert diff <= tol * max(1.0, abs(ref).max()), (prec, k, diff)
        # within each row the terms follow one another in order
        for r in range(n):
            t = tags[got.indptr[r]:got.indptr[r + 1]]
            assert np.all(np.diff(t) >= 0)
        L.close()


@pytest.mark.parametrize("prec,tol", [(qt.F64, 1e-6), (qt.MIXED, 1e-4)])
def test_td_rotating_drive_cavity(ctx, prec, tol):
    """Complex-exponential drive: closed form (frame rotating with the drive) and the oracle."""
    print(f"[gpu] TD driven cavity prec={prec}", flush=True)
    p, H0, terms, c, e_ops = _cavity()
    tl = workloads.tlist(p["t_end"], p["nt"])
    ref = oracle.mesolve_td(H0, terms, c, om.fock_dm(p["N"], 0), tl, e_ops)[0]
    L = qt.Liouvillian(ctx, H0, c, qt.FORM_CSR, prec, h_terms=terms)
    ex, st, _ = qt.mesolve(ctx, L, om.fock_dm(p["N"], 0), tl, e_ops, qt.opts(precision=prec))
    assert st["status"] == 0
    assert np.abs(ex - ref).max() <= tol, np.abs(ex - ref).max()
    z = 1j * (p["omega0"] - p["omega"]) + 0.5 * p["kappa"]
    alpha = (-1j * p["F"] / z) * (1.0 - np.exp(-z * tl))
    assert np.abs(ex[0].real - np.abs(alpha) ** 2).max() <= 1e-4
    assert np.abs(ex[1] - np.exp(-1j * p["omega"] * tl) * alpha).max() <= 1e-4
    L.close()


def _sx_case(kind):
    if kind == "cos":
        return {"kind": "cos", "a": 0.8, "omega": 2.5, "phi": 0.4}
    if kind == "gauss":
        return {"kind": "gauss", "a": 1.1, "t0": 2.0, "sigma": 0.6, "omega": 1.5}
    if kind == "const":
        return {"kind": "const", "a": 0.7 + 0.0j}
    g = np.random.default_rng(3)
    return {"kind": "table", "table": g.uniform(-1.0, 1.0, 12), "table_t0": 0.5, "table_dt": 0.35}


@pytest.mark.parametrize("kind", ["cos", "gauss", "table", "const"])
def test_td_coefficient_kinds_vs_oracle(ctx, kind):
    """Each coefficient kind on a damped qubit with a sigma_x drive (dissipation makes the states
    mixed), FP64 and mixed against the oracle."""
    spec = _sx_case(kind)
    H0 = 0.5 * 1.3 * om.sigmaz()
    c = [np.sqrt(0.2) * om.sigmam()]
    tl = np.linspace(0.0, 4.0, 33)
    rho0 = np.diag([1.0, 0.0]).astype(complex)
    e_ops = [om.sigmaz(), om.sigmam()]
    ref = oracle.mesolve_td(H0, [(om.sigmax(), spec)], c, rho0, tl, e_ops)[0]
    for prec, tol in [(qt.F64, 1e-6), (qt.MIXED, 1e-4)]:
        print(f"[gpu] TD kind={kind} prec={prec}", flush=True)
        L = qt.Liouvillian(ctx, H0, c, qt.FORM_CSR, prec, h_terms=[(om.sigmax(), spec)])
        ex, st, _ = qt.mesolve(ctx, L, rho0, tl, e_ops, qt.opts(precision=prec))
        assert st["status"] == 0
        assert np.abs(ex - ref).max() <= tol, (prec, np.abs(ex - ref).max())
        L.close()


def test_td_collapse_weights_vs_oracle(ctx):
    """Weighted collapse operators (|g(t)|^2 D[C]) together with constant ones."""
    N = 10
    H, c = om.kerr(N, 1.0, 0.5, 0.8, 1.0)
    a = om.destroy(N)
    c_ops = [(c[0], {"kind": "gauss", "a": 1.0 + 0.5j, "t0": 1.5, "sigma": 0.8}), 0.3 * (a @ a).tocsr()]
    tl = workloads.tlist(4.0, 21)
    ref = oracle.mesolve_td(H, [], c_ops, om.fock_dm(N, 0), tl, [om.number(N)])[0]
    for prec, tol in [(qt.F64, 1e-6), (qt.MIXED, 1e-4)]:
        print(f"[gpu] TD collapse weights prec={prec}", flush=True)
        L = qt.Liouvillian(ctx, H, c_ops, qt.FORM_CSR, prec)
        assert L.terms() == 1
        ex, st, _ = qt.mesolve(ctx, L, om.fock_dm(N, 0), tl, [om.number(N)], qt.opts(precision=prec))
        assert st["status"] == 0
        assert np.abs(ex - ref).max() <= tol, (prec, np.abs(ex - ref).max())
        L.close()


SHAPES = [(l, r) for l in (4, 8, 16) for r in (1, 2, 4) if r <= l]
WIDE = [(4, 1), (8, 1), (8, 2), (16, 1)]  # also built with 16-byte matrix loads (cached_matrix = 2)


def test_td_optomechanics_every_launch_form_vs_oracle(ctx):
    """The driven optomechanical system (cos drive on a + a^dag) over a short window, solved alone
    (descriptor in the kernel arguments) and in a batch with a second drive frequency (block table),
    matrix streamed and cached, for every tile shape, against the oracle."""
    base = workloads.optomech_td(t_end=15.0, nt=16)
    ps = [dict(base, Nc=6, Nm=4), dict(base, Nc=6, Nm=4, wd=1.1)]
    refs, probs = [], {qt.F64: [], qt.MIXED: []}
    for p in ps:
        H0, xa, c, n_op = om.optomech(p["Nc"], p["Nm"], p["wc"], p["wm"], p["g"], p["kappa"], p["gamma"])
        d = p["Nc"] * p["Nm"]
        rho0 = np.zeros((d, d), complex)
        rho0[0, 0] = 1.0
        spec = {"kind": "cos", "a": p["F"], "omega": p["wd"]}
        tl = workloads.tlist(p["t_end"], p["nt"])
        refs.append(oracle.mesolve_td(H0, [(xa, spec)], c, rho0, tl, [n_op])[0])
        for prec in (qt.F64, qt.MIXED):
            L = qt.Liouvillian(ctx, H0, c, qt.FORM_CSR, prec, h_terms=[(xa, spec)])
            probs[prec].append((L, rho0, tl, [n_op]))
    for prec, tol in [(qt.F64, 1e-6), (qt.MIXED, 1e-4)]:
        for sel in ([0], [0, 1]):
            plan = qt.MePlan(ctx, [probs[prec][i] for i in sel], qt.opts(precision=prec))
            for (lpr, rg), keep in [(sh, k) for k in (0, 1) for sh in SHAPES] + [(sh, 2) for sh in WIDE]:
                print(f"[gpu] TD optomech n={len(sel)} lpr={lpr} rg={rg} keep={keep} prec={prec}", flush=True)
                plan.set_shape(lpr, rg, 0, keep)
                plan.run()
                for j, i in enumerate(sel):
                    ex, st, _ = plan.result(j)
                    assert st["status"] == 0
                    assert np.abs(ex - refs[i]).max() <= tol, (prec, sel, lpr, rg, keep, np.abs(ex - refs[i]).max())
            plan.close()


@pytest.mark.parametrize("prec,tol", [(qt.F64, 1e-6), (qt.MIXED, 1e-4)])
def test_td_optomechanics_example_at_benched_size(ctx, prec, tol):
    """The optomechanical example exactly as benchmarked (cavity cutoff 10, mechanical cutoff 7:
    n = 4,900; t in [0, 5 / kappa] = [0, 500], 5,000 saves; default tolerances; the shipped tuning
    table and autotuner picking the launch shape) against the stored FP64 oracle solution."""
    import json
    import os
    print(f"[gpu] TD optomech example at benched size prec={prec}", flush=True)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    qt.tune_load(os.path.join(root, "paper_2504_21440_amd", "tuning", "mi355x.json"))
    p = workloads.optomech_td()
    H0, xa, c, n_op = om.optomech(p["Nc"], p["Nm"], p["wc"], p["wm"], p["g"], p["kappa"], p["gamma"])
    d = p["Nc"] * p["Nm"]
    rho0 = np.zeros((d, d), complex)
    rho0[0, 0] = 1.0
    L = qt.Liouvillian(ctx, H0, c, qt.FORM_CSR, prec, h_terms=[(xa, {"kind": "cos", "a": p["F"], "omega": p["wd"]})])
    plan = qt.MePlan(ctx, [(L, rho0, workloads.tlist(p["t_end"], p["nt"]), [n_op])],
                     qt.opts(precision=prec, autotune=True))
    plan.run()
    ex, st, _ = plan.result(0)
    plan.close()
    L.close()
    with open(os.path.join(root, "tests", "golden", "optomech_full.json")) as f:
        g = json.load(f)
    ref = np.array(g["expect_re"]) + 1j * np.array(g["expect_im"])
    assert st["status"] == 0
    err = np.abs(ex - ref).max()
    print(f"[gpu]   max |d<a^dag a>| = {err:.2e} over {p['nt']} saves, {st['n_accept']} steps", flush=True)
    assert err <= tol


def test_td_plan_keeps_constant_problems_bitwise(ctx):
    """A constant problem in a plan that also holds a time-dependent one runs through the weighted
    kernels with the coefficient 1: its results equal those of the constant-only plan bit for bit."""
    print("[gpu] TD plan: constant problem bitwise", flush=True)
    H, cs = qt.model_ising(4, 1.0, 0.7, 0.2)
    e_ops = [om.site_op(4, 0, om.sigmaz())]
    tl = np.linspace(0, 4, 21)
    p, H0, terms, c, ce = _cavity()
    for prec in (qt.F64, qt.MIXED):
        Lc = qt.Liouvillian(ctx, H, cs, qt.FORM_CSR, prec)
        Ltd = qt.Liouvillian(ctx, H0, c, qt.FORM_CSR, prec, h_terms=terms)
        out = []
        for prs in ([(Lc, om.all_up_ket(4), tl, e_ops)],
                    [(Lc, om.all_up_ket(4), tl, e_ops), (Ltd, om.fock_dm(p["N"], 0), tl, ce)]):
            plan = qt.MePlan(ctx, prs, qt.opts(precision=prec))
            plan.set_shape(8, 1)
            plan.run()
            out.append(plan.result(0))
            plan.close()
        np.testing.assert_array_equal(out[0][0], out[1][0])
        assert out[0][1]["n_accept"] == out[1][1]["n_accept"]


def test_td_error_paths(ctx):
    print("[gpu] TD error paths", flush=True)
    p, H0, terms, c, _ = _cavity()
    with pytest.raises(qt.QtError) as e:
        qt.Liouvillian(ctx, H0, c, qt.FORM_DENSE, qt.MIXED, h_terms=terms)
    assert e.value.code == qt.QT_EINVAL
    with pytest.raises(qt.QtError):
        qt.Liouvillian(ctx, H0, c, qt.FORM_CSR, qt.F64, h_terms=[(terms[0][0], {"kind": "gauss", "sigma": 0.0})])
    with pytest.raises(qt.QtError):
        qt.Liouvillian(ctx, H0, c, qt.FORM_CSR, qt.F64,
                       h_terms=[(terms[0][0], {"kind": "table", "table": [], "table_dt": 1.0})])
    with pytest.raises(qt.QtError):
        qt.Liouvillian(ctx, H0, c, qt.FORM_CSR, qt.F64, h_terms=[(terms[0][0], {"kind": "cos"})] * 32)
    L = qt.Liouvillian(ctx, H0, c, qt.FORM_CSR, qt.MIXED, h_terms=terms)
    srv = qt.Server(ctx, pool_bytes=1 << 26, max_slots=4)
    with pytest.raises(qt.QtError) as e:
        srv.submit(L, om.fock_dm(p["N"], 0), np.linspace(0, 1, 3), [])
    assert e.value.code == qt.QT_EINVAL
    srv.close()
    L.close()


# --------------------------------------------------------------------------------------------
# Time-dependent trajectories and Schrodinger evolution
# --------------------------------------------------------------------------------------------
@pytest.mark.parametrize("prec,tol", [(qt.F64, 1e-6), (qt.MIXED, 1e-4)])
def test_td_sesolve_rotating_qubit(ctx, prec, tol):
    """Rabi oscillation under a rotating drive: the oracle and the closed form of the rotating frame."""
    print(f"[gpu] TD sesolve rotating qubit prec={prec}", flush=True)
    w0, w, W = 4.0, 4.4, 1.3
    sz, sm = om.sigmaz(), om.sigmam()
    terms = [(sm.conj().T.tocsr(), {"kind": "exp", "a": 0.5 * W, "omega": -w}),
             (sm, {"kind": "exp", "a": 0.5 * W, "omega": w})]
    tl = np.linspace(0.0, 8.0, 41)
    psi0 = np.array([1, 0], complex)
    ref = oracle.sesolve_td(0.5 * w0 * sz, terms, psi0, tl, [sz, sm])[0]
    ex, st = qt.sesolve(ctx, 0.5 * w0 * sz, psi0, tl, [sz, sm], qt.opts(precision=prec), h_terms=terms)
    assert st["status"] == 0
    assert np.abs(ex - ref).max() <= tol, np.abs(ex - ref).max()
    WR = np.hypot(W, w0 - w)
    assert np.abs(ex[0].real - (1 - 2 * (W / WR) ** 2 * np.sin(WR * tl / 2) ** 2)).max() <= max(tol, 1e-5)


def test_td_weighted_decay_jump_times_exact(ctx):
    """One collapse operator sqrt(g0) cos(om t) sigma_-: trajectory j jumps where
    g0 (t/2 + sin(2 om t) / (4 om)) = -ln r0 (FP64, tight tolerances), as the oracle does."""
    import scipy.optimize as so
    print("[gpu] TD weighted decay jump times", flush=True)
    g0, om_ = 0.4, 1.7
    Lam = lambda t: g0 * (0.5 * t + np.sin(2 * om_ * t) / (4 * om_))
    tl = np.linspace(0, 10, 21)
    seed = 31
    H = sp.csr_matrix((2, 2), dtype=complex)
    c = [(om.sigmam(), {"kind": "cos", "a": np.sqrt(g0), "omega": om_})]
    res = qt.mcsolve(ctx, H, c, np.array([1, 0], complex), tl, [om.sigmaz()], 48, seed,
                     options=qt.opts(abstol=1e-12, reltol=1e-10, precision=qt.F64), want_traj=True,
                     max_jump_record=2)
    seen = 0
    for j in range(48):
        r0, _ = oracle.traj_draw(seed, j, 0)
        target = -np.log(r0)
        if Lam(tl[-1]) > target:
            tstar = so.brentq(lambda t: Lam(t) - target, 0.0, tl[-1], xtol=1e-14)
            assert res["njumps"][j] == 1
            assert abs(res["jump_times"][j, 0] - tstar) < 1e-7
            seen += 1
        else:
            assert res["njumps"][j] == 0
    assert seen > 10


def _td_kerr():
    N = 8
    a = om.destroy(N)
    ad = a.conj().T
    H0 = (2.0 * om.number(N) + 0.5 * (ad @ ad @ a @ a)).tocsr()
    terms = [(ad.tocsr(), {"kind": "exp", "a": 0.6, "omega": -1.5}), (a, {"kind": "exp", "a": 0.6, "omega": 1.5})]
    c_ops = [np.sqrt(0.3) * a, (a, {"kind": "gauss", "a": 0.8, "t0": 2.0, "sigma": 1.0})]
    return N, H0, terms, c_ops


@pytest.mark.parametrize("prec", [qt.F64, qt.MIXED])
def test_td_trajectory_parity_with_oracle(ctx, prec):
    """Same seed, same time-dependent trajectories: jump counts, channels, times and expectations
    equal the oracle's in FP64; in mixed precision nearly every trajectory jumps alike."""
    print(f"[gpu] TD trajectory parity prec={prec}", flush=True)
    N, H0, terms, c_ops = _td_kerr()
    psi0 = np.eye(N, dtype=complex)[0]
    tl = np.linspace(0, 5, 11)
    n, seed = 48, 13
    ref = oracle.mcsolve_td(H0, terms, c_ops, psi0, tl, [om.number(N)], n, seed, max_jump_record=8)
    res = qt.mcsolve(ctx, H0, c_ops, psi0, tl, [om.number(N)], n, seed, options=qt.opts(precision=prec),
                     want_traj=True, max_jump_record=8, h_terms=terms)
    assert ref["njumps"].sum() > n  # the weighted channel and the drive make jumps happen
    if prec == qt.F64:
        np.testing.assert_array_equal(res["njumps"], ref["njumps"])
        for j in range(n):
            m = min(8, int(ref["njumps"][j]))
            np.testing.assert_array_equal(res["jump_channels"][j, :m], ref["jump_channels"][j, :m])
            assert np.abs(res["jump_times"][j, :m] - ref["jump_times"][j, :m]).max(initial=0) < 1e-8
        assert np.abs(res["expect_tr"] - ref["expect_tr"]).max() < 1e-6
    else:
        assert (res["njumps"] == ref["njumps"]).mean() > 0.9


def test_td_ensemble_matches_td_master_equation(ctx):
    """Sec. 3.3 with time-dependent operators: 4,000 mixed-precision trajectories against the oracle's
    time-dependent master equation, within 4 standard errors."""
    print("[gpu] TD ensemble vs TD master equation", flush=True)
    N, H0, terms, c_ops = _td_kerr()
    tl = np.linspace(0, 5, 11)
    me = oracle.mesolve_td(H0, terms, c_ops, om.fock_dm(N, 0), tl, [om.number(N)])[0][0].real
    res = qt.mcsolve(ctx, H0, c_ops, np.eye(N, dtype=complex)[0], tl, [om.number(N)], 4000, 21,
                     options=qt.opts(abstol=1e-8, reltol=1e-6, precision=qt.MIXED), h_terms=terms)
    mean, se = res["mean"][0].real, res["se"][0]
    z = np.abs(mean - me)[1:] / np.maximum(se[1:], 1e-12)
    print(f"[gpu]   max z = {z.max():.2f}", flush=True)
    assert (z > 3).sum() <= 1 and z.max() < 4.5


@pytest.mark.parametrize("prec", [qt.F64, qt.MIXED])
def test_td_folded_step_control_is_bitwise_the_control_kernel(ctx, prec):
    """A time-dependent problem folds its step control, and the coefficient rows of the next step,
    into stage 2 at an even number of steps per graph; an odd number keeps the control kernel.
    Solutions, save times and step counts agree bitwise (with rejected steps from a first step far
    too large), and match the oracle."""
    print(f"[gpu] TD folded step control, prec={prec}", flush=True)
    p, H0, terms, c, e_ops = _cavity()
    tl = workloads.tlist(p["t_end"], p["nt"])
    L = qt.Liouvillian(ctx, H0, c, qt.FORM_CSR, prec, h_terms=terms)
    out = []
    for spl in (16, 15):
        o = qt.opts(precision=prec, h0=2.0, steps_per_launch=spl)
        plan = qt.MePlan(ctx, [(L, om.fock_dm(p["N"], 0), tl, e_ops)], o)
        plan.set_shape(8, 1, 0, 2)
        plan.run()
        plan.run()
        out.append(plan.result(0))
        plan.close()
    (ea, sa, _), (eb, sb, _) = out
    np.testing.assert_array_equal(ea, eb)
    for k in ("n_accept", "n_reject", "n_rhs", "status"):
        assert sa[k] == sb[k], (k, sa[k], sb[k])
    assert sa["status"] == 0 and sa["n_reject"] > 0
    ref = oracle.mesolve_td(H0, terms, c, om.fock_dm(p["N"], 0), tl, e_ops, h0=2.0)[0]
    assert np.abs(ea - ref).max() <= (1e-6 if prec == qt.F64 else 1e-4)
    L.close()

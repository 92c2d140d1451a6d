"""Pins of the oracle's time-dependent master equation (Sec. 3.2 with H(t) = H_0 + sum_i f_i(t) H_i,
the QobjEvo of Sec. 2 and the driven example of Sec. 3.4).

Each coefficient kind is checked against exact mathematics the oracle does not contain:
  * complex exponentials: a frame rotating with the drive makes the problem time independent, so
    the lab-frame solution must match the driven-cavity closed form and the matrix exponential of
    the rotating-frame Liouvillian;
  * cos, Gaussian and sample tables: with H(t) = f(t) sigma_x the Hamiltonians at different times
    commute, so <sigma_z>(t) = cos(2 int_0^t f) with the integral in closed form (sin, erf, the
    trapezoid rule of a piecewise-linear interpolant);
  * constants and collapse weights: a constant coefficient and a unit-modulus collapse coefficient
    must reproduce the time-independent solver, and a constant collapse coefficient g must act as
    |g|^2 on the dissipator.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.special as ssp

import oracle
from oracle import liouvillian as ol
from oracle import models as om
import workloads

TIGHT = dict(abstol=1e-11, reltol=1e-9)


def _sigma_plus():
    return om.sigmam().conj().T.tocsr()


def test_rotating_drive_cavity_closed_form():
    """F (e^{-i w t} a^dag + e^{i w t} a) on omega0 a^dag a: in the frame rotating at w the cavity is
    the linear driven cavity with detuning omega0 - w, whose coherent amplitude is known exactly;
    the lab-frame <a> carries the extra phase e^{-i w t}."""
    p = workloads.driven_cavity_td()
    N, w = p["N"], p["omega"]
    a = om.destroy(N)
    H0 = p["omega0"] * om.number(N)
    terms = [(a.conj().T.tocsr(), {"kind": "exp", "a": p["F"], "omega": -w}),
             (a, {"kind": "exp", "a": p["F"], "omega": w})]
    tl = workloads.tlist(p["t_end"], p["nt"])
    ex, st, rc, _ = oracle.mesolve_td(H0, terms, [np.sqrt(p["kappa"]) * a], om.fock_dm(N, 0), tl,
                                      [om.number(N), a], **TIGHT)
    assert rc == 0
    z = 1j * (p["omega0"] - w) + 0.5 * p["kappa"]
    alpha = (-1j * p["F"] / z) * (1.0 - np.exp(-z * tl))
    np.testing.assert_allclose(ex[0].real, np.abs(alpha) ** 2, atol=1e-8)
    np.testing.assert_allclose(ex[1], np.exp(-1j * w * tl) * alpha, atol=1e-8)
    for t, v in [(1, 0.364779), (2, 0.738058), (5, 0.491607)]:
        assert abs(ex[0, int(round(t * 10))].real - v) < 1e-6


def test_rotating_drive_qubit_matches_rotating_frame_expm():
    """Driven damped qubit H = (w0/2) sz + (W/2)(e^{-i w t} s+ + e^{i w t} s-), C = sqrt(g) s-:
    <sz> and e^{i w t}<s-> equal those of the time-independent rotating-frame problem
    H' = ((w0 - w)/2) sz + (W/2) sx, computed by a matrix exponential."""
    w0, w, W, g = 5.0, 5.3, 1.1, 0.15
    sz, sm, sp_ = om.sigmaz(), om.sigmam(), _sigma_plus()
    H0 = 0.5 * w0 * sz
    terms = [(sp_, {"kind": "exp", "a": 0.5 * W, "omega": -w}), (sm, {"kind": "exp", "a": 0.5 * W, "omega": w})]
    c = [np.sqrt(g) * sm]
    tl = np.linspace(0.0, 6.0, 25)
    rho0 = np.diag([0.0, 1.0]).astype(complex)  # down
    ex, st, rc, _ = oracle.mesolve_td(H0, terms, c, rho0, tl, [sz, sm], **TIGHT)
    assert rc == 0
    Hr = 0.5 * (w0 - w) * sz + 0.5 * W * om.sigmax()
    Lr = ol.liouvillian(Hr, c).toarray()
    v0 = ol.vec(rho0)
    for k, t in enumerate(tl):
        r = ol.unvec(sla.expm(Lr * t) @ v0, 2)
        assert abs(ex[0, k] - np.trace(sz.toarray() @ r)) < 1e-8
        assert abs(np.exp(1j * w * t) * ex[1, k] - np.trace(sm.toarray() @ r)) < 1e-8


def _commuting_sx(spec, tl, theta, atol=1e-8):
    """H(t) = f(t) sigma_x from up: <sigma_z>(t) = cos(2 int_0^t f)."""
    H0 = 0.0 * om.sigmaz()
    ex, st, rc, _ = oracle.mesolve_td(H0, [(om.sigmax(), spec)], [], np.diag([1.0, 0.0]).astype(complex), tl,
                                      [om.sigmaz()], **TIGHT)
    assert rc == 0
    np.testing.assert_allclose(ex[0].real, np.cos(2.0 * theta), atol=atol)
    assert np.abs(ex[0].imag).max() < 1e-12


def test_cos_coefficient_commuting_closed_form():
    a, w, phi = 0.8, 2.5, 0.4
    tl = np.linspace(0.0, 7.0, 36)
    _commuting_sx({"kind": "cos", "a": a, "omega": w, "phi": phi}, tl,
                  a * (np.sin(w * tl + phi) - np.sin(phi)) / w)


def test_gaussian_coefficient_commuting_closed_form():
    """A Gaussian pulse (t0, sigma) times cos(w t): with w = 0 the area is an erf; a pi pulse
    (area pi/2 for f multiplying sigma_x) inverts the spin."""
    sig, t0 = 0.6, 2.0
    amp = (np.pi / 2) / (sig * np.sqrt(2 * np.pi))
    tl = np.linspace(0.0, 4.0, 41)
    theta = amp * sig * np.sqrt(np.pi / 2) * (ssp.erf((tl - t0) / (sig * np.sqrt(2))) + ssp.erf(t0 / (sig * np.sqrt(2))))
    _commuting_sx({"kind": "gauss", "a": amp, "t0": t0, "sigma": sig}, tl, theta)
    assert abs(np.cos(2 * theta[-1]) + 1.0) < 1e-4  # the full pulse inverts


def test_table_coefficient_commuting_trapezoid():
    """Linear interpolation of samples, held at the end values: its integral is the trapezoid rule
    over the nodes plus the partial segment.  The interpolant has kinks at the nodes, which the
    adaptive steps do not know about; the local error there is controlled to the tolerance but no
    longer of fifth order, hence the looser bound."""
    g = np.random.default_rng(3)
    t0, dt, n = 0.5, 0.35, 12
    samples = g.uniform(-1.0, 1.0, n)
    tl = np.linspace(0.0, 6.0, 31)  # starts before the table and ends after it

    def interp(t):
        return np.interp(t, t0 + dt * np.arange(n), samples)

    theta = []
    for t in tl:
        nodes = np.concatenate(([0.0], t0 + dt * np.arange(n)))
        nodes = np.sort(np.concatenate((nodes[nodes < t], [t])))
        theta.append(np.trapezoid(interp(nodes), nodes))
    _commuting_sx({"kind": "table", "table": samples, "table_t0": t0, "table_dt": dt}, tl, np.array(theta),
                  atol=2e-6)


def test_constant_coefficient_equals_static_solver():
    p = workloads.kerr_single()
    N = 12
    H, c = om.kerr(N, p["delta"], p["U"], 0.0, p["kappa"])
    a = om.destroy(N)
    drive = (a + a.conj().T).tocsr()
    tl = workloads.tlist(4.0, 21)
    for spec in ({"kind": "const", "a": p["F"]}, {"kind": "cos", "a": p["F"], "omega": 0.0}):
        td = oracle.mesolve_td(H, [(drive, spec)], c, om.fock_dm(N, 0), tl, [om.number(N)], **TIGHT)[0]
        st = oracle.mesolve(H + p["F"] * drive, c, om.fock_dm(N, 0), tl, [om.number(N)], **TIGHT)[0]
        assert np.abs(td - st).max() < 1e-9


def test_collapse_coefficient_weight_is_modulus_squared():
    N = 10
    H, c = om.kerr(N, 1.0, 0.5, 0.8, 1.0)
    tl = workloads.tlist(4.0, 21)
    ref = oracle.mesolve(H, c, om.fock_dm(N, 0), tl, [om.number(N)], **TIGHT)[0]
    # a unit-modulus phase on the collapse operator leaves the dissipator unchanged
    td = oracle.mesolve_td(H, [], [(c[0], {"kind": "exp", "a": 1.0, "omega": 2.3})], om.fock_dm(N, 0), tl,
                           [om.number(N)], **TIGHT)[0]
    assert np.abs(td - ref).max() < 1e-9
    # a constant coefficient g scales the dissipator by |g|^2
    gq = 0.3 + 0.4j
    td = oracle.mesolve_td(H, [], [(c[0], {"kind": "const", "a": gq})], om.fock_dm(N, 0), tl, [om.number(N)],
                           **TIGHT)[0]
    ref2 = oracle.mesolve(H, [abs(gq) * c[0]], om.fock_dm(N, 0), tl, [om.number(N)], **TIGHT)[0]
    assert np.abs(td - ref2).max() < 1e-9


def test_optomechanics_invariants_short_window():
    """The driven optomechanical system of the time-dependent example over a short window: trace kept,
    photon number real and within the cutoff."""
    p = workloads.optomech_td(t_end=20.0, nt=41)
    H0, xa, c, n_op = om.optomech(p["Nc"], p["Nm"], p["wc"], p["wm"], p["g"], p["kappa"], p["gamma"])
    d = p["Nc"] * p["Nm"]
    rho0 = np.zeros((d, d), complex)
    rho0[0, 0] = 1.0
    tl = workloads.tlist(p["t_end"], p["nt"])
    ex, st, rc, fin = oracle.mesolve_td(H0, [(xa, {"kind": "cos", "a": p["F"], "omega": p["wd"]})], c, rho0, tl,
                                        [n_op], want_final=True)
    assert rc == 0
    assert abs(np.trace(fin) - 1.0) < 1e-9
    assert np.abs(fin - fin.conj().T).max() < 1e-9
    assert np.all(ex[0].real >= -1e-9) and np.all(ex[0].real <= p["Nc"] - 1)
    assert np.abs(ex[0].imag).max() < 1e-9
    assert ex[0, -1].real > 1e-3  # the drive has populated the cavity


# --------------------------------------------------------------------------------------------
# Time-dependent trajectories (Sec. 3.3 with the time-dependent operators of Sec. 2)
# --------------------------------------------------------------------------------------------
def test_td_sesolve_rotating_qubit_rabi_closed_form():
    """No dissipation: in the frame rotating with the drive the qubit precesses about
    (W, 0, w0 - w), so <sz>(t) = 1 - 2 (W/WR)^2 sin^2(WR t / 2) from up, WR^2 = W^2 + (w0 - w)^2."""
    w0, w, W = 4.0, 4.4, 1.3
    sz, sm = om.sigmaz(), om.sigmam()
    terms = [(_sigma_plus(), {"kind": "exp", "a": 0.5 * W, "omega": -w}),
             (sm, {"kind": "exp", "a": 0.5 * W, "omega": w})]
    tl = np.linspace(0.0, 8.0, 41)
    ex, st = oracle.sesolve_td(0.5 * w0 * sz, terms, np.array([1, 0], complex), tl, [sz], **TIGHT)
    assert st == 0
    WR = np.hypot(W, w0 - w)
    np.testing.assert_allclose(ex[0].real, 1 - 2 * (W / WR) ** 2 * np.sin(WR * tl / 2) ** 2, atol=1e-8)


def _weighted_decay(g0, om_):
    """Decay rate |g(t)|^2 = g0 cos^2(om t): the no-jump norm is exp(-Lambda(t)) with
    Lambda(t) = g0 (t/2 + sin(2 om t) / (4 om))."""
    return lambda t: g0 * (0.5 * t + np.sin(2 * om_ * t) / (4 * om_))


def test_td_weighted_collapse_jump_time_is_exact():
    """H = 0, one collapse operator sqrt(g0) cos(om t) sigma_-: trajectory j jumps when
    Lambda(t*) = -ln r0, with r0 its Philox threshold."""
    import scipy.optimize as so
    g0, om_ = 0.4, 1.7
    Lam = _weighted_decay(g0, om_)
    tl = np.linspace(0, 10, 21)
    seed = 31
    res = oracle.mcsolve_td(0.0 * om.sigmaz(), [], [(om.sigmam(), {"kind": "cos", "a": np.sqrt(g0), "omega": om_})],
                            np.array([1, 0], complex), tl, [om.sigmaz()], 48, seed, max_jump_record=2, **TIGHT)
    assert (res["status"] == 0).all()
    seen = 0
    for j in range(48):
        r0, _ = oracle.traj_draw(seed, j, 0)
        target = -np.log(r0)
        if Lam(tl[-1]) > target:
            tstar = so.brentq(lambda t: Lam(t) - target, 0.0, tl[-1], xtol=1e-14)
            assert res["njumps"][j] == 1
            assert abs(res["jump_times"][j, 0] - tstar) < 1e-7, (j, res["jump_times"][j, 0], tstar)
            seen += 1
        else:
            assert res["njumps"][j] == 0
    assert seen > 10


def test_td_channel_choice_uses_weights_at_the_jump_time():
    """Two channels out of one level, C_0 = sqrt(a) |1><0| (constant) and C_1 = sqrt(b) cos(om t)
    |2><0|: the first jump picks channel 0 exactly when u (a + b cos^2(om t*)) <= a, with u the
    trajectory's Philox channel uniform."""
    a_, b_, om_ = 0.5, 0.8, 2.3
    C0 = sp.csr_matrix(([np.sqrt(a_)], ([1], [0])), shape=(3, 3), dtype=complex)
    C1 = sp.csr_matrix(([1.0], ([2], [0])), shape=(3, 3), dtype=complex)
    H = sp.csr_matrix((3, 3), dtype=complex)
    seed, n = 41, 200
    res = oracle.mcsolve_td(H, [], [C0, (C1, {"kind": "cos", "a": np.sqrt(b_), "omega": om_})],
                            np.array([1, 0, 0], complex), np.linspace(0, 40, 3), [C0], n, seed, max_jump_record=1,
                            **TIGHT)
    jumped = np.nonzero(res["njumps"] >= 1)[0]
    assert len(jumped) > 0.95 * n
    for j in jumped:
        ts = res["jump_times"][j, 0]
        u, _ = oracle.traj_draw(seed, j, 1)
        w1 = b_ * np.cos(om_ * ts) ** 2
        want = 0 if u * (a_ + w1) <= a_ else 1
        assert res["jump_channels"][j, 0] == want, (j, u, ts)


def test_td_mc_matches_td_me():
    """Sec. 3.3: the trajectory average reproduces the time-dependent master equation (a driven Kerr
    cavity with a rotating drive and a Gaussian-weighted extra loss channel; the nonlinearity makes
    the jumps matter).  Both at tight tolerances, so the statistics dominate the difference."""
    N = 8
    a = om.destroy(N)
    ad = a.conj().T
    H0 = (2.0 * om.number(N) + 0.5 * (ad @ ad @ a @ a)).tocsr()
    terms = [(a.conj().T.tocsr(), {"kind": "exp", "a": 0.6, "omega": -1.5}), (a, {"kind": "exp", "a": 0.6, "omega": 1.5})]
    c_ops = [np.sqrt(0.3) * a, (a, {"kind": "gauss", "a": 0.8, "t0": 2.0, "sigma": 1.0})]
    tl = np.linspace(0, 5, 11)
    me = oracle.mesolve_td(H0, terms, c_ops, om.fock_dm(N, 0), tl, [om.number(N)], **TIGHT)[0][0].real
    n = 3000
    mc = oracle.mcsolve_td(H0, terms, c_ops, np.eye(N, dtype=complex)[0], tl, [om.number(N)], n, 3, **TIGHT)
    dev = np.abs(mc["mean"][0].real - me)
    se = mc["se"][0]
    assert se[-1] > 1e-3  # the trajectories differ
    assert (dev[1:] <= 4 * se[1:] + 1e-7).all(), (dev, se)

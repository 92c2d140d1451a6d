"""Pins of the oracle's time-dependent master equation (Sec. 3.2 with H(t) = H_0 + sum_i f_i(t) H_i,
the QobjEvo of Sec. 2 and the driven example of Sec. 3.5).

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

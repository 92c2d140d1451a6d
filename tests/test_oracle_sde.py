"""Pins of the oracle's stochastic Schrodinger and master equations under homodyne detection
(Sec. 3.5, Ito form, measurement current J = <S + S^dag> + dW/dt).

Checked against what the mathematics fixes, not against the oracle itself:
  * the Wiener increments: standard normal statistics of the Box-Muller draws;
  * a coherent state under homodyne detection of a lossy cavity stays coherent with the
    deterministic amplitude alpha e^{-(i w + kappa/2) t} in every trajectory, with first-order
    convergence in the step, and its current fluctuates around <X> with unit variance per unit time;
  * measuring a Hermitian S = sqrt(G) sigma_z with H = 0, the state is fixed by the integrated
    current Y: psi ~ exp(S Y - S^2 t) psi0, so <sigma_z> = tanh(2 sqrt(G) Y + atanh <sigma_z>_0);
  * the ensemble average of either equation follows the Lindblad master equation;
  * with no extra collapse operators a pure initial state stays pure, and the SME trajectory equals
    the SSE trajectory driven by the same increments (to the schemes' step error).
"""
from math import factorial

import numpy as np
import pytest
import scipy.stats as ss

import oracle
from oracle import models as om


def _coherent(N, al):
    return np.array([np.exp(-abs(al) ** 2 / 2) * al ** n / np.sqrt(float(factorial(n))) for n in range(N)],
                    complex)


def test_wiener_normals_are_standard_normal():
    z = np.array([oracle.wiener_normals(7, j, s, 0) for j in range(40) for s in range(100)])
    for col in (0, 1):
        assert abs(z[:, col].mean()) < 4 / np.sqrt(len(z))
        assert abs(z[:, col].var() - 1.0) < 0.1
        assert ss.kstest(z[:, col], "norm").pvalue > 1e-3
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < 0.1
    # different pairs, steps and trajectories draw different numbers
    assert oracle.wiener_normals(7, 0, 0, 0) != oracle.wiener_normals(7, 0, 0, 1)
    assert oracle.wiener_normals(7, 0, 0, 0) != oracle.wiener_normals(7, 0, 1, 0)
    assert oracle.wiener_normals(7, 0, 0, 0) != oracle.wiener_normals(7, 1, 0, 0)


def test_sse_coherent_state_closed_form_first_order():
    N, w, kap, al = 20, 1.0, 1.0, 1.0
    a = om.destroy(N)
    tl = np.linspace(0, 3, 31)
    exact = al * np.exp(-(1j * w + kap / 2) * tl)
    errs = []
    for dt in (2e-3, 1e-3, 5e-4):
        r = oracle.ssesolve(w * om.number(N), [np.sqrt(kap) * a], _coherent(N, al), tl, [a, om.number(N)], 8, 1, dt)
        assert r["rc"] == 0
        ex = r["expect_tr"]
        errs.append(np.abs(ex[:, 0, :] - exact).max())
        np.testing.assert_allclose(ex[:, 1, :].real, np.abs(ex[:, 0, :]) ** 2, atol=1e-6)  # still coherent
    assert errs[1] < 3e-3
    assert errs[1] / errs[0] < 0.7 and errs[2] / errs[1] < 0.7  # first order in the step


def test_sse_current_fluctuates_with_unit_variance_per_time():
    N, w, kap, al = 16, 1.0, 1.0, 0.8
    a = om.destroy(N)
    tl = np.linspace(0, 2, 21)
    X = np.sqrt(kap) * (a + a.conj().T)
    r = oracle.ssesolve(w * om.number(N), [np.sqrt(kap) * a], _coherent(N, al), tl, [X], 400, 9, 1e-3)
    J = r["measurement"][:, 0, :]
    # mean <X> over each interval (trapezoid of the exact amplitude) vs the ensemble of currents
    tf = np.linspace(0, 2, 2001)
    xf = 2 * np.sqrt(kap) * (al * np.exp(-(1j * w + kap / 2) * tf)).real
    lens = np.diff(tl)
    xbar = np.array([np.trapezoid(xf[100 * i:100 * i + 101], tf[100 * i:100 * i + 101]) for i in range(20)]) / lens
    z = (J - xbar) * np.sqrt(lens)  # standard normal per interval and trajectory
    assert abs(z.mean()) < 4 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 0.05


def test_sse_hermitian_measurement_filter():
    """H = 0, S = sqrt(G) sz: <sz>(t) = tanh(2 sqrt(G) Y(t) + atanh <sz>_0), Y the integral of the
    recorded current."""
    sz, G = om.sigmaz(), 0.8
    psi0 = np.array([np.sqrt(0.3), np.sqrt(0.7)], complex)
    tl = np.linspace(0, 2, 11)
    errs = []
    for dt in (2e-3, 5e-4):
        r = oracle.ssesolve(0 * sz, [np.sqrt(G) * sz], psi0, tl, [sz], 20, 5, dt)
        J = r["measurement"][:, 0, :]
        Y = np.concatenate([np.zeros((20, 1)), np.cumsum(J * np.diff(tl), axis=1)], axis=1)
        pred = np.tanh(2 * np.sqrt(G) * Y + np.arctanh(0.3 - 0.7))
        errs.append(np.abs(r["expect_tr"][:, 0, :].real - pred).max())
    assert errs[1] < 5e-3 and errs[1] < 0.5 * errs[0], errs


def _driven_qubit():
    return 0.5 * om.sigmax(), [np.sqrt(0.5) * om.sigmam()], np.linspace(0, 4, 21)


def test_sse_ensemble_follows_master_equation():
    H, S, tl = _driven_qubit()
    me = oracle.mesolve(H, S, np.array([1, 0], complex), tl, [om.sigmaz()])[0][0].real
    r = oracle.ssesolve(H, S, np.array([1, 0], complex), tl, [om.sigmaz()], 4000, 3, 2e-3)
    z = np.abs(r["mean"][0].real - me)[1:] / r["se"][0][1:]
    assert (z > 3).sum() <= 1 and z.max() < 4.5, z


def test_sme_ensemble_follows_master_equation():
    H, S, tl = _driven_qubit()
    C = [np.sqrt(0.2) * om.sigmaz()]
    me = oracle.mesolve(H, S + C, np.array([1, 0], complex), tl, [om.sigmaz()])[0][0].real
    r = oracle.smesolve(H, C, S, np.array([1, 0], complex), tl, [om.sigmaz()], 600, 3, 2e-3)
    z = np.abs(r["mean"][0].real - me)[1:] / r["se"][0][1:]
    assert (z > 3).sum() <= 1 and z.max() < 4.5, z


def test_sme_pure_state_follows_the_sse_trajectory():
    """No extra losses: rho stays pure, and with the same Wiener increments the SME and SSE
    trajectories coincide to the step error, which shrinks with the step."""
    H, S, tl = _driven_qubit()
    tl = tl[:11]
    e = [om.sigmaz(), om.sigmax()]
    errs = []
    for dt in (2e-3, 5e-4):
        a = oracle.ssesolve(H, S, np.array([1, 0], complex), tl, e, 6, 4, dt)
        b = oracle.smesolve(H, [], S, np.array([1, 0], complex), tl, e, 6, 4, dt)
        errs.append(np.abs(a["expect_tr"] - b["expect_tr"]).max())
        np.testing.assert_allclose(a["measurement"], b["measurement"], atol=0.05)
    assert errs[1] < 1e-2 and errs[1] < 0.6 * errs[0], errs

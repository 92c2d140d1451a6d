"""Pins of the oracle's Dormand-Prince 5(4) integrator.

The paper never names its integrator; the oracle uses DOPRI5.  The coefficients are pinned here by
the Butcher order conditions (all 17 rooted trees up to order 5 for the propagating weights, all 8
up to order 4 for the embedded weights), which a single mistyped coefficient violates, and by the
observed convergence order on a linear test problem whose exact solution is a matrix exponential.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

import oracle


def _trees(A, b, c):
    """Elementary-weight conditions sum(...) = 1/gamma(t) for trees up to order 5."""
    Ac = A @ c
    Ac2 = A @ (c ** 2)
    Ac3 = A @ (c ** 3)
    AAc = A @ Ac
    AAc2 = A @ Ac2
    AcAc = A @ (c * Ac)
    AAAc = A @ AAc
    return [
        (1, b.sum(), 1),
        (2, b @ c, 2),
        (3, b @ c ** 2, 3), (3, b @ Ac, 6),
        (4, b @ c ** 3, 4), (4, b @ (c * Ac), 8), (4, b @ Ac2, 12), (4, b @ AAc, 24),
        (5, b @ c ** 4, 5), (5, b @ (c ** 2 * Ac), 10), (5, b @ (Ac ** 2), 20), (5, b @ (c * Ac2), 15),
        (5, b @ Ac3, 20), (5, b @ (c * AAc), 30), (5, b @ AcAc, 40), (5, b @ AAc2, 60), (5, b @ AAAc, 120),
    ]


def test_row_sums_and_fsal():
    c, A, b, bh = oracle.tableau()
    np.testing.assert_allclose(A.sum(axis=1), c, atol=1e-15)
    np.testing.assert_array_equal(A[6], b)  # first-same-as-last
    assert bh[6] != 0.0 and b[6] == 0.0
    assert np.all(np.triu(A) == 0.0)  # explicit


def test_order_conditions_fifth_order_weights():
    c, A, b, bh = oracle.tableau()
    for order, val, gamma in _trees(A, b, c):
        assert abs(val - 1.0 / gamma) < 1e-14, (order, val, gamma)


def test_order_conditions_embedded_fourth_order():
    c, A, b, bh = oracle.tableau()
    conds = _trees(A, bh, c)
    for order, val, gamma in conds:
        if order <= 4:
            assert abs(val - 1.0 / gamma) < 1e-14, (order, val, gamma)
    # the embedded pair is genuinely of order 4: at least one fifth-order condition fails
    assert max(abs(v - 1.0 / g) for o, v, g in conds if o == 5) > 1e-6


def test_exact_rational_coefficients():
    """Each coefficient equals its rational value to the last bit (no transcription drift)."""
    c, A, b, bh = oracle.tableau()
    F = Fraction
    exact_b = [F(35, 384), 0, F(500, 1113), F(125, 192), F(-2187, 6784), F(11, 84), 0]
    exact_bh = [F(5179, 57600), 0, F(7571, 16695), F(393, 640), F(-92097, 339200), F(187, 2100), F(1, 40)]
    for x, e in zip(b, exact_b):
        assert x == float(e)
    for x, e in zip(bh, exact_bh):
        assert x == float(e)


def _test_matrix():
    g = np.random.default_rng(1)
    M = g.normal(size=(4, 4)) + 1j * g.normal(size=(4, 4))
    return -0.5 * np.eye(4) + 0.3 * M


def test_observed_order_five():
    M = _test_matrix()
    y0 = np.array([1, 0.5j, -0.25, 0.1 + 0.2j])
    T = 1.0
    exact = sla.expm(M * T) @ y0
    errs = []
    hs = [0.1, 0.05, 0.025]
    for h in hs:
        y, _ = oracle.linear_fixed(M, y0, h, int(round(T / h)))
        errs.append(np.linalg.norm(y - exact))
    p1 = np.log2(errs[0] / errs[1])
    p2 = np.log2(errs[1] / errs[2])
    assert 4.7 < p1 < 5.4 and 4.7 < p2 < 5.4, (p1, p2)


def test_error_estimate_scales_as_h5():
    M = _test_matrix()
    y0 = np.array([1, 0.5j, -0.25, 0.1 + 0.2j])
    e1 = np.linalg.norm(oracle.linear_fixed(M, y0, 0.04, 1)[1])
    e2 = np.linalg.norm(oracle.linear_fixed(M, y0, 0.02, 1)[1])
    assert 4.6 < np.log2(e1 / e2) < 5.4


def test_adaptive_linear_meets_tolerance_and_lands_on_tlist():
    M = _test_matrix()
    y0 = np.array([1, 0.5j, -0.25, 0.1 + 0.2j])
    tl = np.linspace(0, 3, 31)
    out, st, rc = oracle.linear_solve(M, y0, tl, abstol=1e-10, reltol=1e-8)
    assert rc == 0
    for k, t in enumerate(tl):
        np.testing.assert_allclose(out[k], sla.expm(M * t) @ y0, atol=1e-7)
    # tolerance proportionality: 100x tighter tolerance -> error shrinks
    out2, st2, _ = oracle.linear_solve(M, y0, tl, abstol=1e-12, reltol=1e-10)
    e1 = np.abs(out[-1] - sla.expm(M * 3) @ y0).max()
    e2 = np.abs(out2[-1] - sla.expm(M * 3) @ y0).max()
    assert e2 < e1 and st2["n_accept"] > st["n_accept"]


def test_limits_reported():
    M = _test_matrix()
    y0 = np.ones(4, dtype=complex)
    _, st, rc = oracle.linear_solve(M, y0, np.linspace(0, 50, 3), max_steps=3)
    assert rc == 4  # max steps
    _, _, rc = oracle.linear_solve(M, y0, np.array([0.0, 1.0, 1.0]))
    assert rc == 1  # tlist not strictly increasing
    _, _, rc = oracle.linear_solve(np.full((4, 4), np.nan), y0, np.linspace(0, 1, 3))
    assert rc == 6  # non-finite


@pytest.mark.parametrize("n", [1, 2])
def test_single_point_tlist(n):
    M = _test_matrix()
    y0 = np.ones(4, dtype=complex)
    out, st, rc = oracle.linear_solve(M, y0, np.linspace(0, 1, n))
    assert rc == 0
    np.testing.assert_array_equal(out[0], y0)


def test_step_controller_fixed_point():
    """The step-size controller (a reading: DOPRI5's PI law h <- h 0.9 err^-0.17 err_prev^0.04) is
    pinned by its fixed point rather than by its formula.  On y' = i y the rtol-weighted error of a
    step depends on h alone, err(h) = |E(ih)| / rtol with E(z) = z (b - bhat)^T (I - zA)^-1 1 the
    stability-function difference of the pair; a constant err is a fixed point of the law only at
    err* = 0.9^(1 / (0.17 - 0.04)).  So after a short transient every step has the size h* with
    err(h*) = err*, and a long interval T = N h* takes N steps plus the transient.  A changed safety
    factor or exponent (0.17 -> 0.2 shifts h* by 3%), a swapped or sign-flipped exponent, or a
    changed error weighting moves the count far outside the window."""
    c, A, b, bh = oracle.tableau()

    def stab_diff(z):
        return z * ((b - bh) @ np.linalg.solve(np.eye(len(b)) - z * A, np.ones(len(b))))

    rtol = 1e-6
    err_star = 0.9 ** (1.0 / (0.17 - 0.04))
    lo, hi = 1e-4, 2.0
    for _ in range(200):  # |E(ih)| grows with h on this range
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if abs(stab_diff(1j * mid)) / rtol < err_star else (lo, mid)
    h_star = lo
    for n in (1000, 2000):
        _, st, rc = oracle.linear_solve(np.array([[1j]]), np.array([1.0 + 0j]), np.array([0.0, n * h_star]),
                                        abstol=1e-12, reltol=rtol)
        assert rc == 0 and st["n_reject"] == 0
        assert n <= st["n_accept"] <= n + 6, (n, st["n_accept"])

"""Pins of the oracle's steady state (Sec. 3.2, steadystate) against closed forms and invariants."""
import numpy as np
import scipy.sparse as sp

import oracle
from oracle import liouvillian as ol
from oracle import models as om


def test_thermal_oscillator():
    """Loss and gain at rates kappa (n_th + 1) and kappa n_th: the steady state is thermal,
    p_n = n_th^n / (1 + n_th)^(n+1), diagonal, with <n> = n_th (up to the cutoff)."""
    N, kap, nth = 40, 0.7, 0.6
    a = om.destroy(N)
    c = [np.sqrt(kap * (nth + 1)) * a, np.sqrt(kap * nth) * a.conj().T.tocsr()]
    rho = oracle.steadystate(0.9 * om.number(N), c)
    p = nth ** np.arange(N) / (1 + nth) ** (np.arange(N) + 1)
    np.testing.assert_allclose(np.diag(rho).real, p / p.sum(), atol=1e-12)
    assert np.abs(rho - np.diag(np.diag(rho))).max() < 1e-12


def test_resonance_fluorescence():
    """Resonantly driven two-level system, H = (W/2) sx, C = sqrt(g) s-: <sz>_ss = -1/(1 + s) with
    the saturation parameter s = 2 W^2 / g^2, and <s-> = -i (W/g) / (1 + s) on the same footing."""
    W, g = 1.3, 0.7
    rho = oracle.steadystate(0.5 * W * om.sigmax(), [np.sqrt(g) * om.sigmam()])
    s = 2 * W ** 2 / g ** 2
    assert abs(np.trace(om.sigmaz().toarray() @ rho) - (-1 / (1 + s))) < 1e-12
    assert abs(np.trace(om.sigmam().toarray() @ rho) - (-1j * (W / g) / (1 + s))) < 1e-12


def test_driven_cavity_coherent_steady_state():
    """Linear driven cavity: the steady state is the coherent state alpha = -i F / (i Delta + kappa/2)
    (the U = 0 Kerr closed form at t -> infinity)."""
    N, det, F, kap = 25, 0.7, 0.6, 1.0
    H, c = om.kerr(N, det, 0.0, F, kap)
    rho = oracle.steadystate(H, c)
    al = -1j * F / (1j * det + kap / 2)
    a = om.destroy(N).toarray()
    assert abs(np.trace(a @ rho) - al) < 1e-10
    assert abs(np.trace(a.conj().T @ a @ rho) - abs(al) ** 2) < 1e-10


def test_steady_state_invariants_ising():
    H, c = om.ising(4, 1.0, 0.7, 0.2)
    rho = oracle.steadystate(H, c)
    L = ol.liouvillian(H, c)
    assert np.abs(L @ rho.reshape(-1)).max() < 1e-12
    assert abs(np.trace(rho) - 1) < 1e-12
    assert np.abs(rho - rho.conj().T).max() < 1e-12
    assert np.linalg.eigvalsh((rho + rho.conj().T) / 2).min() > -1e-12

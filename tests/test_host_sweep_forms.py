"""Host logic of the sweep's form choice: the a-priori stiffness estimate against the exact
spectral radius of small Kerr-cavity Liouvillians, and the partitions each policy makes."""
import numpy as np
import pytest

from oracle import models as om
import workloads
import paper_2504_21440_amd as qt
from bench import kerr_dense_cost, kerr_spectral_estimate, sweep_forms


def _liouvillian(H, cs):
    """Column-stacked superoperator of the master equation (Sec. 2): vec(A X B) = (B^T kron A) vec X."""
    n = H.shape[0]
    eye = np.eye(n)
    L = -1j * (np.kron(eye, H) - np.kron(H.T, eye))
    for c in cs:
        cdc = c.conj().T @ c
        L += np.kron(c.conj(), c) - 0.5 * np.kron(eye, cdc) - 0.5 * np.kron(cdc.T, eye)
    return L


@pytest.mark.parametrize("i", range(12))
def test_spectral_estimate_tracks_exact_radius(i):
    """The estimate only ranks cavities by cost: it stays within a small factor of the exact
    spectral radius (0.86 to 2.4 on these cavities), not above it."""
    g = np.random.default_rng(100 + i)
    p = {"N": int(g.integers(6, 15)), "delta": float(g.uniform(-2, 2)), "U": float(g.uniform(0, 1)),
         "F": float(g.uniform(0, 2)), "kappa": float(g.uniform(0.5, 2))}
    H, cs = om.kerr(p["N"], p["delta"], p["U"], p["F"], p["kappa"])
    rho = np.abs(np.linalg.eigvals(_liouvillian(H.toarray(), [c.toarray() for c in cs]))).max()
    est = kerr_spectral_estimate(p)
    assert 0.5 * rho <= est <= 3.0 * rho, (p, rho, est)


def test_sweep_form_policies():
    sweep = workloads.kerr_sweep(n=512)
    assert all(f == qt.FORM_DENSE for f in sweep_forms(sweep, "dense"))
    n32 = sweep_forms(sweep, "n32")
    assert all((f == qt.FORM_DENSE) == (p["N"] <= 32) for f, p in zip(n32, sweep))
    cost = np.array([kerr_dense_cost(p) for p in sweep])
    prev = 0
    for f in (0.9, 0.6, 0.3):
        forms = np.array(sweep_forms(sweep, f"stiff{f}"))
        csr = forms == qt.FORM_CSR
        # the CSR set is the costliest cavities, and it only grows as the cut fraction falls
        assert csr[np.argmax(cost)] and cost[csr].min() >= cost[~csr].max()
        assert csr.sum() > prev
        prev = csr.sum()
    # cost grows with the Kerr coefficient and with the padded size
    p = dict(sweep[0], N=40, U=0.2)
    assert kerr_dense_cost(dict(p, U=0.4)) > kerr_dense_cost(p) < kerr_dense_cost(dict(p, N=50))
    with pytest.raises(ValueError):
        sweep_forms(sweep, "bogus")

"""Kernel variants chosen by ensemble size give the same trajectories.

Large complex64 ensembles run the trajectory and stochastic kernels in variants held to fewer
registers (more trajectories in flight per compute unit).  A trajectory's random draws are keyed by
(seed, trajectory index) and its arithmetic does not depend on the variant, so the first k
trajectories of an ensemble above the size threshold must equal, bit for bit, those of a small
ensemble below it: expectation rows, jump counts, jump times and channels, and measurement currents.
The state lengths cover 2, 4 and 8 rows per thread (jump kernel: chains of L = 9, 10, 11; stochastic
kernel: the master equation at d = 30 and 45 and the Schrodinger equation at d = 1,024)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import models as om
import paper_2504_21440_amd as qt

pytestmark = pytest.mark.gpu

MC_LARGE = 2048   # ensembles at least this large take the variant held to 3 (8 rows: 2) waves per SIMD
SDE_LARGE = 300   # more trajectories than compute units: the stochastic variant held to 2 waves per SIMD
SMALL = 48


@pytest.fixture(scope="module")
def ctx():
    print("[gpu] variants: creating context", flush=True)
    c = qt.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("L", [9, 10, 11])
@pytest.mark.parametrize("td", [False, True])
def test_jump_kernel_large_ensemble_variant_is_bitwise(ctx, L, td):
    print(f"[gpu] variants: mcsolve L={L} td={td} ntraj {SMALL} vs {MC_LARGE}", flush=True)
    H, cs = qt.model_ising(L, 1.0, 1.0, 0.4)
    tl = np.linspace(0.0, 0.6, 4)
    e = [om.site_op(L, 0, om.sigmaz()), om.site_op(L, L // 2, om.sigmax())]
    h_terms = None
    if td:
        sx = sum(om.site_op(L, i, om.sigmax()) for i in range(L))
        h_terms = [(sp.csr_matrix(sx), {"kind": "cos", "a": 0.3, "omega": 2.0})]
    o = qt.opts(abstol=1e-6, reltol=1e-4, precision=qt.MIXED)
    psi0 = om.all_up_ket(L)
    res = {}
    for n in (SMALL, MC_LARGE):
        res[n] = qt.mcsolve(ctx, H, cs, psi0, tl, e, n, 77, options=o, want_traj=True, max_jump_record=6,
                            h_terms=h_terms)
    a, b = res[SMALL], res[MC_LARGE]
    np.testing.assert_array_equal(a["expect_tr"], b["expect_tr"][:SMALL])
    np.testing.assert_array_equal(a["njumps"], b["njumps"][:SMALL])
    rec = np.arange(6)[None, :] < np.minimum(a["njumps"], 6)[:, None]  # slots past njumps are unspecified
    np.testing.assert_array_equal(a["jump_times"][rec], b["jump_times"][:SMALL][rec])
    np.testing.assert_array_equal(a["jump_channels"][rec], b["jump_channels"][:SMALL][rec])
    assert a["njumps"].sum() > 0


def _cavity(N, delta=0.5, F=0.7, kappa=1.0):
    a = om.destroy(N)
    H = sp.csr_matrix(delta * (a.conj().T @ a) + F * (a + a.conj().T))
    return H, [sp.csr_matrix(np.sqrt(kappa) * a)], sp.csr_matrix(a + a.conj().T)


@pytest.mark.parametrize("case", ["sme_d30", "sme_d45", "sse_d1024"])
def test_stochastic_kernel_large_ensemble_variant_is_bitwise(ctx, case):
    print(f"[gpu] variants: stochastic {case} ntraj {SMALL} vs {SDE_LARGE}", flush=True)
    tl = np.linspace(0.0, 0.2, 5)
    o = qt.opts(precision=qt.MIXED)
    if case.startswith("sme"):
        N = 30 if case == "sme_d30" else 45
        H, S, X = _cavity(N)
        rho0 = np.zeros((N, N), complex)
        rho0[0, 0] = 1.0
        kw = dict(c_ops=[sp.csr_matrix(np.sqrt(0.2) * om.number(N))], master=True)
        state0, e = rho0, [X]
    else:
        L = 10
        H, _ = qt.model_ising(L, 1.0, 1.0, 0.0)
        S = [sp.csr_matrix(np.sqrt(0.5) * om.site_op(L, 0, om.sigmam()))]
        kw = dict(master=False)
        state0, e = om.all_up_ket(L), [om.site_op(L, 0, om.sigmaz())]
    res = {}
    for n in (SMALL, SDE_LARGE):
        P = qt.SdePlan(ctx, H, S, state0, tl, e, n, 31, 1e-3, options=o, **kw)
        P.run()
        res[n] = P.result(want_traj=True)
        P.close()
    a, b = res[SMALL], res[SDE_LARGE]
    np.testing.assert_array_equal(a["expect_tr"], b["expect_tr"][:SMALL])
    np.testing.assert_array_equal(a["measurement"], b["measurement"][:SMALL])

"""Pins of the oracle's master-equation solver (Sec. 3.2) and of its Liouvillian.

Each test checks the oracle against something other than itself: a closed form, the exact matrix
exponential of an independently assembled superoperator, or an invariant that the definition fixes.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle
from oracle import liouvillian as ol
from oracle import models as om
import workloads


def _coherent_alpha(t, delta, F, kappa):
    """Driven damped linear cavity (U = 0): alpha(t) = alpha_ss (1 - exp(-(i Delta + kappa/2) t)),
    alpha_ss = -i F / (i Delta + kappa/2)."""
    z = 1j * delta + 0.5 * kappa
    return (-1j * F / z) * (1.0 - np.exp(-z * t))


def test_kerr_u0_coherent_closed_form():
    p = workloads.kerr_single(U=0.0)
    N = p["N"]
    H, c = om.kerr(N, p["delta"], 0.0, p["F"], p["kappa"])
    a = om.destroy(N)
    tl = workloads.tlist(p["t_end"], 201)
    ex, st, rc, _ = oracle.mesolve(H, c, om.fock_dm(N, 0), tl, [om.number(N), a],
                                   abstol=1e-12, reltol=1e-10)
    assert rc == 0
    al = _coherent_alpha(tl, p["delta"], p["F"], p["kappa"])
    np.testing.assert_allclose(ex[0].real, np.abs(al) ** 2, atol=1e-9)
    np.testing.assert_allclose(ex[1], al, atol=1e-9)  # the phase pins the sign of -i[H, rho]
    # the values quoted for t = 1, 2, 5, 20 and the steady state F^2 / (Delta^2 + kappa^2/4)
    for t, v in [(1, 0.364779), (2, 0.738058), (5, 0.491607), (20, 0.511981)]:
        assert abs(ex[0, int(round(t * 10))].real - v) < 1e-6
    assert abs(abs(_coherent_alpha(1e9, 1.0, 0.8, 1.0)) ** 2 - 0.8 ** 2 / (1.0 + 0.25)) < 1e-12


def test_kerr_u0_at_config_tolerances():
    p = workloads.kerr_single(U=0.0)
    N = p["N"]
    H, c = om.kerr(N, p["delta"], 0.0, p["F"], p["kappa"])
    tl = workloads.tlist(p["t_end"], p["nt"])
    ex, st, rc, _ = oracle.mesolve(H, c, om.fock_dm(N, 0), tl, [om.number(N)])
    assert rc == 0
    al = _coherent_alpha(tl, p["delta"], p["F"], p["kappa"])
    assert np.abs(ex[0].real - np.abs(al) ** 2).max() < 1e-6


def test_steady_state_photon_number():
    """<n>_ss = F^2 / ((omega_c - omega_d)^2 + gamma^2/4) in the rotating frame (Sec. 5 closed form)."""
    N, det, F, g = 25, 0.7, 0.6, 1.0
    H, c = om.kerr(N, det, 0.0, F, g)
    tl = np.array([0.0, 60.0])
    ex, st, rc, _ = oracle.mesolve(H, c, om.fock_dm(N, 0), tl, [om.number(N)], abstol=1e-10, reltol=1e-8)
    assert abs(ex[0, -1].real - F ** 2 / (det ** 2 + g ** 2 / 4)) < 1e-8


def test_oscillator_fock3_decay():
    """H = omega a^dag a, C = sqrt(gamma) a, psi0 = |3>: <a^dag a> = 3 exp(-gamma t) (Sec. 4 example)."""
    N, w, g = 20, 1.0, 0.1
    a = om.destroy(N)
    H = w * (a.conj().T @ a)
    tl = np.linspace(0, 10, 100)
    ex, st, rc, _ = oracle.mesolve(H, [np.sqrt(g) * a], om.fock_dm(N, 3), tl, [om.number(N)])
    assert rc == 0
    np.testing.assert_allclose(ex[0].real, 3 * np.exp(-g * tl), atol=1e-7)


@pytest.mark.parametrize("L", [2, 3])
def test_ising_no_field_decay(L):
    """h = 0: rho stays diagonal and every <sz_i> = 2 exp(-gamma t) - 1 (pins sigma_- and 'up' = 0)."""
    gam = 0.2
    H, c = om.ising(L, 1.0, 0.0, gam)
    tl = np.linspace(0, 10, 41)
    e_ops = [om.site_op(L, i, om.sigmaz()) for i in range(L)]
    ex, st, rc, fin = oracle.mesolve(H, c, om.all_up_ket(L), tl, e_ops, want_final=True)
    assert rc == 0
    for i in range(L):
        np.testing.assert_allclose(ex[i].real, 2 * np.exp(-gam * tl) - 1, atol=1e-7)
    assert np.abs(fin - np.diag(np.diag(fin))).max() < 1e-12


def _expm_reference(H, c_ops, rho0, tl, e_ops):
    Lm = ol.liouvillian(H, c_ops).toarray()
    d = rho0.shape[0]
    out = np.zeros((len(e_ops), len(tl)), dtype=complex)
    for k, t in enumerate(tl):
        rho = ol.unvec(sla.expm(Lm * t) @ ol.vec(rho0), d)
        for q, O in enumerate(e_ops):
            out[q, k] = np.trace(O.toarray() @ rho)
    return out


def test_expm_kerr_small():
    p = workloads.kerr_single()
    N = 8
    H, c = om.kerr(N, p["delta"], p["U"], p["F"], p["kappa"])
    tl = np.linspace(0, 5, 11)
    e_ops = [om.number(N), om.destroy(N)]
    ex, st, rc, _ = oracle.mesolve(H, c, om.fock_dm(N, 0), tl, e_ops, abstol=1e-12, reltol=1e-10)
    ref = _expm_reference(H, c, om.fock_dm(N, 0), tl, e_ops)
    assert np.abs(ex - ref).max() < 1e-8


def test_expm_ising_small():
    p = workloads.ising_single(L=3)
    H, c = om.ising(3, p["J"], p["h"], p["gamma"])
    tl = np.linspace(0, 4, 9)
    e_ops = [om.site_op(3, i, om.sigmaz()) for i in range(3)] + [om.site_op(3, 1, om.sigmax())]
    rho0 = np.outer(om.all_up_ket(3), om.all_up_ket(3))
    ex, st, rc, _ = oracle.mesolve(H, c, rho0, tl, e_ops, abstol=1e-12, reltol=1e-10)
    ref = _expm_reference(H, c, rho0, tl, e_ops)
    assert np.abs(ex - ref).max() < 1e-8


def _random_ops(d, nc, seed):
    g = np.random.default_rng(seed)
    X = g.normal(size=(d, d)) + 1j * g.normal(size=(d, d))
    H = sp.csr_matrix(X + X.conj().T)
    cs = [sp.csr_matrix(0.4 * (g.normal(size=(d, d)) + 1j * g.normal(size=(d, d)))) for _ in range(nc)]
    return H, cs


def test_expm_random_complex_operators():
    """Complex, non-symmetric collapse operators and a complex Hermitian H: catches a transposed or
    unconjugated operand anywhere in either formulation."""
    H, cs = _random_ops(4, 2, 3)
    rho0 = workloads.random_hermitian_dm(4, 7)
    tl = np.linspace(0, 2, 5)
    e_ops = [sp.csr_matrix(np.eye(4)[[1, 0, 3, 2]] * 1.0 + 0j), H]
    ex, st, rc, _ = oracle.mesolve(H, cs, rho0, tl, e_ops, abstol=1e-12, reltol=1e-10)
    ref = _expm_reference(H, cs, rho0, tl, e_ops)
    assert np.abs(ex - ref).max() < 1e-8


def test_closed_system_is_unitary_conjugation():
    """No collapse operators: rho(t) = U rho0 U^dag with U = exp(-i H t) (Sec. 3.1) -- independent of
    any superoperator."""
    H, _ = _random_ops(5, 0, 11)
    psi = workloads.random_ket(5, 2)
    tl = np.linspace(0, 1.5, 4)
    O = sp.csr_matrix(np.diag(np.arange(5.0)) + 0j)
    ex, st, rc, fin = oracle.mesolve(H, [], psi, tl, [O], abstol=1e-12, reltol=1e-10, want_final=True)
    U = sla.expm(-1j * H.toarray() * tl[-1])
    rho = np.outer(U @ psi, (U @ psi).conj())
    assert np.abs(fin - rho).max() < 1e-9
    assert abs(ex[0, -1] - np.trace(O.toarray() @ rho)) < 1e-9


def test_liouvillian_matches_matrix_free_rhs():
    """The Kronecker-assembled superoperator and the C right-hand side agree on random inputs."""
    for (H, cs), d in [(_random_ops(6, 3, 5), 6), (om.ising(3, 1.0, 0.7, 0.2), 8), (om.kerr(7, 1.0, 0.5, 0.8, 1.0), 7)]:
        Lm = ol.liouvillian(H, cs)
        rho = workloads.random_hermitian_dm(d, 9)
        a = ol.unvec(Lm @ ol.vec(rho), d)
        b = oracle.lindblad_apply(H, cs, rho)
        assert np.abs(a - b).max() < 1e-12
        # trace preservation and Hermiticity preservation of the definition
        assert abs(np.trace(b)) < 1e-12
        assert np.abs(b - b.conj().T).max() < 1e-12
        # and on a non-Hermitian input (no symmetry shortcut anywhere)
        g = np.random.default_rng(d)
        X = g.normal(size=(d, d)) + 1j * g.normal(size=(d, d))
        assert np.abs(ol.unvec(Lm @ ol.vec(X), d) - oracle.lindblad_apply(H, cs, X)).max() < 1e-11


def test_liouvillian_sizes():
    H, c = om.kerr(20, 1.0, 0.5, 0.8, 1.0)
    assert ol.liouvillian(H, c).nnz == 2280
    H, c = om.ising(8, 1.0, 0.7, 0.2)
    Lm = ol.liouvillian(H, c)
    assert Lm.shape == (65536, 65536) and Lm.nnz == 1_245_183


def test_invariants_config_tolerances():
    p = workloads.kerr_single()
    N = p["N"]
    H, c = om.kerr(N, p["delta"], p["U"], p["F"], p["kappa"])
    tl = workloads.tlist(p["t_end"], p["nt"])
    ex, st, rc, fin = oracle.mesolve(H, c, om.fock_dm(N, 0), tl, [om.number(N)], want_final=True)
    assert rc == 0
    assert abs(np.trace(fin) - 1) < 1e-10
    assert np.abs(fin - fin.conj().T).max() < 1e-12
    assert np.linalg.eigvalsh(0.5 * (fin + fin.conj().T)).min() > -1e-7
    # self-convergence: config tolerances vs tight tolerances
    ex2, _, _, _ = oracle.mesolve(H, c, om.fock_dm(N, 0), tl, [om.number(N)], abstol=1e-12, reltol=1e-10)
    assert np.abs(ex - ex2).max() < 1e-5


def test_expect_closed_forms():
    N = 6
    for n in range(N):
        assert abs(oracle.expect_dm(om.number(N), om.fock_dm(N, n)) - n) < 1e-15
        v = np.zeros(N, complex)
        v[n] = 2.0  # unnormalised ket
        assert abs(oracle.expect_ket(om.number(N), v) - n) < 1e-15
    # product state of 3 spins: up, down, up
    psi = np.zeros(8, complex)
    psi[0b010] = 1.0
    vals = [oracle.expect_ket(om.site_op(3, i, om.sigmaz()), psi) for i in range(3)]
    assert vals == [1, -1, 1]
    # Tr(O rho) with a non-Hermitian O pins the index order O_ij rho_ji
    O = sp.csr_matrix(np.array([[0, 1], [0, 0]], dtype=complex))
    rho = np.array([[0.5, 0.2 + 0.1j], [0.3 - 0.4j, 0.5]])
    assert abs(oracle.expect_dm(O, rho) - rho[1, 0]) < 1e-15

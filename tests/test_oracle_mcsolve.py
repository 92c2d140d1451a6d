"""Pins of the oracle's Monte-Carlo wave-function solver (Sec. 3.3) and of its Philox generator."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.stats as ss

import oracle
from oracle import models as om


def test_philox_round_structure():
    """Philox-4x32-10 is a bijection of the counter for a fixed key and differs for adjacent keys
    and counters in about half of the output bits (avalanche)."""
    outs = set()
    flips = []
    for i in range(2000):
        w = oracle.philox([i, 0, 0, 0], [7, 9])
        outs.add(tuple(int(x) for x in w))
        w2 = oracle.philox([i ^ 1, 0, 0, 0], [7, 9])
        flips.append(sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(w, w2)))
    assert len(outs) == 2000
    assert 60 < np.mean(flips) < 68  # 128 bits, ideal 64


def test_philox_uniformity():
    ws = np.array([oracle.philox([i, 3, 1, 0], [123, 456]) for i in range(20000)], dtype=np.uint64)
    for col in range(4):
        bits = ws[:, col] >> np.uint64(24)  # top 8 bits
        counts = np.bincount(bits.astype(np.int64), minlength=256)
        chi2 = ((counts - len(bits) / 256) ** 2 / (len(bits) / 256)).sum()
        assert ss.chi2.sf(chi2, 255) > 1e-4
    u = np.array([oracle.uniform_from_words(a, b) for a, b in ws[:, :2]])
    assert u.min() > 0 and u.max() < 1
    assert ss.kstest(u, "uniform").pvalue > 1e-4


def test_uniform_from_words_range():
    assert oracle.uniform_from_words(0, 0) == 0.5 * 2.0 ** -53
    assert oracle.uniform_from_words(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 0.5 * 2.0 ** -53
    assert 0.0 < oracle.uniform_from_words(0, 0) < oracle.uniform_from_words(0, 64)


def _single_spin():
    gam = 0.7
    H = sp.csr_matrix((2, 2), dtype=complex)
    C = np.sqrt(gam) * om.sigmam()
    return gam, H, [C]


def test_single_spin_jump_time_is_exact():
    """H = 0, C = sqrt(gamma) sigma_-, psi0 = up: |psi(t)|^2 = exp(-gamma t), so the jump happens at
    t* = -ln(r0)/gamma exactly, into channel 0, and at most once."""
    gam, H, cs = _single_spin()
    tl = np.linspace(0, 10, 21)
    seed = 99
    res = oracle.mcsolve(H, cs, np.array([1, 0], complex), tl, [om.sigmaz()], 64, seed, max_jump_record=2,
                         abstol=1e-12, reltol=1e-10)
    loose = oracle.mcsolve(H, cs, np.array([1, 0], complex), tl, [om.sigmaz()], 64, seed, max_jump_record=2)
    assert (res["status"] == 0).all()
    # at the default tolerances the located time carries the integration error only
    np.testing.assert_allclose(loose["jump_times"][:, 0], res["jump_times"][:, 0], atol=1e-6)
    for j in range(64):
        r0, _ = oracle.traj_draw(seed, j, 0)
        tstar = -np.log(r0) / gam
        if tstar < tl[-1]:
            assert res["njumps"][j] == 1
            assert abs(res["jump_times"][j, 0] - tstar) < 1e-8
            assert res["jump_channels"][j, 0] == 0
            sz = res["expect_tr"][j, 0].real
            np.testing.assert_allclose(sz[tl < tstar - 1e-9], 1.0, atol=1e-12)
            np.testing.assert_allclose(sz[tl > tstar + 1e-9], -1.0, atol=1e-12)
        else:
            assert res["njumps"][j] == 0


def test_single_spin_ensemble():
    """<sigma_z>(t) -> 2 exp(-gamma t) - 1 with binomial standard error."""
    gam, H, cs = _single_spin()
    tl = np.linspace(0, 5, 11)
    n = 4000
    res = oracle.mcsolve(H, cs, np.array([1, 0], complex), tl, [om.sigmaz()], n, 5)
    exact = 2 * np.exp(-gam * tl) - 1
    p = np.exp(-gam * tl)
    se = 2 * np.sqrt(p * (1 - p) / n)
    dev = np.abs(res["mean"][0].real - exact)
    assert (dev[1:] <= 4 * se[1:]).all(), (dev, se)
    np.testing.assert_allclose(res["se"][0, 1:], se[1:], rtol=0.1)


def test_channel_choice_frequencies():
    """Two decay channels from one level: P_k = <C_k^dag C_k> / sum (Sec. 3.3) -> channel 0 with
    probability g0/(g0+g1)."""
    g0, g1 = 0.3, 0.9
    # three levels: 0 decays to 1 (rate g0) and to 2 (rate g1)
    C0 = sp.csr_matrix(([np.sqrt(g0)], ([1], [0])), shape=(3, 3), dtype=complex)
    C1 = sp.csr_matrix(([np.sqrt(g1)], ([2], [0])), shape=(3, 3), dtype=complex)
    H = sp.csr_matrix((3, 3), dtype=complex)
    n = 3000
    res = oracle.mcsolve(H, [C0, C1], np.array([1, 0, 0], complex), np.linspace(0, 30, 3), [C0], n, 17,
                         max_jump_record=1)
    jumped = res["njumps"] == 1
    assert jumped.mean() > 0.99
    frac0 = (res["jump_channels"][jumped, 0] == 0).mean()
    p = g0 / (g0 + g1)
    assert abs(frac0 - p) < 4 * np.sqrt(p * (1 - p) / jumped.sum())


def test_mc_matches_me_ising():
    """Sec. 3.3: the trajectory average reproduces the master-equation result."""
    L = 3
    H, cs = om.ising(L, 1.0, 0.7, 0.2)
    Sz = sum(om.site_op(L, i, om.sigmaz()) for i in range(L))
    tl = np.linspace(0, 6, 25)
    me, _, rc, _ = oracle.mesolve(H, cs, om.all_up_ket(L), tl, [Sz])
    n = 3000
    res = oracle.mcsolve(H, cs, om.all_up_ket(L), tl, [Sz], n, 2024)
    assert (res["status"] == 0).all()
    z = np.abs(res["mean"][0].real - me[0].real)[1:] / res["se"][0, 1:]
    assert (z < 4).all() and (z > 3).mean() < 0.1, z
    assert res["njumps"].min() >= 0 and res["njumps"].max() > res["njumps"].min()  # uneven jump counts


def test_mc_matches_me_complex_operators():
    g = np.random.default_rng(8)
    d = 3
    X = g.normal(size=(d, d)) + 1j * g.normal(size=(d, d))
    H = sp.csr_matrix(X + X.conj().T)
    cs = [sp.csr_matrix(0.5 * (g.normal(size=(d, d)) + 1j * g.normal(size=(d, d)))) for _ in range(2)]
    O = sp.csr_matrix(np.diag([1.0, -0.5, 2.0]) + 0j)
    psi0 = np.array([1, 1j, 0]) / np.sqrt(2)
    tl = np.linspace(0, 3, 13)
    me, _, _, _ = oracle.mesolve(H, cs, psi0, tl, [O])
    res = oracle.mcsolve(H, cs, psi0, tl, [O], 3000, 77)
    z = np.abs(res["mean"][0].real - me[0].real)[1:] / res["se"][0, 1:]
    assert (z < 4).all() and (z > 3).mean() < 0.15, z


def test_trajectories_reproducible_and_independent_of_batching():
    L = 3
    H, cs = om.ising(L, 1.0, 0.7, 0.2)
    Sz = sum(om.site_op(L, i, om.sigmaz()) for i in range(L))
    tl = np.linspace(0, 4, 9)
    a = oracle.mcsolve(H, cs, om.all_up_ket(L), tl, [Sz], 40, 11)
    b = oracle.mcsolve(H, cs, om.all_up_ket(L), tl, [Sz], 10, 11, traj0=30)
    np.testing.assert_array_equal(a["expect_tr"][30:], b["expect_tr"])


def test_ensemble_stats_definition():
    """Ensemble mean and standard error of the real part, against their definitions written out:
    mean over trajectories, SE = sqrt(sum (x - mean)^2 / (N - 1) / N); one trajectory gives SE 0."""
    g = np.random.default_rng(17)
    ex = g.normal(size=(37, 2, 5)) + 1j * g.normal(size=(37, 2, 5))
    mean, se = oracle.ensemble_stats(ex)
    n = ex.shape[0]
    for k in range(2):
        for t in range(5):
            xs = [ex[j, k, t] for j in range(n)]
            m = sum(xs) / n
            v = sum((x.real - m.real) ** 2 for x in xs) / (n - 1) / n
            assert abs(mean[k, t] - m) < 1e-14
            assert abs(se[k, t] - v ** 0.5) < 1e-14
    m1, s1 = oracle.ensemble_stats(ex[:1])
    assert np.all(s1 == 0) and np.allclose(m1, ex[0])


def _expm_expect(H, psi0, tlist, e_ops):
    import scipy.linalg as sl
    Hd = H.toarray() if sp.issparse(H) else np.asarray(H)
    psi0 = np.asarray(psi0, complex) / np.linalg.norm(psi0)
    out = np.zeros((len(e_ops), len(tlist)), complex)
    for n, t in enumerate(tlist):
        psi = sl.expm(-1j * Hd * t) @ psi0
        for k, O in enumerate(e_ops):
            Od = O.toarray() if sp.issparse(O) else np.asarray(O)
            out[k, n] = np.vdot(psi, Od @ psi)
    return out


@pytest.mark.parametrize("case", ["random6", "ising3"])
def test_sesolve_matches_matrix_exponential(case):
    """sesolve against psi(t) = expm(-i H t) psi0 (scipy), at tight tolerances."""
    g = np.random.default_rng(23)
    if case == "random6":
        X = g.normal(size=(6, 6)) + 1j * g.normal(size=(6, 6))
        H = sp.csr_matrix(X + X.conj().T)
        psi0 = g.normal(size=6) + 1j * g.normal(size=6)
        e_ops = [sp.csr_matrix(np.diag(np.arange(6.0))), sp.csr_matrix(g.normal(size=(6, 6)))]
    else:
        H, _ = om.ising(3, 1.0, 0.7, 0.2)
        psi0 = om.all_up_ket(3)
        e_ops = [om.site_op(3, 0, om.sigmaz()), om.site_op(3, 1, om.sigmax())]
    tl = np.linspace(0, 3, 16)
    ex, status = oracle.sesolve(H, psi0, tl, e_ops, abstol=1e-12, reltol=1e-10)
    assert status == 0
    assert np.abs(ex - _expm_expect(H, psi0, tl, e_ops)).max() < 1e-8


def test_sesolve_conserves_energy_and_norm_of_expectations():
    """<H> is a constant of the motion; an unnormalised psi0 gives the same expectations."""
    H, _ = om.ising(4, 1.0, 0.9, 0.2)
    g = np.random.default_rng(3)
    psi0 = g.normal(size=16) + 1j * g.normal(size=16)
    tl = np.linspace(0, 4, 9)
    ex, _ = oracle.sesolve(H, psi0, tl, [H], abstol=1e-12, reltol=1e-10)
    assert np.abs(ex[0] - ex[0, 0]).max() < 1e-8
    ex2, _ = oracle.sesolve(H, 3.0 * psi0, tl, [H], abstol=1e-12, reltol=1e-10)
    assert np.abs(ex2 - ex).max() < 1e-9

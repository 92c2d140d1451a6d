"""GPU parity of the master-equation path (CSR superoperator and dense operator form) against the
FP64 oracle.  Bars: max |d<O>| <= 1e-6 in FP64 mode, <= 1e-4 in mixed FP32/FP64 mode."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import liouvillian as ol
from oracle import models as om
import workloads
import paper_2504_21440_amd as qt

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name + ".json")) as f:
        g = json.load(f)
    return g, np.array(g["expect_re"]) + 1j * np.array(g["expect_im"])


@pytest.fixture(scope="module")
def ctx():
    print("[gpu] creating context", flush=True)
    c = qt.Context(0)
    yield c
    c.close()


def _kerr_lib(p):
    return qt.model_kerr(p["N"], p["delta"], p["U"], p["F"], p["kappa"])


def _ising_lib(p):
    return qt.model_ising(p["L"], p["J"], p["h"], p["gamma"])


# --------------------------------------------------------------------------------------------
# Liouvillian assembly on the device vs the Kronecker definition
# --------------------------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["kerr20", "ising4", "ising8", "random6"])
def test_liouvillian_device_assembly(ctx, case):
    print(f"[gpu] liouvillian assembly {case}", flush=True)
    if case == "kerr20":
        H, cs = om.kerr(20, 1.0, 0.5, 0.8, 1.0)
    elif case == "ising4":
        H, cs = om.ising(4, 1.0, 0.7, 0.2)
    elif case == "ising8":
        H, cs = om.ising(8, 1.0, 0.7, 0.2)
    else:
        g = np.random.default_rng(6)
        X = g.normal(size=(6, 6)) + 1j * g.normal(size=(6, 6))
        H = sp.csr_matrix(X + X.conj().T)
        cs = [sp.csr_matrix(g.normal(size=(6, 6)) + 1j * g.normal(size=(6, 6))) for _ in range(2)]
    ref = ol.liouvillian(H, cs)
    for prec, tol in [(qt.F64, 1e-13), (qt.MIXED, 2e-6)]:
        L = qt.Liouvillian(ctx, H, cs, qt.FORM_CSR, prec)
        d, nnz, _ = L.info()
        got = L.export()
        assert nnz == ref.nnz
        diff = abs(got - ref).max()
        assert diff <= tol * max(1.0, abs(ref).max()), (prec, diff)
        L.close()


# --------------------------------------------------------------------------------------------
# CSR form
# --------------------------------------------------------------------------------------------
def test_kerr_u0_closed_form_csr_f64(ctx):
    print("[gpu] kerr U=0 closed form (CSR, FP64)", flush=True)
    p = workloads.kerr_single(U=0.0)
    H, c = _kerr_lib(p)
    L = qt.Liouvillian(ctx, H, c, qt.FORM_CSR, qt.F64)
    tl = workloads.tlist(p["t_end"], p["nt"])
    N = p["N"]
    ex, st, _ = qt.mesolve(ctx, L, om.fock_dm(N, 0), tl, [om.number(N), om.destroy(N)])
    assert st["status"] == 0
    z = 1j * p["delta"] + 0.5 * p["kappa"]
    al = (-1j * p["F"] / z) * (1 - np.exp(-z * tl))
    assert np.abs(ex[0].real - np.abs(al) ** 2).max() < 1e-6
    assert np.abs(ex[1] - al).max() < 1e-6
    ref, ost, _, _ = oracle.mesolve(H, c, om.fock_dm(N, 0), tl, [om.number(N), om.destroy(N)])
    assert np.abs(ex - ref).max() < 1e-6
    assert abs(st["n_accept"] - ost["n_accept"]) <= 2


def test_kerr_config_csr_f64_vs_golden(ctx):
    print("[gpu] kerr N=20 U=0.5 (CSR, FP64) vs stored oracle values", flush=True)
    g, ref = _gold("kerr_n20_u05")
    H, c = _kerr_lib(g)
    L = qt.Liouvillian(ctx, H, c, qt.FORM_CSR, qt.F64)
    tl = workloads.tlist(g["t_end"], g["nt"])
    ex, st, fin = qt.mesolve(ctx, L, om.fock_dm(g["N"], 0), tl, [om.number(g["N"])], want_final=True)
    assert st["status"] == 0
    assert np.abs(ex - ref).max() <= 1e-6
    assert abs(np.trace(fin) - 1) < 1e-10 and np.abs(fin - fin.conj().T).max() < 1e-12


def test_ising_l8_csr_f64_and_mixed_vs_golden(ctx):
    print("[gpu] ising L=8 (CSR) FP64 and mixed vs stored oracle values", flush=True)
    g, ref = _gold("ising_l8")
    H, cs = _ising_lib(g)
    L = g["L"]
    e_ops = [om.site_op(L, i, om.sigmaz()) for i in range(L)]
    tl = workloads.tlist(g["t_end"], g["nt"])
    L64 = qt.Liouvillian(ctx, H, cs, qt.FORM_CSR, qt.F64)
    ex, st, fin = qt.mesolve(ctx, L64, om.all_up_ket(L), tl, e_ops, want_final=True)
    assert st["status"] == 0
    print("[gpu]   FP64 max|d<sz>| =", np.abs(ex - ref).max(), st, flush=True)
    assert np.abs(ex - ref).max() <= 1e-6
    assert abs(np.trace(fin) - 1) < 1e-10
    assert np.linalg.eigvalsh(0.5 * (fin + fin.conj().T)).min() > -1e-7
    L32 = qt.Liouvillian(ctx, H, cs, qt.FORM_CSR, qt.MIXED)
    exm, stm, finm = qt.mesolve(ctx, L32, om.all_up_ket(L), tl, e_ops,
                                options=qt.opts(precision=qt.MIXED), want_final=True)
    print("[gpu]   mixed max|d<sz>| =", np.abs(exm - ref).max(), stm, flush=True)
    assert stm["status"] == 0
    assert np.abs(exm - ref).max() <= 1e-4
    assert abs(np.trace(finm) - 1) < 1e-6


def test_ising_small_live_oracle(ctx):
    """Small chain against the oracle run live (several blocks and a ragged last block)."""
    for Lc, h in [(3, 0.7), (5, 1.1)]:
        H, cs = qt.model_ising(Lc, 1.0, h, 0.2)
        e_ops = [om.site_op(Lc, i, om.sigmaz()) for i in range(Lc)] + [om.site_op(Lc, 0, om.sigmax())]
        tl = np.linspace(0, 6, 31)
        ref, ost, _, _ = oracle.mesolve(H, cs, om.all_up_ket(Lc), tl, e_ops)
        L = qt.Liouvillian(ctx, H, cs, qt.FORM_CSR, qt.F64)
        ex, st, _ = qt.mesolve(ctx, L, om.all_up_ket(Lc), tl, e_ops)
        assert np.abs(ex - ref).max() <= 1e-6
        assert abs(st["n_accept"] - ost["n_accept"]) <= 2


def test_complex_operators_csr(ctx):
    g = np.random.default_rng(12)
    d = 7
    X = g.normal(size=(d, d)) + 1j * g.normal(size=(d, d))
    H = sp.csr_matrix(X + X.conj().T)
    cs = [sp.csr_matrix(0.4 * (g.normal(size=(d, d)) + 1j * g.normal(size=(d, d)))) for _ in range(2)]
    rho0 = workloads.random_hermitian_dm(d, 3)
    O = sp.csr_matrix(g.normal(size=(d, d)) + 1j * g.normal(size=(d, d)))  # non-Hermitian e_op
    tl = np.linspace(0, 3, 13)
    ref, _, _, _ = oracle.mesolve(H, cs, rho0, tl, [O])
    L = qt.Liouvillian(ctx, H, cs, qt.FORM_CSR, qt.F64)
    ex, st, _ = qt.mesolve(ctx, L, rho0, tl, [O])
    assert np.abs(ex - ref).max() <= 1e-6


# --------------------------------------------------------------------------------------------
# dense operator form (MFMA)
# --------------------------------------------------------------------------------------------
@pytest.mark.parametrize("N,prec", [(20, qt.F64), (37, qt.F64), (48, qt.F64), (20, qt.MIXED), (80, qt.MIXED),
                                    (10, qt.MIXED), (64, qt.MIXED), (1, qt.MIXED)])
def test_kerr_dense_vs_oracle(ctx, N, prec):
    print(f"[gpu] dense kerr N={N} prec={prec}", flush=True)
    p = dict(workloads.kerr_single(), N=N)
    H, c = _kerr_lib(p)
    tl = workloads.tlist(p["t_end"], 41)
    ref, ost, _, _ = oracle.mesolve(H, c, om.fock_dm(N, 0), tl, [om.number(N), om.destroy(N)])
    L = qt.Liouvillian(ctx, H, c, qt.FORM_DENSE, prec)
    ex, st, fin = qt.mesolve(ctx, L, om.fock_dm(N, 0), tl, [om.number(N), om.destroy(N)],
                             options=qt.opts(precision=prec), want_final=True)
    assert st["status"] == 0
    err = np.abs(ex - ref).max()
    print(f"[gpu]   max|d<O>| = {err:.3e}  gpu steps {st['n_accept']}  oracle steps {ost['n_accept']}", flush=True)
    assert err <= (1e-6 if prec == qt.F64 else 1e-4)
    assert abs(np.trace(fin) - 1) < (1e-10 if prec == qt.F64 else 1e-5)


def test_dense_complex_operators_f64(ctx):
    g = np.random.default_rng(21)
    d = 19
    X = g.normal(size=(d, d)) + 1j * g.normal(size=(d, d))
    H = sp.csr_matrix(0.3 * (X + X.conj().T))
    cs = [sp.csr_matrix(0.3 * (g.normal(size=(d, d)) + 1j * g.normal(size=(d, d)))) for _ in range(3)]
    rho0 = workloads.random_hermitian_dm(d, 5)
    O = sp.csr_matrix(np.diag(np.arange(d, dtype=float)) + 0j)
    tl = np.linspace(0, 2, 9)
    ref, _, _, _ = oracle.mesolve(H, cs, rho0, tl, [O])
    L = qt.Liouvillian(ctx, H, cs, qt.FORM_DENSE, qt.F64)
    ex, st, _ = qt.mesolve(ctx, L, rho0, tl, [O])
    assert np.abs(ex - ref).max() <= 1e-6


@pytest.mark.parametrize("d,prec,kinds", [(77, qt.MIXED, "rc"), (33, qt.MIXED, "c"), (45, qt.F64, ""),
                                          (64, qt.MIXED, "rrr"), (40, qt.F64, "cr")])
def test_dense_operator_mixes_vs_oracle(ctx, d, prec, kinds):
    """The dense kernel's product paths: real collapse operators (two real products per complex
    one), complex ones (four), several channels (running sum between channels) and none, at padded
    sizes up to 80, against the oracle."""
    print(f"[gpu] dense operators d={d} prec={prec} channels={kinds or 'none'}", flush=True)
    g = np.random.default_rng(100 + d)
    X = g.normal(size=(d, d)) + 1j * g.normal(size=(d, d))
    H = sp.csr_matrix(0.1 * (X + X.conj().T))
    cs = []
    for k in kinds:
        C = 0.15 * g.normal(size=(d, d))
        if k == "c":
            C = C + 0.15j * g.normal(size=(d, d))
        cs.append(sp.csr_matrix(C))
    rho0 = workloads.random_hermitian_dm(d, 4)
    O = sp.csr_matrix(np.diag(np.arange(d, dtype=float)) + 0j)
    tl = np.linspace(0, 1, 6)
    ref, _, _, _ = oracle.mesolve(H, cs, rho0, tl, [O])
    L = qt.Liouvillian(ctx, H, cs, qt.FORM_DENSE, prec)
    ex, st, fin = qt.mesolve(ctx, L, rho0, tl, [O], options=qt.opts(precision=prec), want_final=True)
    assert st["status"] == 0
    err = np.abs(ex - ref).max() / max(1.0, np.abs(ref).max())
    print(f"[gpu]   relative max|d<O>| = {err:.3e}", flush=True)
    assert err <= (1e-6 if prec == qt.F64 else 1e-4)
    # Hermitian by construction: off the diagonal each element is its mirror's conjugate exactly
    np.testing.assert_array_equal(np.triu(fin, 1), np.triu(fin.conj().T, 1))
    assert np.abs(np.diag(fin).imag).max() < (1e-10 if prec == qt.F64 else 1e-5)


# --------------------------------------------------------------------------------------------
# batches: every result is the same alone and in the mix
# --------------------------------------------------------------------------------------------
def test_batch_alone_vs_mix_bitwise(ctx):
    print("[gpu] batch alone vs mix", flush=True)
    sweep = workloads.kerr_sweep(n=6, seed=9, n_min=10, n_max=40)
    probs = []
    for p in sweep:
        H, c = _kerr_lib(p)
        probs.append((qt.Liouvillian(ctx, H, c, qt.FORM_DENSE, qt.MIXED), om.fock_dm(p["N"], 0),
                      workloads.tlist(p["t_end"], 21), [om.number(p["N"])]))
    for Lc, h in [(4, 0.5), (5, 0.9)]:
        H, cs = qt.model_ising(Lc, 1.0, h, 0.2)
        probs.append((qt.Liouvillian(ctx, H, cs, qt.FORM_CSR, qt.MIXED), om.all_up_ket(Lc),
                      np.linspace(0, 10, 21), [om.site_op(Lc, 0, om.sigmaz())]))
    o = qt.opts(precision=qt.MIXED)

    def solve(prs):
        plan = qt.MePlan(ctx, prs, o)
        plan.set_shape(8, 1)  # one CSR shape for both, so the reduction orders agree
        plan.run()
        out = [plan.result(i) for i in range(len(prs))]
        plan.close()
        return out

    mix = solve(probs)
    for i, pr in enumerate(probs):
        alone = solve([pr])[0]
        np.testing.assert_array_equal(alone[0], mix[i][0])
        assert alone[1]["n_accept"] == mix[i][1]["n_accept"]


SHAPES = [(l, r) for l in (4, 8, 16) for r in (1, 2, 4) if r <= l]
WIDE = [(4, 1), (8, 1), (8, 2), (16, 1)]  # also built with 16-byte matrix loads (cached_matrix = 2)
# every (shape, block order, matrix load kind) the CSR kernels are built with
LAUNCHES = [(sh, x, k) for k in (0, 1) for x in (0, 1) for sh in SHAPES] + [(sh, x, 2) for x in (0, 1) for sh in WIDE]


def test_csr_every_tile_shape_vs_oracle(ctx):
    """Each (lanes per row, rows per lane group) shape of the CSR kernels against the oracle, on two
    chains solved together (1024 and 64 rows: partial last blocks for every shape)."""
    chains = [(5, 0.9), (3, 0.7)]
    tl = np.linspace(0, 4, 21)
    refs, probs = [], {qt.F64: [], qt.MIXED: []}
    for Lc, h in chains:
        H, cs = qt.model_ising(Lc, 1.0, h, 0.2)
        e_ops = [om.site_op(Lc, i, om.sigmaz()) for i in range(Lc)]
        refs.append(oracle.mesolve(H, cs, om.all_up_ket(Lc), tl, e_ops)[0])
        for prec in (qt.F64, qt.MIXED):
            probs[prec].append((qt.Liouvillian(ctx, H, cs, qt.FORM_CSR, prec), om.all_up_ket(Lc), tl, e_ops))
    for prec, tol in [(qt.F64, 1e-6), (qt.MIXED, 1e-4)]:
        plan = qt.MePlan(ctx, probs[prec], qt.opts(precision=prec))
        for (lpr, rg), xcd, keep in LAUNCHES:
            print(f"[gpu] CSR shape lpr={lpr} rg={rg} xcd={xcd} keep={keep} prec={prec}", flush=True)
            plan.set_shape(lpr, rg, xcd, keep)
            assert plan.shape()[:4] == (lpr, rg, 0, keep)  # two problems: round-robin order
            plan.run()
            for i, ref in enumerate(refs):
                ex, st, _ = plan.result(i)
                assert st["status"] == 0
                assert np.abs(ex - ref).max() <= tol, (lpr, rg, prec, i, np.abs(ex - ref).max())
        plan.close()
    with pytest.raises(qt.QtError):
        plan = qt.MePlan(ctx, probs[qt.F64][:1], qt.opts())
        plan.set_shape(8, 8)
    with pytest.raises(qt.QtError):  # 16-byte loads are not built for 4 rows per lane group
        plan = qt.MePlan(ctx, probs[qt.F64][:1], qt.opts())
        plan.set_shape(8, 4, 0, 2)


def test_ising_l10_hbm_sized_every_shape_vs_golden(ctx):
    """The HBM-sized Liouvillian the SpMV bandwidth is measured on (1,048,576 rows, 24.6 M nnz),
    integrated over a short window with every tile shape, FP64 and mixed, against stored oracle
    values."""
    g, ref = _gold("ising_l10_short")
    H, cs = _ising_lib(g)
    e_ops = [om.site_op(10, 0, om.sigmaz()), om.site_op(10, 4, om.sigmax())]
    tl = np.linspace(0.0, g["t_end"], g["nt"])
    for prec, tol in [(qt.F64, 1e-6), (qt.MIXED, 1e-4)]:
        Lo = qt.Liouvillian(ctx, H, cs, qt.FORM_CSR, prec)
        assert Lo.info()[1] == 24_641_535
        plan = qt.MePlan(ctx, [(Lo, om.all_up_ket(10), tl, e_ops)], qt.opts(precision=prec))
        for (lpr, rg), xcd, keep in LAUNCHES:
            print(f"[gpu] L=10 shape lpr={lpr} rg={rg} xcd={xcd} keep={keep} prec={prec}", flush=True)
            plan.set_shape(lpr, rg, xcd, keep)
            assert plan.shape()[:4] == (lpr, rg, xcd, keep)
            plan.run()
            ex, st, _ = plan.result(0)
            assert st["status"] == 0
            assert np.abs(ex - ref).max() <= tol, (lpr, rg, prec, np.abs(ex - ref).max())
        plan.close()
        Lo.close()


def test_ising_batch_16_mixed_vs_golden(ctx):
    """Sixteen L=8 chains in one plan (the batched configuration of the benchmark), mixed precision
    at the accuracy-matched tolerance (rtol 1e-4, atol 1e-6): stored oracle values for three
    members, the trace-bounded range of <sigma_z> for all."""
    with open(os.path.join(GOLD, "ising_batch_members.json")) as f:
        gold = json.load(f)
    batch = workloads.ising_batch(n=16)
    probs = []
    for p in batch:
        H, cs = qt.model_ising(p["L"], p["J"], p["h"], p["gamma"])
        probs.append((qt.Liouvillian(ctx, H, cs, qt.FORM_CSR, qt.MIXED), om.all_up_ket(8),
                      workloads.tlist(p["t_end"], p["nt"]), [om.site_op(8, i, om.sigmaz()) for i in range(8)]))
    plan = qt.MePlan(ctx, probs, qt.opts(abstol=1e-6, reltol=1e-4, precision=qt.MIXED))
    plan.run()
    for i in range(16):
        ex, st, _ = plan.result(i)
        assert st["status"] == 0
        assert np.all(np.abs(ex.real) <= 1 + 1e-4)
    for g in gold["members"]:
        ref = np.array(g["expect_re"]) + 1j * np.array(g["expect_im"])
        err = np.abs(plan.result(g["index"])[0] - ref).max()
        print(f"[gpu]   batch member {g['index']} (h={g['h']:.2f}): max|d<sz>| = {err:.2e}", flush=True)
        assert err <= 1e-4
    plan.close()


def test_plan_rerun_is_deterministic(ctx):
    H, cs = qt.model_ising(6, 1.0, 0.7, 0.2)
    L = qt.Liouvillian(ctx, H, cs, qt.FORM_CSR, qt.MIXED)
    plan = qt.MePlan(ctx, [(L, om.all_up_ket(6), np.linspace(0, 5, 11), [om.site_op(6, 2, om.sigmaz())])],
                     qt.opts(precision=qt.MIXED))
    plan.run()
    a = plan.result(0)[0]
    plan.run()
    b = plan.result(0)[0]
    np.testing.assert_array_equal(a, b)


# --------------------------------------------------------------------------------------------
# edge cases and error paths
# --------------------------------------------------------------------------------------------
def test_single_time_point_and_unnormalised_state(ctx):
    H, c = qt.model_kerr(8, 1.0, 0.5, 0.8, 1.0)
    rho0 = 2.5 * om.fock_dm(8, 1)
    for form in (qt.FORM_CSR, qt.FORM_DENSE):
        L = qt.Liouvillian(ctx, H, c, form, qt.F64)
        ex, st, _ = qt.mesolve(ctx, L, rho0, np.array([0.3]), [om.number(8)])
        assert st["status"] == 0 and abs(ex[0, 0] - 2.5) < 1e-14
        tl = np.linspace(0, 2, 5)
        ex, st, _ = qt.mesolve(ctx, L, rho0, tl, [om.number(8)])
        ref, _, _, _ = oracle.mesolve(H, c, rho0, tl, [om.number(8)])
        assert np.abs(ex - ref).max() <= 1e-6


def test_error_paths(ctx):
    H, c = qt.model_kerr(8, 1.0, 0.5, 0.8, 1.0)
    L = qt.Liouvillian(ctx, H, c, qt.FORM_CSR, qt.F64)
    with pytest.raises(qt.QtError) as e:
        qt.mesolve(ctx, L, om.fock_dm(8, 0), np.array([0.0, 1.0, 1.0]), [om.number(8)])
    assert e.value.code == qt.QT_EINVAL
    with pytest.raises(qt.QtError) as e:
        qt.mesolve(ctx, L, om.fock_dm(8, 0), np.linspace(0, 20, 3), [om.number(8)], options=qt.opts(max_steps=3))
    assert e.value.code == qt.QT_EMAXSTEPS
    Hn = H.copy()
    Hn.data[0] = np.nan
    with pytest.raises(qt.QtError) as e:
        qt.Liouvillian(ctx, Hn, c, qt.FORM_CSR, qt.F64)
    assert e.value.code == qt.QT_EINVAL
    with pytest.raises(qt.QtError) as e:
        qt.mesolve(ctx, L, om.fock_dm(8, 0), np.linspace(0, 1, 3), [om.number(8)],
                   options=qt.opts(precision=qt.MIXED))
    assert e.value.code == qt.QT_EINVAL  # precision mismatch
    with pytest.raises(qt.QtError):
        qt.Liouvillian(ctx, *qt.model_kerr(100, 1.0, 0.5, 0.8, 1.0), qt.FORM_DENSE, qt.MIXED)


def test_expect_on_device_state(ctx):
    from hipmem import DeviceArray
    d = 12
    g = np.random.default_rng(2)
    rho = workloads.random_hermitian_dm(d, 4)
    O = sp.csr_matrix(g.normal(size=(d, d)) + 1j * g.normal(size=(d, d)))
    ref = oracle.expect_dm(O, rho)
    a = DeviceArray(rho)
    assert abs(qt.expect(ctx, O, a.address, d, False, qt.F64) - ref) < 1e-12
    a32 = DeviceArray(rho.astype(np.complex64))
    assert abs(qt.expect(ctx, O, a32.address, d, False, qt.MIXED) - ref) < 1e-5
    psi = workloads.random_ket(d, 8) * 1.7
    k = DeviceArray(psi)
    assert abs(qt.expect(ctx, O, k.address, d, True, qt.F64) - oracle.expect_ket(O, psi)) < 1e-12
    for x in (a, a32, k):
        x.free()


def test_autotune_chooses_a_kernel_shape_and_keeps_parity(ctx, tmp_path):
    print("[gpu] autotune CSR + dense", flush=True)
    H, cs = qt.model_ising(6, 1.0, 0.7, 0.2)
    e_ops = [om.site_op(6, 2, om.sigmaz())]
    tl = np.linspace(0, 3, 11)
    ref = oracle.mesolve(H, cs, om.all_up_ket(6), tl, e_ops)[0]
    Hk, ck = qt.model_kerr(20, 1.0, 0.5, 0.8, 1.0)
    refk = oracle.mesolve(Hk, ck, om.fock_dm(20, 0), tl, [om.number(20)])[0]
    o = qt.opts(precision=qt.MIXED, autotune=True)
    probs = [(qt.Liouvillian(ctx, H, cs, qt.FORM_CSR, qt.MIXED), om.all_up_ket(6), tl, e_ops),
             (qt.Liouvillian(ctx, Hk, ck, qt.FORM_DENSE, qt.MIXED), om.fock_dm(20, 0), tl, [om.number(20)])]
    plan = qt.MePlan(ctx, probs, o)
    lpr, rg, xcd, keep, waves = plan.shape()
    assert (lpr, rg) in SHAPES and xcd in (0, 1) and keep in (0, 1, 2) and waves in (1, 2, 4)
    assert keep < 2 or (lpr, rg) in WIDE
    plan.run()
    assert np.abs(plan.result(0)[0] - ref).max() <= 1e-4
    assert np.abs(plan.result(1)[0] - refk).max() <= 1e-4
    path = tmp_path / "tune.json"
    qt.tune_save(str(path))
    table = json.loads(path.read_text())
    assert [lpr, rg, xcd, keep] in table.values()
    assert table.get("dense:mixed:np32:waves") == [waves]
    plan.close()


@pytest.mark.parametrize("prec", [qt.F64, qt.MIXED])
def test_folded_step_control_is_bitwise_the_control_kernel(ctx, prec):
    """One constant problem with runs of 4 stored entries takes its step control inside the next
    step's stage-2 launch (double-buffered control record); an odd number of steps per graph keeps
    the separate control launch.  Both take the same decisions in the same reduction order, so the
    solutions, save times and step counts agree bitwise -- with rejected steps (a first step far too
    large) and with the trace renormalisation of the mixed path -- and match the oracle."""
    print(f"[gpu] folded step control vs control kernel, prec={prec}", flush=True)
    H, cs = qt.model_ising(6, 1.0, 0.8, 0.2)
    e_ops = [om.site_op(6, 0, om.sigmaz()), om.site_op(6, 3, om.sigmax())]
    tl = np.linspace(0.0, 3.0, 13)
    Lo = qt.Liouvillian(ctx, H, cs, qt.FORM_CSR, prec)
    out = []
    for spl in (16, 15):  # 16: folded control; 15 (odd): the control kernel
        o = qt.opts(abstol=1e-8, reltol=1e-6, precision=prec, h0=0.5, steps_per_launch=spl)
        plan = qt.MePlan(ctx, [(Lo, om.all_up_ket(6), tl, e_ops)], o)
        plan.set_shape(8, 2, 0, 2)
        plan.run()
        plan.run()  # a second run from the start: the record buffers are reset
        out.append(plan.result(0))
        plan.close()
    (ea, sa, _), (eb, sb, _) = out
    np.testing.assert_array_equal(ea, eb)
    for k in ("n_accept", "n_reject", "n_rhs", "status"):
        assert sa[k] == sb[k], (k, sa[k], sb[k])
    assert sa["status"] == 0 and sa["n_reject"] > 0
    Ho, co = om.ising(6, 1.0, 0.8, 0.2)
    ref = oracle.mesolve(Ho, co, om.all_up_ket(6), tl, e_ops, abstol=1e-8, reltol=1e-6, h0=0.5)[0]
    assert np.abs(ea - ref).max() <= (1e-6 if prec == qt.F64 else 1e-4)
    Lo.close()

"""The allocation-free expectation value (qt_expect_noalloc) against qt_expect, through the C ABI.

Both entry points run the same kernel on the same canonical operator, so their results agree
bitwise; each is also checked against the FP64 oracle.  Two calls in a row, the second with a
smaller operator and state, show that the shared scratch array holds no state a call depends on.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import paper_2504_21440_amd as qt
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    print("[gpu] no-alloc: creating context", flush=True)
    c = qt.Context(0)
    yield c
    c.close()


def _random_op(d, density, seed):
    g = np.random.default_rng(seed)
    A = sp.random(d, d, density=density, random_state=seed, format="csr")
    A.data = g.normal(size=A.nnz) + 1j * g.normal(size=A.nnz)
    A.sort_indices()
    return A.tocsr()


@pytest.mark.parametrize("d1,d2", [(96, 12), (40, 7)])
def test_noalloc_expect_matches_qt_expect_on_two_calls(ctx, d1, d2):
    from hipmem import DeviceArray
    for d, dens, seed in ((d1, 0.6, 11), (d2, 0.9, 12)):
        print(f"[gpu] no-alloc expect d={d} density={dens} seed={seed}", flush=True)
        O = _random_op(d, dens, seed)
        rho = workloads.random_hermitian_dm(d, seed)
        psi = workloads.random_ket(d, seed + 100) * 1.3
        cases = [(DeviceArray(rho), False, qt.F64, oracle.expect_dm(O, rho), 1e-12),
                 (DeviceArray(rho.astype(np.complex64)), False, qt.MIXED, oracle.expect_dm(O, rho), 1e-5),
                 (DeviceArray(psi), True, qt.F64, oracle.expect_ket(O, psi), 1e-12)]
        for arr, is_ket, prec, ref, tol in cases:
            a = qt.expect(ctx, O, arr.address, d, is_ket, prec)
            b = qt.expect_noalloc(ctx, O, arr.address, d, is_ket, prec)
            assert a == b, (d, is_ket, prec, a, b)
            assert abs(b - ref) <= tol * max(1.0, abs(ref)), (d, is_ket, prec, b, ref)
            arr.free()


def test_noalloc_expect_rejects_operators_beyond_the_scratch(ctx):
    from hipmem import DeviceArray
    d = 400_000  # 12 (d + 1) + 20 d bytes > 8 MiB: refused on the host before any device work
    print(f"[gpu] no-alloc size limit d={d}", flush=True)
    O = sp.identity(d, dtype=np.complex128, format="csr")
    psi = np.zeros(d, np.complex128)
    psi[0] = 1.0
    arr = DeviceArray(psi)
    with pytest.raises(qt.QtError) as ei:
        qt.expect_noalloc(ctx, O, arr.address, d, True, qt.F64)
    assert ei.value.code == qt.QT_ENOMEM
    # a call within the limit still works afterwards
    small = sp.identity(16, dtype=np.complex128, format="csr")
    assert qt.expect_noalloc(ctx, small, arr.address, 16, True, qt.F64) == 1.0
    arr.free()

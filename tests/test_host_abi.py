"""Host-side parts of the C ABI (no GPU): exported symbols, model operators, argument checks."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2504_21440_amd as qt
from oracle import models as om

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "qtamd.h")).read()
    decl = r"^(?:qt_status|void|const char \*)\s*(qt_[a-z0-9_]+)\s*\("
    return sorted(set(re.findall(decl, src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    L = qt.lib()
    names = _declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(qt.EXPORTED)


def test_version_and_default_opts():
    assert b"gfx950" in qt.lib().qt_version()
    o = qt.Opts()
    qt.lib().qt_opts_default(ctypes.byref(o))
    assert (o.abstol, o.reltol, o.max_steps, o.h0, o.precision, o.form) == (1e-8, 1e-6, 1_000_000, 0.0, 0, 0)


def _close(A, B):
    return abs(A - B).max() <= 1e-14 * max(1.0, abs(B).max())


@pytest.mark.parametrize("N,U", [(1, 0.5), (5, 0.0), (20, 0.5), (80, 0.9)])
def test_kerr_operators_match_oracle_builder(N, U):
    H, c = qt.model_kerr(N, 1.3, U, 0.8, 0.7)
    H2, c2 = om.kerr(N, 1.3, U, 0.8, 0.7)
    assert _close(H, H2) and _close(c[0], c2[0])


@pytest.mark.parametrize("L", [1, 2, 6, 10])
def test_ising_operators_match_oracle_builder(L):
    H, cs = qt.model_ising(L, 1.0, 0.7, 0.2)
    H2, cs2 = om.ising(L, 1.0, 0.7, 0.2)
    assert _close(H, H2)
    assert len(cs) == L
    for a, b in zip(cs, cs2):
        assert _close(a, b)


def test_model_argument_errors():
    with pytest.raises(qt.QtError) as e:
        qt.model_kerr(0, 1, 1, 1, 1)
    assert e.value.code == qt.QT_EINVAL
    with pytest.raises(qt.QtError):
        qt.model_ising(0, 1, 1, 1)


def test_tuning_table_roundtrip(tmp_path):
    """The autotuner table persists as JSON; unsupported shapes in a file are ignored on load."""
    src = tmp_path / "in.json"
    src.write_text(
        '{\n'
        '  "csr:mixed:n20:r19": [16, 2, 1, 1],\n'
        '  "csr:f64:n12:r7": [4, 4],\n'
        '  "csr:f64:n13:r7": [4, 8],\n'      # rows per group above the lanes: not a kernel shape
        '  "csr:f64:n14:r7": [32, 1],\n'     # 32 lanes per row: not a kernel shape
        '  "dense:mixed:np32:waves": [4],\n'
        '  "dense:mixed:np48": [2],\n'       # the older waves-per-row form of the key
        '  "dense:mixed:np80:waves": [3],\n'  # 3 waves are not built for this size
        '  "dense:f64:np48:waves": [8]\n'    # 8 waves are not built for FP64
        '}\n')
    qt.tune_load(str(src))
    out = tmp_path / "out.json"
    qt.tune_save(str(out))
    import json
    table = json.loads(out.read_text())
    assert table["csr:mixed:n20:r19"] == [16, 2, 1, 1]
    assert table["csr:f64:n12:r7"] == [4, 4, 0, 0]  # a two-number entry reads as round-robin, streamed
    assert table["dense:mixed:np32:waves"] == [4]
    for bad in ("csr:f64:n13:r7", "csr:f64:n14:r7", "dense:mixed:np48", "dense:mixed:np80:waves",
                "dense:f64:np48:waves"):
        assert bad not in table
    with pytest.raises(qt.QtError):
        qt.tune_load(str(tmp_path / "missing.json"))

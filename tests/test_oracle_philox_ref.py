"""Pin of the oracle's Philox-4x32-10 against rocRAND's host-callable Philox engine.

rocRAND's engine keys Philox with the 64-bit seed and places the 'subsequence' in counter words
2-3 and offset/4 in counter words 0-1, so the oracle's draw for (seed, trajectory j, event m),
counter (j_lo, j_hi, m, 0), is the engine's first block at subsequence m and offset 4 j.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def refbin(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    out = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.check_call([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", "-o", out,
                           os.path.join(HERE, "philox_ref.cpp")])
    return out


def test_philox_matches_rocrand_engine(refbin):
    g = np.random.default_rng(3)
    cases = [(0, 0, 0), (1, 0, 0), (2**64 - 1, 5, 4 * 7), (20250430, 3, 4 * 123456789)]
    cases += [(int(g.integers(0, 2**63)), int(g.integers(0, 1000)), 4 * int(g.integers(0, 2**40)))
              for _ in range(200)]
    inp = "".join(f"{s} {m} {o}\n" for s, m, o in cases)
    res = subprocess.run([refbin], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for (s, m, o), line in zip(cases, res):
        ref = [int(x) for x in line.split()]
        j = o // 4
        key = [s & 0xFFFFFFFF, s >> 32]
        ctr = [j & 0xFFFFFFFF, j >> 32, m & 0xFFFFFFFF, m >> 32]
        assert [int(x) for x in oracle.philox(ctr, key)] == ref, (s, m, o)

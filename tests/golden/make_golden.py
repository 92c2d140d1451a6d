"""Writes the stored expected values under tests/golden/ by calling only the oracle.

Run from the repository root:  python tests/golden/make_golden.py [name ...]
Each file records the workload parameters, tolerances and the oracle's statistics beside the values.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import models as om  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def _write(name, meta, expect):
    path = os.path.join(OUT, name + ".json")
    meta = dict(meta)
    meta["expect_re"] = np.asarray(expect).real.tolist()
    meta["expect_im"] = np.asarray(expect).imag.tolist()
    with open(path, "w") as f:
        json.dump(meta, f)
    print("wrote", path)


def ising_me(L, h, gamma, t_end, nt, e_kind, abstol, reltol, name):
    H, cs = om.ising(L, 1.0, h, gamma)
    if e_kind == "sz_each":
        e_ops = [om.site_op(L, i, om.sigmaz()) for i in range(L)]
    else:
        e_ops = [sum(om.site_op(L, i, om.sigmaz()) for i in range(L))]
    tl = workloads.tlist(t_end, nt)
    t0 = time.time()
    ex, st, rc, _ = oracle.mesolve(H, cs, om.all_up_ket(L), tl, e_ops, abstol=abstol, reltol=reltol)
    assert rc == 0, rc
    _write(name, {"workload": "ising", "L": L, "J": 1.0, "h": h, "gamma": gamma, "t_end": t_end, "nt": nt,
                  "e_ops": e_kind, "abstol": abstol, "reltol": reltol, "oracle_stats": st,
                  "oracle_seconds": time.time() - t0, "source": "oracle.mesolve"}, ex)


def kerr_me(U, abstol, reltol, name):
    p = workloads.kerr_single(U=U)
    N = p["N"]
    H, cs = om.kerr(N, p["delta"], p["U"], p["F"], p["kappa"])
    tl = workloads.tlist(p["t_end"], p["nt"])
    t0 = time.time()
    ex, st, rc, _ = oracle.mesolve(H, cs, om.fock_dm(N, 0), tl, [om.number(N)], abstol=abstol, reltol=reltol)
    assert rc == 0
    _write(name, dict(p, abstol=abstol, reltol=reltol, oracle_stats=st, oracle_seconds=time.time() - t0,
                      source="oracle.mesolve"), ex)


def sweep_sample_indices(n=512, extra=6, seed=11):
    """Instances of the 512-cavity sweep checked one by one: the smallest and largest cutoff and a
    seeded random draw of the others."""
    Ns = np.array([p["N"] for p in workloads.kerr_sweep(n=n)])
    pick = [int(Ns.argmin()), int(Ns.argmax())]
    g = np.random.Generator(np.random.PCG64(seed))
    for i in g.permutation(n):
        if len(pick) >= 2 + extra:
            break
        if int(i) not in pick:
            pick.append(int(i))
    return pick


def kerr_sweep_samples(name):
    sweep = workloads.kerr_sweep(n=512)
    out = {"workload": "kerr_sweep", "n": 512, "abstol": 1e-8, "reltol": 1e-6, "source": "oracle.mesolve",
           "instances": []}
    for i in sweep_sample_indices():
        p = sweep[i]
        H, cs = om.kerr(p["N"], p["delta"], p["U"], p["F"], p["kappa"])
        tl = workloads.tlist(p["t_end"], p["nt"])
        t0 = time.time()
        ex, st, rc, _ = oracle.mesolve(H, cs, om.fock_dm(p["N"], 0), tl, [om.number(p["N"])])
        assert rc == 0
        out["instances"].append(dict(p, index=i, oracle_stats=st, oracle_seconds=time.time() - t0,
                                     expect_re=ex.real.tolist(), expect_im=ex.imag.tolist()))
        print("sweep instance", i, "N", p["N"], st)
    path = os.path.join(OUT, name + ".json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


def ising_l10_short(name):
    """The HBM-sized chain (L = 10: 1,048,576 Liouville rows) over a short window."""
    L, h, gamma = 10, 1.0, 0.1
    H, cs = om.ising(L, 1.0, h, gamma)
    e_ops = [om.site_op(L, 0, om.sigmaz()), om.site_op(L, 4, om.sigmax())]
    tl = np.linspace(0.0, 0.3, 4)
    t0 = time.time()
    ex, st, rc, _ = oracle.mesolve(H, cs, om.all_up_ket(L), tl, e_ops)
    assert rc == 0
    _write(name, {"workload": "ising", "L": L, "J": 1.0, "h": h, "gamma": gamma, "t_end": 0.3, "nt": 4,
                  "e_ops": "sz_0,sx_4", "abstol": 1e-8, "reltol": 1e-6, "oracle_stats": st,
                  "oracle_seconds": time.time() - t0, "source": "oracle.mesolve"}, ex)


def ising_batch_members(name, members=(0, 7, 15)):
    """Members of the 16-chain batch (h = 0.3 + 0.08 i), <sigma_z^i> at 100 times."""
    batch = workloads.ising_batch(n=16)
    out = {"workload": "ising_batch", "n": 16, "abstol": 1e-8, "reltol": 1e-6, "source": "oracle.mesolve",
           "members": []}
    for i in members:
        p = batch[i]
        H, cs = om.ising(p["L"], p["J"], p["h"], p["gamma"])
        e_ops = [om.site_op(p["L"], k, om.sigmaz()) for k in range(p["L"])]
        ex, st, rc, _ = oracle.mesolve(H, cs, om.all_up_ket(p["L"]), workloads.tlist(p["t_end"], p["nt"]), e_ops)
        assert rc == 0
        out["members"].append(dict(p, index=i, oracle_stats=st, expect_re=ex.real.tolist(),
                                   expect_im=ex.imag.tolist()))
    path = os.path.join(OUT, name + ".json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


JOBS = {
    "ising_batch_members": lambda: ising_batch_members("ising_batch_members"),
    "kerr_sweep_samples": lambda: kerr_sweep_samples("kerr_sweep_samples"),
    "ising_l10_short": lambda: ising_l10_short("ising_l10_short"),
    "kerr_n20_u05": lambda: kerr_me(0.5, 1e-8, 1e-6, "kerr_n20_u05"),
    "ising_l8": lambda: ising_me(8, 0.7, 0.2, 10.0, 100, "sz_each", 1e-8, 1e-6, "ising_l8"),
    "ising_l8_tight": lambda: ising_me(8, 0.7, 0.2, 10.0, 100, "sz_each", 1e-12, 1e-10, "ising_l8_tight"),
    "ising_l10_me": lambda: ising_me(10, 1.0, 0.1, 10.0, 100, "sz_sum", 1e-8, 1e-6, "ising_l10_me"),
}

if __name__ == "__main__":
    oracle.build()
    for n in (sys.argv[1:] or list(JOBS)):
        JOBS[n]()

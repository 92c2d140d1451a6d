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


def _serving_ref(p):
    """Oracle reference of one served request (abstol 1e-10, reltol 1e-8): <a^dag a> of a Kerr cavity
    from vacuum, or <sigma_z> of the first spin of a chain from all up, at 100 times."""
    tl = workloads.tlist(p["t_end"], p["nt"])
    t0 = time.time()
    if p["kind"] == "kerr":
        H, cs = om.kerr(p["N"], p["delta"], p["U"], p["F"], p["kappa"])
        ex, st, rc, _ = oracle.mesolve(H, cs, om.fock_dm(p["N"], 0), tl, [om.number(p["N"])], abstol=1e-10,
                                       reltol=1e-8)
    else:
        H, cs = om.ising(p["L"], p["J"], p["h"], p["gamma"])
        ex, st, rc, _ = oracle.mesolve(H, cs, om.all_up_ket(p["L"]), tl, [om.site_op(p["L"], 0, om.sigmaz())],
                                       abstol=1e-10, reltol=1e-8)
    assert rc == 0, (p, rc)
    return dict(p, oracle_stats=st, oracle_seconds=time.time() - t0, expect_re=ex.real.tolist(),
                expect_im=ex.imag.tolist())


def _one_thread_worker():
    os.environ["OMP_NUM_THREADS"] = "1"


def serving_trace_refs(name, n=240, workers=None):
    """References for the first n requests of the served stream (request parameters do not depend
    on the offered load, only the arrival times do), one single-threaded oracle solve per request,
    solved in parallel processes."""
    import multiprocessing as mp
    trace = workloads.serving_trace(n=n)
    # largest problems first so that the pool's tail is short
    order = sorted(range(n), key=lambda i: -(trace[i]["N"] ** 2 * (1 + trace[i]["U"]) if trace[i]["kind"] == "kerr"
                                              else 4.0 ** trace[i]["L"] * 3))
    ctx = mp.get_context("fork")
    with ctx.Pool(workers or int(os.environ.get("GOLDEN_WORKERS", os.cpu_count())), initializer=_one_thread_worker) as pool:
        res = pool.map(_serving_ref, [trace[i] for i in order], chunksize=1)
    refs = [None] * n
    for i, r in zip(order, res):
        refs[i] = r
    out = {"workload": "serving_trace", "n": n, "abstol": 1e-10, "reltol": 1e-8, "source": "oracle.mesolve",
           "e_op": "kerr: a^dag a; ising: sigma_z of spin 0", "requests": refs}
    path = os.path.join(OUT, name + ".json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


def sesolve_l10(name, abstol=1e-12, reltol=1e-10):
    """Closed L = 10 chain (J = 1, h = 1, all up), <sum sigma_z> at 100 times over t in [0, 10]."""
    p = workloads.ising_mc()
    L = p["L"]
    H, _ = om.ising(L, p["J"], p["h"], p["gamma"])
    Sz = sum(om.site_op(L, i, om.sigmaz()) for i in range(L))
    tl = workloads.tlist(p["t_end"], p["nt"])
    t0 = time.time()
    ex, rc = oracle.sesolve(H, om.all_up_ket(L), tl, [Sz], abstol=abstol, reltol=reltol)
    assert rc == 0, rc
    _write(name, {"workload": "sesolve_ising", "L": L, "J": p["J"], "h": p["h"], "t_end": p["t_end"], "nt": p["nt"],
                  "e_ops": "sz_sum", "abstol": abstol, "reltol": reltol,
                  "oracle_seconds": time.time() - t0, "source": "oracle.sesolve"}, ex)


def optomech_full(name):
    """The driven optomechanical example over its whole window (t in [0, 5 / kappa], 5000 saves of
    <a^dag a>) at the default tolerances (abstol 1e-8, reltol 1e-6)."""
    p = workloads.optomech_td()
    H0, xa, c_ops, n_op = om.optomech(p["Nc"], p["Nm"], p["wc"], p["wm"], p["g"], p["kappa"], p["gamma"])
    d = p["Nc"] * p["Nm"]
    tl = workloads.tlist(p["t_end"], p["nt"])
    t0 = time.time()
    ex, st, rc, _ = oracle.mesolve_td(H0, [(xa, {"kind": "cos", "a": p["F"], "omega": p["wd"]})], c_ops,
                                      om.fock_dm(d, 0), tl, [n_op])
    assert rc == 0, rc
    _write(name, dict(p, abstol=1e-8, reltol=1e-6, oracle_stats=st, oracle_seconds=time.time() - t0,
                      source="oracle.mesolve_td"), ex)


def jc_homodyne_traj(name, ntraj=2):
    """The first trajectories of the homodyne example (cavity cutoff 20, step 1e-3 over t in
    [0, 2 pi], 400 saves), stochastic Schrodinger and master equations, FP64: <X> per save time
    and the measurement current per interval."""
    p = workloads.jc_homodyne()
    H, S, C, X, psi0 = om.jc_homodyne(p["N"], p["wc"], p["wq"], p["g"], p["kappa"], p["gamma"], p["kappa_phi"],
                                      p["alpha"])
    tl = workloads.tlist(p["t_end"], p["nt"])
    out = dict(p, ntraj_stored=ntraj, source="oracle.ssesolve / oracle.smesolve")
    for key, fn in [("sse", lambda: oracle.ssesolve(H, S, psi0, tl, [X], ntraj, p["seed"], p["dt"])),
                    ("sme", lambda: oracle.smesolve(H, C, S, psi0, tl, [X], ntraj, p["seed"], p["dt"]))]:
        t0 = time.time()
        r = fn()
        assert r["rc"] == 0, r["rc"]
        out[key] = {"expect_re": r["expect_tr"].real.tolist(), "expect_im": r["expect_tr"].imag.tolist(),
                    "measurement": r["measurement"].tolist(), "oracle_seconds": time.time() - t0}
        print(key, "done", time.time() - t0)
    path = os.path.join(OUT, name + ".json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


JOBS = {
    "jc_homodyne_traj": lambda: jc_homodyne_traj("jc_homodyne_traj"),
    "sesolve_l10_tight": lambda: sesolve_l10("sesolve_l10_tight"),
    "optomech_full": lambda: optomech_full("optomech_full"),
    "serving_trace240": lambda: serving_trace_refs("serving_trace240"),
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

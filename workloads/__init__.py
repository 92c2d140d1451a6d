"""Seeded synthetic workloads: parameter records only.

This module is shared by the HIP path's tests and benchmark and by the oracle side.  It holds no
arithmetic of the method: it draws model parameters, sizes, time grids and arrival times from seeded
NumPy PCG64 generators and returns plain records.  Each side builds its own operators from them.

Workloads (shapes of the paper's examples: the driven Kerr oscillator and the dissipative Ising
chain of the performance section, the decaying oscillator of the GPU section):
  * ``kerr_single``: N = 20, Delta = 1, U = 0.5, F = 0.8, kappa = 1, rho0 = |0><0|, t in [0, 20],
    200 save points (the U = 0 variant relaxes to a coherent state).
  * ``ising_single``: L = 8, J = 1, h = 0.7, gamma = 0.2, all spins up, t in [0, 10], 100 saves of
    <sigma_z^i>.
  * ``ising_mc``: L = 10, J = 1, h = 1, gamma = 0.1, 10,000 trajectories, t in [0, 10], 100 saves
    of <sum_i sigma_z^i>.
  * ``kerr_sweep``: 512 Kerr cavities, N ~ U{10..80}, Delta ~ U[-2, 2], U ~ U[0, 1], F ~ U[0, 2],
    kappa ~ U[0.5, 2], vacuum start, t in [0, 20], 100 saves of <a^dag a>.
  * ``serving_trace``: Poisson arrivals; 70% Kerr (as the sweep), 30% Ising chains with L ~ U{4..9},
    J = 1, h ~ U[0.3, 1.5], gamma ~ U[0.05, 0.5].
  * ``driven_cavity_td``: a lossy cavity omega0 a^dag a driven by F (e^{-i omega t} a^dag + h.c.),
    omega0 = 4, omega = 3 (detuning 1), F = 0.8, kappa = 1, N = 15, t in [0, 5], 51 saves.
  * ``optomech_td``: the driven optomechanical system of the time-dependent example (cavity
    cutoff 10, mechanical cutoff 7, omega_c = 1, omega_m = 2, g = 0.05, kappa = gamma = 0.01,
    drive F cos(omega_d t) (a + a^dag) with F = 10 kappa and omega_d = omega_c), vacuum start,
    t in [0, 5 / kappa], 5000 saves of <a^dag a>; ``optomech_sweep`` draws omega_d values around
    omega_c for a batch of such problems over a shorter window.
  * ``jc_homodyne``: the homodyne example (cavity cutoff 20, omega_c = omega_q = 5, g = 0.1,
    kappa = 1 measured through S = sqrt(kappa) a, qubit decay gamma = 2 and cavity dephasing
    kappa_phi = 0.3 as extra losses of the master-equation variant), cavity in the coherent state
    alpha = 2 and qubit excited, t in [0, 10 pi / omega_c] with 400 saves, 500 trajectories, step 1e-3.
"""
import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def tlist(t_end, n):
    return np.linspace(0.0, float(t_end), int(n))


def kerr_single(U=0.5):
    return {"kind": "kerr", "N": 20, "delta": 1.0, "U": float(U), "F": 0.8, "kappa": 1.0,
            "t_end": 20.0, "nt": 200}


def ising_single(L=8, h=0.7):
    return {"kind": "ising", "L": int(L), "J": 1.0, "h": float(h), "gamma": 0.2, "t_end": 10.0, "nt": 100}


def ising_mc(L=10, ntraj=10_000, seed=20250430):
    return {"kind": "ising", "L": int(L), "J": 1.0, "h": 1.0, "gamma": 0.1, "t_end": 10.0, "nt": 100,
            "ntraj": int(ntraj), "seed": int(seed)}


def kerr_sweep(n=512, seed=4, n_min=10, n_max=80):
    g = _rng(seed)
    out = []
    for _ in range(n):
        out.append({"kind": "kerr", "N": int(g.integers(n_min, n_max + 1)), "delta": float(g.uniform(-2, 2)),
                    "U": float(g.uniform(0, 1)), "F": float(g.uniform(0, 2)), "kappa": float(g.uniform(0.5, 2)),
                    "t_end": 20.0, "nt": 100})
    return out


def ising_batch(n=16, L=8):
    """n chains that differ only in the transverse field, h = 0.3 + 0.08 i."""
    return [dict(ising_single(L=L, h=0.3 + 0.08 * i)) for i in range(n)]


def serving_trace(n=2000, qps=100.0, seed=5, kerr_frac=0.7):
    g = _rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += float(g.exponential(1.0 / qps))
        if g.uniform() < kerr_frac:
            p = {"kind": "kerr", "N": int(g.integers(10, 81)), "delta": float(g.uniform(-2, 2)),
                 "U": float(g.uniform(0, 1)), "F": float(g.uniform(0, 2)), "kappa": float(g.uniform(0.5, 2)),
                 "t_end": 20.0, "nt": 100}
        else:
            p = {"kind": "ising", "L": int(g.integers(4, 10)), "J": 1.0, "h": float(g.uniform(0.3, 1.5)),
                 "gamma": float(g.uniform(0.05, 0.5)), "t_end": 10.0, "nt": 100}
        p["arrival"] = t
        p["id"] = i
        out.append(p)
    return out


def driven_cavity_td():
    return {"kind": "cavity_td", "N": 15, "omega0": 4.0, "omega": 3.0, "F": 0.8, "kappa": 1.0, "t_end": 5.0,
            "nt": 51}


def optomech_td(t_end=None, nt=5000):
    kappa = 0.01
    return {"kind": "optomech", "Nc": 10, "Nm": 7, "wc": 1.0, "wm": 2.0, "g": 0.05, "kappa": kappa,
            "gamma": 0.01, "F": 10 * kappa, "wd": 1.0, "t_end": (5.0 / kappa) if t_end is None else float(t_end),
            "nt": int(nt)}


def optomech_sweep(n=64, seed=7, t_end=100.0, nt=200, Nc=10, Nm=7):
    """n optomechanical problems whose drive frequency omega_d ~ U[0.8, 1.2] omega_c."""
    g = _rng(seed)
    out = []
    for _ in range(n):
        p = optomech_td(t_end=t_end, nt=nt)
        p.update({"wd": float(g.uniform(0.8, 1.2)), "Nc": int(Nc), "Nm": int(Nm)})
        out.append(p)
    return out


def jc_homodyne():
    return {"kind": "jc", "N": 20, "wc": 5.0, "wq": 5.0, "g": 0.1, "kappa": 1.0, "gamma": 2.0, "kappa_phi": 0.3,
            "alpha": 2.0, "t_end": 10 * np.pi / 5.0, "nt": 400, "ntraj": 500, "seed": 2025, "dt": 1e-3}


def random_hermitian_dm(d, seed):
    """A random full-rank density matrix (Wishart draw), for one-shot RHS checks."""
    g = _rng(seed)
    X = g.normal(size=(d, d)) + 1j * g.normal(size=(d, d))
    rho = X @ X.conj().T
    return rho / np.trace(rho).real


def random_ket(d, seed):
    g = _rng(seed)
    v = g.normal(size=d) + 1j * g.normal(size=d)
    return v / np.linalg.norm(v)

"""Operators of the model systems, built independently for the oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Conventions (arXiv:2504.21440, Sec. 2 and the constructor table of App. C):
  * ``destroy(N)``: a|n> = sqrt(n)|n-1>, Fock basis 0..N-1.
  * spin-1/2 basis: index 0 = "up" (sigma_z = +1, the excited state of Sec. 3.1),
    index 1 = "down"; sigma_- = |down><up| lowers up to down.
  * ``tensor`` is the Kronecker product with the first factor most significant.

Model Hamiltonians of the benchmark workloads:
  * driven Kerr cavity (Sec. 6): H = Delta a^dag a + (U/2) a^dag a^dag a a + F (a + a^dag),
    C = sqrt(kappa) a;
  * open transverse-field Ising chain (Secs. 4 and 6):
    H = J sum_i sz_i sz_{i+1} + h sum_i sx_i, C_i = sqrt(gamma) sm_i;
  * driven optomechanical system (Sec. 3.4, time-dependent example), cavity a (cutoff Nc) first:
    H_0 = wc a^dag a + wm b^dag b + (g/2)(a + a^dag)^2 (b + b^dag), drive term (a + a^dag) with
    coefficient F cos(wd t), C = sqrt(kappa) a and sqrt(gamma) b.
"""
import numpy as np
import scipy.sparse as sp


def destroy(N):
    return sp.diags(np.sqrt(np.arange(1, N, dtype=float)), 1, shape=(N, N), format="csr").astype(complex)


def qeye(N):
    return sp.identity(N, dtype=complex, format="csr")


def sigmax():
    return sp.csr_matrix(np.array([[0, 1], [1, 0]], dtype=complex))


def sigmaz():
    return sp.csr_matrix(np.array([[1, 0], [0, -1]], dtype=complex))


def sigmam():
    return sp.csr_matrix(np.array([[0, 0], [1, 0]], dtype=complex))


def tensor(*ops):
    out = ops[0]
    for op in ops[1:]:
        out = sp.kron(out, op, format="csr")
    return sp.csr_matrix(out)


def site_op(L, i, op):
    """op acting on spin i (0-based, i = 0 most significant) of an L-spin chain."""
    return tensor(*[op if k == i else qeye(2) for k in range(L)])


def kerr(N, delta, U, F, kappa):
    a = destroy(N)
    ad = a.conj().T
    H = delta * (ad @ a) + 0.5 * U * (ad @ ad @ a @ a) + F * (a + ad)
    return sp.csr_matrix(H), [sp.csr_matrix(np.sqrt(kappa) * a)]


def ising(L, J, h, gamma):
    H = sp.csr_matrix((2 ** L, 2 ** L), dtype=complex)
    for i in range(L - 1):
        H = H + J * (site_op(L, i, sigmaz()) @ site_op(L, i + 1, sigmaz()))
    for i in range(L):
        H = H + h * site_op(L, i, sigmax())
    c_ops = [sp.csr_matrix(np.sqrt(gamma) * site_op(L, i, sigmam())) for i in range(L)]
    return sp.csr_matrix(H), c_ops


def optomech(Nc, Nm, wc, wm, g, kappa, gamma):
    """(H_0, drive operator a + a^dag, c_ops, cavity photon number) of the optomechanical system."""
    a = tensor(destroy(Nc), qeye(Nm))
    b = tensor(qeye(Nc), destroy(Nm))
    ad, bd = a.conj().T, b.conj().T
    xa = a + ad
    H = wc * (ad @ a) + wm * (bd @ b) + 0.5 * g * (xa @ xa) @ (b + bd)
    c_ops = [sp.csr_matrix(np.sqrt(kappa) * a), sp.csr_matrix(np.sqrt(gamma) * b)]
    return sp.csr_matrix(H), sp.csr_matrix(xa), c_ops, sp.csr_matrix(ad @ a)


def jc_homodyne(N, wc, wq, g, kappa, gamma, kappa_phi, alpha):
    """The homodyne-detection example (Sec. 3.5): a cavity (cutoff N, first factor) coupled to a
    qubit, H = wc a^dag a + (wq/2) sz + g (a^dag sm + a sm^dag); measured operator sqrt(kappa) a; extra
    losses of the master-equation variant sqrt(gamma) sm and sqrt(kappa_phi) a^dag a; the observable
    sqrt(kappa) (a + a^dag); initial state the coherent state alpha (real) times the excited qubit.
    Returns (H, [S], c_ops, X, psi0)."""
    from math import exp, factorial, sqrt
    a = tensor(destroy(N), qeye(2))
    sm = tensor(qeye(N), sigmam())
    sz = tensor(qeye(N), sigmaz())
    ad = a.conj().T
    H = wc * (ad @ a) + 0.5 * wq * sz + g * (ad @ sm + a @ sm.conj().T)
    S = [sp.csr_matrix(np.sqrt(kappa) * a)]
    c_ops = [sp.csr_matrix(np.sqrt(gamma) * sm), sp.csr_matrix(np.sqrt(kappa_phi) * (ad @ a))]
    X = sp.csr_matrix(np.sqrt(kappa) * (a + ad))
    coh = np.array([exp(-alpha ** 2 / 2) * alpha ** n / sqrt(float(factorial(n))) for n in range(N)])
    psi0 = np.kron(coh, np.array([1.0, 0.0])).astype(complex)
    return sp.csr_matrix(H), S, c_ops, X, psi0


def number(N):
    a = destroy(N)
    return sp.csr_matrix(a.conj().T @ a)


def fock_dm(N, n):
    rho = np.zeros((N, N), dtype=complex)
    rho[n, n] = 1.0
    return rho


def all_up_ket(L):
    psi = np.zeros(2 ** L, dtype=complex)
    psi[0] = 1.0
    return psi

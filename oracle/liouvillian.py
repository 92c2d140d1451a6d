"""Liouvillian superoperator from its Kronecker definition.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

With the row-major vectorisation v[i*d + j] = rho_ij one has vec(A X B) = (A kron B^T) vec(X),
so the generator of the master equation (Sec. 3.2, eq. eq-lindblad-master-equation, with the
trace-preserving anticommutator form of the dissipator) is

  L = -i (H kron I - I kron H^T)
      + sum_k [ C_k kron conj(C_k) - 1/2 (C_k^dag C_k) kron I - 1/2 I kron (C_k^dag C_k)^T ].

Exact zeros produced by cancellation are removed, so ``nnz`` counts stored non-zeros.
"""
import numpy as np
import scipy.sparse as sp


def liouvillian(H, c_ops):
    H = sp.csr_matrix(H, dtype=complex)
    d = H.shape[0]
    Id = sp.identity(d, dtype=complex, format="csr")
    L = -1j * (sp.kron(H, Id) - sp.kron(Id, H.T))
    for C in c_ops:
        C = sp.csr_matrix(C, dtype=complex)
        CdC = C.conj().T @ C
        L = L + sp.kron(C, C.conj()) - 0.5 * sp.kron(CdC, Id) - 0.5 * sp.kron(Id, CdC.T)
    L = sp.csr_matrix(L)
    L.sum_duplicates()
    L.eliminate_zeros()
    L.sort_indices()
    return L


def vec(rho):
    """Row-major vectorisation."""
    return np.ascontiguousarray(rho).reshape(-1)


def unvec(v, d):
    return np.asarray(v).reshape(d, d)

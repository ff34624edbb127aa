"""Dense Jordan-Wigner brute force: an independent check of the oracle.

Ladder operators are built from Kronecker products of 2x2 matrices on the
full Fock space (qubit P <-> bit P of a basis index), so signs come from the
textbook Z-string construction and not from any occupation-count formula.
The Hamiltonian is assembled from operator products,
H = sum h_PQ a+_P a_Q + 1/2 sum (PQ|RS) a+_P a+_R a_S a_Q,
via spin-summed excitation operators E_pq, and then restricted to a fixed
(n_alpha, n_beta) sector.  Only small spaces (up to 16 spin-orbitals).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

_I = sp.identity(2, format="csr")
_Z = sp.csr_matrix(np.array([[1.0, 0.0], [0.0, -1.0]]))
# sigma^- : |1> -> |0>  (basis order |0>, |1>)
_LOWER = sp.csr_matrix(np.array([[0.0, 1.0], [0.0, 0.0]]))


def annihilators(nso: int):
    """a_P for P = 0..nso-1 as sparse (2^nso x 2^nso) matrices."""
    ops = []
    for P in range(nso):
        factors = []
        for Q in range(nso - 1, -1, -1):  # kron puts the first factor on the highest bit
            if Q < P:
                factors.append(_Z)
            elif Q == P:
                factors.append(_LOWER)
            else:
                factors.append(_I)
        m = factors[0]
        for f in factors[1:]:
            m = sp.kron(m, f, format="csr")
        ops.append(m.tocsr())
    return ops


def sector_basis(n: int, n_alpha: int, n_beta: int):
    """Sorted keys of the (n_alpha, n_beta) sector, interleaved spin-orbitals."""
    keys = []
    for k in range(1 << (2 * n)):
        a = bin(k & int("01" * n, 2)).count("1")
        b = bin(k & int("10" * n, 2)).count("1")
        if a == n_alpha and b == n_beta:
            keys.append(k)
    return np.array(keys, dtype=np.int64)


class DenseProblem:
    def __init__(self, n, n_alpha, n_beta, h, eri, ecore=0.0):
        self.n, self.nso = n, 2 * n
        self.basis = sector_basis(n, n_alpha, n_beta)
        self.index = {int(k): i for i, k in enumerate(self.basis)}
        self.a = annihilators(self.nso)
        self.ad = [m.T.tocsr() for m in self.a]
        dim_full = 1 << self.nso
        idx = self.basis
        # E_pq preserves the alpha and beta electron counts, so the sector is
        # invariant and products may be formed after restriction.
        E = {}
        for p in range(n):
            for q in range(n):
                m = sp.csr_matrix((dim_full, dim_full))
                for s in range(2):
                    m = m + self.ad[2 * p + s] @ self.a[2 * q + s]
                E[(p, q)] = m.tocsr()[idx][:, idx].tocsr()
        dim = len(idx)
        H = sp.csr_matrix((dim, dim))
        for p in range(n):
            for q in range(n):
                if h[p, q] != 0.0:
                    H = H + h[p, q] * E[(p, q)]
        # 1/2 sum_pqrs (pq|rs) (E_pq E_rs - delta_qr E_ps)
        for p in range(n):
            for q in range(n):
                F = sp.csr_matrix((dim, dim))
                for r in range(n):
                    for s in range(n):
                        F = F + eri[p, q, r, s] * E[(r, s)]
                H = H + 0.5 * (E[(p, q)] @ F)
        for p in range(n):
            for s in range(n):
                coef = sum(eri[p, q, q, s] for q in range(n))
                H = H - 0.5 * coef * E[(p, s)]
        H = H + ecore * sp.identity(dim, format="csr")
        self.H = H.toarray()
        self._E = None

    # operators -----------------------------------------------------------
    def excitation(self, row):
        """T of a pool row as a full-space sparse matrix."""
        P, Q, R, S = (int(x) for x in row)
        if R < 0:
            return (self.ad[P] @ self.a[Q]).tocsr()
        return (self.ad[P] @ self.ad[Q] @ self.a[S] @ self.a[R]).tocsr()

    def generator_sparse(self, row):
        """A = T - T^dagger restricted to the sector (sparse)."""
        T = self.excitation(row)
        A = (T - T.T).tocsr()
        idx = self.basis
        return A[idx][:, idx].tocsr()

    def generator(self, row):
        """A = T - T^dagger restricted to the sector (dense)."""
        return self.generator_sparse(row).toarray()

    def vec(self, state: dict):
        v = np.zeros(len(self.basis))
        for k, a in state.items():
            v[self.index[int(k)]] = a
        return v

    def ref_vec(self, ref_key: int):
        v = np.zeros(len(self.basis))
        v[self.index[int(ref_key)]] = 1.0
        return v

    def fci(self):
        return float(np.linalg.eigvalsh(self.H)[0])

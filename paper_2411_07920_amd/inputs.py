"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the method itself: it draws integrals,
enumerates the operator-pool index table, draws ansatz operator lists and
parameters, and draws synthetic sparse states.  Phases, matrix elements,
gates, energies and gradients live elsewhere (the oracle and the HIP library
compute them independently from these arrays).

Conventions (the paper leaves them open; they are fixed here):

* ``n`` spatial orbitals, ``2n`` spin-orbitals, spin-orbital index
  ``P = 2p + sigma`` (sigma = 0 for alpha, 1 for beta).  Bit ``P`` of a uint64
  key is the occupation of spin-orbital ``P``.
* The reference determinant is the lowest ``n_elec`` spin-orbitals
  (``2**n_elec - 1``), a closed-shell aufbau determinant.
* Integrals stand in for the molecular-orbital integrals of step 1 of the
  ADAPT procedure (Sec. II.C): ``h`` symmetric with a sorted diagonal in
  [-2, 1] and N(0, 0.05) off-diagonals, ``(pq|rs) = sum_L B^L_pq B^L_rs`` with
  symmetric ``B^L ~ N(0, 0.1)`` (8-fold symmetric and positive semidefinite as
  a pair matrix), chemists' notation, row-major ``eri[p, q, r, s]``.
* Pool: the generalized singles and doubles of Sec. II.C in spin-orbital form.
  Singles ``T = a+_P a_Q`` with ``P > Q`` and equal spin, row ``(P, Q, -1, -1)``.
  Doubles ``T = a+_P a+_Q a_S a_R`` with ``P > Q``, ``R > S``, disjoint index
  sets, equal spin multisets of ``(P, Q)`` and ``(R, S)`` and ``(P, Q) > (R, S)``
  lexicographically (one operator per generator up to sign), row
  ``(P, Q, R, S)``.  Singles come first, then doubles, each sorted
  lexicographically; the row index is the pool index.
"""
from __future__ import annotations

import dataclasses
import hashlib
from math import comb

import numpy as np

__all__ = [
    "Config",
    "CONFIGS",
    "make_integrals",
    "enumerate_pool",
    "pool_count",
    "draw_ansatz",
    "reference_key",
    "sector_size",
    "draw_synthetic_state",
    "draw_random_keys",
    "array_digest",
]


@dataclasses.dataclass(frozen=True)
class Config:
    """One synthetic workload: integral shape, electrons, ansatz and threshold."""

    name: str
    n: int              # spatial orbitals
    n_elec: int         # electrons (n_alpha = n_beta = n_elec // 2)
    rank: int           # number of B^L factors in the ERI
    n_ops: int          # ansatz length M
    theta_lo: float
    theta_hi: float
    eps: float
    seed_int: int
    seed_ansatz: int

    @property
    def n_so(self) -> int:
        return 2 * self.n


# Workloads: 12/28/40/40/52 spin-orbitals with 4/10/12/12/16 electrons.
CONFIGS = {
    "c1": Config("c1", 6, 4, 6, 30, -0.1, 0.1, 0.0, 1001, 2001),
    "c2": Config("c2", 14, 10, 14, 100, -0.05, 0.05, 1e-6, 1002, 2002),
    "c3": Config("c3", 20, 12, 20, 200, -0.05, 0.05, 1e-7, 1003, 2003),
    "c4": Config("c4", 20, 12, 20, 150, -0.05, 0.05, 1e-7, 1004, 2004),
    "c5": Config("c5", 26, 16, 26, 300, -0.05, 0.05, 1e-8, 1005, 2005),
}


def make_integrals(n: int, rank: int, seed: int):
    """Draw (h, eri) for ``n`` spatial orbitals.

    Draw order: the sorted diagonal of h, the strict upper triangle of h, then
    for each of the ``rank`` factors the upper triangle (with diagonal) of B.
    Returns float64 arrays ``h[n, n]`` and ``eri[n, n, n, n]`` (C order).
    """
    rng = np.random.default_rng(seed)
    h = np.zeros((n, n))
    h[np.diag_indices(n)] = np.sort(rng.uniform(-2.0, 1.0, n))
    iu = np.triu_indices(n, 1)
    off = rng.normal(0.0, 0.05, len(iu[0]))
    h[iu] = off
    h[(iu[1], iu[0])] = off
    eri = np.zeros((n, n, n, n))
    iu0 = np.triu_indices(n, 0)
    for _ in range(rank):
        b = np.zeros((n, n))
        v = rng.normal(0.0, 0.1, len(iu0[0]))
        b[iu0] = v
        b[(iu0[1], iu0[0])] = v
        eri += np.multiply.outer(b, b)
    return h, eri


def _spin(P: int) -> int:
    return P & 1


def enumerate_pool(n: int) -> np.ndarray:
    """Index table ``int32[K, 4]`` of the generalized singles and doubles pool."""
    nso = 2 * n
    singles = []
    for P in range(nso):
        for Q in range(P):
            if _spin(P) == _spin(Q):
                singles.append((P, Q, -1, -1))
    pairs = [(P, Q) for P in range(nso) for Q in range(P)]
    doubles = []
    for (P, Q) in pairs:
        sp = sorted((_spin(P), _spin(Q)))
        for (R, S) in pairs:
            if not (P, Q) > (R, S):
                continue
            if len({P, Q, R, S}) != 4:
                continue
            if sorted((_spin(R), _spin(S))) != sp:
                continue
            doubles.append((P, Q, R, S))
    singles.sort()
    doubles.sort()
    return np.array(singles + doubles, dtype=np.int32).reshape(-1, 4)


def pool_count(n: int) -> tuple[int, int]:
    """Closed-form (singles, doubles) counts of :func:`enumerate_pool`."""
    singles = 2 * comb(n, 2)
    same_spin = 2 * (comb(n, 2) * comb(n - 2, 2) // 2)
    opposite = n * n * (n - 1) * (n - 1) // 2
    return singles, same_spin + opposite


def reference_key(n_elec: int) -> int:
    """Aufbau reference: the lowest ``n_elec`` spin-orbitals occupied."""
    return (1 << n_elec) - 1


def sector_size(n: int, n_alpha: int, n_beta: int) -> int:
    """Number of determinants with fixed alpha and beta electron counts."""
    return comb(n, n_alpha) * comb(n, n_beta)


def draw_ansatz(n_pool: int, n_ops: int, lo: float, hi: float, seed: int):
    """Operator indices (distinct, applied in list order) and parameters."""
    rng = np.random.default_rng(seed)
    ops = rng.choice(n_pool, n_ops, replace=False).astype(np.int32)
    theta = rng.uniform(lo, hi, n_ops)
    return ops, theta


def _strings(n: int, k: int) -> np.ndarray:
    """All n-bit masks with k bits set (one spin's occupation strings), ascending."""
    if n <= 26:
        x = np.arange(1 << n, dtype=np.uint32)
        pc = np.zeros_like(x, dtype=np.uint8)
        for b in range(n):
            pc += ((x >> np.uint32(b)) & np.uint32(1)).astype(np.uint8)
        return x[pc == k].astype(np.uint64)
    from itertools import combinations
    out = [sum(1 << i for i in c) for c in combinations(range(n), k)]
    return np.array(sorted(out), dtype=np.uint64)


def _spread(mask: np.ndarray, n: int, offset: int) -> np.ndarray:
    """Place bit p of a spatial mask at spin-orbital 2p + offset."""
    out = np.zeros_like(mask, dtype=np.uint64)
    for p in range(n):
        bit = (mask >> np.uint64(p)) & np.uint64(1)
        out |= bit << np.uint64(2 * p + offset)
    return out


def draw_synthetic_state(n: int, n_alpha: int, n_beta: int, count: int, seed: int):
    """``count`` distinct determinants drawn uniformly from the (n_alpha, n_beta)
    sector (an alpha string and a beta string, each uniform), random signs and
    log-uniform magnitudes in [1e-8, 1e-2].

    Returns ``(keys uint64[count], amps float64[count])`` in draw order (not
    sorted).  A structure-free stand-in for a large truncated state.
    """
    rng = np.random.default_rng(seed)
    total = sector_size(n, n_alpha, n_beta)
    if count > total:
        raise ValueError("count exceeds sector size")
    sa = _spread(_strings(n, n_alpha), n, 0)
    sb = sa if n_beta == n_alpha else None
    sb = _spread(_strings(n, n_beta), n, 1) if sb is None else (sa << np.uint64(1))
    keys = np.zeros(0, dtype=np.uint64)
    while len(keys) < count:
        need = int((count - len(keys)) * 1.05) + 16
        k = sa[rng.integers(0, len(sa), need)] | sb[rng.integers(0, len(sb), need)]
        keys = np.concatenate([keys, k])
        _, first = np.unique(keys, return_index=True)
        keys = keys[np.sort(first)]
    keys = keys[:count]
    mag = 10.0 ** rng.uniform(-8.0, -2.0, count)
    sign = np.where(rng.random(count) < 0.5, -1.0, 1.0)
    return keys, mag * sign


def draw_random_keys(count: int, seed: int) -> np.ndarray:
    """uint32 random priorities (used to pick the random share of a screened pool)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2**32, count, dtype=np.uint64).astype(np.uint32)


def array_digest(*arrays) -> str:
    """SHA-256 over the raw bytes of the given arrays (input provenance)."""
    m = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        m.update(str(a.dtype).encode())
        m.update(str(a.shape).encode())
        m.update(a.tobytes())
    return m.hexdigest()

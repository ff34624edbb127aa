"""Spin-complemented generators (Sec. III) on the SWCS library.

For a pool operator T (singles a+_P a_Q, doubles a+_P a+_Q a_S a_R) its spin
complement T' replaces every spin-orbital by the same spatial orbital with
the other spin, in the same operator order.  The complemented generator is
G = A(T) + A(T'), A(X) = X - X^dagger.  The pool holds T' in canonical form
as row k' with A(T') = sign * A_k'.

When T and T' touch disjoint spin-orbitals (singles, same-spin doubles, and
opposite-spin doubles whose spatial indices are all distinct) the two parts
are even operators on disjoint modes and commute, so
exp(theta G) = exp(theta A_k) exp(sign theta A_k'): two gates with one shared
parameter.  A row that is its own complement is one gate.  An opposite-spin
double with two indices on one spatial orbital (p = q, r = s, p = s or q = r,
not a self-complement) shares spin-orbitals with its complement; the parts do
not commute, and the library applies exp(theta G) as one exact gate (a
determinant both parts act on turns with its two images at frequency
sqrt(2) theta).

All arithmetic on states runs in the library (swcs_apply_generators with rows
(k, k', sign)); this module builds the generator list and combines the pool
gradients, which are linear in the generator: g_G = g_k + sign * g_k'.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import scipy.optimize


@dataclasses.dataclass
class GeneratorPool:
    first: np.ndarray    # int32 [G] first pool row
    second: np.ndarray   # int32 [G] second pool row, -1 for one-row generators
    sign: np.ndarray     # float64 [G] factor of the second row (0 when there is none)
    overlap: np.ndarray  # bool [G] the two rows share spin-orbitals (one exact gate)

    def __len__(self):
        return len(self.first)


def complement_row(row):
    """(canonical pool row of the spin complement of `row`, sign) with
    A(T') = sign * A(row')."""
    P, Q, R, S = (int(x) for x in row)
    if R < 0:  # same-spin single: the order P > Q is kept by the flip
        return (P ^ 1, Q ^ 1, -1, -1), 1.0
    A, B, C, D = P ^ 1, Q ^ 1, R ^ 1, S ^ 1  # T' = a+_A a+_B a_D a_C
    sign = 1.0
    if A < B:
        A, B, sign = B, A, -sign
    if C < D:
        C, D, sign = D, C, -sign
    if (A, B) > (C, D):
        return (A, B, C, D), sign
    # the pool holds the adjoint orientation: A(row) = -A(T') * sign
    return (C, D, A, B), -sign


def spin_complemented(pool, overlapping=True) -> GeneratorPool:
    """Every pool row paired with its spin complement.  overlapping=False
    keeps rows that share spin-orbitals with their complement as separate
    one-row generators (the commuting pairs only)."""
    pool = np.asarray(pool)
    index = {tuple(int(x) for x in r): k for k, r in enumerate(pool)}
    seen = np.zeros(len(pool), dtype=bool)
    first, second, sign, over = [], [], [], []
    for k, r in enumerate(pool):
        if seen[k]:
            continue
        row2, s = complement_row(r)
        k2 = index[row2]
        seen[k] = seen[k2] = True
        modes = {int(x) for x in r if x >= 0}
        modes2 = {int(x) for x in row2 if x >= 0}
        if k2 == k:
            first.append(k), second.append(-1), sign.append(0.0), over.append(False)
        elif modes & modes2 and not overlapping:
            for kk in (k, k2):
                first.append(kk), second.append(-1), sign.append(0.0), over.append(False)
        else:
            first.append(k), second.append(k2), sign.append(s), over.append(bool(modes & modes2))
    return GeneratorPool(np.array(first, dtype=np.int32), np.array(second, dtype=np.int32),
                         np.array(sign, dtype=np.float64), np.array(over, dtype=bool))


def gen_rows(gp: GeneratorPool, gens) -> np.ndarray:
    """int32 [M, 3] rows (k, k', sign) of generators `gens` for the library's
    generator chain (k' = -1 for one-row generators)."""
    g = np.asarray(gens, dtype=np.int64)
    rows = np.empty((len(g), 3), dtype=np.int32)
    rows[:, 0] = gp.first[g]
    rows[:, 1] = gp.second[g]
    rows[:, 2] = np.where(gp.second[g] >= 0, gp.sign[g], 1.0).astype(np.int32)
    return rows


def generator_gradients(gp: GeneratorPool, g_pool) -> np.ndarray:
    g = np.asarray(g_pool, dtype=np.float64)
    out = g[gp.first].copy()
    two = gp.second >= 0
    out[two] += gp.sign[two] * g[gp.second[two]]
    return out


def expand(gp: GeneratorPool, gens, theta):
    """Gate list (pool rows, angles) of commuting generators `gens` with
    angles `theta`, first generator applied first (a generator whose rows
    overlap is not a product of gates: use gen_rows)."""
    ops, ang = [], []
    if np.any(gp.overlap[np.asarray(gens, dtype=np.int64)]):
        raise ValueError("generators with overlapping rows are one gate each: use gen_rows")
    for j, t in zip(np.asarray(gens, dtype=np.int64).tolist(), np.asarray(theta, dtype=np.float64).tolist()):
        ops.append(int(gp.first[j]))
        ang.append(t)
        if gp.second[j] >= 0:
            ops.append(int(gp.second[j]))
            ang.append(float(gp.sign[j]) * t)
    return np.array(ops, dtype=np.int32), np.array(ang, dtype=np.float64)


def contract(gp: GeneratorPool, gens, dE_gates) -> np.ndarray:
    """Per-generator parameter gradients from the per-gate ones."""
    out = []
    p = 0
    for j in np.asarray(gens, dtype=np.int64).tolist():
        d = dE_gates[p]
        p += 1
        if gp.second[j] >= 0:
            d += float(gp.sign[j]) * dE_gates[p]
            p += 1
        out.append(d)
    return np.array(out, dtype=np.float64)


class TiedEnergy:
    """E and dE/dtheta over generator parameters (the library's generator
    chain).  A call at exactly the previous angles returns the previous result
    without touching the context, whose state is then still at those angles."""

    def __init__(self, ctx, gp: GeneratorPool, gens, eps=0.0):
        self.ctx, self.gp, self.gens, self.eps = ctx, gp, list(gens), eps
        self.rows = gen_rows(gp, self.gens)
        self.evals = 0
        self._last = None

    def __call__(self, theta):
        theta = np.array(theta, dtype=np.float64)
        if self._last is not None and np.array_equal(theta, self._last[0]):
            return self._last[1], self._last[2].copy()
        self.ctx.apply_generators(self.rows, theta, self.eps)
        dE, E = self.ctx.param_gradients(len(theta))
        self.evals += 1
        d = np.array(dE, dtype=np.float64)
        self._last = (theta, E, d)
        return E, d.copy()


_FIT9 = (np.arange(9) - 4) * (2.0 * np.pi / 9.0)


def seed_new_angle(ctx, gp: GeneratorPool, gens, theta, eps):
    """Start angle of the newest generator when the state is pruned.  A new
    angle at exactly 0 sits on a plateau (the partners it creates at small
    angles are dropped), where a gradient optimizer does not move.  Without
    pruning E is a trigonometric polynomial of degree 2 per gate in this
    angle, so at most 4 for a two-gate generator; nine samples fit it and
    its minimum on a grid is the start (for a generator whose rows overlap
    the frequencies are not integers and the fit is only a guide).  Returns
    (theta, evaluations)."""
    Es = []
    rows = gen_rows(gp, gens)
    for t in _FIT9:
        th = np.array(theta, dtype=np.float64)
        th[-1] = t
        ctx.apply_generators(rows, th, eps)
        Es.append(ctx.energy()[0])
    X = np.stack([np.ones(9)] + [f(m * _FIT9) for m in range(1, 5) for f in (np.cos, np.sin)], axis=1)
    coef = np.linalg.solve(X, np.array(Es))
    grid = np.linspace(-np.pi, np.pi, 4097)
    G = np.stack([np.ones_like(grid)] + [f(m * grid) for m in range(1, 5) for f in (np.cos, np.sin)], axis=1)
    out = np.array(theta, dtype=np.float64)
    out[-1] = float(grid[int(np.argmin(G @ coef))])
    return out, 9


def run_adapt_spin(ctx, gp: GeneratorPool, eps=0.0, max_iter=20, grad_tol=1e-2, vqe_gtol=1e-6,
                   vqe_maxiter=200, rel_tol=1e-9, log=None):
    """ADAPT-VQE (Fig. 1) over spin-complemented generators: full-pool gradients
    from the library, the generator of largest |g| appended with angle 0 (values
    within rel_tol * max |g| tie and go to the lower generator index), its
    angle seeded by seed_new_angle when the state is pruned, then L-BFGS over
    all generator angles.  Returns (generators, theta, history)."""
    gens, theta, hist = [], np.zeros(0), []
    for it in range(max_iter):
        t0 = time.perf_counter()
        n_det = ctx.apply_generators(gen_rows(gp, gens), theta, eps)
        E = ctx.energy()[0]
        g = generator_gradients(gp, ctx.pool_gradients())
        a = np.abs(g)
        top = a.max()
        j = int(np.flatnonzero(a >= top - rel_tol * max(top, 1e-300))[0])
        rec = {"iter": it, "E": E, "n_det": int(n_det), "gen": j, "gmax": float(a[j]),
               "gnorm": float(np.linalg.norm(g))}
        if grad_tol is not None and rec["gnorm"] < grad_tol:
            rec["converged"] = True
            hist.append(rec)
            if log:
                log(rec)
            break
        gens.append(j)
        start = np.append(theta, 0.0)
        extra = 0
        if eps > 0.0:
            start, extra = seed_new_angle(ctx, gp, gens, start, eps)
        f = TiedEnergy(ctx, gp, gens, eps)
        r = scipy.optimize.minimize(f, start, jac=True, method="L-BFGS-B",
                                    options={"gtol": vqe_gtol, "ftol": 1e-15, "maxiter": vqe_maxiter})
        f.evals += extra
        theta = np.array(r.x)
        rec.update(E_after=float(r.fun), vqe_evals=f.evals, t_iter=time.perf_counter() - t0)
        hist.append(rec)
        if log:
            log(rec)
    return gens, theta, hist

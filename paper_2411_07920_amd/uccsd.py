"""MP2-ordered UCCSD workload on the SWCS library (Sec. II.A, Eqs. 1-3).

The factorized UCCSD ansatz applies one unitary exp(theta_I A_I) per
occupied -> virtual single or double excitation of a closed-shell reference.
The doubles act first, largest MP2 amplitude first, starting from their MP2
amplitudes; the singles follow in orbital-index order, starting from 0.

MP2 amplitudes come from the library's own kernels.  At the reference, the
pool gradient of an excitation generator A_k (A_k|ref> = s_k|D>, s_k = +-1) is
g_k = 2 s_k <D|H|ref>.  With the Moller-Plesset partition
H0 = sum_P f_{P/2,P/2} n_P (the closed-shell Fock diagonal the library
exports), the first-order coefficient of D is <D|H|ref> / Delta_k,
Delta_k = E0(ref) - E0(D) = f_i + f_j - f_a - f_b.  Hence
theta_k = g_k / (2 Delta_k), whatever the sign convention of A_k, and the
MP2 energy is E2 = sum_k g_k^2 / (4 Delta_k).

The VQE over all parameters is ``adapt.preoptimize`` (adjoint gradients,
L-BFGS or BFGS).
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class UccsdAnsatz:
    ops: np.ndarray        # int32 pool indices, index 0 applied first
    theta: np.ndarray      # float64 starting parameters (MP2 amplitudes; singles 0)
    e_ref: float           # energy of the reference determinant
    e2: float              # MP2 correlation energy
    n_doubles: int
    n_singles: int


def _excitation(row, occ):
    """(occupied, virtual) spin-orbitals of a pool row that excites the
    reference in one of its two orientations, else None."""
    P, Q, R, S = (int(x) for x in row)
    cre = (P, Q) if R >= 0 else (P,)
    ann = (R, S) if R >= 0 else (Q,)
    if all(a in occ for a in ann) and not any(c in occ for c in cre):
        return ann, cre
    if all(c in occ for c in cre) and not any(a in occ for a in ann):
        return cre, ann
    return None


def order_by_magnitude(values, idx, rel_tol=1e-9):
    """Positions of `values` by decreasing |value|; a run of values within
    rel_tol * max|value| of its first member counts as equal and goes by
    ascending `idx` (spin-symmetric amplitudes are equal up to rounding)."""
    a = np.abs(np.asarray(values, dtype=np.float64))
    idx = np.asarray(idx)
    if len(a) == 0:
        return np.zeros(0, dtype=np.int64)
    order = np.lexsort((idx, -a))
    tol = rel_tol * a.max()
    out = []
    i = 0
    while i < len(order):
        j = i + 1
        while j < len(order) and a[order[i]] - a[order[j]] <= tol:
            j += 1
        run = order[i:j]
        out.extend(run[np.argsort(idx[run], kind="stable")].tolist())
        i = j
    return np.array(out, dtype=np.int64)


def mp2_ordered_uccsd(ctx, pool, ref, n_spatial, rel_tol=1e-9) -> UccsdAnsatz:
    """The UCCSD operator list of `pool` for the closed-shell reference `ref`,
    ordered and initialized from MP2 (see the module docstring).  Leaves the
    context's current state at the reference."""
    pool = np.asarray(pool)
    ref = int(ref)
    occ = {P for P in range(2 * n_spatial) if (ref >> P) & 1}
    f = np.asarray(ctx.fock_diagonal(), dtype=np.float64)
    doubles, gaps, singles = [], [], []
    for k in range(len(pool)):
        ex = _excitation(pool[k], occ)
        if ex is None:
            continue
        o, v = ex
        if len(o) == 1:
            singles.append((o[0], v[0], k))
            continue
        doubles.append(k)
        gaps.append(sum(f[P >> 1] for P in o) - sum(f[P >> 1] for P in v))
    doubles = np.array(doubles, dtype=np.int32)
    gaps = np.array(gaps, dtype=np.float64)
    ctx.set_state(np.array([ref], dtype=np.uint64), np.array([1.0]))
    e_ref = float(ctx.energy()[0])
    g = np.asarray(ctx.pool_gradients(doubles), dtype=np.float64) if len(doubles) else np.zeros(0)
    theta_d = g / (2.0 * gaps)
    e2 = float(np.sum(g * g / (4.0 * gaps)))
    pos = order_by_magnitude(theta_d, doubles, rel_tol)
    singles.sort()
    ops = np.concatenate([doubles[pos], np.array([k for _, _, k in singles], dtype=np.int32)])
    theta = np.concatenate([theta_d[pos], np.zeros(len(singles))])
    return UccsdAnsatz(ops=ops.astype(np.int32), theta=theta, e_ref=e_ref, e2=e2,
                       n_doubles=len(doubles), n_singles=len(singles))


def spin_complemented_uccsd(ans: UccsdAnsatz, gp):
    """The UCCSD ansatz over spin-complemented generators (Sec. III; see
    ``spin.py``).  For a closed-shell reference the complement of an
    occupied -> virtual excitation is one as well, with the MP2 amplitude of
    the same excitation read with flipped spins, so a complement pair becomes
    one generator with one parameter at the first member's position in the
    MP2 order; self-complementary rows stay single.  Returns (generators,
    theta) for ``spin.gen_rows`` / ``spin.TiedEnergy``."""
    ops = np.asarray(ans.ops).tolist()
    pos = {k: i for i, k in enumerate(ops)}
    gen_of = {}
    for j in range(len(gp)):
        gen_of[int(gp.first[j])] = j
        if gp.second[j] >= 0:
            gen_of[int(gp.second[j])] = j
    gens, theta, taken = [], [], set()
    for i, k in enumerate(ops):
        j = gen_of[k]
        if j in taken:
            continue
        if gp.second[j] >= 0 and (int(gp.first[j]) not in pos or int(gp.second[j]) not in pos):
            raise ValueError("a complement pair is not within the UCCSD operators")
        taken.add(j)
        gens.append(j)
        # the generator's angle multiplies its first gate
        k1 = int(gp.first[j])
        theta.append(float(ans.theta[pos[k1]]))
    return np.array(gens, dtype=np.int64), np.array(theta, dtype=np.float64)

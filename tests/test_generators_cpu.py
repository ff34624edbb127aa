"""The oracle's spin-complemented generators (Sec. III) pinned by dense
Jordan-Wigner brute force: one generator G = A_k + s A_k' whose rows overlap
is exp(theta G) from scipy's expm; chains of generators against the dense
product; the generator adjoint against central finite differences (eps = 0)
and against the per-row adjoint of the same chain written as single rows
(commuting pairs, eps > 0)."""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle
from dense_jw import DenseProblem
from paper_2411_07920_amd import spin
from paper_2411_07920_amd.inputs import enumerate_pool, make_integrals, reference_key


def _setup(n, ne, seed):
    h, eri = make_integrals(n, n, seed)
    pool = enumerate_pool(n)
    dense = DenseProblem(n, ne // 2, ne // 2, h, eri)
    orc = oracle.Oracle(n, ne // 2, ne // 2, h, eri)
    gp = spin.spin_complemented(pool)
    return h, eri, pool, dense, orc, gp


@pytest.fixture(scope="module")
def p12():
    return _setup(6, 4, 7)


@pytest.fixture(scope="module")
def p16():
    return _setup(8, 8, 1101)


def _gmat(dense, pool, row):
    k1, k2, s = (int(x) for x in row)
    G = dense.generator(pool[k1])
    if k2 >= 0:
        G = G + s * dense.generator(pool[k2])
    return G


def test_every_overlapping_generator_is_expm(p12):
    """All overlapping complement pairs at 12 spin-orbitals, on full random
    vectors of the 225-determinant sector: exp(theta G) and G psi."""
    h, eri, pool, dense, orc, gp = p12
    rng = np.random.default_rng(1)
    over = np.flatnonzero(gp.overlap)
    assert len(over) == 120
    rows = spin.gen_rows(gp, over)
    for row in rows:
        G = _gmat(dense, pool, row)
        assert np.abs(G @ G @ G + G).max() > 0.5  # the one-row closed form does not hold
        v = rng.normal(size=len(dense.basis))
        st = oracle.OracleState.from_arrays(dense.basis.astype(np.uint64), v)
        th = float(rng.uniform(-1.3, 1.3))
        out = oracle.Oracle.apply_gen(st, pool, row, th)
        assert np.abs(dense.vec(out.as_dict()) - scipy.linalg.expm(th * G) @ v).max() < 1e-13
        gs = oracle.Oracle.apply_gen_sum(st, pool, row)
        assert np.abs(dense.vec(gs.as_dict()) - G @ v).max() < 1e-13


def test_overlapping_generators_16so_sampled(p16):
    h, eri, pool, dense, orc, gp = p16
    rng = np.random.default_rng(2)
    over = rng.choice(np.flatnonzero(gp.overlap), 12, replace=False)
    for row in spin.gen_rows(gp, over):
        G = dense.generator_sparse(pool[row[0]]) + row[2] * dense.generator_sparse(pool[row[1]])
        v = rng.normal(size=len(dense.basis))
        st = oracle.OracleState.from_arrays(dense.basis.astype(np.uint64), v)
        th = float(rng.uniform(-1.3, 1.3))
        out = oracle.Oracle.apply_gen(st, pool, row, th)
        w = scipy.sparse.linalg.expm_multiply(th * G, v)
        assert np.abs(dense.vec(out.as_dict()) - w).max() < 1e-12


def _mixed_chain(gp, rng, m):
    singles = np.flatnonzero(gp.second < 0)
    comm = np.flatnonzero((gp.second >= 0) & ~gp.overlap)
    over = np.flatnonzero(gp.overlap)
    gens = np.concatenate([rng.choice(singles, m // 3), rng.choice(comm, m // 3), rng.choice(over, m - 2 * (m // 3))])
    rng.shuffle(gens)
    return gens


def test_generator_chain_matches_dense(p12):
    h, eri, pool, dense, orc, gp = p12
    rng = np.random.default_rng(3)
    gens = _mixed_chain(gp, rng, 30)
    rows = spin.gen_rows(gp, gens)
    theta = rng.uniform(-0.8, 0.8, len(gens))
    ref = reference_key(4)
    st = oracle.Oracle.apply_gen_ansatz(pool, rows, theta, 0.0, ref)
    v = dense.ref_vec(ref)
    for row, t in zip(rows, theta):
        v = scipy.linalg.expm(t * _gmat(dense, pool, row)) @ v
    assert np.abs(dense.vec(st.as_dict()) - v).max() < 1e-13
    _, a = st.export()
    assert abs((a * a).sum() - 1.0) < 1e-13


def test_generator_adjoint_central_fd(p12):
    h, eri, pool, dense, orc, gp = p12
    rng = np.random.default_rng(4)
    gens = _mixed_chain(gp, rng, 18)
    rows = spin.gen_rows(gp, gens)
    theta = rng.uniform(-0.6, 0.6, len(gens))
    ref = reference_key(4)
    dE, E = orc.gen_param_gradients(pool, rows, theta, 0.0, ref)
    assert abs(E - orc.energy(oracle.Oracle.apply_gen_ansatz(pool, rows, theta, 0.0, ref))[0]) < 1e-13
    hs = 1e-5
    for i in range(len(theta)):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += hs
        tm[i] -= hs
        fd = (orc.energy(oracle.Oracle.apply_gen_ansatz(pool, rows, tp, 0.0, ref))[0]
              - orc.energy(oracle.Oracle.apply_gen_ansatz(pool, rows, tm, 0.0, ref))[0]) / (2 * hs)
        assert abs(fd - dE[i]) < 1e-8, (i, fd, dE[i])


def test_commuting_generators_equal_their_rows(p16):
    """With only single rows and commuting pairs, the generator chain is the
    plain chain of its rows (row 2 at s theta), state and pruning included,
    and each generator derivative is d/dtheta_k + s d/dtheta_k' of that chain
    (eps > 0)."""
    h, eri, pool, dense, orc, gp = p16
    rng = np.random.default_rng(5)
    cand = np.flatnonzero(~gp.overlap)
    gens = rng.choice(cand, 24, replace=False)
    rows = spin.gen_rows(gp, gens)
    theta = rng.uniform(-0.7, 0.7, len(gens))
    ops, ang, own, fac = [], [], [], []
    for i, (k1, k2, s) in enumerate(rows.tolist()):
        ops.append(k1), ang.append(theta[i]), own.append(i), fac.append(1.0)
        if k2 >= 0:
            ops.append(k2), ang.append(s * theta[i]), own.append(i), fac.append(float(s))
    eps, ref = 1e-3, reference_key(8)
    a = oracle.Oracle.apply_gen_ansatz(pool, rows, theta, eps, ref)
    b = oracle.Oracle.apply_ansatz(pool, np.array(ops), np.array(ang), eps, ref)
    assert a.as_dict() == b.as_dict()
    dE, _ = orc.gen_param_gradients(pool, rows, theta, eps, ref)
    d_rows, _ = orc.param_gradients(pool, np.array(ops), np.array(ang), eps, ref)
    want = np.zeros(len(theta))
    np.add.at(want, own, np.array(fac) * d_rows)
    assert np.abs(dE - want).max() < 1e-13

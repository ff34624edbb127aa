"""Spin-complemented generators (Sec. III): the pairing and its sign against
dense Jordan-Wigner operators built from the definition, the product formula
of commuting parts, the singlet character of complemented singles, and the
tied-parameter ADAPT driver on a CPU stand-in context backed by the oracle."""
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp

import oracle
from dense_jw import DenseProblem, annihilators
from paper_2411_07920_amd import spin
from paper_2411_07920_amd.inputs import enumerate_pool, make_integrals, reference_key

N = 4  # spatial orbitals: 8 spin-orbitals, 256-dimensional Fock space


@pytest.fixture(scope="module")
def setup():
    pool = enumerate_pool(N)
    a = annihilators(2 * N)
    ad = [m.T.tocsr() for m in a]
    gp = spin.spin_complemented(pool)
    return pool, a, ad, gp


def _T(row, a, ad):
    P, Q, R, S = (int(x) for x in row)
    if R < 0:
        return (ad[P] @ a[Q]).tocsr()
    return (ad[P] @ ad[Q] @ a[S] @ a[R]).tocsr()


def _A(T):
    return (T - T.T).tocsr()


def test_every_row_in_exactly_one_generator(setup):
    pool, a, ad, gp = setup
    used = np.concatenate([gp.first, gp.second[gp.second >= 0]])
    assert np.array_equal(np.sort(used), np.arange(len(pool)))
    # singles and same-spin doubles always pair with their complement
    paired = set(gp.first[gp.second >= 0].tolist()) | set(gp.second[gp.second >= 0].tolist())
    for k, (P, Q, R, S) in enumerate(pool.tolist()):
        same_spin = R < 0 or len({P & 1, Q & 1, R & 1, S & 1}) == 1
        if same_spin:
            assert k in paired


def test_complement_sign_matches_definition(setup):
    """A_k + sign A_k' equals A(T) + A(T') with T' the spin flip of T written
    in the same operator order, for every two-gate generator."""
    pool, a, ad, gp = setup
    for j in range(len(gp)):
        k, k2, s = int(gp.first[j]), int(gp.second[j]), float(gp.sign[j])
        P, Q, R, S = (int(x) for x in pool[k])
        if R < 0:
            Tf = (ad[P ^ 1] @ a[Q ^ 1]).tocsr()
        else:
            Tf = (ad[P ^ 1] @ ad[Q ^ 1] @ a[S ^ 1] @ a[R ^ 1]).tocsr()
        if k2 < 0:
            continue
        lhs = _A(_T(pool[k], a, ad)) + s * _A(_T(pool[k2], a, ad))
        rhs = _A(_T(pool[k], a, ad)) + _A(Tf)
        assert abs(lhs - rhs).max() == 0.0, (pool[k], pool[k2], s)


def test_paired_parts_commute_exactly_when_disjoint(setup):
    """Pairs on disjoint spin-orbitals commute; pairs marked overlapping do
    not (so they need the one-gate exponential); keeping the overlapping ones
    apart leaves only commuting pairs."""
    pool, a, ad, gp = setup
    n_over = 0
    for j in range(len(gp)):
        if gp.second[j] < 0:
            continue
        A1 = _A(_T(pool[gp.first[j]], a, ad))
        A2 = _A(_T(pool[gp.second[j]], a, ad))
        comm = abs(A1 @ A2 - A2 @ A1).max()
        if gp.overlap[j]:
            n_over += 1
            assert comm > 0.0
        else:
            assert comm == 0.0
    assert n_over > 0
    gp2 = spin.spin_complemented(pool, overlapping=False)
    assert not gp2.overlap.any() and len(gp2) == len(gp) + n_over


def test_product_formula_and_singlet_singles(setup):
    pool, a, ad, gp = setup
    rng = np.random.default_rng(5)
    psi = rng.normal(size=1 << (2 * N))
    psi /= np.linalg.norm(psi)
    # S^2 = S- S+ + Sz (Sz + 1) on the full Fock space
    Sp = sum((ad[2 * p] @ a[2 * p + 1]) for p in range(N))
    Sz = 0.5 * sum((ad[2 * p] @ a[2 * p]) - (ad[2 * p + 1] @ a[2 * p + 1]) for p in range(N))
    I = sp.identity(1 << (2 * N), format="csr")
    S2 = (Sp.T @ Sp + Sz @ (Sz + I)).tocsr()
    theta = 0.37
    for j in rng.choice(np.flatnonzero((gp.second >= 0) & ~gp.overlap), 12, replace=False):
        A1 = _A(_T(pool[gp.first[j]], a, ad)).toarray()
        A2 = _A(_T(pool[gp.second[j]], a, ad)).toarray()
        G = A1 + gp.sign[j] * A2
        exact = scipy.linalg.expm(theta * G) @ psi
        prod = scipy.linalg.expm(gp.sign[j] * theta * A2) @ (scipy.linalg.expm(theta * A1) @ psi)
        assert np.abs(exact - prod).max() < 1e-12
        if pool[gp.first[j]][2] < 0:
            Gs = sp.csr_matrix(G)
            assert abs(S2 @ Gs - Gs @ S2).max() < 1e-12


class OracleContext:
    """The slice of swcs.Context the spin driver uses, on the oracle."""

    def __init__(self, n, ne, h, eri, pool):
        self.orc = oracle.Oracle(n, ne // 2, ne // 2, h, eri)
        self.pool, self.ref = pool, reference_key(ne)

    def apply_ansatz(self, ops, theta, eps=0.0, ncut=0):
        self.ops, self.theta, self.eps, self.gens = np.array(ops), np.array(theta), eps, None
        self.st = oracle.Oracle.apply_ansatz(self.pool, self.ops, self.theta, eps, self.ref)
        return len(self.st)

    def apply_generators(self, gens, theta, eps=0.0, ncut=0):
        self.gens, self.theta, self.eps = np.array(gens, dtype=np.int32), np.array(theta), eps
        self.st = oracle.Oracle.apply_gen_ansatz(self.pool, self.gens, self.theta, eps, self.ref)
        return len(self.st)

    def energy(self):
        return self.orc.energy(self.st)

    def pool_gradients(self, subset=None):
        return self.orc.pool_gradients(self.st, self.pool, subset=subset)

    def param_gradients(self, M):
        if self.gens is not None:
            return self.orc.gen_param_gradients(self.pool, self.gens, self.theta, self.eps, self.ref)
        return self.orc.param_gradients(self.pool, self.ops, self.theta, self.eps, self.ref)


def test_generator_gradients_are_dense_commutators(setup):
    """g_G = <psi|[H, G]|psi> / <psi|psi> on a state of a few gates."""
    n, ne = N, 4
    h, eri = make_integrals(n, n, 88)
    pool = enumerate_pool(n)
    gp = spin.spin_complemented(pool)
    ctx = OracleContext(n, ne, h, eri, pool)
    gens = [int(x) for x in np.flatnonzero(gp.second >= 0)[:6]] + \
        [int(x) for x in np.flatnonzero(gp.overlap)[:3]]
    ctx.apply_generators(spin.gen_rows(gp, gens), np.linspace(0.1, 0.6, len(gens)))
    g = spin.generator_gradients(gp, ctx.pool_gradients())
    dense = DenseProblem(n, ne // 2, ne // 2, h, eri)
    keys, amps = ctx.st.export()
    v = dense.vec(dict(zip(keys.tolist(), amps.tolist())))
    for j in range(0, len(gp), 7):
        G = dense.generator(pool[gp.first[j]])
        if gp.second[j] >= 0:
            G = G + gp.sign[j] * dense.generator(pool[gp.second[j]])
        expect = v @ (dense.H @ G - G @ dense.H) @ v / (v @ v)
        assert abs(g[j] - expect) < 1e-12


def test_spin_adapt_driver_on_stand_in():
    n, ne = N, 4
    h, eri = make_integrals(n, n, 77)
    pool = enumerate_pool(n)
    gp = spin.spin_complemented(pool)
    ctx = OracleContext(n, ne, h, eri, pool)
    gens, theta, hist = spin.run_adapt_spin(ctx, gp, max_iter=8, grad_tol=1e-3)
    Es = [r.get("E_after", r["E"]) for r in hist]
    assert all(b <= a + 1e-10 for a, b in zip(Es, Es[1:]))
    f = spin.TiedEnergy(ctx, gp, gens)
    E, dE = f(theta)
    assert np.abs(dE).max() < 1e-5
    assert E >= DenseProblem(n, ne // 2, ne // 2, h, eri).fci() - 1e-10
    # tied gradients against a central difference of the tied energy
    k = len(theta) - 1
    e = np.zeros_like(theta)
    e[k] = 1e-5
    fd = (f(theta + e)[0] - f(theta - e)[0]) / 2e-5
    assert abs(fd - f(theta)[1][k]) < 1e-8

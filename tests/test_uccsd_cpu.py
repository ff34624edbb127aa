"""Pins of the oracle's MP2-ordered UCCSD ansatz (Sec. II.A) and the host
logic of the product's UCCSD driver (run on a CPU stand-in context).

The oracle takes first-order coefficients <D|H|ref> / (E0(ref) - E0(D)) with
H0 = sum_P f_pp n_P.  Pinned by: the closed-shell spatial-orbital MP2 energy
formula (no determinants involved); the Fock diagonal against energy
differences of N +- 1 electron determinants (Koopmans with frozen orbitals);
and the first-order coefficients against the dense Jordan-Wigner Hamiltonian
and dense exp(theta A) of each operator.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle
from dense_jw import DenseProblem
from paper_2411_07920_amd import uccsd
from paper_2411_07920_amd.inputs import CONFIGS, enumerate_pool, make_integrals, reference_key


def _problem(name):
    c = CONFIGS[name]
    h, eri = make_integrals(c.n, c.rank, c.seed_int)
    na = c.n_elec // 2
    return c.n, na, h, eri, enumerate_pool(c.n), reference_key(c.n_elec)


def _fock_diag(h, eri, n_occ):
    return np.diag(oracle.fock_spatial(h, eri, n_occ))


def spatial_mp2(h, eri, n_occ, f):
    """Closed-shell MP2 energy in spatial orbitals:
    sum_{ij occ, ab vir} (ia|jb) [2 (ia|jb) - (ib|ja)] / (f_i + f_j - f_a - f_b)."""
    n = h.shape[0]
    occ, vir = range(n_occ), range(n_occ, n)
    e2 = 0.0
    for i in occ:
        for j in occ:
            for a in vir:
                for b in vir:
                    iajb, ibja = eri[i, a, j, b], eri[i, b, j, a]
                    e2 += iajb * (2.0 * iajb - ibja) / (f[i] + f[j] - f[a] - f[b])
    return e2


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_mp2_energy_matches_spatial_formula(name):
    n, na, h, eri, pool, ref = _problem(name)
    orc = oracle.Oracle(n, na, na, h, eri)
    ops, theta, e2 = oracle.mp2_uccsd(orc, pool, ref)
    f = _fock_diag(h, eri, na)
    expect = spatial_mp2(h, eri, na, f)
    assert abs(e2 - expect) < 1e-12 * max(1.0, abs(expect))
    # negative when every virtual f_aa lies above every occupied f_ii (true
    # for c1; the synthetic c2 reference is not aufbau and E2 is positive)
    if f[na:].min() > f[:na].max():
        assert e2 < 0.0


def test_fock_diagonal_is_koopmans_energy_difference():
    """f_aa = E(ref + a) - E(ref) for a virtual, f_ii = E(ref) - E(ref - i)
    for an occupied spin-orbital (single determinants, frozen orbitals)."""
    n, na, h, eri, pool, ref = _problem("c1")
    f = _fock_diag(h, eri, na)
    e_ref = oracle.Oracle(n, na, na, h, eri).hmat(ref, ref)
    up = oracle.Oracle(n, na + 1, na, h, eri)
    down = oracle.Oracle(n, na - 1, na, h, eri)
    for p in range(n):
        P = 2 * p  # alpha spin-orbital of spatial orbital p
        if (ref >> P) & 1:
            key = ref ^ (1 << P)
            assert abs((e_ref - down.hmat(key, key)) - f[p]) < 1e-12
        else:
            key = ref | (1 << P)
            assert abs((up.hmat(key, key) - e_ref) - f[p]) < 1e-12


def test_first_order_coefficients_match_dense():
    """For every double of c1: asin of <D| exp(theta_k A_k) |ref> (dense expm of
    the dense generator) equals <D|H|ref> / (E0(ref) - E0(D)) from the dense
    Jordan-Wigner Hamiltonian; singles have theta 0."""
    n, na, h, eri, pool, ref = _problem("c1")
    orc = oracle.Oracle(n, na, na, h, eri)
    ops, theta, e2 = oracle.mp2_uccsd(orc, pool, ref)
    dense = DenseProblem(n, na, na, h, eri)
    f = _fock_diag(h, eri, na)
    v0 = dense.ref_vec(ref)
    i0 = dense.index[int(ref)]

    def e0(key):
        return sum(f[P >> 1] for P in range(2 * n) if (key >> P) & 1)

    n_doubles = 0
    e2_dense = 0.0
    for k, t in zip(ops.tolist(), theta.tolist()):
        A = dense.generator(pool[k])
        out = A @ v0
        hit = np.flatnonzero(out)
        assert len(hit) == 1
        D = int(dense.basis[hit[0]])
        if pool[k][2] < 0:
            assert t == 0.0
            continue
        n_doubles += 1
        c = (scipy.linalg.expm(t * A) @ v0)[hit[0]]
        t_dense = dense.H[hit[0], i0] / (e0(ref) - e0(D))
        e2_dense += dense.H[hit[0], i0] ** 2 / (e0(ref) - e0(D))
        assert abs(math.asin(c) - t_dense) < 1e-12
    assert n_doubles == 76
    assert abs(e2 - e2_dense) < 1e-12


def test_uccsd_order_properties():
    n, na, h, eri, pool, ref = _problem("c2")
    orc = oracle.Oracle(n, na, na, h, eri)
    ops, theta, e2 = oracle.mp2_uccsd(orc, pool, ref)
    is_double = pool[ops][:, 2] >= 0
    nd = int(is_double.sum())
    # 2 C(5,2) C(9,2) + 5^2 9^2 doubles, 2 * 5 * 9 singles
    assert nd == 2745 and len(ops) - nd == 90
    assert is_double[:nd].all() and not is_double[nd:].any()
    a = np.abs(theta[:nd])
    assert np.all(a[1:] <= a[:-1] + 1e-9 * a.max())
    assert np.all(theta[nd:] == 0.0)
    assert len(set(ops.tolist())) == len(ops)


class OracleContext:
    """The slice of swcs.Context that the UCCSD driver uses, on the oracle."""

    def __init__(self, n, na, h, eri, pool, ref):
        self.n = n
        self.h, self.eri, self.na = h, eri, na
        self.orc = oracle.Oracle(n, na, na, h, eri)
        self.pool, self.ref = pool, ref

    def fock_diagonal(self):
        return _fock_diag(self.h, self.eri, self.na)

    def set_state(self, keys, amps):
        self.st = oracle.OracleState.from_arrays(keys, amps)

    def energy(self):
        return self.orc.energy(self.st)

    def pool_gradients(self, subset=None):
        return self.orc.pool_gradients(self.st, self.pool, subset=subset)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_driver_host_logic_matches_oracle(name):
    """The product driver (pool gradients at the reference divided by twice
    the zeroth-order gap) on a stand-in context gives the oracle's ansatz."""
    n, na, h, eri, pool, ref = _problem(name)
    ctx = OracleContext(n, na, h, eri, pool, ref)
    ans = uccsd.mp2_ordered_uccsd(ctx, pool, ref, n)
    ops, theta, e2 = oracle.mp2_uccsd(ctx.orc, pool, ref)
    assert np.array_equal(ans.ops, ops)
    # relative: near-zero gaps of the non-aufbau c2 reference give |theta| ~ 20
    assert np.all(np.abs(ans.theta - theta) <= 1e-12 * np.maximum(1.0, np.abs(theta)))
    assert abs(ans.e2 - e2) < 1e-12 * max(1.0, abs(e2))
    assert abs(ans.e_ref - ctx.orc.hmat(ref, ref)) < 1e-12


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_spin_complemented_uccsd(name):
    """Complement pairs of UCCSD operators carry amplitudes theta_k' =
    sign * theta_k, so the tied ansatz starts from the MP2 amplitudes of every
    operator; each UCCSD operator appears in exactly one generator."""
    from paper_2411_07920_amd import spin
    n, na, h, eri, pool, ref = _problem(name)
    ctx = OracleContext(n, na, h, eri, pool, ref)
    ans = uccsd.mp2_ordered_uccsd(ctx, pool, ref, n)
    gp = spin.spin_complemented(pool)
    gens, theta = uccsd.spin_complemented_uccsd(ans, gp)
    rows = spin.gen_rows(gp, gens)
    ops, ang = [], []
    for (k1, k2, sg), t in zip(rows.tolist(), theta.tolist()):
        ops.append(k1), ang.append(t)
        if k2 >= 0:
            ops.append(k2), ang.append(sg * t)
    assert sorted(ops) == sorted(ans.ops.tolist())
    mp2 = dict(zip(ans.ops.tolist(), ans.theta.tolist()))
    assert all(abs(a - mp2[k]) <= 1e-12 * max(1.0, abs(mp2[k])) for k, a in zip(ops, ang))
    assert len(gens) < len(ans.ops)
    assert gp.overlap[gens].any()     # overlapping complement pairs are tied too

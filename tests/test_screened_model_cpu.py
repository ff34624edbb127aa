"""The determinant-major screened pool-gradient passes (query, push,
contract; ADAPT step 4, Sec. II.C), modelled on the host, against the oracle
on the c2 state: a 6,000-operator subset, unbatched and split into key-hash
batches.  Pins the algorithm the HIP path follows (linking operator from the
generator table, the sign a_k(D), the diagonal term, the batch partition)."""
import numpy as np
import pytest

import oracle
import screened_model as sm
from paper_2411_07920_amd.inputs import (CONFIGS, draw_ansatz, enumerate_pool, make_integrals,
                                         reference_key)


@pytest.fixture(scope="module")
def c2():
    c = CONFIGS["c2"]
    h, eri = make_integrals(c.n, c.rank, c.seed_int)
    pool = enumerate_pool(c.n)
    ops, theta = draw_ansatz(len(pool), c.n_ops, c.theta_lo, c.theta_hi, c.seed_ansatz)
    ref = reference_key(c.n_elec)
    st = oracle.Oracle.apply_ansatz(pool, ops, theta, c.eps, ref)
    orc = oracle.Oracle(c.n, c.n_elec // 2, c.n_elec // 2, h, eri)
    keys, amps = st.export()
    return dict(h=h, eri=eri, pool=pool, st=st, orc=orc, keys=keys, amps=amps)


def test_generator_table_inverts_linking(c2):
    """Every pool row is found again from the holes and particles of the
    connection it makes: T acts when its annihilated orbitals are the holes,
    T^dagger when its created orbitals are."""
    pool = c2["pool"]
    tab, npairs = sm.generator_table(pool, 28)
    P, Q, R, S = (pool[:, j].astype(np.int64) for j in range(4))
    single = R < 0
    h0 = np.where(single, Q, np.minimum(R, S))
    h1 = np.where(single, Q, np.maximum(R, S))
    p0 = np.where(single, P, np.minimum(P, Q))
    p1 = np.where(single, P, np.maximum(P, Q))
    nh = np.where(single, 1, 2)
    k, t, *_ = sm.linking_operator(tab, npairs, nh, h0, h1, p0, p1)
    assert np.array_equal(k, np.arange(len(pool))) and t.all()
    k2, t2, *_ = sm.linking_operator(tab, npairs, nh, p0, p1, h0, h1)
    assert np.array_equal(k2, np.arange(len(pool))) and not t2.any()


@pytest.mark.parametrize("nbatch", [1, 5])
def test_screened_model_matches_oracle_c2(c2, nbatch):
    rng = np.random.default_rng(12)
    rng.choice(len(c2["pool"]), 500, replace=False)   # the GPU test draws 500 first
    subset = np.sort(rng.choice(len(c2["pool"]), 6000, replace=False)).astype(np.int32)
    g = sm.screened_gradients(c2["keys"], c2["amps"], c2["pool"], subset, c2["h"], c2["eri"], nbatch)
    g_ref = c2["orc"].pool_gradients(c2["st"], c2["pool"], subset=subset)
    assert np.abs(g_ref).max() > 1e-3
    assert np.abs(g - g_ref).max() < 1e-12

"""The sort-and-join pool gradient (ADAPT step 4, Sec. II.C) modelled on the
host against the oracle: records encoded and decoded the way the kernels do,
grouped by their hash bucket, sigma and g formed per group.  Pins the record
layout, the decoding from the fields and lists alone, the identity between
pool operators and connections, and the diagonal record."""
import numpy as np
import pytest

import join_model as jm
import oracle
from paper_2411_07920_amd.inputs import (CONFIGS, draw_ansatz, draw_synthetic_state, enumerate_pool,
                                         make_integrals, reference_key)


@pytest.mark.parametrize("name,orbital", [("c1", None), ("c2", None), ("c1", False), ("c2", False)])
def test_join_model_matches_oracle(name, orbital):
    c = CONFIGS[name]
    h, eri = make_integrals(c.n, c.rank, c.seed_int)
    pool = enumerate_pool(c.n)
    ops, theta = draw_ansatz(len(pool), c.n_ops, c.theta_lo, c.theta_hi, c.seed_ansatz)
    na = (c.n_elec + 1) // 2
    nb = c.n_elec // 2
    st = oracle.Oracle.apply_ansatz(pool, ops, theta, c.eps, reference_key(c.n_elec))
    orc = oracle.Oracle(c.n, na, nb, h, eri)
    keys, amps = st.export()
    g, X_dec, X_enum, fmt = jm.join_gradients(keys, amps, pool, h, eri, na, nb, orbital)
    assert fmt[3] == (orbital is None)  # orbital fields fit these small states
    assert np.array_equal(X_dec, X_enum)
    g_ref = orc.pool_gradients(st, pool)
    assert np.abs(g_ref).max() > 1e-3
    assert np.abs(g - g_ref).max() < 1e-12


def test_join_model_open_shell_and_dead_entries():
    """Unequal spin counts (every class size differs) and pruned entries in
    storage, which emit nothing; both record formats."""
    n, na, nb = 6, 3, 2
    h, eri = make_integrals(n, n, 1203)
    pool = enumerate_pool(n)
    keys, amps = draw_synthetic_state(n, na, nb, 40, 4203)
    amps = amps.copy()
    amps[[3, 17, 25]] = np.nan
    alive = ~np.isnan(amps)
    st = oracle.OracleState.from_arrays(keys[alive], amps[alive])
    orc = oracle.Oracle(n, na, nb, h, eri)
    g_ref = orc.pool_gradients(st, pool)
    for orbital in (None, False):
        g, X_dec, X_enum, fmt = jm.join_gradients(keys, amps, pool, h, eri, na, nb, orbital)
        assert np.array_equal(X_dec, X_enum)
        assert np.abs(g - g_ref).max() < 1e-12

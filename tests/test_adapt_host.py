"""Host logic of the ADAPT-VQE / pre-optimization drivers, run on the CPU
against a stand-in context backed by the oracle (no GPU involved)."""
import numpy as np
import pytest

import oracle
from paper_2411_07920_amd import adapt
from paper_2411_07920_amd.inputs import enumerate_pool, make_integrals, reference_key


class OracleContext:
    """Implements the slice of swcs.Context the drivers use, on the oracle."""

    def __init__(self, n, ne, h, eri, pool):
        self.orc = oracle.Oracle(n, ne // 2, ne // 2, h, eri)
        self.pool = pool
        self.ref = reference_key(ne)
        self.K = len(pool)
        self.calls = {"apply": 0, "pool": 0, "param": 0}

    def apply_ansatz(self, ops, theta, eps=0.0, ncut=0):
        self.calls["apply"] += 1
        self.ops, self.theta, self.eps, self.ncut = np.array(ops), np.array(theta), eps, ncut
        self.st = oracle.Oracle.apply_ansatz(self.pool, self.ops, self.theta, eps, self.ref, ncut)
        return len(self.st)

    def energy(self):
        return self.orc.energy(self.st)

    def pool_gradients(self, subset=None):
        self.calls["pool"] += 1
        return self.orc.pool_gradients(self.st, self.pool, subset=subset)

    def param_gradients(self, M):
        self.calls["param"] += 1
        return self.orc.param_gradients(self.pool, self.ops, self.theta, self.eps, self.ref, self.ncut)


@pytest.fixture(scope="module")
def problem():
    n, ne = 4, 4
    h, eri = make_integrals(n, n, 77)
    pool = enumerate_pool(n)
    return n, ne, h, eri, pool


def test_adapt_decreases_energy_and_converges(problem):
    n, ne, h, eri, pool = problem
    ctx = OracleContext(n, ne, h, eri, pool)
    cfg = adapt.AdaptConfig(eps=0.0, max_iter=12, grad_tol=1e-3, optimizer="lbfgs")
    ops, theta, hist = adapt.run_adapt(ctx, len(pool), cfg)
    Es = [r["E"] for r in hist]
    assert all(b <= a + 1e-10 for a, b in zip(Es, Es[1:]))
    # the selected operator is the argmax of the exact pool gradient
    for r in hist:
        assert r["full"] and r["n_exact"] == len(pool)
    # the VQE optimum has a vanishing gradient
    ctx.apply_ansatz(ops, theta)
    dE, _ = ctx.param_gradients(len(ops))
    assert np.abs(dE).max() < 1e-5
    # never below the exact ground state of the 36-determinant sector
    from dense_jw import DenseProblem
    assert hist[-1]["E"] >= DenseProblem(n, 2, 2, h, eri).fci() - 1e-10


@pytest.mark.parametrize("method", ["bfgs", "lbfgs", "bfgs2", "bfgs2f"])
def test_optimizers_reach_stationary_points(problem, method):
    n, ne, h, eri, pool = problem
    ctx = OracleContext(n, ne, h, eri, pool)
    cfg = adapt.AdaptConfig(eps=0.0, max_iter=4, grad_tol=None, optimizer=method)
    ops, theta, hist = adapt.run_adapt(ctx, len(pool), cfg)
    assert len(ops) == 4
    ctx.apply_ansatz(ops, theta)
    dE, _ = ctx.param_gradients(len(ops))
    if method == "bfgs2f":
        assert abs(dE[-1]) < 1e-5      # only the newest parameter is optimized
    else:
        assert np.abs(dE).max() < 1e-5


def test_adapt_first_operator_is_largest_hf_gradient(problem):
    n, ne, h, eri, pool = problem
    ctx = OracleContext(n, ne, h, eri, pool)
    ctx.apply_ansatz(np.zeros(0, np.int32), np.zeros(0))
    g = ctx.pool_gradients()
    cfg = adapt.AdaptConfig(eps=0.0, max_iter=1, grad_tol=None)
    ops, _, _ = adapt.run_adapt(ctx, len(pool), cfg)
    assert ops[0] == int(np.argmax(np.abs(g)))


def test_preoptimize_lbfgs_lowers_energy(problem):
    n, ne, h, eri, pool = problem
    ctx = OracleContext(n, ne, h, eri, pool)
    rng = np.random.default_rng(1)
    ops = rng.choice(len(pool), 8, replace=False).astype(np.int32)
    th0 = rng.uniform(-0.05, 0.05, 8)
    cfg = adapt.AdaptConfig(eps=1e-4, optimizer="lbfgs")
    ctx.apply_ansatz(ops, th0, 1e-4)
    E0 = ctx.energy()[0]
    th, E, trace, evals = adapt.preoptimize(ctx, ops, th0, cfg)
    assert E <= E0 + 1e-12 and evals >= 2
    assert all(b <= a + 1e-9 for a, b in zip(trace, trace[1:]))


def test_pruned_adapt_leaves_the_zero_plateau(problem):
    """With eps pruning a new parameter at 0 creates only zero partners, which
    are dropped, so the pruned energy is flat there; the driver must still
    lower the energy beyond the reference."""
    n, ne, h, eri, pool = problem
    ctx = OracleContext(n, ne, h, eri, pool)
    cfg = adapt.AdaptConfig(eps=1e-4, max_iter=5, grad_tol=None, optimizer="lbfgs")
    ops, theta, hist = adapt.run_adapt(ctx, len(pool), cfg)
    ctx.apply_ansatz(np.zeros(0, np.int32), np.zeros(0), 1e-4)
    e_ref = ctx.energy()[0]
    assert hist[-1]["E_after"] < e_ref - 1e-3
    assert np.all(np.abs(theta) > 0)
    ctx.apply_ansatz(ops, theta, 1e-4)
    assert len(ctx.st) > 1


def test_seed_last_parameter_is_exact_without_pruning(problem):
    n, ne, h, eri, pool = problem
    ctx = OracleContext(n, ne, h, eri, pool)
    rng = np.random.default_rng(4)
    ops = rng.choice(len(pool), 5, replace=False).astype(np.int32)
    th = rng.uniform(-0.3, 0.3, 5)
    cfg = adapt.AdaptConfig(eps=0.0)
    seeded, _ = adapt.seed_last_parameter(ctx, ops, th, cfg)
    grid = np.linspace(-np.pi, np.pi, 721)
    Es = []
    for t in grid:
        x = th.copy(); x[-1] = t
        ctx.apply_ansatz(ops, x)
        Es.append(ctx.energy()[0])
    x = th.copy(); x[-1] = seeded[-1]
    ctx.apply_ansatz(ops, x)
    assert ctx.energy()[0] <= min(Es) + 1e-6


def test_select_operator_ties_go_to_smallest_index():
    g = np.array([0.1, -0.5, 0.5 * (1 + 1e-13), 0.2])
    assert adapt.select_operator(g, np.arange(4)) == 1
    idx = np.array([9, 4, 7, 1])
    assert adapt.select_operator(np.array([0.5, 0.1, -0.5, 0.0]), idx) == 2
    assert adapt.select_operator(np.array([0.3, 0.5, 0.1]), np.arange(3)) == 1


def test_bootstrap_ncut_restart(problem):
    """Bootstrap N_CUT (Sec. IV): ADAPT at a small N_CUT, then a restart at a
    larger N_CUT from the final ansatz (ops0 / theta0).  The restart's first
    energy is the seeded ansatz's energy at the larger N_CUT, and the energy
    keeps decreasing."""
    n, ne, h, eri, pool = problem
    ctx = OracleContext(n, ne, h, eri, pool)
    cfg1 = adapt.AdaptConfig(ncut=6, max_iter=4, grad_tol=None, optimizer="lbfgs")
    ops1, th1, hist1 = adapt.run_adapt(ctx, len(pool), cfg1)
    cfg2 = adapt.AdaptConfig(ncut=30, max_iter=3, grad_tol=None, optimizer="lbfgs")
    ops2, th2, hist2 = adapt.run_adapt(ctx, len(pool), cfg2, ops0=ops1, theta0=th1)
    assert ops2[: len(ops1)].tolist() == ops1.tolist() and len(ops2) == len(ops1) + 3
    ctx.apply_ansatz(ops1, th1, 0.0, 30)
    assert abs(hist2[0]["E"] - ctx.energy()[0]) < 1e-12
    Es = [r["E_after"] for r in hist2]
    assert all(b <= a + 1e-10 for a, b in zip([hist2[0]["E"]] + Es, Es))
    assert hist1[0]["n_det"] <= 6 and hist2[-1]["n_det"] <= 30


def test_adapt_checkpoint_resume(problem, tmp_path):
    """A run split into segments through its checkpoint (3 iterations, then
    the rest up to 6) chooses the same operators and reaches the same
    parameters and energies as one uninterrupted run; a time limit stops a
    segment at an iteration boundary; a converged run is not continued."""
    import dataclasses
    n, ne, h, eri, pool = problem
    cfg = adapt.AdaptConfig(eps=1e-4, max_iter=6, grad_tol=None, optimizer="lbfgs")
    ops_a, th_a, hist_a = adapt.run_adapt(OracleContext(n, ne, h, eri, pool), len(pool), cfg)
    path = str(tmp_path / "adapt.npz")
    o1, _, h1 = adapt.run_adapt(OracleContext(n, ne, h, eri, pool), len(pool),
                                dataclasses.replace(cfg, max_iter=3), checkpoint=path)
    assert len(h1) == 3 and o1.tolist() == ops_a[:3].tolist()
    # a segment with a zero time limit still completes one iteration
    o2, _, h2 = adapt.run_adapt(OracleContext(n, ne, h, eri, pool), len(pool), cfg,
                                checkpoint=path, time_limit=0.0)
    assert len(h2) == 4
    ops_b, th_b, hist_b = adapt.run_adapt(OracleContext(n, ne, h, eri, pool), len(pool), cfg,
                                          checkpoint=path)
    assert ops_b.tolist() == ops_a.tolist()
    assert np.array_equal(th_b, th_a)
    assert [r["E_after"] for r in hist_b] == [r["E_after"] for r in hist_a]
    # converged runs are final
    path2 = str(tmp_path / "conv.npz")
    cfg_c = adapt.AdaptConfig(eps=0.0, max_iter=40, grad_tol=1e-1, optimizer="lbfgs")
    oc, tc, hc = adapt.run_adapt(OracleContext(n, ne, h, eri, pool), len(pool), cfg_c, checkpoint=path2)
    assert hc[-1].get("converged")
    ctx = OracleContext(n, ne, h, eri, pool)
    od, td, hd = adapt.run_adapt(ctx, len(pool), cfg_c, checkpoint=path2)
    assert od.tolist() == oc.tolist() and ctx.calls["apply"] == 0

"""Spin-complemented ADAPT (Sec. III) on the GPU library: the run over
complemented generators chooses the same generators and reaches the same
energies as the same driver on the oracle, and the generator gradients of the
GPU pool equal the oracle's."""
import numpy as np
import pytest

from paper_2411_07920_amd import spin
from paper_2411_07920_amd.inputs import CONFIGS, enumerate_pool, make_integrals, reference_key

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swcs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_07920_amd import swcs as mod
    mod.load()
    return mod


@pytest.mark.parametrize("name,eps,iters", [("c1", 0.0, 8), ("c2", 1e-6, 4)])
def test_spin_adapt_follows_oracle_driver(swcs, name, eps, iters):
    from test_spin_cpu import OracleContext
    c = CONFIGS[name]
    h, eri = make_integrals(c.n, c.rank, c.seed_int)
    pool = enumerate_pool(c.n)
    gp = spin.spin_complemented(pool)
    gpu = swcs.make_context(c.n, c.n_elec // 2, c.n_elec // 2, h, eri, pool, reference_key(c.n_elec))
    cpu = OracleContext(c.n, c.n_elec, h, eri, pool)
    g_gpu, th_gpu, hist_gpu = spin.run_adapt_spin(gpu, gp, eps=eps, max_iter=iters, grad_tol=None)
    g_cpu, th_cpu, hist_cpu = spin.run_adapt_spin(cpu, gp, eps=eps, max_iter=iters, grad_tol=None)
    assert g_gpu == g_cpu
    for a, b in zip(hist_gpu, hist_cpu):
        assert abs(a["gmax"] - b["gmax"]) < 1e-9
        assert abs(a["E_after"] - b["E_after"]) < 1e-7
    # generator gradients of the final GPU state against the oracle's
    ops, ang = spin.expand(gp, g_gpu, th_gpu)
    gpu.apply_ansatz(ops, ang, eps)
    cpu.apply_ansatz(ops, ang, eps)
    gg = spin.generator_gradients(gp, gpu.pool_gradients())
    gc = spin.generator_gradients(gp, cpu.pool_gradients())
    assert np.abs(gg - gc).max() < 1e-10
    gpu.close()

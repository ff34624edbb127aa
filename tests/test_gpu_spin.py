"""Spin-complemented generators (Sec. III) on the GPU library: chains with
overlapping complement pairs (one exact gate each) against the oracle, bit
for bit, with energies and per-generator adjoint gradients; the ADAPT run over
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
    rows = spin.gen_rows(gp, g_gpu)
    gpu.apply_generators(rows, th_gpu, eps)
    cpu.apply_generators(rows, th_gpu, eps)
    gg = spin.generator_gradients(gp, gpu.pool_gradients())
    gc = spin.generator_gradients(gp, cpu.pool_gradients())
    assert np.abs(gg - gc).max() < 1e-10
    gpu.close()


def _spreading_gens(gp, pool, ref, n_gens, rng, theta_max):
    """Generators chosen to act on the current support (every third one a
    pair that overlaps), so the state spreads."""
    import oracle
    rows_all = spin.gen_rows(gp, np.arange(len(gp)))
    over = set(np.flatnonzero(gp.overlap).tolist())

    def acts(row, key):
        P, Q, R, S = (int(x) for x in row)
        cre = [P, Q] if R >= 0 else [P]
        ann = [R, S] if R >= 0 else [Q]
        occ = lambda x: (key >> x) & 1
        return (all(occ(a) for a in ann) and not any(occ(c) for c in cre)) or \
               (all(occ(c) for c in cre) and not any(occ(a) for a in ann))

    gens, theta, support = [], [], [ref]
    for i in range(n_gens):
        key = support[rng.integers(len(support))]
        cands = [j for j in range(len(gp)) if acts(pool[gp.first[j]], key) and ((i % 3 == 0) == (j in over))]
        if not cands:
            cands = [j for j in range(len(gp)) if acts(pool[gp.first[j]], key)]
        gens.append(int(cands[rng.integers(len(cands))]))
        theta.append(float(rng.uniform(-theta_max, theta_max)))
        st = oracle.Oracle.apply_gen_ansatz(pool, rows_all[gens], np.array(theta), 0.0, ref)
        support = st.export()[0].tolist()
    return np.array(gens), np.array(theta)


@pytest.mark.parametrize("n,ne,n_gens,eps,ncut", [(6, 4, 30, 0.0, 0), (6, 4, 30, 0.0, 60),
                                                  (8, 8, 70, 0.0, 0), (8, 8, 70, 1e-4, 0)])
def test_generator_chain_parity(swcs, n, ne, n_gens, eps, ncut):
    """Chains of spin-complemented generators, overlapping pairs as one exact
    gate: state bit for bit, energy, one adjoint derivative per generator and
    the pool gradients, against the oracle.  The 16-spin-orbital chains grow
    the state past the initial capacity."""
    import oracle
    h, eri = make_integrals(n, n, 1400 + n)
    pool = enumerate_pool(n)
    gp = spin.spin_complemented(pool)
    ref = reference_key(ne)
    rng = np.random.default_rng(n * 100 + n_gens)
    gens, theta = _spreading_gens(gp, pool, ref, n_gens, rng, 0.8)
    rows = spin.gen_rows(gp, gens)
    assert gp.overlap[gens].sum() >= n_gens // 4
    st = oracle.Oracle.apply_gen_ansatz(pool, rows, theta, eps, ref, ncut)
    orc = oracle.Oracle(n, ne // 2, ne // 2, h, eri)
    ctx = swcs.make_context(n, ne // 2, ne // 2, h, eri, pool, ref)
    print(f"[spin] generators n={n} ne={ne} M={n_gens} eps={eps} ncut={ncut}: {len(st)} dets", flush=True)
    assert ctx.apply_generators(rows, theta, eps, ncut) == len(st)
    k, a = ctx.get_state()
    k_ref, a_ref = st.export()
    assert np.array_equal(k, k_ref)
    assert np.array_equal(a, a_ref), np.abs(a - a_ref).max()
    E = ctx.energy()[0]
    assert abs(E - orc.energy(st)[0]) < 1e-10
    dE, E2 = ctx.param_gradients(len(theta))
    dE_ref, E_ref = orc.gen_param_gradients(pool, rows, theta, eps, ref, ncut)
    assert abs(E2 - E_ref) < 1e-10
    assert np.abs(dE - dE_ref).max() < 1e-10
    g = ctx.pool_gradients()
    assert np.abs(g - orc.pool_gradients(st, pool)).max() < 1e-10
    if n == 8 and eps == 0.0:
        assert len(st) > 4096
    ctx.close()

"""GPU parity of the screener kernels against the float64 numpy oracle.

Bars (float32 kernels): features within 1e-6 relative, MLP forward within
1e-5 relative, MLP gradients within 1e-4 relative, Adam within 1e-6, and the
selected index set identical to the oracle's.
"""
import numpy as np
import pytest

import oracle
from paper_2411_07920_amd.inputs import (CONFIGS, draw_ansatz, draw_random_keys, enumerate_pool,
                                         make_integrals, reference_key)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_07920_amd import swcs
    c = CONFIGS["c2"]
    h, eri = make_integrals(c.n, c.rank, c.seed_int)
    pool = enumerate_pool(c.n)
    ops, theta = draw_ansatz(len(pool), c.n_ops, c.theta_lo, c.theta_hi, c.seed_ansatz)
    ref = reference_key(c.n_elec)
    ctx = swcs.make_context(c.n, 5, 5, h, eri, pool, ref)
    ctx.apply_ansatz(ops, theta, c.eps)
    yield dict(torch=torch, swcs=swcs, ctx=ctx, h=h, eri=eri, pool=pool, ops=ops, theta=theta,
               c=c, ref=ref)
    ctx.close()


def rel(a, b):
    return np.abs(a - b).max() / max(1e-30, np.abs(b).max())


def test_features(env):
    torch, ctx, pool = env["torch"], env["ctx"], env["pool"]
    K = len(pool)
    rng = np.random.default_rng(1)
    prev = np.where(rng.random(K) < 0.3, rng.random(K), 0.0).astype(np.float32)
    age = rng.integers(0, 30, K).astype(np.float32)
    cnt = rng.integers(0, 3, K).astype(np.float32)
    dev = lambda a: torch.from_numpy(a).cuda()
    out = torch.zeros((K, 16), dtype=torch.float32, device="cuda")
    ctx.features(dev(prev), dev(age), dev(cnt), out)
    torch.cuda.synchronize()
    c = env["c"]
    orc = oracle.Oracle(c.n, 5, 5, env["h"], env["eri"])
    st = oracle.Oracle.apply_ansatz(pool, env["ops"], env["theta"], c.eps, env["ref"])
    fock = oracle.fock_spatial(env["h"], env["eri"], 5)
    F = oracle.features(pool, fock, env["eri"], orc.occupations(st), prev.astype(np.float64),
                        age.astype(np.float64), cnt.astype(np.float64))
    got = out.cpu().numpy().astype(np.float64)
    for j in range(16):
        scale = max(1e-30, np.abs(F[:, j]).max())
        assert np.abs(got[:, j] - F[:, j]).max() / scale < 2e-6, j


def test_mlp_forward_backward(env):
    torch, ctx, swcs = env["torch"], env["ctx"], env["swcs"]
    assert swcs.mlp_param_count() == oracle.N_PARAMS
    rng = np.random.default_rng(2)
    w = oracle.mlp_init(3)
    w[oracle.LAYOUT["b1"][0]:oracle.LAYOUT["b1"][0] + 128] = rng.normal(0, 0.1, 128)
    w[oracle.LAYOUT["b2"][0]:oracle.LAYOUT["b2"][0] + 128] = rng.normal(0, 0.1, 128)
    w32 = w.astype(np.float32)
    for B in (1, 31, 32, 77, 1000):
        x = rng.normal(size=(B, 16)).astype(np.float32)
        dy = rng.normal(size=B).astype(np.float32)
        W = torch.from_numpy(w32).cuda()
        X = torch.from_numpy(x).cuda()
        Y = torch.zeros(B, device="cuda")
        A = torch.zeros((B, 256), device="cuda")
        ctx.mlp_forward(W, X, Y, A)
        dW = torch.zeros(oracle.N_PARAMS, device="cuda")
        ctx.mlp_backward(W, X, A, torch.from_numpy(dy).cuda(), dW)
        torch.cuda.synchronize()
        y_ref, cache = oracle.mlp_forward(w32.astype(np.float64), x.astype(np.float64))
        g_ref = oracle.mlp_backward(w32.astype(np.float64), cache, dy.astype(np.float64))
        assert rel(Y.cpu().numpy(), y_ref) < 1e-5
        assert rel(dW.cpu().numpy(), g_ref) < 1e-4


def test_mse_and_adam(env):
    torch, ctx = env["torch"], env["ctx"]
    rng = np.random.default_rng(4)
    y = rng.normal(size=500).astype(np.float32)
    t = rng.normal(size=500).astype(np.float32)
    dy = torch.zeros(500, device="cuda")
    loss = torch.zeros(1, device="cuda")
    ctx.mse(torch.from_numpy(y).cuda(), torch.from_numpy(t).cuda(), dy, loss)
    torch.cuda.synchronize()
    assert abs(loss.item() - np.mean((y.astype(np.float64) - t) ** 2)) < 1e-5
    assert rel(dy.cpu().numpy(), 2 * (y.astype(np.float64) - t) / 500) < 1e-6
    P = oracle.N_PARAMS
    w = rng.normal(size=P)
    m = np.zeros(P)
    v = np.zeros(P)
    Wd = torch.from_numpy(w.astype(np.float32)).cuda()
    Md = torch.zeros(P, device="cuda")
    Vd = torch.zeros(P, device="cuda")
    for step in range(1, 4):
        g = rng.normal(size=P)
        w, m, v = oracle.adam_step(w, m, v, g, 1e-3, 0.9, 0.999, 1e-8, step)
        ctx.adam_step(Wd, Md, Vd, torch.from_numpy(g.astype(np.float32)).cuda(), 1e-3, 0.9, 0.999,
                      1e-8, step)
    torch.cuda.synchronize()
    assert np.abs(Wd.cpu().numpy() - w).max() < 1e-5


def test_select_matches_oracle(env):
    torch, ctx = env["torch"], env["ctx"]
    # single-workgroup path up to 131,072 operators, sort-based path above;
    # ties in both keys; no top or no random share
    cases = [(10, 0.05, 0.01), (1000, 0.05, 0.01), (22750, 0.05, 0.01), (22750, 0.0, 0.02),
             (22750, 0.03, 0.0), (101650, 0.05, 0.01), (150000, 0.05, 0.01)]
    for K, ft, fr in cases:
        rng = np.random.default_rng(K)
        score = rng.normal(size=K).astype(np.float32)
        score[::7] = score[3]  # ties
        rnd = draw_random_keys(K, 99)
        rnd[::5] = rnd[2]  # ties
        n_top, n_rand = int(np.ceil(ft * K)), int(np.ceil(fr * K))
        out = torch.zeros(n_top + n_rand, dtype=torch.int32, device="cuda")
        ctx.select(torch.from_numpy(score).cuda(), torch.from_numpy(rnd.astype(np.int32)).cuda(),
                   n_top, n_rand, out)
        torch.cuda.synchronize()
        ref = oracle.select_subset(score, rnd, ft, fr)
        assert out.cpu().numpy().tolist() == ref.tolist(), (K, ft, fr)


def test_select_degenerate_scores(env):
    """Scores that share their leading digits: all equal (the candidates stay
    above the LDS list size until the index digits), three distinct values,
    and one value per 5,000 operators; random keys with heavy ties."""
    torch, ctx = env["torch"], env["ctx"]
    K = 22750
    rng = np.random.default_rng(77)
    cases = [np.full(K, 0.25, dtype=np.float32),
             rng.choice(np.array([-1.5, 0.5, 0.75], dtype=np.float32), K),
             (np.arange(K) // 5000).astype(np.float32) * np.float32(0.001)]
    for c_i, score in enumerate(cases):
        for rnd in (draw_random_keys(K, 5 + c_i), np.full(K, 7, dtype=np.uint32)):
            n_top, n_rand = int(np.ceil(0.05 * K)), int(np.ceil(0.01 * K))
            out = torch.zeros(n_top + n_rand, dtype=torch.int32, device="cuda")
            ctx.select(torch.from_numpy(score).cuda(), torch.from_numpy(rnd.astype(np.int32)).cuda(),
                       n_top, n_rand, out)
            torch.cuda.synchronize()
            ref = oracle.select_subset(score, rnd, 0.05, 0.01)
            assert out.cpu().numpy().tolist() == ref.tolist(), c_i


def test_add_feature(env):
    """Score / target offset by one feature column, both signs, ragged
    length, with and without shrinking the existing values."""
    torch, ctx = env["torch"], env["ctx"]
    rng = np.random.default_rng(9)
    for n in (1, 255, 1000):
        feat = rng.normal(size=(n, 16)).astype(np.float32)
        v0 = rng.normal(size=n).astype(np.float32)
        for col, sign, scale in ((10, 1, 1.0), (3, -1, 1.0), (10, 1, 0.375), (10, 1, 0.0)):
            v = torch.from_numpy(v0.copy()).cuda()
            ctx.add_feature(v, torch.from_numpy(feat).cuda(), col, sign, scale)
            torch.cuda.synchronize()
            expect = np.float32(scale) * v0 + np.float32(sign) * feat[:, col]
            assert np.array_equal(v.cpu().numpy(), expect)

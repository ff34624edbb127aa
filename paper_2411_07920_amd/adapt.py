"""ADAPT-VQE and classical pre-optimization drivers on the SWCS library.

The ADAPT loop follows Sec. II.C (Fig. 1): with the integrals (step 1), the
pool (step 2) and the reference (step 3) set on a context, each iteration
computes the pool gradient (step 4), stops when its norm is below the
threshold (step 5), appends the operator of largest |g| with parameter 0 at
the end of the ansatz (step 6) and re-optimizes the parameters (step 7).
The state is pruned after every unitary by the context's rule (eps or N_CUT).

VQE optimizers (Sec. II.B uses BFGS; Sec. IV.D proposes BFGS-2 / BFGS-2F):
  "bfgs"   scipy BFGS over all parameters
  "lbfgs"  scipy L-BFGS-B over all parameters
  "bfgs2"  (1) optimize only the new parameter from 0, others frozen,
           (2) BFGS over all parameters
  "bfgs2f" step (1) only
The gradient tolerance is the paper's convergence threshold of 1e-6.  When
the state is pruned, a newly appended parameter is first moved off the
zero-slope plateau at 0 by a five-point trigonometric fit (see
seed_last_parameter).

With a screener, the pool gradient of step 4 is evaluated exactly only for
the operators the learned network ranks highest (top 5 %) plus a random 1 %,
with the full pool every `full_every` iterations and in the first
`warm_full` iterations; `shadow_full` additionally evaluates the full pool
(untimed) to measure whether the selected operator matches.
"""
from __future__ import annotations

import dataclasses
import json
import os
import time

import numpy as np
import scipy.optimize


@dataclasses.dataclass
class AdaptConfig:
    eps: float = 0.0
    ncut: int = 0
    max_iter: int = 50
    grad_tol: float | None = 1e-2      # stop when ||g||_2 < grad_tol (None: run max_iter)
    optimizer: str = "lbfgs"
    vqe_gtol: float = 1e-6
    vqe_maxiter: int = 200
    screener: bool = False
    frac_top: float = 0.05
    frac_rand: float = 0.01
    full_every: int = 10
    warm_full: int = 3
    shadow_full: bool = False
    seed: int = 3000
    train_steps: int = 30


class Energy:
    """E(theta) and dE/dtheta of a fixed operator list on a context.  A call
    at exactly the angles of the previous call returns its result without
    touching the context, whose current state is then still the one at
    those angles (optimizer callbacks re-query the accepted point)."""

    def __init__(self, ctx, ops, eps, ncut):
        self.ctx, self.ops, self.eps, self.ncut = ctx, np.asarray(ops, dtype=np.int32), eps, ncut
        self.evals = 0
        self.time = 0.0
        self._last = None

    def __call__(self, theta):
        theta = np.array(theta, dtype=np.float64)
        if self._last is not None and np.array_equal(theta, self._last[0]):
            return self._last[1], self._last[2].copy()
        t = time.perf_counter()
        self.ctx.apply_ansatz(self.ops, theta, self.eps, self.ncut)
        dE, E = self.ctx.param_gradients(len(self.ops))
        self.evals += 1
        self.time += time.perf_counter() - t
        self._last = (theta, E, np.array(dE))
        return E, dE


class EnergyOnly:
    """E(theta) without gradients (one apply + one sigma)."""

    def __init__(self, ctx, ops, eps, ncut):
        self.ctx, self.ops, self.eps, self.ncut = ctx, np.asarray(ops, dtype=np.int32), eps, ncut
        self.evals = 0

    def __call__(self, theta):
        self.ctx.apply_ansatz(self.ops, np.asarray(theta, dtype=np.float64), self.eps, self.ncut)
        self.evals += 1
        return self.ctx.energy()[0]


_FIT_T = np.array([-2.0, -1.0, 0.0, 1.0, 2.0]) * (np.pi / 5.0)


def seed_last_parameter(ctx, ops, theta, cfg: AdaptConfig):
    """Starting value for a newly appended parameter.

    Without pruning, E as a function of one parameter is a trigonometric
    polynomial with frequencies 0, 1 and 2 (A has eigenvalues 0 and +-i), so
    five samples fix it.  With pruning, a parameter at exactly 0 sits on a
    plateau (the partners it creates are dropped for small angles), where
    the pruned energy has zero slope; the fitted polynomial, minimized on a
    grid, gives a starting point off that plateau.  Returns (theta, evals)."""
    f = EnergyOnly(ctx, ops, cfg.eps, cfg.ncut)
    base = np.array(theta, dtype=np.float64)
    Es = []
    for t in _FIT_T:
        th = base.copy()
        th[-1] = t
        Es.append(f(th))
    X = np.stack([np.ones(5), np.cos(_FIT_T), np.sin(_FIT_T), np.cos(2 * _FIT_T),
                  np.sin(2 * _FIT_T)], axis=1)
    a = np.linalg.solve(X, np.array(Es))
    grid = np.linspace(-np.pi, np.pi, 4097)
    model = a[0] + a[1] * np.cos(grid) + a[2] * np.sin(grid) + a[3] * np.cos(2 * grid) + \
        a[4] * np.sin(2 * grid)
    out = base.copy()
    out[-1] = float(grid[int(np.argmin(model))])
    return out, f.evals


def optimize(ctx, ops, theta0, cfg: AdaptConfig, method=None, seed_new=False):
    """VQE step: returns (theta, E, n_evals, seconds).  With seed_new, the
    last parameter is first set by seed_last_parameter (used after ADAPT
    appends an operator at 0 while the state is pruned)."""
    method = method or cfg.optimizer
    f = Energy(ctx, ops, cfg.eps, cfg.ncut)
    theta = np.array(theta0, dtype=np.float64)
    if len(theta) == 0:
        E, _ = f(theta)
        return theta, E, f.evals, f.time
    extra = 0
    if seed_new:
        theta, extra = seed_last_parameter(ctx, ops, theta, cfg)
    if method in ("bfgs2", "bfgs2f"):
        base = theta.copy()

        def one(x):
            th = base.copy()
            th[-1] = x[0]
            E, dE = f(th)
            return E, dE[-1:]

        r = scipy.optimize.minimize(one, theta[-1:], jac=True, method="BFGS",
                                    options={"gtol": cfg.vqe_gtol, "maxiter": cfg.vqe_maxiter})
        theta[-1] = r.x[0]
        if method == "bfgs2f":
            E, _ = f(theta)
            return theta, E, f.evals + extra, f.time
        method = "bfgs"
    if method == "bfgs":
        r = scipy.optimize.minimize(f, theta, jac=True, method="BFGS",
                                    options={"gtol": cfg.vqe_gtol, "maxiter": cfg.vqe_maxiter})
    elif method == "lbfgs":
        # ftol ~ 0 so that the gradient tolerance decides convergence
        r = scipy.optimize.minimize(f, theta, jac=True, method="L-BFGS-B",
                                    options={"gtol": cfg.vqe_gtol, "ftol": 1e-15,
                                             "maxiter": cfg.vqe_maxiter})
    else:
        raise ValueError(f"unknown optimizer {method}")
    theta = np.array(r.x)
    E, _ = f(theta)  # leave the context at the optimum
    return theta, E, f.evals + extra, f.time


def select_operator(g, idx, rel_tol=1e-9):
    """Position of the operator to append: largest |g|, where values within
    rel_tol * max|g| of the maximum count as ties (spin-symmetric pairs are
    exactly degenerate and differ only by rounding) and ties go to the
    smallest pool index."""
    a = np.abs(np.asarray(g, dtype=np.float64))
    top = a.max()
    cand = np.flatnonzero(a >= top - rel_tol * max(top, 1e-300))
    return int(cand[np.argmin(np.asarray(idx)[cand])])


def save_checkpoint(path, it_next, ops, theta, history, last_absg, scr, finished):
    """Write the state of an ADAPT run after an iteration: ansatz, parameters,
    history, the stale-ranking record and the screener (arrays in an .npz,
    scalars as JSON; nothing pickled).  Written to a temporary file and
    renamed, so an interrupted write leaves the previous checkpoint."""
    arrays = {"ops": np.asarray(ops, dtype=np.int32), "theta": np.asarray(theta, dtype=np.float64)}
    if last_absg is not None:
        arrays["last_absg"] = last_absg
    meta = {"it_next": it_next, "history": history, "finished": finished, "screener": None}
    if scr is not None:
        sa, ss = scr.state()
        arrays.update({"scr_" + k: v for k, v in sa.items()})
        meta["screener"] = ss
    arrays["meta_json"] = np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8)
    tmp = path + ".tmp.npz"
    np.savez(tmp, **arrays)
    os.replace(tmp, path)


def load_checkpoint(path):
    with np.load(path, allow_pickle=False) as z:
        arrays = {k: z[k] for k in z.files}
    meta = json.loads(arrays.pop("meta_json").tobytes().decode())
    return arrays, meta


def run_adapt(ctx, K: int, cfg: AdaptConfig, ops0=None, theta0=None, log=None, checkpoint=None,
              time_limit=None):
    """ADAPT-VQE; returns (ops, theta, history).  `ctx` has integrals, pool
    (K operators) and reference set.  ops0 / theta0 seed the ansatz (bootstrap
    restarts reuse a previous final ansatz).

    checkpoint: path of an .npz file written after every iteration; if it
    exists when the run starts, the run continues from it (operators,
    parameters, history, screener weights, Adam moments, replay buffer and
    random generator state) up to cfg.max_iter iterations in all, so a long
    run can proceed in segments; a run that converged is not continued.
    time_limit: seconds after which the run stops at the end of an iteration
    (the checkpoint then holds everything needed to continue)."""
    from .screener import Screener

    ops = list(ops0) if ops0 is not None else []
    theta = np.array(theta0 if theta0 is not None else [], dtype=np.float64)
    scr = Screener(ctx, K, cfg.seed, cfg.frac_top, cfg.frac_rand,
                   train_steps=cfg.train_steps) if cfg.screener else None
    history = []
    # last exact |g| of every operator (the information a stale-ranking
    # heuristic would select with; shadow runs only)
    last_absg = np.zeros(K) if cfg.shadow_full else None
    it0 = 0
    if checkpoint is not None and os.path.exists(checkpoint):
        arrays, meta = load_checkpoint(checkpoint)
        ops = arrays["ops"].astype(np.int64).tolist()
        theta = arrays["theta"].astype(np.float64)
        history = meta["history"]
        it0 = int(meta["it_next"])
        if last_absg is not None and "last_absg" in arrays:
            last_absg = arrays["last_absg"].astype(np.float64)
        if scr is not None and meta["screener"] is not None:
            scr.load_state({k[4:]: v for k, v in arrays.items() if k.startswith("scr_")}, meta["screener"])
        if meta["finished"]:
            return np.array(ops, dtype=np.int32), theta, history
    t_start = time.perf_counter()
    for it in range(it0, cfg.max_iter):
        if time_limit is not None and it > it0 and time.perf_counter() - t_start > time_limit:
            break
        rec = {"iter": it}
        t0 = time.perf_counter()
        n_det = ctx.apply_ansatz(np.array(ops, dtype=np.int32), theta, cfg.eps, cfg.ncut)
        E_cur, _, _ = ctx.energy()
        t1 = time.perf_counter()
        full = (scr is None) or it < cfg.warm_full or (it % cfg.full_every == 0)
        if full:
            g = ctx.pool_gradients()
            idx = np.arange(K, dtype=np.int32)
            gsel = g
            rec_idx, rec_g = idx, gsel
            if scr is not None:
                scr.compute_features(ops)
        else:
            scr.compute_features(ops)
            scr.scores()
            idx_d = scr.select()
            g_d = scr.exact_gradients(idx_d)
            idx = idx_d.cpu().numpy()
            gsel = g_d.cpu().numpy()
            rec_idx, rec_g = idx_d, g_d
        t2 = time.perf_counter()
        # sizing of the pass (keys, table slots, key-hash batches, repeats)
        # when the context reports it
        if hasattr(ctx, "pool_stats"):
            rec["pool_stats"] = ctx.pool_stats()
        kpos = select_operator(gsel, idx)
        kstar = int(idx[kpos])
        gnorm = float(np.linalg.norm(gsel))
        rec.update(E=E_cur, n_det=int(n_det), full=full, kstar=kstar, gmax=float(abs(gsel[kpos])),
                   gnorm=gnorm, n_exact=int(len(idx)), t_state=t1 - t0, t_pool=t2 - t1)
        if scr is not None:
            scr.record(rec_idx, rec_g)
            t3 = time.perf_counter()
            rec["loss"] = scr.train()
            rec["t_train"] = time.perf_counter() - t3
            rec["lam"] = scr.lam
        if cfg.shadow_full and not full:
            g_all = ctx.pool_gradients()
            ks = int(select_operator(g_all, np.arange(K)))
            rec["shadow_kstar"] = ks
            rec["shadow_match"] = bool(ks == kstar)
            rec["shadow_gnorm"] = float(np.linalg.norm(g_all))
            # baselines with the same number of exact gradients: a random
            # subset, and the operators with the largest last exact |g|
            budget = len(idx)
            rnd = np.random.default_rng((cfg.seed, it)).choice(K, budget, replace=False)
            stale = np.argsort(-last_absg, kind="stable")[:budget]
            rec["random_hit"] = bool(np.any(rnd == ks))
            rec["stale_hit"] = bool(np.any(stale == ks))
        if last_absg is not None:
            last_absg[np.asarray(idx)] = np.abs(np.asarray(gsel))
        if cfg.grad_tol is not None and full and gnorm < cfg.grad_tol:
            rec["converged"] = True
            history.append(rec)
            if log:
                log(rec)
            if checkpoint is not None:
                save_checkpoint(checkpoint, it + 1, ops, theta, history, last_absg, scr, True)
            break
        ops.append(kstar)
        theta = np.append(theta, 0.0)
        t4 = time.perf_counter()
        pruned = cfg.eps > 0.0 or cfg.ncut > 0
        theta, E_new, nev, _ = optimize(ctx, ops, theta, cfg, seed_new=pruned)
        rec.update(E_after=E_new, vqe_evals=nev, t_vqe=time.perf_counter() - t4,
                   n_params=len(ops), t_iter=time.perf_counter() - t0)
        history.append(rec)
        if log:
            log(rec)
        if checkpoint is not None:
            save_checkpoint(checkpoint, it + 1, ops, theta, history, last_absg, scr, False)
    return np.array(ops, dtype=np.int32), theta, history


def preoptimize(ctx, ops, theta0, cfg: AdaptConfig, log=None):
    """Classical pre-optimization of a fixed ansatz (L-BFGS by default),
    recording the energy after every optimizer step."""
    f = Energy(ctx, ops, cfg.eps, cfg.ncut)
    trace = []

    def cb(xk):
        E, _ = f(xk)
        trace.append(E)
        if log:
            log({"step": len(trace), "E": E})

    method = "L-BFGS-B" if cfg.optimizer == "lbfgs" else "BFGS"
    opts = {"gtol": cfg.vqe_gtol, "maxiter": cfg.vqe_maxiter}
    if method == "L-BFGS-B":
        opts["ftol"] = 1e-15
    r = scipy.optimize.minimize(f, np.asarray(theta0, dtype=np.float64), jac=True, method=method,
                                callback=cb, options=opts)
    E, _ = f(r.x)
    return np.array(r.x), E, trace, f.evals

"""Benchmark of the SWCS hot path on one MI355X.

One step = one pass of the whole hot path over the synthetic 52-spin-orbital
workload (26 spatial orbitals, 16 electrons, (pq|rs) of rank 26, 300-gate
ansatz with theta ~ U(-0.05, 0.05), eps = 1e-8, generalized singles and
doubles pool of 301,600 operators; --workload picks another):

  1. apply the ansatz from the reference with pruning (300 gates),
  2. energy through the projected sigma vector,
  3. exact pool gradients of the full pool (external sigma + contraction),
  4. adjoint parameter gradients (sqrt(M) checkpoints, recompute, reverse),
  5. learned screener: features, MLP scores for the pool, top 5 % + 1 %
     random selection, exact gradients of the selection and one training
     step (forward, MSE, backward, Adam) on them.

Prints one JSON line.  `value` is determinant-excitation applies per second
over the whole step: the number of (determinant, gate) applications the step
performs (forward gates, adjoint recompute gates and reverse gates, each
counted by the kept determinants entering the gate) divided by the step time.
The same step on the 28-spin-orbital workload and the HBM-path kernels on a
16M-determinant synthetic state are reported beside it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2411_07920_amd.inputs import (CONFIGS, array_digest, draw_ansatz,  # noqa: E402
                                         draw_random_keys, enumerate_pool, make_integrals,
                                         reference_key)

HBM_PEAK_GBS = 8000.0


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c5", choices=sorted(CONFIGS))
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 28-spin-orbital step and the large-state kernels")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-times", dest="kernel_times", action="store_false",
                    help="skip the per-kernel HIP-event passes")
    ap.add_argument("--profile-phase", default=None,
                    help="run only this phase in a loop (for counter collection)")
    ap.add_argument("--adapt", default=None, choices=sorted(CONFIGS),
                    help="instead of the step benchmark: ADAPT iteration time, screened vs "
                         "full pool, on this workload (prints its own JSON line)")
    ap.add_argument("--iters", type=int, default=150)
    ap.add_argument("--adapt-segment", default=None, choices=sorted(CONFIGS),
                    help="instead of the step benchmark: one screened ADAPT run on this workload "
                         "that continues from --checkpoint if it exists, writes it after every "
                         "iteration and stops after --time-limit seconds (a long run in segments)")
    ap.add_argument("--checkpoint", default=None, help="checkpoint file of --adapt-segment")
    ap.add_argument("--time-limit", type=float, default=None, help="seconds per --adapt-segment run")
    ap.add_argument("--large-state", type=int, default=16_000_000,
                    help="determinants of the synthetic state for the HBM-path gate and sigma "
                         "measurement added to the step line (0 = skip)")
    ap.add_argument("--huge-state", type=int, default=100_000_000,
                    help="determinants of a second synthetic state for the gate alone, added to the "
                         "step line (0 = skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 1 GiB device buffer five times (reference kernel for the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--uccsd", default=None, choices=sorted(CONFIGS),
                    help="instead of the step benchmark: MP2-ordered UCCSD on this workload "
                         "(ansatz build, energy + adjoint gradient evaluation, L-BFGS steps)")
    ap.add_argument("--spin", action="store_true",
                    help="with --uccsd: spin-complemented generators (one angle per complement pair)")
    ap.add_argument("--eps", type=float, default=None,
                    help="pruning threshold for --uccsd (default: the workload's)")
    ap.add_argument("--vqe-iters", type=int, default=20,
                    help="L-BFGS iterations for --uccsd")
    ap.add_argument("--preopt", default=None, choices=sorted(CONFIGS),
                    help="instead of the step benchmark: classical pre-optimization (L-BFGS with "
                         "adjoint gradients) of this workload's fixed ansatz at its eps and at "
                         "--ref-eps")
    ap.add_argument("--ref-eps", type=float, default=1e-8,
                    help="reference pruning threshold for --preopt")
    ap.add_argument("--micro", type=int, default=0,
                    help="instead of the step benchmark: gate and sigma kernels on a synthetic "
                         "state of this many determinants (52 spin-orbitals, 16 electrons)")
    return ap.parse_args()


class Workload:
    def __init__(self, name):
        c = CONFIGS[name]
        self.c = c
        self.h, self.eri = make_integrals(c.n, c.rank, c.seed_int)
        self.pool = enumerate_pool(c.n)
        self.ops, self.theta = draw_ansatz(len(self.pool), c.n_ops, c.theta_lo, c.theta_hi,
                                           c.seed_ansatz)
        self.ref = reference_key(c.n_elec)
        self.na = c.n_elec // 2
        self.K = len(self.pool)
        self.n_top = int(math.ceil(0.05 * self.K))
        self.n_rand = int(math.ceil(0.01 * self.K))
        self.rand = draw_random_keys(self.K, 3000 + int(name[1:]))
        self.digest = array_digest(self.h, self.eri, self.pool, self.ops, self.theta)


def applies_in_step(n_in, seg, lds):
    """(forward, adjoint) determinant-gate applications of one step: the
    forward chain, then the adjoint's recomputation (every gate of a segment
    is replayed from its checkpoint on the HBM path; the single-workgroup path
    stops a segment's replay before its last gate) and its reverse sweep."""
    M = len(n_in)
    fwd = int(n_in.sum())
    recompute = 0
    for g in range(M):
        seg_lo = (g // seg) * seg
        seg_hi = min(M, seg_lo + seg)
        if not lds or g < seg_hi - 1:
            recompute += int(n_in[g])
    return fwd, recompute + fwd


def gpu_bench(args, wl):
    import torch
    from paper_2411_07920_amd import swcs

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ctx = swcs.make_context(wl.c.n, wl.na, wl.na, wl.h, wl.eri, wl.pool, wl.ref, stream=stream)
    dev = "cuda"
    K = wl.K
    P = swcs.mlp_param_count()
    rng = np.random.default_rng(3000)
    w0 = np.zeros(P, dtype=np.float32)
    # He-normal initial weights (the values do not change the work done)
    w0[: 16 * 128] = rng.normal(0, math.sqrt(2 / 16), 16 * 128)
    off = 16 * 128 + 128
    w0[off: off + 128 * 128] = rng.normal(0, math.sqrt(2 / 128), 128 * 128)
    off += 128 * 128 + 128
    w0[off: off + 128] = rng.normal(0, math.sqrt(2 / 128), 128)
    W = torch.from_numpy(w0).to(dev)
    Mt = torch.zeros(P, device=dev)
    Vt = torch.zeros(P, device=dev)
    dW = torch.zeros(P, device=dev)
    prev = torch.zeros(K, device=dev)
    age = torch.zeros(K, device=dev)
    count = torch.zeros(K, device=dev)
    feat = torch.zeros((K, 16), device=dev)
    score = torch.zeros(K, device=dev)
    rnd = torch.from_numpy(wl.rand.astype(np.int32)).to(dev)
    nsel = wl.n_top + wl.n_rand
    sel = torch.zeros(nsel, dtype=torch.int32, device=dev)
    gsel = torch.zeros(nsel, dtype=torch.float64, device=dev)
    xs = torch.zeros((nsel, 16), device=dev)
    ys = torch.zeros(nsel, device=dev)
    act = torch.zeros((nsel, 256), device=dev)
    tgt = torch.zeros(nsel, device=dev)
    dy = torch.zeros(nsel, device=dev)
    loss = torch.zeros(1, device=dev)
    M = len(wl.ops)
    state = {"adam": 0}

    def phase_apply():
        return ctx.apply_ansatz(wl.ops, wl.theta, wl.c.eps)

    def phase_energy():
        return ctx.energy()

    def phase_pool():
        return ctx.pool_gradients()

    def phase_adjoint():
        return ctx.param_gradients(M)

    def phase_screener():
        ctx.features(prev, age, count, feat)
        ctx.mlp_forward(W, feat, score)
        ctx.add_feature(score, feat, 10, +1)  # score = log10 last |g| + network
        ctx.select(score, rnd, wl.n_top, wl.n_rand, sel)
        # exact gradients of the selection and the network's residual targets
        # log10(|g| + 1e-12) - feature 10, stream-ordered on the device
        ctx.pool_gradients_device(sel, gsel)
        ctx.log_abs(gsel, tgt)
        torch.index_select(feat, 0, sel.long(), out=xs)
        ctx.add_feature(tgt, xs, 10, -1)
        ctx.mlp_forward(W, xs, ys, act)
        ctx.mse(ys, tgt, dy, loss)
        ctx.mlp_backward(W, xs, act, dy, dW)
        state["adam"] += 1
        ctx.adam_step(W, Mt, Vt, dW, 1e-3, 0.9, 0.999, 1e-8, state["adam"])

    phases = [("apply", phase_apply), ("energy", phase_energy), ("pool_gradients", phase_pool),
              ("adjoint", phase_adjoint), ("screener", phase_screener)]

    if args.profile_phase:
        fn = dict(phases)[args.profile_phase]
        phase_apply()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        print(json.dumps({"profile_phase": args.profile_phase, "steps": args.steps}))
        return None

    def step(events=None):
        for i, (name, fn) in enumerate(phases):
            if events is not None:
                events[i][0].record(stream)
            fn()
            if events is not None:
                events[i][1].record(stream)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        progress(f"{wl.c.name}: warm-up step {i + 1} done")
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in phases] for _ in range(args.steps)]
    torch.cuda.synchronize()
    retries0 = torch.cuda.memory_stats().get("num_alloc_retries", 0)
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(ev[s])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # cache flushes of the caching allocator (each frees and synchronizes)
    alloc_retries = torch.cuda.memory_stats().get("num_alloc_retries", 0) - retries0
    ms_step = (t1 - t0) * 1e3 / args.steps
    progress(f"{wl.c.name}: {args.steps} timed steps, {ms_step:.2f} ms per step")
    phase_ms = {name: float(np.mean([ev[s][i][0].elapsed_time(ev[s][i][1]) for s in range(args.steps)]))
                for i, (name, _) in enumerate(phases)}
    phase_max_ms = {name: float(np.max([ev[s][i][0].elapsed_time(ev[s][i][1]) for s in range(args.steps)]))
                    for i, (name, _) in enumerate(phases)}

    # Work counts of one step.
    n_det = phase_apply()
    n_in = ctx.gate_sizes(M)
    stored, alive = ctx.state_counts()
    phase_pool()
    pool_table = ctx.pool_stats()
    seg = max(1, int(math.ceil(math.sqrt(M))))
    fwd_applies, adj_applies = applies_in_step(n_in, seg, int(n_in.max(initial=1)) <= 4096)
    applies = fwd_applies + adj_applies

    # Per-kernel GPU time of one step: the library records HIP events on the
    # context stream around every launch of the selected kernel.
    kern = {}
    reps = 3
    for kname in ("chain_lds", "gate", "adjoint_lds", "adjoint_replay_lds", "gate_replay", "adjoint_rec", "sigma_proj",
                  "holepair", "sigma_push", "sigma_push_into", "pool_contract", "contract_ops", "select",
                  "join_emit", "join_sort", "join_reduce", "join_terms"):
        if not args.kernel_times:
            break
        ctx.timer_start(kname)
        for _ in range(reps):
            step()
        launches, total = ctx.timer_stop()
        progress(f"{wl.c.name}: kernel times of {kname}")
        if launches:
            kern[kname] = {"launches_per_step": launches / reps, "ms_per_step": total / reps,
                           "us_per_launch": 1e3 * total / launches}
    ctx.close()
    return dict(ms_step=ms_step, phase_ms=phase_ms, phase_max_ms=phase_max_ms, alloc_retries=alloc_retries,
                n_det=n_det, n_in=n_in, applies=applies,
                fwd_applies=fwd_applies, adj_applies=adj_applies, kernels=kern, seg=seg,
                stored=stored, pool_table=pool_table)


def algorithmic_bytes(kname, wl, r):
    """Lower-bound bytes the method must move per launch of a kernel: 8 B per
    stored determinant scanned by a gate (the key test; also per determinant
    and gate for the LDS adjoint's replay and reverse sweeps); 16 B per (source,
    connection) read-modify-write of the external sigma table; 8 B per probe
    of a hash table and 16 B per source determinant read; for the selection,
    a score and a random key per operator in and the chosen indices out.
    Whole-pool gradients by sort and join: 8 B per (source, connection)
    record written (plus 16 B per source read) by the emit; 16 B per record
    and radix pass (read and written once) by the sort; 8 B per record read
    and 8 B per gradient update by the join; the binned gradient terms (8 B
    value and 2 B operator index per pair record) read once by their sum."""
    from paper_2411_07920_amd.inputs import sector_size  # noqa: F401
    n_in = r["n_in"]
    M = len(n_in)
    n = r["n_det"]
    na = wl.na
    from math import comb
    nv = wl.c.n - na
    C = 2 * na * nv + 2 * comb(na, 2) * comb(nv, 2) + na * na * nv * nv
    if kname in ("chain_lds",):
        return 8.0 * n_in.sum()                      # whole chain per launch
    if kname in ("gate", "gate_replay", "adjoint_rec"):
        return 8.0 * n_in.sum() / M                  # one gate per launch
    if kname in ("adjoint_lds", "adjoint_replay_lds"):
        return 8.0 * n_in.sum()                      # reverse sweep / all segment replays
    if kname == "sigma_proj":
        return n * (C * 8.0 + 16.0)
    if kname in ("sigma_push", "sigma_push_into"):
        return n * ((C + 1) * 16.0 + 16.0)
    if kname == "pool_contract":
        return n * (C * 8.0 + 16.0)
    if kname == "contract_ops":
        return n * 16.0 + wl.n_top * 0.0
    if kname == "join_terms":
        return n * C * 10.0
    if kname in ("join_emit", "join_sort", "join_reduce"):
        R = n * (C + 1)
        if kname == "join_emit":
            return R * 8.0 + n * 16.0
        if kname == "join_sort":
            kb = 8
            while kb < 24 and (R >> kb) > 256:
                kb += 8
            return R * 16.0 * (kb // 8)
        return R * 8.0 + n * C * 8.0
    if kname == "select":
        return wl.K * 8.0 + (wl.n_top + wl.n_rand) * 4.0  # scores and random keys in, indices out
    return 0.0


def cpu_baseline(wl, fwd_applies, adj_applies):
    """The oracle timed on the host on a bounded sample of one step, scaled
    to the whole step.  The forward chain runs in full.  The other parts are
    timed on samples of the final state and scaled by its size: sigma_P rows
    (energy), the external sigma of sampled source determinants and the
    generator applications of sampled operators (pool gradients, full pool
    plus the screener's 6 % subset); the adjoint is the oracle's forward
    states, one sigma_P and a reverse sweep of one more chain."""
    import oracle
    orc = oracle.Oracle(wl.c.n, wl.na, wl.na, wl.h, wl.eri)
    t = time.perf_counter()
    st = oracle.Oracle.apply_ansatz(wl.pool, wl.ops, wl.theta, wl.c.eps, wl.ref)
    t_apply = time.perf_counter() - t
    keys, amps = st.export()
    n = len(keys)
    rng = np.random.default_rng(0)
    rows = rng.choice(n, min(n, 1000), replace=False)
    t = time.perf_counter()
    orc.sigma_at(st, keys[rows])
    t_energy = (time.perf_counter() - t) * n / len(rows)
    # pool gradients: external sigma of n_src sources (one operator), then
    # the same plus n_ops more operators, whose difference is the generator
    # applications of n_ops operators over the n_src determinants
    src = np.sort(rng.choice(n, min(n, 100), replace=False))
    sub = oracle.OracleState.from_arrays(keys[src], amps[src])
    n_ops = min(wl.K, 3000)
    ops_s = np.sort(rng.choice(wl.K, n_ops + 1, replace=False)).astype(np.int32)
    t = time.perf_counter()
    orc.pool_gradients(sub, wl.pool, subset=ops_s[:1])
    t_ext = time.perf_counter() - t
    t = time.perf_counter()
    orc.pool_gradients(sub, wl.pool, subset=ops_s)
    t_both = time.perf_counter() - t
    t_gen = max(t_both - t_ext, 0.0) / n_ops          # one operator over len(src) determinants
    frac = 1.0 + (wl.n_top + wl.n_rand) / wl.K
    t_pool = t_ext * n / len(src) + frac * t_gen * wl.K * n / len(src)
    t_adj = 2.0 * t_apply + t_energy
    t_step = t_apply + t_energy + t_pool + t_adj
    return {
        "value": (fwd_applies + adj_applies) / t_step,
        "unit": "determinant-excitation applies/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"one step of the same workload ({n} determinants): forward chain in full "
                   f"({t_apply:.2f} s); energy from {len(rows)} sigma_P rows; pool gradients from the "
                   f"external sigma of {len(src)} sources and {n_ops} operators' generator "
                   f"applications over them; adjoint as two chains plus one sigma_P; every part "
                   f"scaled to the full state and pool; estimated step {t_step:.1f} s"),
    }


def adapt_bench(args):
    """ADAPT-VQE from the reference: full-pool arm, screened arm (both timed)
    and a screened validation arm that also evaluates the full pool on every
    iteration (untimed) to measure selection agreement and two baselines at
    the same exact-gradient budget: the fraction of screened iterations whose
    full-pool choice lies in a random subset, or among the operators with the
    largest last exact |g| (the choice a stale ranking would find)."""
    import torch
    from paper_2411_07920_amd import adapt, swcs

    torch.cuda.set_device(0)
    wl = Workload(args.adapt)
    c = wl.c

    def fresh():
        return swcs.make_context(c.n, wl.na, wl.na, wl.h, wl.eri, wl.pool, wl.ref,
                                 stream=torch.cuda.current_stream())

    def arm(screened, shadow, iters):
        ctx = fresh()
        cfg = adapt.AdaptConfig(eps=c.eps, max_iter=iters, grad_tol=None, optimizer="lbfgs",
                                screener=screened, shadow_full=shadow, seed=3000 + int(args.adapt[1:]))
        t = time.perf_counter()
        name = "screened" + ("+shadow" if shadow else "") if screened else "full"

        def log(r):
            print(f"[adapt {name}] it={r['iter']} E={r.get('E_after', r['E']):.10f} "
                  f"k={r['kstar']} exact={r['n_exact']} pool={1e3 * r['t_pool']:.1f}ms "
                  f"vqe={1e3 * r.get('t_vqe', 0.0):.1f}ms evals={r.get('vqe_evals', 0)} n_det={r['n_det']} "
                  f"batches={r.get('pool_stats', {}).get('batches', 0)} "
                  f"passes={r.get('pool_stats', {}).get('passes', 0)}", file=sys.stderr, flush=True)

        ops, theta, hist = adapt.run_adapt(ctx, wl.K, cfg, log=log)
        wall = time.perf_counter() - t
        ctx.apply_ansatz(ops, theta, c.eps)
        E = ctx.energy()[0]
        n_det = ctx.apply_ansatz(ops, theta, c.eps)
        ctx.close()
        return ops, theta, hist, wall, E, n_det

    iters = args.iters
    arm(False, False, min(iters, 5))  # untimed warm-up: code load, clocks, first allocations
    _, _, h_full, w_full, E_full, nd_full = arm(False, False, iters)
    ops_s, _, h_scr, w_scr, E_scr, nd_scr = arm(True, False, iters)
    _, _, h_val, _, E_val, _ = arm(True, True, iters)

    def mean(h, key, pred=lambda r: True):
        v = [r[key] for r in h if key in r and pred(r)]
        return float(np.mean(v)) if v else None

    screened_iters = [r for r in h_val if not r["full"]]
    match = [r["shadow_match"] for r in screened_iters]
    out = {
        "metric": "ADAPT iteration time, screened vs full pool",
        "workload": f"{args.adapt}: {c.n_so} spin-orbitals, {c.n_elec} electrons, eps={c.eps:g}, "
                    f"pool {wl.K}, {iters} iterations, L-BFGS VQE",
        "full": {"wall_s": w_full, "iter_ms": 1e3 * w_full / iters,
                 "pool_ms": 1e3 * mean(h_full, "t_pool"), "vqe_ms": 1e3 * mean(h_full, "t_vqe"),
                 "E_final": E_full, "n_det_final": nd_full},
        "screened": {"wall_s": w_scr, "iter_ms": 1e3 * w_scr / iters,
                     "pool_ms_screened_iters": 1e3 * mean(h_scr, "t_pool", lambda r: not r["full"]),
                     "pool_ms_full_iters": 1e3 * mean(h_scr, "t_pool", lambda r: r["full"]),
                     "train_ms": 1e3 * mean(h_scr, "t_train"), "vqe_ms": 1e3 * mean(h_scr, "t_vqe"),
                     "E_final": E_scr, "n_det_final": nd_scr},
        "validation": {"screened_iterations": len(match),
                       "same_operator_frac": float(np.mean(match)) if match else None,
                       "random_subset_hit_frac": (float(np.mean([r["random_hit"] for r in screened_iters]))
                                                  if match else None),
                       "stale_top_hit_frac": (float(np.mean([r["stale_hit"] for r in screened_iters]))
                                              if match else None),
                       "E_final": E_val},
        "dE_final_screened_minus_full": E_scr - E_full,
    }
    print(json.dumps(out))


def adapt_segment(args):
    """One segment of a long screened ADAPT run (the learned screener with the
    workload's eps and L-BFGS), resumed from and saved to args.checkpoint, up
    to args.iters iterations in all; prints one JSON line for the segment."""
    import torch
    from paper_2411_07920_amd import adapt, swcs

    torch.cuda.set_device(0)
    wl = Workload(args.adapt_segment)
    c = wl.c
    ctx = swcs.make_context(c.n, wl.na, wl.na, wl.h, wl.eri, wl.pool, wl.ref,
                            stream=torch.cuda.current_stream())
    cfg = adapt.AdaptConfig(eps=c.eps, max_iter=args.iters, grad_tol=None, optimizer="lbfgs",
                            screener=True, shadow_full=False, seed=3000 + int(args.adapt_segment[1:]))
    done = []

    def log(r):
        done.append(r)
        ps = r.get("pool_stats", {})
        print(f"[adapt segment] it={r['iter']} E={r.get('E_after', r['E']):.10f} k={r['kstar']} "
              f"exact={r['n_exact']} pool={1e3 * r['t_pool']:.1f}ms vqe={1e3 * r.get('t_vqe', 0.0):.1f}ms "
              f"n_det={r['n_det']} pool_keys={ps.get('keys', 0):.3g} slots={ps.get('table_slots', 0)} "
              f"batches={ps.get('batches', 0)} passes={ps.get('passes', 0)}", file=sys.stderr, flush=True)

    t = time.perf_counter()
    ops, theta, hist = adapt.run_adapt(ctx, wl.K, cfg, log=log, checkpoint=args.checkpoint,
                                       time_limit=args.time_limit)
    wall = time.perf_counter() - t
    last = hist[-1] if hist else {}
    print(json.dumps({
        "metric": "ADAPT segment (screened)",
        "workload": f"{args.adapt_segment}: {c.n_so} spin-orbitals, {c.n_elec} electrons, eps={c.eps:g}, "
                    f"pool {wl.K}",
        "iterations_total": len(hist), "iterations_this_segment": len(done), "target": args.iters,
        "wall_s": wall, "E_last": last.get("E_after", last.get("E")), "n_det_last": last.get("n_det"),
        "ms_per_iteration_this_segment": 1e3 * wall / max(1, len(done)),
    }))
    ctx.close()


def large_state_bench(N, sigma=True):
    """Gate and sigma_P kernels on a structure-free synthetic state of N
    determinants in the 52-spin-orbital, 16-electron sector (uniform alpha and
    beta strings, log-uniform |c|): eight double-excitation gates at eps = 0
    on the HBM path, then sigma_P by hole-pair grouping (and by enumeration
    when N <= 2,000,000).  Gate bytes per gate: 8 B per input entry (the key
    test every entry needs), 16 B per entry the operator acts on (amplitude
    read and written) and 16 B per new entry (key and amplitude); the active
    count of each gate is counted by the gate kernel.  At 16M
    determinants the counter-measured HBM traffic of a gate and of one
    sigma_P call (profiles/pmc_traffic.txt) is divided by the measured times
    as well."""
    import torch
    from math import comb
    from paper_2411_07920_amd import swcs
    from paper_2411_07920_amd.inputs import draw_synthetic_state

    torch.cuda.set_device(0)
    wl = Workload("c5")
    c = wl.c
    keys, amps = draw_synthetic_state(c.n, wl.na, wl.na, N, 4005)
    ctx = swcs.make_context(c.n, wl.na, wl.na, wl.h, wl.eri, wl.pool, wl.ref,
                            stream=torch.cuda.current_stream())
    out = {"n_det": N, "workload": f"synthetic state, {N} determinants, 52 spin-orbitals, "
                                   f"16 electrons, uniform sector sample, |c| in [1e-8, 1e-2]"}
    nv = c.n - wl.na
    C = 2 * wl.na * nv + 2 * comb(wl.na, 2) * comb(nv, 2) + wl.na * wl.na * nv * nv
    ctx.set_state(keys, amps)
    for method in ("hole_pairs", "enumerate"):
        if not sigma or (method == "enumerate" and N > 2_000_000):
            continue
        ctx.set_sigma_method(method)
        ctx.energy()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        ctx.energy()
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1)
        out["sigma_" + method] = {"ms": ms, "rows_per_s": N / (ms * 1e-3), "connections_per_row": C}
        if method == "hole_pairs" and N == 16_000_000:
            tb = measured_traffic("sigma_hole_pairs", "synthetic16M")
            out["sigma_" + method]["traffic_bytes_per_call"] = tb
            if tb is not None:
                gbps = tb / (ms * 1e-3) / 1e9
                out["sigma_" + method]["traffic_GBps"] = gbps
                out["sigma_" + method]["traffic_frac_hbm"] = gbps / HBM_PEAK_GBS
    ctx.set_sigma_method("auto")
    rng = np.random.default_rng(4005)
    doubles = np.flatnonzero(wl.pool[:, 2] >= 0)
    ops = rng.choice(doubles, 8).astype(np.int32)
    theta = rng.uniform(-0.3, 0.3, len(ops))
    # The gates' active counts come from the gate kernels themselves.  A gate
    # that would overflow the capacity returns at once and is launched again
    # after the host grows the state, so time is summed per gate.
    ctx.timer_start("gate")
    n_out = ctx.apply_gates(ops, theta, 0.0)
    launches, ms = ctx.timer_stop()
    n_in = ctx.gate_sizes(len(ops)).astype(np.float64)
    n_act = ctx.gate_active(len(ops)).astype(np.float64)
    after = np.append(n_in[1:], n_out)
    n_new = np.maximum(after - n_in, 0.0)
    nbytes = float((8.0 * n_in + 16.0 * n_act + 16.0 * n_new).sum())
    us = 1e3 * ms / len(ops)
    gbps = nbytes / len(ops) / (us * 1e-6) / 1e9
    out["gate"] = {"gates": len(ops), "launches": launches, "us_per_gate": us,
                   "dets_per_s": float(n_in.sum()) / (ms * 1e-3),
                   "active_frac": float(n_act.sum() / n_in.sum()),
                   "new_per_gate": float(n_new.mean()),
                   "algorithmic_bytes_per_gate": nbytes / len(ops),
                   "achieved_GBps": gbps, "frac_hbm": gbps / HBM_PEAK_GBS,
                   "n_det_in": int(n_in[0]), "n_det_out": int(n_out)}
    if N % 1_000_000 == 0:
        tb = measured_traffic("gate", f"synthetic{N // 1_000_000}M")
        out["gate"]["traffic_bytes_per_launch"] = tb
        if tb is not None:
            gbps = tb / (us * 1e-6) / 1e9
            out["gate"]["traffic_GBps"] = gbps
            out["gate"]["traffic_frac_hbm"] = gbps / HBM_PEAK_GBS
            out["gate"]["traffic_over_algorithmic"] = tb / (nbytes / len(ops))
    ctx.close()
    return out


def preopt_bench(args):
    """Classical pre-optimization of a fixed ansatz (the workload's operators
    and starting angles): L-BFGS over all parameters with adjoint gradients
    and sqrt(M) checkpoints, at the workload's eps and at --ref-eps, up to
    --vqe-iters iterations each.  Reports the energy after every optimizer
    step, the state size and the time per energy + gradient evaluation (mean
    of three at the starting angles after one untimed), and the error of the
    eps run against the --ref-eps run: final energies, and the eps optimum
    re-evaluated at --ref-eps."""
    import torch
    from paper_2411_07920_amd import adapt, swcs

    torch.cuda.set_device(0)
    wl = Workload(args.preopt)
    c = wl.c
    ctx = swcs.make_context(c.n, wl.na, wl.na, wl.h, wl.eri, wl.pool, wl.ref,
                            stream=torch.cuda.current_stream())
    runs = {}
    for eps in (c.eps if args.eps is None else args.eps, args.ref_eps):
        n_det = ctx.apply_ansatz(wl.ops, wl.theta, eps)
        _, E0 = ctx.param_gradients(len(wl.ops))
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            ctx.apply_ansatz(wl.ops, wl.theta, eps)
            ctx.param_gradients(len(wl.ops))
        torch.cuda.synchronize()
        t_eval = (time.perf_counter() - t) / 3
        print(f"[preopt eps={eps:g}] {n_det} determinants at the starting angles, E {E0:.10f}, "
              f"{1e3 * t_eval:.1f} ms per energy + gradient", file=sys.stderr, flush=True)
        cfg = adapt.AdaptConfig(eps=eps, optimizer="lbfgs", vqe_maxiter=args.vqe_iters)

        def log(r, eps=eps):
            print(f"[preopt eps={eps:g}] L-BFGS step {r['step']}: E {r['E']:.10f}", file=sys.stderr,
                  flush=True)

        t = time.perf_counter()
        theta, E, trace, evals = adapt.preoptimize(ctx, wl.ops, wl.theta, cfg, log=log)
        wall = time.perf_counter() - t
        n_final = ctx.apply_ansatz(wl.ops, theta, eps)
        runs[eps] = {"eps": eps, "n_det_start": int(n_det), "E_start": E0, "eval_ms": 1e3 * t_eval,
                     "iterations": len(trace), "evaluations": evals, "wall_s": wall,
                     "energy_per_step": trace, "E_final": E, "n_det_final": int(n_final),
                     "theta": theta}
    e_main, e_ref = list(runs)
    ctx.apply_ansatz(wl.ops, runs[e_main]["theta"], e_ref)
    E_cross = ctx.energy()[0]
    for r in runs.values():
        r.pop("theta")
    out = {
        "metric": "classical pre-optimization: energy per L-BFGS step and time per energy + gradient",
        "workload": f"{args.preopt}: {c.n_so} spin-orbitals, {c.n_elec} electrons, {len(wl.ops)}-operator "
                    f"ansatz, theta0 in [{c.theta_lo:g}, {c.theta_hi:g}], L-BFGS with adjoint gradients",
        "runs": list(runs.values()),
        "E_final_minus_ref_run": runs[e_main]["E_final"] - runs[e_ref]["E_final"],
        "eps_optimum_at_ref_eps": E_cross,
        "eps_optimum_at_ref_eps_minus_ref_run": E_cross - runs[e_ref]["E_final"],
    }
    print(json.dumps(out))
    ctx.close()
    return out


def uccsd_bench(args):
    """MP2-ordered UCCSD (Sec. II.A) on one workload: the ansatz from the
    library's pool gradients at the reference and its Fock diagonal (doubles by
    decreasing MP2 amplitude, then singles), the time of one energy + adjoint
    gradient evaluation at the MP2 parameters (apply of the whole ansatz with
    pruning, sigma_P, reverse sweep; mean of three after one untimed), and the
    energy after each of up to --vqe-iters L-BFGS iterations."""
    import torch
    from paper_2411_07920_amd import adapt, swcs, uccsd

    torch.cuda.set_device(0)
    wl = Workload(args.uccsd)
    c = wl.c
    eps = c.eps if args.eps is None else args.eps
    ctx = swcs.make_context(c.n, wl.na, wl.na, wl.h, wl.eri, wl.pool, wl.ref,
                            stream=torch.cuda.current_stream())
    t = time.perf_counter()
    ans = uccsd.mp2_ordered_uccsd(ctx, wl.pool, wl.ref, c.n)
    t_build = time.perf_counter() - t
    print(f"[uccsd] {args.uccsd}: {len(ans.ops)} operators ({ans.n_doubles} doubles), "
          f"E_ref {ans.e_ref:.10f}, E2 {ans.e2:.10f}, build {t_build:.3f} s", file=sys.stderr, flush=True)
    n_det = ctx.apply_ansatz(ans.ops, ans.theta, eps)
    _, E0 = ctx.param_gradients(len(ans.ops))
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(3):
        ctx.apply_ansatz(ans.ops, ans.theta, eps)
        ctx.param_gradients(len(ans.ops))
    torch.cuda.synchronize()
    t_eval = (time.perf_counter() - t) / 3
    print(f"[uccsd] {n_det} determinants, E(MP2 parameters) {E0:.10f}, "
          f"{1e3 * t_eval:.1f} ms per energy + gradient", file=sys.stderr, flush=True)
    cfg = adapt.AdaptConfig(eps=eps, optimizer="lbfgs", vqe_maxiter=args.vqe_iters)

    def log(r):
        print(f"[uccsd] L-BFGS step {r['step']}: E {r['E']:.10f}", file=sys.stderr, flush=True)

    t = time.perf_counter()
    n_params = len(ans.ops)
    if args.spin:
        # one angle per spin-complemented generator
        import scipy.optimize
        from paper_2411_07920_amd import spin
        gp = spin.spin_complemented(wl.pool)
        gens, th0 = uccsd.spin_complemented_uccsd(ans, gp)
        n_params = len(gens)
        f = spin.TiedEnergy(ctx, gp, gens, eps)
        trace = []

        def cb(xk):
            trace.append(float(f(xk)[0]))
            log({"step": len(trace), "E": trace[-1]})

        r = scipy.optimize.minimize(f, th0, jac=True, method="L-BFGS-B", callback=cb,
                                    options={"gtol": 1e-6, "ftol": 1e-15, "maxiter": args.vqe_iters})
        E, evals = float(r.fun), f.evals
        n_final = ctx.apply_generators(spin.gen_rows(gp, gens), r.x, eps)
    else:
        theta, E, trace, evals = adapt.preoptimize(ctx, ans.ops, ans.theta, cfg, log=log)
        n_final = ctx.apply_ansatz(ans.ops, theta, eps)
    t_vqe = time.perf_counter() - t
    out = {
        "metric": "MP2-ordered UCCSD: energy + adjoint gradient evaluation time and VQE energies",
        "workload": f"{args.uccsd}: {c.n_so} spin-orbitals, {c.n_elec} electrons, eps={eps:g}, "
                    f"{len(ans.ops)} operators ({ans.n_doubles} doubles, {ans.n_singles} singles), "
                    f"{n_params} parameters" + (" (spin-complemented)" if args.spin else ""),
        "e_ref": ans.e_ref, "e2": ans.e2, "e_mp2": ans.e_ref + ans.e2,
        "ansatz_build_s": t_build,
        "E_mp2_parameters": E0, "n_det_mp2_parameters": int(n_det),
        "eval_ms": 1e3 * t_eval,
        "vqe": {"iterations": len(trace), "evaluations": evals, "wall_s": t_vqe,
                "energy_per_step": trace, "E_final": E, "n_det_final": int(n_final)},
    }
    print(json.dumps(out))
    ctx.close()
    return out


def micro_bench(args):
    # above 32M determinants the hole-pair records (and their sort buffer) no
    # longer fit beside the state, and enumeration would take minutes
    out = large_state_bench(args.micro, sigma=args.micro <= 32_000_000)
    out["metric"] = "kernel rates on a synthetic state"
    print(json.dumps(out))


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic.txt")
CSRC = os.path.join(ROOT, "paper_2411_07920_amd", "csrc")


def sources_digest(names):
    import hashlib
    m = hashlib.sha256()
    for name in names:
        with open(os.path.join(CSRC, name), "rb") as f:
            m.update(f.read())
    return m.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel
    calibration), or None when there is none or the kernel's sources have
    changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if line.startswith("#") or "=" not in line:
                continue
            kv = dict(tok.split("=", 1) for tok in line.split())
            if kv.get("kernel") != kernel or kv.get("workload") != workload:
                continue
            if sources_digest(kv["sources"].split(",")) != kv["sources_sha256"]:
                return None
            return float(kv["bytes_per_launch"])
    return None


def copy_calibration():
    import torch
    torch.cuda.set_device(0)
    n = 1 << 28
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 5}))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    if args.adapt:
        adapt_bench(args)
        return
    if args.adapt_segment:
        adapt_segment(args)
        return
    if args.uccsd:
        uccsd_bench(args)
        return
    if args.preopt:
        preopt_bench(args)
        return
    if args.micro:
        micro_bench(args)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    wl = Workload(args.workload)
    r = gpu_bench(args, wl)
    if r is None:
        return
    M = len(wl.ops)
    kern = r["kernels"]
    line = {
        "metric": "determinant-excitation applies/s",
        "value": r["applies"] / (r["ms_step"] * 1e-3),
        "unit": "determinant-excitation applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl.c.n_so} spin-orbitals, {wl.c.n_elec} electrons, "
                               f"{M}-gate ansatz, eps={wl.c.eps:g}, pool {wl.K}",
                   "n_det_final": r["n_det"], "n_stored_final": r["stored"],
                   "applies_per_step": r["applies"], "input_sha256": wl.digest[:16]},
        "pool_table": r["pool_table"],
        "phases_ms": {k: round(v, 4) for k, v in r["phase_ms"].items()},
        "phases_max_ms": {k: round(v, 4) for k, v in r["phase_max_ms"].items()},
        "alloc_retries": r["alloc_retries"],
    }
    if kern:
        dom = max(kern, key=lambda k: kern[k]["ms_per_step"])
        per_launch_s = kern[dom]["us_per_launch"] * 1e-6
        bytes_launch = algorithmic_bytes(dom, wl, r)
        achieved = bytes_launch / per_launch_s / 1e9
        tb = measured_traffic(dom, args.workload)
        line["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": achieved / HBM_PEAK_GBS, "traffic": tb,
                            "kernel": dom, "us_per_launch": kern[dom]["us_per_launch"],
                            "algorithmic_bytes_per_launch": bytes_launch,
                            "traffic_over_algorithmic": (tb / bytes_launch) if tb else None}
        line["kernels_ms_per_step"] = {k: round(v["ms_per_step"], 4) for k, v in kern.items()}
    if not args.no_cpu_baseline:
        progress("oracle baseline")
        line["cpu_baseline"] = cpu_baseline(wl, r["fwd_applies"], r["adj_applies"])
    if not args.no_extras and args.workload != "c2":
        a2 = argparse.Namespace(steps=20, warmup=3, profile_phase=None, kernel_times=False)
        wl2 = Workload("c2")
        r2 = gpu_bench(a2, wl2)
        line["extra_c2_step"] = {"workload": f"c2: {wl2.c.n_so} spin-orbitals, {wl2.c.n_elec} electrons, "
                                             f"{len(wl2.ops)}-gate ansatz, eps={wl2.c.eps:g}, pool {wl2.K}",
                                 "ms_per_step": r2["ms_step"],
                                 "applies_per_s": r2["applies"] / (r2["ms_step"] * 1e-3),
                                 "n_det_final": r2["n_det"],
                                 "phases_ms": {k: round(v, 4) for k, v in r2["phase_ms"].items()}}
    if args.large_state and not args.no_extras:
        progress("large state")
        line["large_state"] = large_state_bench(args.large_state)
    if args.huge_state and not args.no_extras:
        progress("huge state")
        line["huge_state_gate"] = large_state_bench(args.huge_state, sigma=False)
    print(json.dumps(line))


if __name__ == "__main__":
    main()

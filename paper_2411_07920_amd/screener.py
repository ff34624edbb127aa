"""Learned operator-pool screener driven by the library's float32 kernels.

The ADAPT step ranks the pool by the derivative of the energy with respect to
each operator appended at the end of the ansatz (Sec. II.C, step 4).  The
screener predicts log10 |g_k| from sixteen cheap per-operator features, so
that exact gradients are evaluated only for the top-scored fraction plus a
random share; the exact gradients that result are its training data (online,
Adam, mean squared error).  The prediction is feature 10 -- log10 of the
operator's last exact |g| -- plus the output of a 16 -> 128 -> 128 -> 1 ReLU
network, which therefore learns how each gradient has changed since it was
last evaluated; an untrained network ranks by the last exact gradients.  The
network output enters the score multiplied by lam in {0, 1/4, 1/2, 3/4, 1},
chosen on held-out data for the job the score does: at every full-pool
iteration, before the network is trained on it, each lam's score ranks all
operators and the number ranked above the one ADAPT selects is recorded; lam
is the value with the smallest sum of log(1 + rank) so far (ties to the
smaller).  A network that does not help find the selected operator leaves the
ranking by the last exact gradients unchanged.

All arithmetic runs in libswcs kernels (features, forward, MSE, backward,
Adam, selection); torch only holds the device buffers.
"""
from __future__ import annotations

import math

import numpy as np


class Screener:
    def __init__(self, ctx, K: int, seed: int, frac_top=0.05, frac_rand=0.01, lr=1e-3,
                 buffer_rows=65536, train_steps=30):
        import torch
        from . import swcs

        self.torch = torch
        self.ctx = ctx
        self.K = K
        self.frac_top, self.frac_rand = frac_top, frac_rand
        self.n_top = int(math.ceil(frac_top * K))
        self.n_rand = int(math.ceil(frac_rand * K))
        self.lr = lr
        self.train_steps = train_steps
        self.rng = np.random.default_rng(seed)
        P = swcs.mlp_param_count()
        w = np.zeros(P, dtype=np.float32)
        # He-normal hidden layers, zero biases and a zero output layer: the
        # untrained network adds nothing to the last exact log10 |g|
        w[: 16 * 128] = self.rng.normal(0, math.sqrt(2 / 16), 16 * 128)
        o = 16 * 128 + 128
        w[o: o + 128 * 128] = self.rng.normal(0, math.sqrt(2 / 128), 128 * 128)
        dev = "cuda"
        self.W = torch.from_numpy(w).to(dev)
        self.m = torch.zeros(P, device=dev)
        self.v = torch.zeros(P, device=dev)
        self.dW = torch.zeros(P, device=dev)
        self.adam_t = 0
        self.feat = torch.zeros((K, 16), device=dev)
        self.score = torch.zeros(K, device=dev)
        self.prev_absg = torch.zeros(K, device=dev)
        self.age = torch.zeros(K, device=dev)
        self.count = torch.zeros(K, device=dev)
        self.buf_x = torch.zeros((buffer_rows, 16), device=dev)
        self.buf_t = torch.zeros(buffer_rows, device=dev)
        self.buf_n = 0
        self.buf_pos = 0
        self.buffer_rows = buffer_rows
        self.loss = torch.zeros(1, device=dev)
        self.lam = 0.0  # weight of the network in the score (see module docstring)
        self.lam_grid = np.array([0.0, 0.25, 0.5, 0.75, 1.0])
        self.lam_cost = np.zeros(len(self.lam_grid))
        self.lam_history = []

    # -- per-iteration bookkeeping ------------------------------------------
    def compute_features(self, ansatz_ops):
        torch = self.torch
        cnt = np.bincount(np.asarray(ansatz_ops, dtype=np.int64), minlength=self.K).astype(np.float32)
        self.count.copy_(torch.from_numpy(cnt))
        self.ctx.features(self.prev_absg, self.age, self.count, self.feat)

    RESIDUAL_COL = 10  # log10 of the last exact |g|

    def scores(self):
        self.ctx.mlp_forward(self.W, self.feat, self.score)
        self.ctx.add_feature(self.score, self.feat, self.RESIDUAL_COL, +1, self.lam)
        return self.score

    def select(self):
        """Selected pool indices: (int32 device tensor, host array)."""
        torch = self.torch
        rnd = self.rng.integers(0, 2 ** 32, self.K, dtype=np.uint64).astype(np.uint32)
        rnd_d = torch.from_numpy(rnd.view(np.int32)).cuda()
        out = torch.zeros(self.n_top + self.n_rand, dtype=torch.int32, device="cuda")
        self.ctx.select(self.score, rnd_d, self.n_top, self.n_rand, out)
        return out

    def exact_gradients(self, idx_d):
        """Exact pool gradients of the selection (float64 device tensor)."""
        g = self.torch.zeros(idx_d.shape[0], dtype=self.torch.float64, device="cuda")
        self.ctx.pool_gradients_device(idx_d, g)
        return g

    def record(self, idx, g):
        """Exact gradients g for pool indices idx (features of this iteration);
        device tensors or host arrays."""
        torch = self.torch
        rows = torch.as_tensor(np.asarray(idx) if not torch.is_tensor(idx) else idx,
                               device="cuda").long()
        g_d = torch.as_tensor(np.asarray(g, dtype=np.float64) if not torch.is_tensor(g) else g,
                              device="cuda").double()
        x = self.feat.index_select(0, rows)
        t = torch.empty(len(rows), dtype=torch.float32, device="cuda")
        self.ctx.log_abs(g_d, t)
        self.ctx.add_feature(t, x, self.RESIDUAL_COL, -1)  # residual target of the network
        if len(rows) == self.K:
            self._update_lam(rows, g_d)
        n = len(rows)
        for s in range(0, n, self.buffer_rows):
            xs, ts = x[s:s + self.buffer_rows], t[s:s + self.buffer_rows]
            m = len(ts)
            end = self.buf_pos + m
            if end <= self.buffer_rows:
                self.buf_x[self.buf_pos:end] = xs
                self.buf_t[self.buf_pos:end] = ts
            else:
                first = self.buffer_rows - self.buf_pos
                self.buf_x[self.buf_pos:] = xs[:first]
                self.buf_t[self.buf_pos:] = ts[:first]
                self.buf_x[: m - first] = xs[first:]
                self.buf_t[: m - first] = ts[first:]
            self.buf_pos = end % self.buffer_rows
            self.buf_n = min(self.buffer_rows, self.buf_n + m)
        # per-operator history used by the features
        self.age += 1.0
        self.age[rows] = 0.0
        self.prev_absg[rows] = g_d.abs().float()

    def _update_lam(self, rows, g_d):
        """Held-out choice of lam at a full-pool iteration (rows = every
        operator, g_d their exact gradients), before training on it: for each
        lam on the grid, the number of operators whose score f10 + lam * y
        exceeds that of the operator of largest |g|."""
        torch = self.torch
        y = torch.zeros(self.K, device="cuda")
        self.ctx.mlp_forward(self.W, self.feat, y)
        yh = y.cpu().numpy().astype(np.float64)
        f10 = self.feat[:, self.RESIDUAL_COL].cpu().numpy().astype(np.float64)
        absg = np.zeros(self.K)
        absg[rows.cpu().numpy()] = g_d.abs().cpu().numpy()
        k = int(np.argmax(absg))
        for j, lam in enumerate(self.lam_grid):
            s = f10 + lam * yh
            self.lam_cost[j] += np.log1p(np.count_nonzero(s > s[k]))
        self.lam = float(self.lam_grid[int(np.argmin(self.lam_cost))])
        self.lam_history.append(self.lam)

    # -- checkpoint / resume ------------------------------------------------
    def state(self):
        """Everything that decides later iterations: network, Adam moments and
        step, replay buffer, per-operator history, lam bookkeeping and the
        random generator (arrays and JSON-able scalars)."""
        arrays = {
            "W": self.W.cpu().numpy(), "m": self.m.cpu().numpy(), "v": self.v.cpu().numpy(),
            "prev_absg": self.prev_absg.cpu().numpy(), "age": self.age.cpu().numpy(),
            "buf_x": self.buf_x[: self.buf_n].cpu().numpy(), "buf_t": self.buf_t[: self.buf_n].cpu().numpy(),
            "lam_cost": self.lam_cost.copy(),
        }
        scalars = {"adam_t": self.adam_t, "buf_n": self.buf_n, "buf_pos": self.buf_pos, "lam": self.lam,
                   "lam_history": list(self.lam_history), "rng": self.rng.bit_generator.state}
        return arrays, scalars

    def load_state(self, arrays, scalars):
        torch = self.torch
        for name in ("W", "m", "v", "prev_absg", "age"):
            getattr(self, name).copy_(torch.from_numpy(np.asarray(arrays[name], dtype=np.float32)))
        n = int(scalars["buf_n"])
        if n:
            self.buf_x[:n] = torch.from_numpy(np.asarray(arrays["buf_x"], dtype=np.float32))
            self.buf_t[:n] = torch.from_numpy(np.asarray(arrays["buf_t"], dtype=np.float32))
        self.buf_n, self.buf_pos = n, int(scalars["buf_pos"])
        self.adam_t = int(scalars["adam_t"])
        self.lam = float(scalars["lam"])
        self.lam_cost = np.asarray(arrays["lam_cost"], dtype=np.float64).copy()
        self.lam_history = list(scalars["lam_history"])
        self.rng.bit_generator.state = scalars["rng"]

    def train(self):
        """Full-batch Adam steps on the replay buffer; returns the last loss."""
        torch = self.torch
        B = self.buf_n
        if B == 0:
            return float("nan")
        x, t = self.buf_x[:B], self.buf_t[:B]
        y = torch.zeros(B, device="cuda")
        act = torch.zeros((B, 256), device="cuda")
        dy = torch.zeros(B, device="cuda")
        for _ in range(self.train_steps):
            self.ctx.mlp_forward(self.W, x, y, act)
            self.ctx.mse(y, t, dy, self.loss)
            self.ctx.mlp_backward(self.W, x, act, dy, self.dW)
            self.adam_t += 1
            self.ctx.adam_step(self.W, self.m, self.v, self.dW, self.lr, 0.9, 0.999, 1e-8, self.adam_t)
        return float(self.loss.item())

"""Python face of the CPU oracle (TEST INFRASTRUCTURE ONLY).

The sparse-state oracle is plain C++ (``oracle_swcs.cpp``) reached through
ctypes; the screener oracle (features, MLP forward/backward, Adam, selection)
is plain float64 numpy in this file.  Nothing here is imported by the product
path, which must fail loudly if its HIP library is missing.

Parity status (what pins each function; the pins live in ``tests/``):

==========================  ===================================================
function                    pinned by
==========================  ===================================================
hmat                        dense Jordan-Wigner H in the sector (brute force)
apply_gate / apply_ansatz   scipy expm on dense A_k; norm preservation;
                            particle-number and S_z invariants
energy                      closed-form Hartree-Fock energy; one-gate 2x2
                            closed form; variational bound vs dense FCI
sigma_projected             psi x psi double loop over hmat; dense H psi
pool_gradients              closed form at HF; FD of an appended gate; dense
                            <psi|[H, A_k]|psi>
param_gradients             central FD (eps = 0); trigonometric 5-point fit;
                            last-parameter identity; masked FD (eps > 0)
apply_ansatz with ncut      dense expm chain pruned by a full sort after every
                            gate; exact ties (theta = 0 gates) keep the
                            smaller keys for every ncut
occupations                 dense Jordan-Wigner number operators; sums equal
                            the alpha and beta electron counts
mlp_forward / mlp_backward  finite differences in float64
adam_step                   closed forms for a constant gradient and for a
                            single gradient followed by zeros (steps 1-6)
features / fock_spatial     every feature of every c1 operator against its
                            definition written out per operator, occupations
                            from the dense vector
select_subset               hand-computed case with ties
mp2_uccsd                   closed-shell spatial MP2 energy formula; first-
                            order coefficients of the dense Hamiltonian
==========================  ===================================================
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

__all__ = [
    "build", "load", "Oracle", "OracleState",
    "mlp_init", "mlp_forward", "mlp_backward", "mlp_loss_grad", "adam_step",
    "fock_spatial", "features", "select_subset", "mp2_uccsd", "N_PARAMS", "LAYOUT",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_swcs.cpp")
_LIB = os.path.join(_HERE, "liboracle_swcs.so")


def build(force: bool = True) -> str:
    """Compile the C++ oracle with g++ (no fused multiply-add contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
               "-o", _LIB + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    vp, i64, i32p = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)
    dp, u64p, u64 = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint64
    sig = {
        "orc_problem_create": (vp, [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_double]),
        "orc_problem_destroy": (None, [vp]),
        "orc_state_create": (vp, [u64p, dp, i64]),
        "orc_state_destroy": (None, [vp]),
        "orc_state_size": (i64, [vp]),
        "orc_state_export": (None, [vp, u64p, dp]),
        "orc_hmat": (ctypes.c_double, [vp, u64, u64]),
        "orc_apply_gate": (vp, [vp, i32p, ctypes.c_double, ctypes.c_double]),
        "orc_apply_gate_truncate": (vp, [vp, i32p, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, i64, dp]),
        "orc_apply_generator": (vp, [vp, i32p]),
        "orc_apply_ansatz": (vp, [i32p, i32p, dp, i64, ctypes.c_double, i64, u64, dp]),
        "orc_energy": (None, [vp, vp, dp, dp, dp]),
        "orc_sigma_projected": (None, [vp, vp, dp]),
        "orc_sigma_at": (None, [vp, vp, u64p, i64, dp]),
        "orc_pool_gradients": (None, [vp, vp, i32p, i64, i32p, i64, dp]),
        "orc_param_gradients": (None, [vp, i32p, i32p, dp, i64, ctypes.c_double, i64, u64, dp, dp]),
        "orc_energy_frozen": (ctypes.c_double, [vp, i32p, i32p, dp, dp, i64, ctypes.c_double, i64, u64]),
        "orc_forward_sizes": (None, [i32p, i32p, dp, i64, ctypes.c_double, i64, u64,
                                     ctypes.POINTER(ctypes.c_int64)]),
        "orc_occupations": (None, [vp, vp, dp]),
        "orc_apply_gen": (vp, [vp, i32p, i32p, ctypes.c_double, ctypes.c_double, i64, dp]),
        "orc_apply_gen_sum": (vp, [vp, i32p, i32p]),
        "orc_apply_gen_ansatz": (vp, [i32p, i32p, dp, i64, ctypes.c_double, i64, u64]),
        "orc_gen_param_gradients": (None, [vp, i32p, i32p, dp, i64, ctypes.c_double, i64, u64, dp, dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleState:
    """A sparse state held by the oracle (ordered map of key -> amplitude)."""

    def __init__(self, handle):
        self._h = handle
        self._lib = load()

    @classmethod
    def from_arrays(cls, keys, amps):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        amps = _f64(amps)
        lib = load()
        return cls(lib.orc_state_create(_p(keys, ctypes.c_uint64), _p(amps, ctypes.c_double), len(keys)))

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.orc_state_destroy(self._h)
            self._h = None

    def __len__(self):
        return int(self._lib.orc_state_size(self._h))

    def export(self):
        """(keys uint64, amps float64) sorted by key."""
        n = len(self)
        keys = np.zeros(n, dtype=np.uint64)
        amps = np.zeros(n, dtype=np.float64)
        self._lib.orc_state_export(self._h, _p(keys, ctypes.c_uint64), _p(amps, ctypes.c_double))
        return keys, amps

    def as_dict(self):
        k, a = self.export()
        return dict(zip(k.tolist(), a.tolist()))


class Oracle:
    """One problem (integrals + electron counts) for the oracle."""

    def __init__(self, n, n_alpha, n_beta, h, eri, ecore=0.0):
        self.n, self.n_alpha, self.n_beta = n, n_alpha, n_beta
        self._h_arr = _f64(h)
        self._eri_arr = _f64(eri)
        self._lib = load()
        self._h = self._lib.orc_problem_create(n, n_alpha, n_beta, _p(self._h_arr, ctypes.c_double),
                                               _p(self._eri_arr, ctypes.c_double), float(ecore))

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.orc_problem_destroy(self._h)
            self._h = None

    # -- matrix elements -------------------------------------------------
    def hmat(self, bra: int, ket: int) -> float:
        return float(self._lib.orc_hmat(self._h, int(bra), int(ket)))

    # -- gates and ansatz ------------------------------------------------
    @staticmethod
    def apply_gate(state: OracleState, row, c: float, sn: float) -> OracleState:
        row = _i32(row)
        return OracleState(load().orc_apply_gate(state._h, _p(row, ctypes.c_int32), c, sn))

    @staticmethod
    def apply_gate_truncate(state, row, c, sn, eps=0.0, ncut=0):
        row = _i32(row)
        d2 = ctypes.c_double(0.0)
        h = load().orc_apply_gate_truncate(state._h, _p(row, ctypes.c_int32), c, sn, eps, int(ncut),
                                           ctypes.byref(d2))
        return OracleState(h), d2.value

    @staticmethod
    def apply_generator(state, row) -> OracleState:
        row = _i32(row)
        return OracleState(load().orc_apply_generator(state._h, _p(row, ctypes.c_int32)))

    @staticmethod
    def apply_ansatz(pool, ops, theta, eps, ref, ncut=0):
        pool, ops, theta = _i32(pool), _i32(ops), _f64(theta)
        d2 = ctypes.c_double(0.0)
        h = load().orc_apply_ansatz(_p(pool, ctypes.c_int32), _p(ops, ctypes.c_int32),
                                    _p(theta, ctypes.c_double), len(ops), float(eps), int(ncut),
                                    int(ref), ctypes.byref(d2))
        st = OracleState(h)
        st.dropped_sq = d2.value
        return st

    @staticmethod
    def forward_sizes(pool, ops, theta, eps, ref, ncut=0):
        pool, ops, theta = _i32(pool), _i32(ops), _f64(theta)
        out = np.zeros(len(ops) + 1, dtype=np.int64)
        load().orc_forward_sizes(_p(pool, ctypes.c_int32), _p(ops, ctypes.c_int32),
                                 _p(theta, ctypes.c_double), len(ops), float(eps), int(ncut), int(ref),
                                 _p(out, ctypes.c_int64))
        return out

    # -- energy, sigma ---------------------------------------------------
    def energy(self, state):
        nu, no, e = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._lib.orc_energy(self._h, state._h, ctypes.byref(nu), ctypes.byref(no), ctypes.byref(e))
        return e.value, nu.value, no.value

    def sigma_projected(self, state):
        out = np.zeros(len(state))
        self._lib.orc_sigma_projected(self._h, state._h, _p(out, ctypes.c_double))
        return out

    def sigma_at(self, state, keys):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        out = np.zeros(len(keys))
        self._lib.orc_sigma_at(self._h, state._h, _p(keys, ctypes.c_uint64), len(keys),
                               _p(out, ctypes.c_double))
        return out

    # -- gradients -------------------------------------------------------
    def pool_gradients(self, state, pool, subset=None):
        pool = _i32(pool)
        if subset is None:
            out = np.zeros(len(pool))
            self._lib.orc_pool_gradients(self._h, state._h, _p(pool, ctypes.c_int32), len(pool),
                                         None, 0, _p(out, ctypes.c_double))
        else:
            subset = _i32(subset)
            out = np.zeros(len(subset))
            self._lib.orc_pool_gradients(self._h, state._h, _p(pool, ctypes.c_int32), len(pool),
                                         _p(subset, ctypes.c_int32), len(subset),
                                         _p(out, ctypes.c_double))
        return out

    def param_gradients(self, pool, ops, theta, eps, ref, ncut=0):
        pool, ops, theta = _i32(pool), _i32(ops), _f64(theta)
        out = np.zeros(len(ops))
        e = ctypes.c_double()
        self._lib.orc_param_gradients(self._h, _p(pool, ctypes.c_int32), _p(ops, ctypes.c_int32),
                                      _p(theta, ctypes.c_double), len(ops), float(eps), int(ncut),
                                      int(ref), _p(out, ctypes.c_double), ctypes.byref(e))
        return out, e.value

    def energy_frozen(self, pool, ops, theta_ref, theta_eval, eps, ref, ncut=0):
        pool, ops = _i32(pool), _i32(ops)
        tr, te = _f64(theta_ref), _f64(theta_eval)
        return float(self._lib.orc_energy_frozen(self._h, _p(pool, ctypes.c_int32),
                                                 _p(ops, ctypes.c_int32), _p(tr, ctypes.c_double),
                                                 _p(te, ctypes.c_double), len(ops), float(eps),
                                                 int(ncut), int(ref)))

    # -- spin-complemented generators (rows (k1, k2, s); k2 < 0: k1 alone) --
    @staticmethod
    def apply_gen(state, pool, gen3, theta, eps=0.0, ncut=0):
        pool, g = _i32(pool), _i32(gen3)
        d2 = ctypes.c_double(0.0)
        h = load().orc_apply_gen(state._h, _p(pool, ctypes.c_int32), _p(g, ctypes.c_int32), float(theta),
                                 float(eps), int(ncut), ctypes.byref(d2))
        return OracleState(h)

    @staticmethod
    def apply_gen_sum(state, pool, gen3):
        pool, g = _i32(pool), _i32(gen3)
        return OracleState(load().orc_apply_gen_sum(state._h, _p(pool, ctypes.c_int32),
                                                    _p(g, ctypes.c_int32)))

    @staticmethod
    def apply_gen_ansatz(pool, gens, theta, eps, ref, ncut=0):
        pool, gens, theta = _i32(pool), _i32(gens), _f64(theta)
        h = load().orc_apply_gen_ansatz(_p(pool, ctypes.c_int32), _p(gens, ctypes.c_int32),
                                        _p(theta, ctypes.c_double), len(theta), float(eps), int(ncut),
                                        int(ref))
        return OracleState(h)

    def gen_param_gradients(self, pool, gens, theta, eps, ref, ncut=0):
        pool, gens, theta = _i32(pool), _i32(gens), _f64(theta)
        out = np.zeros(len(theta))
        e = ctypes.c_double()
        self._lib.orc_gen_param_gradients(self._h, _p(pool, ctypes.c_int32), _p(gens, ctypes.c_int32),
                                          _p(theta, ctypes.c_double), len(theta), float(eps), int(ncut),
                                          int(ref), _p(out, ctypes.c_double), ctypes.byref(e))
        return out, e.value

    def occupations(self, state):
        out = np.zeros(2 * self.n)
        self._lib.orc_occupations(self._h, state._h, _p(out, ctypes.c_double))
        return out


# ---------------------------------------------------------------------------
# Screener oracle (float64 numpy).  The network is 16 -> 128 -> 128 -> 1 with
# ReLU; parameters are one flat vector laid out W1[16,128], b1[128],
# W2[128,128], b2[128], W3[128], b3[1] (row-major, input index first).
# ---------------------------------------------------------------------------
N_IN, N_H = 16, 128
LAYOUT = {
    "W1": (0, (N_IN, N_H)),
    "b1": (N_IN * N_H, (N_H,)),
    "W2": (N_IN * N_H + N_H, (N_H, N_H)),
    "b2": (N_IN * N_H + N_H + N_H * N_H, (N_H,)),
    "W3": (N_IN * N_H + 2 * N_H + N_H * N_H, (N_H,)),
    "b3": (N_IN * N_H + 3 * N_H + N_H * N_H, (1,)),
}
N_PARAMS = N_IN * N_H + 3 * N_H + N_H * N_H + 1   # 18,817


def _unpack(w):
    return {k: w[o:o + int(np.prod(s))].reshape(s) for k, (o, s) in LAYOUT.items()}


def mlp_init(seed: int) -> np.ndarray:
    """He-normal weights from a seed, zero biases (float64)."""
    rng = np.random.default_rng(seed)
    w = np.zeros(N_PARAMS)
    p = _unpack(w)
    p["W1"][...] = rng.normal(0.0, np.sqrt(2.0 / N_IN), (N_IN, N_H))
    p["W2"][...] = rng.normal(0.0, np.sqrt(2.0 / N_H), (N_H, N_H))
    p["W3"][...] = rng.normal(0.0, np.sqrt(2.0 / N_H), (N_H,))
    return w


def mlp_forward(w, x):
    """Returns (y[B], cache) with cache = (x, z1, a1, z2, a2)."""
    p = _unpack(np.asarray(w, dtype=np.float64))
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ p["W1"] + p["b1"]
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ p["W2"] + p["b2"]
    a2 = np.maximum(z2, 0.0)
    y = a2 @ p["W3"] + p["b3"][0]
    return y, (x, z1, a1, z2, a2)


def mlp_backward(w, cache, dy):
    """Gradient of sum(dy * y) with respect to the flat parameter vector."""
    p = _unpack(np.asarray(w, dtype=np.float64))
    x, z1, a1, z2, a2 = cache
    g = np.zeros(N_PARAMS)
    gp = _unpack(g)
    dy = np.asarray(dy, dtype=np.float64)
    gp["W3"][...] = a2.T @ dy
    gp["b3"][...] = dy.sum()
    da2 = np.outer(dy, p["W3"])
    dz2 = da2 * (z2 > 0)
    gp["W2"][...] = a1.T @ dz2
    gp["b2"][...] = dz2.sum(axis=0)
    da1 = dz2 @ p["W2"].T
    dz1 = da1 * (z1 > 0)
    gp["W1"][...] = x.T @ dz1
    gp["b1"][...] = dz1.sum(axis=0)
    return g


def mlp_loss_grad(w, x, target):
    """Mean squared error and its gradient."""
    y, cache = mlp_forward(w, x)
    r = y - np.asarray(target, dtype=np.float64)
    loss = float(np.mean(r * r))
    dy = 2.0 * r / len(r)
    return loss, mlp_backward(w, cache, dy)


def adam_step(w, m, v, g, lr, b1, b2, eps, step):
    """One Adam update (Kingma & Ba) with bias correction; returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def fock_spatial(h, eri, n_occ):
    """Closed-shell Fock matrix f_pq = h_pq + sum_{j<n_occ} [2(pq|jj) - (pj|jq)]."""
    h = np.asarray(h)
    eri = np.asarray(eri)
    j = np.arange(n_occ)
    return h + 2.0 * eri[:, :, j, j].sum(axis=2) - eri[:, j, j, :].sum(axis=1)


def features(pool, fock, eri, occ, prev_absg, age, count):
    """Sixteen screener features per pool operator (float64).

    f0-f3  Fock diagonal of the spatial orbitals of P, Q, R, S (0 when absent)
    f4     |(pr|qs)| for doubles, |f_pq| for singles (spatial indices)
    f5-f8  occupation <n_P> of the spin-orbitals P, Q, R, S (0 when absent)
    f9     previous exact |g_k| (0 if never computed)
    f10    log10(previous |g_k| + 1e-16)
    f11    iterations since the last exact value / 10
    f12-14 one-hot type: single, same-spin double, opposite-spin double
    f15    occurrences of k in the ansatz
    """
    pool = np.asarray(pool)
    K = len(pool)
    F = np.zeros((K, 16))
    diag = np.diag(fock)
    for k in range(K):
        P, Q, R, S = (int(t) for t in pool[k])
        idx = [P, Q, R, S]
        for t in range(4):
            if idx[t] >= 0:
                F[k, t] = diag[idx[t] >> 1]
                F[k, 5 + t] = occ[idx[t]]
        if R < 0:
            F[k, 4] = abs(fock[P >> 1, Q >> 1])
            F[k, 12] = 1.0
        else:
            F[k, 4] = abs(eri[P >> 1, R >> 1, Q >> 1, S >> 1])
            if (P & 1) == (Q & 1):
                F[k, 13] = 1.0
            else:
                F[k, 14] = 1.0
        F[k, 9] = prev_absg[k]
        F[k, 10] = np.log10(prev_absg[k] + 1e-16)
        F[k, 11] = age[k] / 10.0
        F[k, 15] = count[k]
    return F


def select_subset(score, rand_key, frac_top=0.05, frac_rand=0.01):
    """Indices of the top ceil(frac_top K) scores (ties: smaller index first)
    plus the ceil(frac_rand K) remaining operators with the smallest random
    keys (ties: smaller index), returned sorted ascending."""
    score = np.asarray(score)
    K = len(score)
    n_top = int(np.ceil(frac_top * K))
    n_rand = int(np.ceil(frac_rand * K))
    order = sorted(range(K), key=lambda k: (-float(score[k]), k))
    top = set(order[:n_top])
    rest = [k for k in range(K) if k not in top]
    rest.sort(key=lambda k: (int(rand_key[k]), k))
    chosen = sorted(top | set(rest[:n_rand]))
    return np.array(chosen, dtype=np.int32)


def mp2_uccsd(orc, pool, ref, rel_tol=1e-9):
    """MP2-ordered UCCSD ansatz of a closed-shell reference (Sec. II.A, Eqs. 1-3).

    Zeroth-order Hamiltonian: H0 = sum_P f_{P/2, P/2} n_P with f the
    closed-shell Fock matrix of the reference (fock_spatial), so every
    determinant is an eigenvector of H0 with E0(D) = sum of f_pp over its
    spin-orbitals.  The first-order coefficient of a doubly excited D is
    t_D = <D|H|ref> / (E0(ref) - E0(D)) and the MP2 energy is
    E2 = sum_D <D|H|ref>^2 / (E0(ref) - E0(D)) over the doubles.  The pool
    operator k whose generator takes ref to D (A_k|ref> = s_k|D>, s_k = +-1,
    either orientation of T_k) gets theta_k = s_k t_D, so that
    exp(theta_k A_k)|ref> equals ref + t_D D to first order.  Singles get 0
    (the paper's MP2 has no single amplitudes).

    Order (index 0 is applied first): doubles by decreasing |theta| (values
    within rel_tol * max |theta| of the first of a run count as equal and go
    by pool index), then the singles by ascending (occupied, virtual)
    spin-orbital.  Returns (ops int32, theta float64, e2)."""
    if orc.n_alpha != orc.n_beta:
        raise ValueError("closed-shell reference needed")
    f = np.diag(fock_spatial(orc._h_arr, orc._eri_arr, orc.n_alpha))
    nso = 2 * orc.n
    ref = int(ref)
    occ = {P for P in range(nso) if (ref >> P) & 1}

    def e0(key):
        return sum(f[P >> 1] for P in range(nso) if (key >> P) & 1)

    ref_state = OracleState.from_arrays(np.array([ref], dtype=np.uint64), np.array([1.0]))
    doubles, singles, e2 = [], [], 0.0
    for k, row in enumerate(np.asarray(pool).tolist()):
        P, Q, R, S = row
        cre = [P, Q] if R >= 0 else [P]
        ann = [R, S] if R >= 0 else [Q]
        fwd = all(a in occ for a in ann) and not any(c in occ for c in cre)
        rev = all(c in occ for c in cre) and not any(a in occ for a in ann)
        if not (fwd or rev):
            continue
        o, v = (ann, cre) if fwd else (cre, ann)
        if R < 0:
            singles.append((o[0], v[0], k))
            continue
        D = ref
        for x in o + v:
            D ^= 1 << x
        keys, amps = Oracle.apply_generator(ref_state, np.asarray(row)).export()
        hit = np.flatnonzero(keys == np.uint64(D))
        if len(hit) != 1 or abs(abs(amps[hit[0]]) - 1.0) > 0.0:
            raise AssertionError("generator does not take the reference to D")
        s = float(amps[hit[0]])
        hDr = orc.hmat(D, ref)
        dE = e0(ref) - e0(D)
        doubles.append((s * hDr / dE, k))
        e2 += hDr * hDr / dE
    # doubles: |theta| descending, near-equal runs by pool index
    a = {k: abs(t) for t, k in doubles}
    theta_of = {k: t for t, k in doubles}
    order = sorted(a, key=lambda k: (-a[k], k))
    tol = rel_tol * (max(a.values()) if a else 0.0)
    ops = []
    i = 0
    while i < len(order):
        j = i + 1
        while j < len(order) and a[order[i]] - a[order[j]] <= tol:
            j += 1
        ops += sorted(order[i:j])
        i = j
    theta = [theta_of[k] for k in ops]
    for _, _, k in sorted(singles):
        ops.append(k)
        theta.append(0.0)
    return np.array(ops, dtype=np.int32), np.array(theta, dtype=np.float64), e2

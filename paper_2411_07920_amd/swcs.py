"""Thin Python binding of libswcs (argument marshalling only).

Every computation runs in the HIP kernels of ``libswcs.so``; this module
converts numpy arrays / torch tensors to pointers, checks return codes and
raises :class:`SwcsError` with the library's message.  Importing it without
the built library fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import math
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libswcs.so")

SWCS_OK = 0
SWCS_E_INVALID = -1
SWCS_E_STATE = -2
SWCS_E_OOM = -3
SWCS_E_CAPACITY = -4
SWCS_E_DEVICE = -5
SWCS_E_UNSUPPORTED = -6
KERNELS = {"chain_lds": 1, "gate": 2, "sigma_proj": 3, "sigma_push": 4, "pool_contract": 5,
           "adjoint_lds": 6, "gate_replay": 7, "adjoint_rec": 8, "sigma_push_into": 9,
           "contract_ops": 10, "holepair": 11, "adjoint_replay_lds": 12, "select": 13,
           "join_emit": 14, "join_sort": 15, "join_reduce": 16,
           "join_terms": 17}
SIGMA_METHODS = {"auto": 0, "enumerate": 1, "hole_pairs": 2, "pairs": 3}
POOL_METHODS = {"auto": 0, "table": 1, "join": 2}
_NAMES = {0: "SWCS_OK", -1: "SWCS_E_INVALID", -2: "SWCS_E_STATE", -3: "SWCS_E_OOM",
          -4: "SWCS_E_CAPACITY", -5: "SWCS_E_DEVICE", -6: "SWCS_E_UNSUPPORTED"}


class SwcsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_f = ctypes.c_float

# name -> (restype, argtypes); mirrors include/swcs.h
SIGNATURES = {
    "swcs_version": (ctypes.c_char_p, []),
    "swcs_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(_vp)]),
    "swcs_destroy": (None, [_vp]),
    "swcs_last_error": (ctypes.c_char_p, [_vp]),
    "swcs_set_stream": (ctypes.c_int, [_vp, _vp]),
    "swcs_set_capacity": (ctypes.c_int, [_vp, _i64, ctypes.c_int]),
    "swcs_set_allocator": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "swcs_set_table_budget": (ctypes.c_int, [_vp, _i64]),
    "swcs_set_sigma_method": (ctypes.c_int, [_vp, ctypes.c_int]),
    "swcs_set_pool_method": (ctypes.c_int, [_vp, ctypes.c_int]),
    "swcs_set_integrals": (ctypes.c_int, [_vp, _dp, _dp, ctypes.c_double]),
    "swcs_set_reference": (ctypes.c_int, [_vp, ctypes.c_uint64]),
    "swcs_set_pool": (ctypes.c_int, [_vp, _i32p, _i64]),
    "swcs_apply_ansatz": (ctypes.c_int, [_vp, _i32p, _dp, _i64, ctypes.c_double, _i64, _i64p]),
    "swcs_apply_gates": (ctypes.c_int, [_vp, _i32p, _dp, _i64, ctypes.c_double, _i64, _i64p]),
    "swcs_apply_generators": (ctypes.c_int, [_vp, _i32p, _dp, _i64, ctypes.c_double, _i64, _i64p]),
    "swcs_set_state": (ctypes.c_int, [_vp, _u64p, _dp, _i64]),
    "swcs_get_state": (ctypes.c_int, [_vp, _u64p, _dp, _i64, _i64p]),
    "swcs_energy": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
    "swcs_energy_noalloc": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
    "swcs_sigma_projected": (ctypes.c_int, [_vp, _u64p, _dp, _i64, _i64p]),
    "swcs_pool_gradients": (ctypes.c_int, [_vp, _i32p, _i64, _dp]),
    "swcs_pool_gradients_device": (ctypes.c_int, [_vp, _vp, _i64, _vp]),
    "swcs_log_abs": (ctypes.c_int, [_vp, _vp, _i64, _vp]),
    "swcs_add_feature": (ctypes.c_int, [_vp, _vp, _vp, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_float]),
    "swcs_param_gradients": (ctypes.c_int, [_vp, _dp, _dp]),
    "swcs_gate_sizes": (ctypes.c_int, [_vp, _i64p, _i64]),
    "swcs_state_counts": (ctypes.c_int, [_vp, _i64p, _i64p]),
    "swcs_compact": (ctypes.c_int, [_vp, _i64p]),
    "swcs_gate_active": (ctypes.c_int, [_vp, _i64p, _i64]),
    "swcs_pool_stats": (ctypes.c_int, [_vp, _dp, _i64p, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "swcs_occupations": (ctypes.c_int, [_vp, _dp]),
    "swcs_fock_diagonal": (ctypes.c_int, [_vp, _dp]),
    "swcs_timer_start": (ctypes.c_int, [_vp, ctypes.c_int]),
    "swcs_timer_stop": (ctypes.c_int, [_vp, _i64p, _dp]),
    "swcs_mlp_param_count": (ctypes.c_int64, []),
    "swcs_features": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "swcs_mlp_forward": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _vp]),
    "swcs_mlp_backward": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _i64, _vp]),
    "swcs_mse": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _vp]),
    "swcs_adam_step": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _i64, _f, _f, _f, _f, ctypes.c_int]),
    "swcs_select": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i64, _i64, _vp]),
}


def load():
    """Load libswcs.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _dev(t):
    """Device pointer of a torch tensor (or an int address)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("screener calls take device tensors")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


# Device memory callbacks (include/swcs.h: swcs_alloc_fn, swcs_free_fn).
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

# Contexts still open; closed at interpreter exit while torch (whose
# allocator may own their memory) is still alive.
_OPEN = weakref.WeakSet()


@atexit.register
def _close_all():
    for ctx in list(_OPEN):
        try:
            ctx.close()
        except Exception:
            pass


def version() -> str:
    return load().swcs_version().decode()


def mlp_param_count() -> int:
    return int(load().swcs_mlp_param_count())


class Context:
    """One SWCS problem on one HIP device (see include/swcs.h)."""

    def __init__(self, n_spatial: int, n_alpha: int, n_beta: int, device: int = 0):
        self._lib = load()
        h = _vp()
        rc = self._lib.swcs_create(n_spatial, n_alpha, n_beta, device, ctypes.byref(h))
        if rc != SWCS_OK:
            raise SwcsError(rc, self._lib.swcs_last_error(None).decode())
        self._h = h
        self.n, self.n_alpha, self.n_beta = n_spatial, n_alpha, n_beta
        self.device = device
        self._keep = []
        self._alloc_cb = None
        _OPEN.add(self)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.swcs_destroy(self._h)
            self._h = None
            if getattr(self, "_torch_memory", False):
                # the library sizes its tables from the device's free memory
                # (plus what it handed back itself); blocks a closed context
                # leaves in PyTorch's cache would be invisible to the next one
                import torch
                torch.cuda.empty_cache()
        self._alloc_cb = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc):
        if rc != SWCS_OK:
            raise SwcsError(rc, self._lib.swcs_last_error(self._h).decode())

    # -- set-up ---------------------------------------------------------
    def set_stream(self, stream):
        """stream: a torch.cuda.Stream, an int hipStream_t, or None."""
        if stream is None:
            ptr = None
        elif isinstance(stream, int):
            ptr = stream
        else:
            ptr = stream.cuda_stream
        self._check(self._lib.swcs_set_stream(self._h, ptr))

    def set_capacity(self, max_dets: int, allow_regrow: bool = True):
        self._check(self._lib.swcs_set_capacity(self._h, int(max_dets), 1 if allow_regrow else 0))

    def set_allocator(self, alloc, free):
        """Route the library's device allocations through Python callables
        alloc(nbytes) -> int address (0 on failure) and free(address);
        (None, None) restores hipMalloc / hipFree."""
        if alloc is None and free is None:
            self._check(self._lib.swcs_set_allocator(self._h, None, None, None))
            self._alloc_cb = None
            return

        def _a(nbytes, _user):
            try:
                return int(alloc(int(nbytes))) or None
            except Exception:  # reported to the library as an allocation failure
                return None

        def _f(ptr, _user):
            try:
                free(int(ptr))
            except Exception:
                pass

        cbs = (ALLOC_FN(_a), FREE_FN(_f))
        self._check(self._lib.swcs_set_allocator(self._h, ctypes.cast(cbs[0], _vp),
                                                 ctypes.cast(cbs[1], _vp), None))
        # blocks allocated through these callbacks are freed through them, up
        # to swcs_destroy: keep every pair alive for the context's lifetime
        self._keep.append(cbs)
        self._alloc_cb = cbs

    def use_torch_allocator(self, stream=None):
        """Device memory from PyTorch's caching allocator, bound to `stream`
        (default: the current torch stream of the context's device), which is
        also made the context stream, so blocks the library frees are reused
        only in that stream's order."""
        import torch
        dev = self.device
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        self.set_stream(st)
        # blocks already cached by PyTorch would not show as free device memory
        torch.cuda.empty_cache()
        self._torch_memory = True

        def alloc(nbytes):
            return torch.cuda.caching_allocator_alloc(nbytes, dev, st)

        def free(ptr):
            torch.cuda.caching_allocator_delete(ptr)

        self.set_allocator(alloc, free)

    def set_table_budget(self, nbytes: int):
        """Cap on the pool-gradient sigma table in bytes (0 = from free memory)."""
        self._check(self._lib.swcs_set_table_budget(self._h, int(nbytes)))

    def set_sigma_method(self, method: str):
        """'auto', 'enumerate' or 'hole_pairs' (how sigma_P is formed)."""
        self._check(self._lib.swcs_set_sigma_method(self._h, SIGMA_METHODS[method]))

    def set_pool_method(self, method: str):
        """'auto', 'table' or 'join' (how whole-pool gradients are formed)."""
        self._check(self._lib.swcs_set_pool_method(self._h, POOL_METHODS[method]))

    def set_integrals(self, h, eri, e_core: float = 0.0):
        h = np.ascontiguousarray(h, dtype=np.float64)
        eri = np.ascontiguousarray(eri, dtype=np.float64)
        n = self.n
        if h.shape != (n, n) or eri.shape != (n, n, n, n):
            raise ValueError("integral shapes must be (n, n) and (n, n, n, n)")
        self._check(self._lib.swcs_set_integrals(self._h, _ptr(h, ctypes.c_double),
                                                 _ptr(eri, ctypes.c_double), float(e_core)))

    def set_reference(self, det: int):
        self._check(self._lib.swcs_set_reference(self._h, int(det)))

    def set_pool(self, rows):
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        if rows.ndim != 2 or rows.shape[1] != 4:
            raise ValueError("pool must be int32[K, 4]")
        self.K = len(rows)
        self._check(self._lib.swcs_set_pool(self._h, _ptr(rows, ctypes.c_int32), len(rows)))

    # -- state ----------------------------------------------------------
    def apply_ansatz(self, ops, theta, eps: float = 0.0, ncut: int = 0) -> int:
        ops = np.ascontiguousarray(ops, dtype=np.int32)
        theta = np.ascontiguousarray(theta, dtype=np.float64)
        if ops.shape != theta.shape or ops.ndim != 1:
            raise ValueError("ops and theta must be 1-D of equal length")
        out = ctypes.c_int64()
        self._check(self._lib.swcs_apply_ansatz(self._h, _ptr(ops, ctypes.c_int32),
                                                _ptr(theta, ctypes.c_double), len(ops), float(eps),
                                                int(ncut), ctypes.byref(out)))
        return int(out.value)

    def apply_gates(self, ops, theta, eps: float = 0.0, ncut: int = 0) -> int:
        ops = np.ascontiguousarray(ops, dtype=np.int32)
        theta = np.ascontiguousarray(theta, dtype=np.float64)
        if ops.shape != theta.shape or ops.ndim != 1:
            raise ValueError("ops and theta must be 1-D of equal length")
        out = ctypes.c_int64()
        self._check(self._lib.swcs_apply_gates(self._h, _ptr(ops, ctypes.c_int32),
                                               _ptr(theta, ctypes.c_double), len(ops), float(eps),
                                               int(ncut), ctypes.byref(out)))
        return int(out.value)

    def apply_generators(self, gens, theta, eps: float = 0.0, ncut: int = 0) -> int:
        """Chain of spin-complemented generators: int32 rows (k1, k2, s), k2 = -1
        for a single pool row (include/swcs.h: swcs_apply_generators)."""
        gens = np.ascontiguousarray(gens, dtype=np.int32).reshape(-1, 3)
        theta = np.ascontiguousarray(theta, dtype=np.float64)
        if len(gens) != len(theta) or theta.ndim != 1:
            raise ValueError("gens must be [M, 3] and theta [M]")
        out = ctypes.c_int64()
        self._check(self._lib.swcs_apply_generators(self._h, _ptr(gens, ctypes.c_int32),
                                                    _ptr(theta, ctypes.c_double), len(theta), float(eps),
                                                    int(ncut), ctypes.byref(out)))
        return int(out.value)

    def set_state(self, keys, amps):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        amps = np.ascontiguousarray(amps, dtype=np.float64)
        if keys.shape != amps.shape:
            raise ValueError("keys and amps must have equal length")
        self._check(self._lib.swcs_set_state(self._h, _ptr(keys, ctypes.c_uint64),
                                             _ptr(amps, ctypes.c_double), len(keys)))

    def get_state(self):
        """(keys uint64, amps float64), sorted ascending by key."""
        n = ctypes.c_int64()
        rc = self._lib.swcs_get_state(self._h, None, None, 0, ctypes.byref(n))
        if rc not in (SWCS_OK, SWCS_E_INVALID):
            self._check(rc)
        cnt = int(n.value)
        keys = np.zeros(cnt, dtype=np.uint64)
        amps = np.zeros(cnt, dtype=np.float64)
        self._check(self._lib.swcs_get_state(self._h, _ptr(keys, ctypes.c_uint64),
                                             _ptr(amps, ctypes.c_double), cnt, ctypes.byref(n)))
        return keys, amps

    # -- energy and gradients ------------------------------------------
    def energy(self):
        """(E, numer, norm2)."""
        e, nu, no = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(self._lib.swcs_energy(self._h, ctypes.byref(e), ctypes.byref(nu),
                                          ctypes.byref(no)))
        return e.value, nu.value, no.value

    def energy_noalloc(self):
        """(E, numer, norm2) with no device allocation (fixed library scratch)."""
        e, nu, no = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(self._lib.swcs_energy_noalloc(self._h, ctypes.byref(e), ctypes.byref(nu),
                                                  ctypes.byref(no)))
        return e.value, nu.value, no.value

    def sigma_projected(self):
        """(keys, sigma_P) on the kept determinants, sorted by key."""
        n = ctypes.c_int64()
        rc = self._lib.swcs_sigma_projected(self._h, None, None, 0, ctypes.byref(n))
        if rc not in (SWCS_OK, SWCS_E_INVALID):
            self._check(rc)
        cnt = int(n.value)
        keys = np.zeros(cnt, dtype=np.uint64)
        sig = np.zeros(cnt, dtype=np.float64)
        self._check(self._lib.swcs_sigma_projected(self._h, _ptr(keys, ctypes.c_uint64),
                                                   _ptr(sig, ctypes.c_double), cnt, ctypes.byref(n)))
        return keys, sig

    def pool_gradients(self, subset=None):
        if subset is None:
            out = np.zeros(self.K)
            self._check(self._lib.swcs_pool_gradients(self._h, None, 0, _ptr(out, ctypes.c_double)))
        else:
            subset = np.ascontiguousarray(subset, dtype=np.int32)
            out = np.zeros(len(subset))
            self._check(self._lib.swcs_pool_gradients(self._h, _ptr(subset, ctypes.c_int32),
                                                      len(subset), _ptr(out, ctypes.c_double)))
        return out

    def param_gradients(self, M: int):
        """(dE/dtheta[M], E) of the last apply_ansatz."""
        out = np.zeros(max(M, 1))
        e = ctypes.c_double()
        self._check(self._lib.swcs_param_gradients(self._h, _ptr(out, ctypes.c_double),
                                                   ctypes.byref(e)))
        return out[:M], e.value

    def gate_sizes(self, M: int):
        out = np.zeros(max(M, 1), dtype=np.int64)
        self._check(self._lib.swcs_gate_sizes(self._h, _ptr(out, ctypes.c_int64), M))
        return out[:M]

    def gate_active(self, M: int):
        """Entries each gate's operator acted on (multi-block gates; 0 in the LDS chain)."""
        out = np.zeros(max(M, 1), dtype=np.int64)
        self._check(self._lib.swcs_gate_active(self._h, _ptr(out, ctypes.c_int64), M))
        return out[:M]

    def state_counts(self):
        """(stored entries, alive entries) of the current state."""
        st, al = ctypes.c_int64(), ctypes.c_int64()
        self._check(self._lib.swcs_state_counts(self._h, ctypes.byref(st), ctypes.byref(al)))
        return int(st.value), int(al.value)

    def compact(self):
        """Drop the pruned entries from storage (include/swcs.h: swcs_compact);
        returns the stored count afterwards."""
        st = ctypes.c_int64()
        self._check(self._lib.swcs_compact(self._h, ctypes.byref(st)))
        return int(st.value)

    def pool_stats(self):
        """Sizing of the last pool-gradient pass (include/swcs.h: swcs_pool_stats)."""
        k, sl = ctypes.c_double(), ctypes.c_int64()
        b, p, sc = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self._lib.swcs_pool_stats(self._h, ctypes.byref(k), ctypes.byref(sl), ctypes.byref(b),
                                              ctypes.byref(p), ctypes.byref(sc)))
        return {"keys": k.value, "table_slots": int(sl.value), "batches": int(b.value),
                "passes": int(p.value), "screened": bool(sc.value)}

    def occupations(self):
        out = np.zeros(2 * self.n)
        self._check(self._lib.swcs_occupations(self._h, _ptr(out, ctypes.c_double)))
        return out

    def fock_diagonal(self):
        """Closed-shell Fock diagonal f_pp of the n spatial orbitals."""
        out = np.zeros(self.n)
        self._check(self._lib.swcs_fock_diagonal(self._h, _ptr(out, ctypes.c_double)))
        return out

    # -- measurement ----------------------------------------------------
    def timer_start(self, kernel: str):
        self._check(self._lib.swcs_timer_start(self._h, KERNELS[kernel]))

    def timer_stop(self):
        """(launches, total_ms) of the kernel timed since timer_start."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        self._check(self._lib.swcs_timer_stop(self._h, ctypes.byref(n), ctypes.byref(ms)))
        return int(n.value), float(ms.value)

    # -- screener (device tensors) --------------------------------------
    def features(self, prev_absg, age, count, out):
        self._check(self._lib.swcs_features(self._h, _dev(prev_absg), _dev(age), _dev(count),
                                            _dev(out)))

    def mlp_forward(self, W, x, y, act=None):
        B = int(x.shape[0])
        self._check(self._lib.swcs_mlp_forward(self._h, _dev(W), _dev(x), B, _dev(y), _dev(act)))

    def mlp_backward(self, W, x, act, dy, dW):
        B = int(x.shape[0])
        self._check(self._lib.swcs_mlp_backward(self._h, _dev(W), _dev(x), _dev(act), _dev(dy), B,
                                                _dev(dW)))

    def mse(self, y, t, dy, loss):
        self._check(self._lib.swcs_mse(self._h, _dev(y), _dev(t), int(y.shape[0]), _dev(dy),
                                       _dev(loss)))

    def pool_gradients_device(self, subset, g):
        """Pool gradients of the int32 device tensor `subset` into the float64
        device tensor `g`, stream-ordered (no host synchronization)."""
        self._check(self._lib.swcs_pool_gradients_device(self._h, _dev(subset), int(subset.shape[0]),
                                                         _dev(g)))

    def log_abs(self, g, t):
        self._check(self._lib.swcs_log_abs(self._h, _dev(g), int(g.shape[0]), _dev(t)))

    def add_feature(self, v, feat, col, sign, scale=1.0):
        """v = scale * v + sign * feat[:, col] (float32 device tensors, feat of
        16 columns, 0 <= scale <= 1)."""
        if feat.shape[0] < v.shape[0] or feat.shape[1] != 16:
            raise ValueError("feat must have 16 columns and at least len(v) rows")
        self._check(self._lib.swcs_add_feature(self._h, _dev(v), _dev(feat), int(v.shape[0]), int(col),
                                               int(sign), float(scale)))

    def adam_step(self, W, m, v, dW, lr, b1, b2, eps, step):
        self._check(self._lib.swcs_adam_step(self._h, _dev(W), _dev(m), _dev(v), _dev(dW),
                                             int(W.numel()), float(lr), float(b1), float(b2),
                                             float(eps), int(step)))

    def select(self, score, rand, n_top, n_rand, out_idx):
        K = int(score.shape[0])
        self._check(self._lib.swcs_select(self._h, _dev(score), _dev(rand), K, int(n_top),
                                          int(n_rand), _dev(out_idx)))


def make_context(n, n_alpha, n_beta, h, eri, pool, ref, device=0, e_core=0.0, stream=None,
                 torch_memory=True):
    """A context with integrals, reference and pool set.  By default its device
    memory comes from PyTorch's caching allocator on `stream` (default: the
    current torch stream); torch_memory=False keeps hipMalloc."""
    ctx = Context(n, n_alpha, n_beta, device)
    if torch_memory:
        ctx.use_torch_allocator(stream)
    elif stream is not None:
        ctx.set_stream(stream)
    ctx.set_integrals(h, eri, e_core)
    ctx.set_reference(ref)
    ctx.set_pool(pool)
    return ctx


def _autograd_function():
    import torch

    class AnsatzEnergy(torch.autograd.Function):
        """E(theta) of an ansatz on a Context; backward = adjoint gradients.

        forward(theta (float64 CPU tensor), ctx_obj, ops, eps, ncut) -> E
        """

        @staticmethod
        def forward(fctx, theta, swcs_ctx, ops, eps, ncut):
            th = theta.detach().cpu().numpy().astype(np.float64)
            swcs_ctx.apply_ansatz(ops, th, eps, ncut)
            dE, E = swcs_ctx.param_gradients(len(th))
            fctx.save_for_backward(torch.from_numpy(dE))
            return torch.tensor(E, dtype=torch.float64)

        @staticmethod
        def backward(fctx, grad_out):
            (dE,) = fctx.saved_tensors
            return grad_out * dE, None, None, None, None

    return AnsatzEnergy


def ansatz_energy(theta, swcs_ctx, ops, eps=0.0, ncut=0):
    """torch autograd entry: E(theta) with adjoint backward."""
    return _autograd_function().apply(theta, swcs_ctx, ops, eps, ncut)

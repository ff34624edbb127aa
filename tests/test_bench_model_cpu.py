"""The algorithmic-byte model behind the bench line's roofline, checked on
the CPU against the counts it is built from: the connection count of a
determinant with 8 alpha and 8 beta electrons in 26 spatial orbitals, the
record count of the whole-pool join, and the per-kernel byte formulas."""
import os
import sys
from math import comb

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


class _C:
    n = 26
    name = "c5"


class _Wl:
    c = _C()
    na = 8
    K = 301_600
    n_top = 15_080
    n_rand = 3_016


def test_join_and_gate_bytes():
    import bench
    n = 52_031                                          # determinants kept at c5
    C = 2 * 8 * 18 + 2 * comb(8, 2) * comb(18, 2) + 8 * 8 * 18 * 18
    assert C == 29_592                                  # singles + same-spin + opposite-spin doubles
    R = n * (C + 1)                                     # one record per connection and one per determinant
    n_in = np.full(300, 50_000, dtype=np.int64)
    r = {"n_in": n_in, "n_det": n}
    wl = _Wl()
    assert bench.algorithmic_bytes("join_reduce", wl, r) == R * 8 + n * C * 8 == 24_635_637_880
    assert bench.algorithmic_bytes("join_emit", wl, r) == R * 8 + n * 16
    # 24 bucket bits for about 256 records per bucket: three 8-bit passes
    assert bench.algorithmic_bytes("join_sort", wl, r) == R * 16 * 3
    assert bench.algorithmic_bytes("join_terms", wl, r) == n * C * 10
    assert bench.algorithmic_bytes("gate", wl, r) == 8 * 50_000
    assert bench.algorithmic_bytes("chain_lds", wl, r) == 8 * 50_000 * 300
    assert bench.algorithmic_bytes("select", wl, r) == wl.K * 8 + (wl.n_top + wl.n_rand) * 4

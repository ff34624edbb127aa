"""Host model of the library's sort-and-join pool gradient (test
infrastructure; shares no code with the oracle or the HIP library).

The HIP path (k_join.hip) evaluates the whole-pool gradient of ADAPT step 4
(Sec. II.C), g_k = (2/<psi|psi>) sum_D psi(D) a_k(D) sigma(X_k(D)), from one
64-bit record per (alive D, connection X) pair plus one per alive D:

  emit:   record = (d << (kb + bj)) | (field << kb) | (mix64(X) & (2^kb - 1)), with
          either orbital fields (bj = 24: h0 | h1 << 6 | p0 << 12 | p1 << 18, all
          ones for D itself) when they fit the word, or rank fields
          (bj = 3 + bh + bp: (class << (bh + bp)) | (hole set << bp) | particle
          set, class 7 for D itself);
  sort:   stable, by the kb bucket bits only;
  join:   per run of whole buckets, sigma(X) summed over the run's records
          (H_{X D} psi(D), or H_{D D} psi(D) for class 7), then
          psi(D) a_k(D) sigma(X) added to g[k] for every pair record.

This module builds the same records with numpy, in the enumeration order of
the kernels (class, then hole set, then particle set; pair sets by the
triangular index y (y - 1) / 2 + x, x < y), sorts them the same way, and
decodes every record from its fields and the lists alone.  It models the
encoding and the algorithm, not the concurrency.
"""
from __future__ import annotations

import numpy as np

import screened_model as sm


def _tri_pairs(m):
    """(x, y), x < y, of triangular indices 0 .. m (m - 1) / 2 - 1."""
    out = []
    y = 1
    while len(out) < m * (m - 1) // 2:
        for x in range(y):
            out.append((x, y))
        y += 1
    return np.array(out[: m * (m - 1) // 2], dtype=np.int64).reshape(-1, 2)


def lists_of(D, n):
    """occ_a, occ_b, vir_a, vir_b spin-orbitals of D (ascending)."""
    occ_a = [2 * p for p in range(n) if (D >> (2 * p)) & 1]
    occ_b = [2 * p + 1 for p in range(n) if (D >> (2 * p + 1)) & 1]
    vir_a = [2 * p for p in range(n) if not (D >> (2 * p)) & 1]
    vir_b = [2 * p + 1 for p in range(n) if not (D >> (2 * p + 1)) & 1]
    return occ_a, occ_b, vir_a, vir_b


def class_sizes(na, nb, va, vb):
    nh = [na, nb, na * (na - 1) // 2, nb * (nb - 1) // 2, na * nb]
    np_ = [va, vb, va * (va - 1) // 2, vb * (vb - 1) // 2, va * vb]
    return nh, np_


def _bits_for(v):
    b = 1
    while b < 64 and (v >> b) != 0:
        b += 1
    return b


def record_format(n, na, nb, n_stored, R, orbital=None):
    """(kb, bh, bp, orb, fits); orbital=None picks orbital fields when they fit."""
    va, vb = n - na, n - nb
    nh, np_ = class_sizes(na, nb, va, vb)
    bh = _bits_for(max(max(nh), 1) - 1)
    bp = _bits_for(max(max(np_), 1) - 1)
    kb = 8
    while kb < 24 and (R >> kb) > 256:
        kb += 8
    bd = _bits_for(max(n_stored - 1, 0))
    orb = (kb + 24 + bd <= 64) if orbital is None else orbital
    fits = kb + (24 if orb else 3 + bh + bp) + bd <= 64
    return kb, bh, bp, orb, fits


def hole_particle_sets(D, n, na, nb):
    """Per class: hole sets and particle sets as (first, second) spin-orbital
    arrays in the kernels' order (singles repeat the orbital)."""
    oa, ob, xa, xb = (np.array(v, dtype=np.int64) for v in lists_of(D, n))
    hp = []
    for o, x in ((oa, xa), (ob, xb)):
        hp.append(((o, o), (x, x)))
    for o, x in ((oa, xa), (ob, xb)):
        th, tp = _tri_pairs(len(o)), _tri_pairs(len(x))
        hp.append(((o[th[:, 0]], o[th[:, 1]]), (x[tp[:, 0]], x[tp[:, 1]])))
    i, j = np.divmod(np.arange(len(oa) * len(ob)), len(ob))
    a, b = np.divmod(np.arange(len(xa) * len(xb)), len(xb))
    h0, h1 = np.minimum(oa[i], ob[j]), np.maximum(oa[i], ob[j])
    p0, p1 = np.minimum(xa[a], xb[b]), np.maximum(xa[a], xb[b])
    hp.append(((h0, h1), (p0, p1)))
    return hp


def emit(keys, amps, n, na, nb, orbital=None):
    """Records (uint64), each record's X by direct enumeration, and the
    format, in storage order of the alive entries."""
    keys = np.asarray(keys, dtype=np.uint64)
    alive = np.flatnonzero(~np.isnan(np.asarray(amps)))
    va, vb = n - na, n - nb
    nh, np_ = class_sizes(na, nb, va, vb)
    C = sum(a * b for a, b in zip(nh, np_))
    R = len(alive) * (C + 1)
    kb, bh, bp, orb, fits = record_format(n, na, nb, len(keys), R, orbital)
    assert fits
    one = np.uint64(1)
    out, xs = [], []
    for d in alive.tolist():
        D = int(keys[d])
        sets = hole_particle_sets(D, n, na, nb)
        for c, ((h0, h1), (p0, p1)) in enumerate(sets):
            if len(h0) == 0 or len(p0) == 0:
                continue
            hi, pi = np.divmod(np.arange(len(h0) * len(p0)), len(p0))
            hm = (one << h0[hi].astype(np.uint64)) | (one << h1[hi].astype(np.uint64))
            pm = (one << p0[pi].astype(np.uint64)) | (one << p1[pi].astype(np.uint64))
            X = np.uint64(D) ^ hm ^ pm
            if orb:
                field = (h0[hi].astype(np.uint64) | (h1[hi].astype(np.uint64) << np.uint64(6))
                         | (p0[pi].astype(np.uint64) << np.uint64(12)) | (p1[pi].astype(np.uint64) << np.uint64(18)))
            else:
                field = ((np.uint64(c) << np.uint64(bh + bp)) | (hi.astype(np.uint64) << np.uint64(bp))
                         | pi.astype(np.uint64))
            out.append(rec(d, field, X, kb, bh, bp, orb))
            xs.append(X)
        self_field = 0xFFFFFF if orb else 7 << (bh + bp)
        out.append(rec(d, np.array([self_field], dtype=np.uint64), np.array([D], dtype=np.uint64), kb, bh, bp, orb))
        xs.append(np.array([D], dtype=np.uint64))
    recs = np.concatenate(out)
    assert len(recs) == R
    return recs, np.concatenate(xs), (kb, bh, bp, orb)


def rec(d, field, X, kb, bh, bp, orb):
    bucket = sm.mix64(X) & np.uint64((1 << kb) - 1)
    bj = 24 if orb else 3 + bh + bp
    return (np.uint64(d) << np.uint64(kb + bj)) | (field << np.uint64(kb)) | bucket


def decode(recs, fmt, keys, n, na, nb):
    """(d, class, X, nh, h0, h1, p0, p1) of every record, from its fields and
    D's lists only."""
    kb, bh, bp, orb = fmt
    va, vb = n - na, n - nb
    bj = 24 if orb else 3 + bh + bp
    f = (recs >> np.uint64(kb)) & np.uint64((1 << bj) - 1)
    d = (recs >> np.uint64(kb + bj)).astype(np.int64)
    keys = np.asarray(keys, dtype=np.uint64)
    if orb:
        fi = f.astype(np.int64)
        h0, h1, p0, p1 = fi & 63, (fi >> 6) & 63, (fi >> 12) & 63, (fi >> 18) & 63
        c = np.where(fi == 0xFFFFFF, 7, 0)
        nh = np.where(h0 == h1, 1, 2)
        one = np.uint64(1)
        D = keys[d]
        hm = (one << h0.astype(np.uint64)) | (one << h1.astype(np.uint64))
        pm = (one << p0.astype(np.uint64)) | (one << p1.astype(np.uint64))
        X = np.where(c == 7, D, D ^ hm ^ pm)
        return d, c, X, nh, h0, h1, p0, p1
    pi = (f & np.uint64((1 << bp) - 1)).astype(np.int64)
    hi = ((f >> np.uint64(bp)) & np.uint64((1 << bh) - 1)).astype(np.int64)
    c = ((f >> np.uint64(bp + bh)) & np.uint64(7)).astype(np.int64)
    L = np.array([sum(lists_of(int(k), n), []) for k in keys.tolist()], dtype=np.int64)
    oa, ob, xa, xb = 0, na, na + nb, na + nb + va
    tri = _tri_pairs(max(na, nb, va, vb))
    h0 = np.zeros(len(recs), dtype=np.int64)
    h1, p0, p1 = h0.copy(), h0.copy(), h0.copy()
    nh = np.where(c < 2, 1, 2)
    for cl in range(5):
        m = c == cl
        Ld, H, P = L[d[m]], hi[m], pi[m]
        rows = np.arange(m.sum())
        if cl < 2:
            ho, po = (oa, xa) if cl == 0 else (ob, xb)
            a = Ld[rows, ho + H]
            b = Ld[rows, po + P]
            h0[m], h1[m], p0[m], p1[m] = a, a, b, b
        elif cl < 4:
            ho, po = (oa, xa) if cl == 2 else (ob, xb)
            h0[m], h1[m] = Ld[rows, ho + tri[H, 0]], Ld[rows, ho + tri[H, 1]]
            p0[m], p1[m] = Ld[rows, po + tri[P, 0]], Ld[rows, po + tri[P, 1]]
        else:
            i, j = np.divmod(H, nb)
            a, b = np.divmod(P, vb)
            ha, hb = Ld[rows, oa + i], Ld[rows, ob + j]
            pa, pb = Ld[rows, xa + a], Ld[rows, xb + b]
            h0[m], h1[m] = np.minimum(ha, hb), np.maximum(ha, hb)
            p0[m], p1[m] = np.minimum(pa, pb), np.maximum(pa, pb)
    one = np.uint64(1)
    D = keys[d]
    hm = (one << h0.astype(np.uint64)) | (one << h1.astype(np.uint64))
    pm = (one << p0.astype(np.uint64)) | (one << p1.astype(np.uint64))
    X = np.where(c == 7, D, D ^ hm ^ pm)
    return d, c, X, nh, h0, h1, p0, p1


def join_gradients(keys, amps, pool, h, eri, na, nb, orbital=None):
    """Whole-pool g by emit, sort and join; also returns every record's X as
    decoded from its fields and as enumerated when it was emitted (same
    order), and the record format."""
    n = h.shape[0]
    keys = np.asarray(keys, dtype=np.uint64)
    amps = np.asarray(amps, dtype=np.float64)
    recs, X_enum, fmt = emit(keys, amps, n, na, nb, orbital)
    kb = fmt[0]
    order = np.argsort(recs & np.uint64((1 << kb) - 1), kind="stable")
    recs, X_enum = recs[order], X_enum[order]
    d, c, X, nh, h0, h1, p0, p1 = decode(recs, fmt, keys, n, na, nb)
    # sigma over the records of each X (the buckets hold every record of an X)
    v = np.zeros(len(recs))
    pair = c != 7
    for dd in np.unique(d).tolist():
        m = np.flatnonzero((d == dd) & pair)
        v[m] = sm.elements(int(keys[dd]), nh[m], h0[m], h1[m], p0[m], p1[m], h, eri) * amps[dd]
        s = np.flatnonzero((d == dd) & ~pair)
        v[s] = sm.diagonal(int(keys[dd]), h, eri) * amps[dd]
    ux, inv = np.unique(X, return_inverse=True)
    sigma = np.zeros(len(ux))
    np.add.at(sigma, inv, v)
    tab, npairs = sm.generator_table(pool, 2 * n)
    k, t, P, Q, R, S = sm.linking_operator(tab, npairs, nh[pair], h0[pair], h1[pair], p0[pair], p1[pair])
    Dp, Xp = keys[d[pair]], X[pair]
    a = np.where(t, sm.phase_T(Dp, P, Q, R, S), -sm.phase_T(Xp, P, Q, R, S))
    g = np.zeros(len(pool))
    ok = k >= 0
    np.add.at(g, k[ok], (amps[d[pair]] * a * sigma[inv[pair]])[ok])
    return 2.0 * g / float(np.sum(amps[~np.isnan(amps)] ** 2)), X, X_enum, fmt

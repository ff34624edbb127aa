"""Host model of the library's determinant-major screened pool gradient
(test infrastructure; shares no code with the oracle or the HIP library).

The HIP path evaluates g_k = (2/<psi|psi>) sum_D psi(D) a_k(D) sigma(X_k(D))
for a selected subset of pool operators (ADAPT step 4, Sec. II.C) in three
passes over the stored determinants:

  1. query:    every connection X of every alive D whose linking operator k
               (the pool operator taking D to X, found through the direct
               generator table) is selected puts X into a hash table;
  2. push:     every alive D' adds H_{X D'} psi(D') to each connection X (and
               H_{D'D'} psi(D') to D' itself) that is already in the table;
  3. contract: every (D, X, k selected) adds psi(D) a_k(D) sigma(X) to g[k],
               a_k(D) = +<X|T_k|D> when T_k acts on D, -<X|T_k^dagger|D>
               when T_k^dagger does.

Keys may be split into batches by a hash of X; each batch repeats the three
passes on its own keys.  This module walks the same passes with numpy on the
host, keyed by sorted arrays instead of hash tables, with the generator table
indexed the way the kernels index it.  It models the algorithm (which
connections, which operator, which sign, which batch), not the concurrency.
"""
from __future__ import annotations

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def mix64(x):
    """The 64-bit finalizer the library hashes keys with (SplitMix64 style)."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        x = x ^ (x >> np.uint64(30))
        x = x * np.uint64(0xBF58476D1CE4E5B9)
        x = x ^ (x >> np.uint64(27))
        x = x * np.uint64(0x94D049BB133111EB)
        x = x ^ (x >> np.uint64(31))
    return x


def batch_of(X, nbatch):
    h = mix64(np.asarray(X, dtype=np.uint64) ^ np.uint64(0x9E3779B97F4A7C15))
    return ((h >> np.uint64(32)) % np.uint64(nbatch)).astype(np.int64)


def _pair(a, b):
    return a * (a - 1) // 2 + b


def generator_table(pool, nso):
    """(P, Q, R, S) -> pool index, -1 where the pool has no operator: singles
    at pair(P, Q), doubles at npairs + tri(pair(P, Q)) + pair(R, S)."""
    npairs = nso * (nso - 1) // 2
    tab = np.full(npairs + npairs * (npairs - 1) // 2, -1, dtype=np.int64)
    for k, (P, Q, R, S) in enumerate(np.asarray(pool).tolist()):
        if R < 0:
            tab[_pair(P, Q)] = k
        else:
            pq, rs = _pair(P, Q), _pair(R, S)
            tab[npairs + pq * (pq - 1) // 2 + rs] = k
    return tab, npairs


def _below(D, P):
    """Occupied spin-orbitals of D below P (vectorized over P or D)."""
    one = np.uint64(1)
    mask = (one << np.asarray(P, dtype=np.uint64)) - one
    return np.bitwise_count(np.asarray(D, dtype=np.uint64) & mask).astype(np.int64)


def connections(D, n):
    """All spin-conserving singles and doubles of D: arrays (X, nh, h0, h1,
    p0, p1) with holes h0 <= h1 and particles p0 <= p1 (h0 == h1, p0 == p1
    for singles)."""
    occ = [P for P in range(2 * n) if (D >> P) & 1]
    vir = [P for P in range(2 * n) if not (D >> P) & 1]
    rows = []
    for spin in (0, 1):
        for i in (P for P in occ if P & 1 == spin):
            for a in (P for P in vir if P & 1 == spin):
                rows.append((1, i, i, a, a))
    hp = [(x, y) for ix, x in enumerate(occ) for y in occ[ix + 1:]]
    pp = [(x, y) for ix, x in enumerate(vir) for y in vir[ix + 1:]]
    for (x, y) in hp:
        for (a, b) in pp:
            if sorted((x & 1, y & 1)) == sorted((a & 1, b & 1)):
                rows.append((2, x, y, a, b))
    r = np.array(rows, dtype=np.int64)
    one = np.uint64(1)
    Du = np.uint64(D)
    hm = (one << r[:, 1].astype(np.uint64)) | (one << r[:, 2].astype(np.uint64))
    pm = (one << r[:, 3].astype(np.uint64)) | (one << r[:, 4].astype(np.uint64))
    X = Du ^ hm ^ pm
    return X, r[:, 0], r[:, 1], r[:, 2], r[:, 3], r[:, 4]


def linking_operator(tab, npairs, nh, h0, h1, p0, p1):
    """Pool index k (or -1), whether T (not T^dagger) acts on D, and the
    operator's (P, Q, R, S), from the connection's holes and particles."""
    single = nh == 1
    t1 = p0 > h0
    t2 = p1 > h1
    t = np.where(single, t1, t2)
    P = np.where(single, np.where(t1, p0, h0), np.where(t2, p1, h1))
    Q = np.where(single, np.where(t1, h0, p0), np.where(t2, p0, h0))
    R = np.where(single, -1, np.where(t2, h1, p1))
    S = np.where(single, -1, np.where(t2, h0, p0))
    pq = _pair(P, Q)
    rs = _pair(np.maximum(R, 1), np.maximum(S, 0))
    slot = np.where(single, pq, npairs + pq * (pq - 1) // 2 + rs)
    return tab[slot], t, P, Q, R, S


def phase_T(D, P, Q, R, S):
    """Sign of T = a+_P a+_Q a_S a_R (or a+_P a_Q when R < 0) acting on D,
    the rightmost ladder operator first."""
    D = np.asarray(D, dtype=np.uint64) * np.ones(len(P), dtype=np.uint64)
    one = np.uint64(1)
    s = np.zeros(len(P), dtype=np.int64)
    single = R < 0
    # single: a_Q then a+_P
    s1 = _below(D, Q)
    x1 = D ^ (one << Q.astype(np.uint64))
    s1 = s1 + _below(x1, P)
    # double: a_R, a_S, a+_Q, a+_P
    Rs, Ss = np.maximum(R, 0).astype(np.uint64), np.maximum(S, 0).astype(np.uint64)
    s2 = _below(D, Rs)
    x2 = D ^ (one << Rs)
    s2 = s2 + _below(x2, Ss)
    x2 = x2 ^ (one << Ss)
    s2 = s2 + _below(x2, Q)
    x2 = x2 ^ (one << Q.astype(np.uint64))
    s2 = s2 + _below(x2, P)
    s = np.where(single, s1, s2)
    return np.where(s & 1, -1.0, 1.0)


def elements(D, nh, h0, h1, p0, p1, h, eri):
    """<X|H|D> for the connections of D (Slater-Condon, spatial integrals)."""
    n = h.shape[0]
    occ = np.array([P for P in range(2 * n) if (D >> P) & 1], dtype=np.int64)
    out = np.zeros(len(nh))
    s = np.flatnonzero(nh == 1)
    if len(s):
        I, A = h0[s], p0[s]
        sign = (_below(D, I) + _below(np.uint64(D) ^ (np.uint64(1) << I.astype(np.uint64)), A)) & 1
        a, i, q = A // 2, I // 2, occ // 2
        v = h[a, i] + eri[a[:, None], i[:, None], q[None, :], q[None, :]].sum(1)
        same = ((occ[None, :] ^ A[:, None]) & 1) == 0
        v = v - (eri[a[:, None], q[None, :], q[None, :], i[:, None]] * same).sum(1)
        out[s] = np.where(sign, -v, v)
    d = np.flatnonzero(nh == 2)
    if len(d):
        I, J, A, B = h0[d], h1[d], p0[d], p1[d]
        one = np.uint64(1)
        x = np.uint64(D) ^ (one << I.astype(np.uint64))
        sg = _below(D, I) + _below(x, J)
        x = x ^ (one << J.astype(np.uint64))
        sg = sg + _below(x, B)
        x = x ^ (one << B.astype(np.uint64))
        sg = sg + _below(x, A)

        def so(P, Q, R, S):
            ok = (((P ^ Q) & 1) == 0) & (((R ^ S) & 1) == 0)
            return np.where(ok, eri[P // 2, Q // 2, R // 2, S // 2], 0.0)

        v = so(A, I, B, J) - so(A, J, B, I)
        out[d] = np.where(sg & 1, -v, v)
    return out


def diagonal(D, h, eri):
    n = h.shape[0]
    occ = [P for P in range(2 * n) if (D >> P) & 1]
    e = sum(h[P // 2, P // 2] for P in occ)
    for P in occ:
        for Q in occ:
            e += 0.5 * eri[P // 2, P // 2, Q // 2, Q // 2]
            if (P ^ Q) & 1 == 0:
                e -= 0.5 * eri[P // 2, Q // 2, Q // 2, P // 2]
    return e


def screened_gradients(keys, amps, pool, subset, h, eri, nbatch=1):
    """g for the operators of `subset` by the three passes, summed over
    `nbatch` key-hash batches."""
    n = h.shape[0]
    nso = 2 * n
    tab, npairs = generator_table(pool, nso)
    selected = np.zeros(len(pool), dtype=bool)
    selected[np.asarray(subset)] = True
    conns = [connections(int(D), n) for D in np.asarray(keys).tolist()]
    links = [linking_operator(tab, npairs, *c[1:]) for c in conns]
    g = np.zeros(len(pool))
    for b in range(nbatch):
        # pass 1: query keys of this batch
        q = []
        for (X, *_), (k, *_r) in zip(conns, links):
            m = (k >= 0)
            m[m] = selected[k[m]]
            if nbatch > 1:
                m &= batch_of(X, nbatch) == b
            q.append(X[m])
        Qk = np.unique(np.concatenate(q)) if q else np.zeros(0, dtype=np.uint64)
        sig = np.zeros(len(Qk))

        def lookup(X):
            i = np.searchsorted(Qk, X)
            i = np.minimum(i, max(len(Qk) - 1, 0))
            hit = (Qk[i] == X) if len(Qk) else np.zeros(len(X), dtype=bool)
            return i, hit

        # pass 2: push sigma into the query keys
        for D, psi, (X, nh, h0, h1, p0, p1) in zip(np.asarray(keys).tolist(), amps, conns):
            i, hit = lookup(np.array([D], dtype=np.uint64))
            if hit[0]:
                sig[i[0]] += diagonal(D, h, eri) * psi
            i, hit = lookup(X)
            if hit.any():
                H = elements(D, nh[hit], h0[hit], h1[hit], p0[hit], p1[hit], h, eri)
                np.add.at(sig, i[hit], H * psi)
        # pass 3: contract
        for D, psi, (X, *_), (k, t, P, Q, R, S) in zip(np.asarray(keys).tolist(), amps, conns, links):
            m = k >= 0
            m[m] = selected[k[m]]
            i, hit = lookup(X)
            m &= hit
            if not m.any():
                continue
            a = np.where(t[m], phase_T(D, P[m], Q[m], R[m], S[m]),
                         -phase_T(X[m], P[m], Q[m], R[m], S[m]))
            np.add.at(g, k[m], psi * a * sig[i[m]])
    norm2 = float(np.dot(amps, amps))
    return 2.0 * g[np.asarray(subset)] / norm2

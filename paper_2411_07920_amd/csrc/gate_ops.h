// Per-entry logic of one gate exp(theta A), A = T - T^dagger, and of its
// reverse (adjoint) step, shared by the multi-block kernels that keep the
// state in HBM and the single-workgroup kernels that keep it in LDS.
//
// A gate pairs each determinant D on which T acts with X = T D, with sign
// s = <X|T|D>, and rotates the pair:
//   psi'(D) = c psi(D) - s sn psi(X),   psi'(X) = c psi(X) + s sn psi(D)
// (c = cos theta, sn = sin theta): the exact exp(theta A), because T^2 = 0 and
// A^3 = -A (each unitary is evaluated exactly, Sec. II.B).  Everything else is
// unchanged.  Pruning (drop |c| < eps, after every unitary as in Fig. 1) is
// applied to the touched entries.
//
// Ownership rule (race-free in-place update): the pair (D, X) is handled by
// the thread of D whenever D is stored (alive or dead); otherwise by the
// thread of X, which then appends D.  Lookups only target keys stored before
// the gate started, and keys appended by a gate are new and distinct.
#pragma once

#include "swcs_internal.h"

namespace swcs {

struct GateOut {
  bool append;
  u64 key;
  double val;
  long long dalive;
  // The pair this thread owned (active = at least one member was in the
  // state before the gate): entry positions (kNoEntry if not stored; an
  // appended member is filled in by the caller), values before the gate
  // (dead if not in the state) and the sign s = <X|T|D>.
  bool active;
  u64 iD, iX;
  double a_old, b_old;
  int s;
  bool acts;  // T or T^dagger acts on this thread's entry (the gate's active count)
};

constexpr u64 kNoEntry = ~0ULL;

// One logged pair of a gate, consumed by the reverse (adjoint) step.
struct PairRec {
  unsigned iD, iX;  // 0xffffffff = not stored
  int s;
  unsigned pad;
  double a_old, b_old;
};

// One logged star {C, L1, L2} of a generator gate whose rows overlap
// (k_generator.hip): stored positions (0xffffffff = not stored), the signs
// alpha, beta of G C = alpha L1 + beta L2, and the values before the gate
// (dead if not in the state).
struct StarRec {
  unsigned iC, i1, i2;
  signed char al, be;
  unsigned short pad;
  double xc, x1, x2;
};

// Store: key(i), amp(i), set_amp(i, v), find(key) -> index or -1.
template <class Store>
__device__ inline GateOut gate_entry(Store& S, u64 i, const OpDesc& op, double c, double sn,
                                     double eps) {
  GateOut o{false, 0ULL, 0.0, 0, false, kNoEntry, kNoEntry, 0.0, 0.0, 0, false};
  const u64 D = S.key(i);
  const bool isT = ((D & op.ann) == op.ann) && ((D & op.cre) == 0);
  const bool isTd = ((D & op.cre) == op.cre) && ((D & op.ann) == 0);
  o.acts = isT || isTd;
  const u64 pair_mask = op.ann | op.cre;
  if (isT) {
    const u64 X = D ^ pair_mask;
    const long long j = S.find(X);
    const double araw = S.amp(i);
    const double braw = (j >= 0) ? S.amp((u64)j) : dead_value();
    const bool aliveD = !is_dead(araw), aliveX = !is_dead(braw);
    if (aliveD || aliveX) {
      const double s = (double)phase_of_T(op, D);
      const double a = aliveD ? araw : 0.0;
      const double b = aliveX ? braw : 0.0;
      const double nd = c * a - s * (sn * b);
      const double nx = c * b + s * (sn * a);
      const bool keepD = !(fabs(nd) < eps);
      const bool keepX = !(fabs(nx) < eps);
      S.set_amp(i, keepD ? nd : dead_value());
      if (j >= 0) {
        S.set_amp((u64)j, keepX ? nx : dead_value());
      } else if (keepX) {
        o.append = true;
        o.key = X;
        o.val = nx;
      }
      o.dalive = (long long)keepD - (long long)aliveD + (long long)keepX - (long long)aliveX;
      o.active = true;
      o.iD = i;
      o.iX = (j >= 0) ? (u64)j : kNoEntry;
      o.a_old = araw;
      o.b_old = braw;
      o.s = (int)s;
    }
  } else if (isTd) {
    const u64 Dsrc = D ^ pair_mask;
    const long long j = S.find(Dsrc);
    // When Dsrc is stored its thread owns the pair and may be writing this
    // entry; only read it when this thread is the owner.
    if (j < 0) {
      const double braw = S.amp(i);
      if (!is_dead(braw)) {
        const double s = (double)phase_of_T(op, Dsrc);
        const double a = 0.0, b = braw;
        const double nd = c * a - s * (sn * b);
        const double nx = c * b + s * (sn * a);
        const bool keepD = !(fabs(nd) < eps);
        const bool keepX = !(fabs(nx) < eps);
        S.set_amp(i, keepX ? nx : dead_value());
        if (keepD) {
          o.append = true;
          o.key = Dsrc;
          o.val = nd;
        }
        o.dalive = (long long)keepD + (long long)keepX - 1LL;
        o.active = true;
        o.iD = kNoEntry;
        o.iX = i;
        o.a_old = dead_value();
        o.b_old = braw;
        o.s = (int)s;
      }
    }
  }
  return o;
}

// Reverse step of one logged pair: with a, b the pair's values before the
// gate and mu after it, contributes mu^T P U'(theta) (a, b) to dE/dtheta and
// overwrites mu with U(theta)^T mu restricted to the pair members that were
// in the state before the gate.
template <class Mu>
__device__ inline double adjoint_pair(const PairRec& r, Mu& mu, double c, double sn) {
  const bool aliveD = !is_dead(r.a_old), aliveX = !is_dead(r.b_old);
  const double a = aliveD ? r.a_old : 0.0, b = aliveX ? r.b_old : 0.0;
  const double s = (double)r.s;
  const double muD = (r.iD != 0xffffffffu) ? mu.get(r.iD) : 0.0;
  const double muX = (r.iX != 0xffffffffu) ? mu.get(r.iX) : 0.0;
  if (r.iD != 0xffffffffu) mu.set(r.iD, aliveD ? (c * muD + s * sn * muX) : 0.0);
  if (r.iX != 0xffffffffu) mu.set(r.iX, aliveX ? (c * muX - s * sn * muD) : 0.0);
  return muD * (-sn * a - s * c * b) + muX * (-sn * b + s * c * a);
}

__device__ inline PairRec make_rec(const GateOut& o) {
  PairRec r;
  r.iD = (o.iD == kNoEntry) ? 0xffffffffu : (unsigned)o.iD;
  r.iX = (o.iX == kNoEntry) ? 0xffffffffu : (unsigned)o.iX;
  r.s = o.s;
  r.pad = 0;
  r.a_old = o.a_old;
  r.b_old = o.b_old;
  return r;
}

// ---------------------------------------------------------------- N_CUT
// Order used by N_CUT pruning: larger |c| first, ties broken by the smaller
// key.  Encoded as the 128-bit value (bits of |c|, ~key), compared as
// unsigned; "keep the ncut largest" keeps the entries whose value is >= the
// ncut-th largest.  Found by an MSB-first radix select over 16 digits of 8 bits.
__device__ inline void ncut_value(double a, u64 key, u64* hi, u64* lo) {
  *hi = (u64)__double_as_longlong(fabs(a));
  *lo = ~key;
}

__device__ inline unsigned ncut_digit(u64 hi, u64 lo, int d) {
  return d < 8 ? (unsigned)((hi >> (56 - 8 * d)) & 255u) : (unsigned)((lo >> (120 - 8 * d)) & 255u);
}

struct NcutState {
  u64 phi, plo, mhi, mlo;  // prefix of the selected value and its known-bit mask
  unsigned k;              // rank still to find inside the current prefix
  unsigned skip;           // 1: keep everything (fewer than ncut alive, or chain stopped)
  unsigned pad[2];
  unsigned hist[256];
};

__device__ inline bool ncut_matches(const NcutState& st, u64 hi, u64 lo) {
  return ((hi & st.mhi) == st.phi) && ((lo & st.mlo) == st.plo);
}

// After the digit histogram of pass d: choose the digit holding rank k
// (counted from the largest) and extend the prefix; sets skip when fewer
// than k values remain (then nothing is pruned).
__device__ inline void ncut_pick(NcutState& st, int d) {
  unsigned cum = 0;
  int v = -1;
  for (int x = 255; x >= 0; --x) {
    const unsigned h = st.hist[x];
    if (cum + h >= st.k) {
      v = x;
      break;
    }
    cum += h;
  }
  if (v < 0) {
    st.skip = 1;
    return;
  }
  st.k -= cum;
  if (d < 8) {
    st.phi |= (u64)v << (56 - 8 * d);
    st.mhi |= 255ULL << (56 - 8 * d);
  } else {
    st.plo |= (u64)v << (120 - 8 * d);
    st.mlo |= 255ULL << (120 - 8 * d);
  }
}

// ---------------------------------------------------------------- stores
struct GlobalStore {
  u64* keys;
  double* amps;
  const HashSlot* hash;
  u64 hmask;
  __device__ u64 key(u64 i) const { return keys[i]; }
  __device__ double amp(u64 i) const { return amps[i]; }
  __device__ void set_amp(u64 i, double v) { amps[i] = v; }
  __device__ long long find(u64 k) const { return hash_find(hash, hmask, k); }
};

struct GlobalMu {
  double* p;
  __device__ double get(u64 i) const { return p[i]; }
  __device__ void set(u64 i, double v) { p[i] = v; }
};

// LDS-resident state: keys / amps arrays and an index hash whose slots hold
// (position + 1), 0 = empty; keys are compared through the keys array.
struct LdsStore {
  u64* keys;
  double* amps;
  int* slots;
  unsigned smask;
  __device__ u64 key(u64 i) const { return keys[i]; }
  __device__ double amp(u64 i) const { return amps[i]; }
  __device__ void set_amp(u64 i, double v) { amps[i] = v; }
  __device__ long long find(u64 k) const {
    unsigned h = (unsigned)mix64(k) & smask;
    while (true) {
      const int v = slots[h];
      if (v == 0) return -1;
      if (keys[v - 1] == k) return (long long)(v - 1);
      h = (h + 1) & smask;
    }
  }
  // The key must already be written at keys[idx].
  __device__ void insert(u64 k, int idx) {
    unsigned h = (unsigned)mix64(k) & smask;
    while (atomicCAS(&slots[h], 0, idx + 1) != 0) h = (h + 1) & smask;
  }
};

struct LdsMu {
  double* p;
  __device__ double get(u64 i) const { return p[i]; }
  __device__ void set(u64 i, double v) { p[i] = v; }
};

// gate_entry for N entries of one thread in the HBM kernels: entry j is
// idx[j] when use[j] (idx[j] < n always).  The entries go through each
// stage together -- keys; first index probes with the entries' own
// amplitudes; partner amplitudes -- so that their memory requests overlap;
// outputs are exactly those of gate_entry.  A T^dagger entry loads its own
// amplitude before knowing whether it owns the pair; when it does not, the
// value (possibly being rewritten by the owner) is discarded unused.
template <int N>
__device__ inline void gate_entries_list(const GlobalStore& S, const u64 (&idx)[N], const bool (&use)[N],
                                         const OpDesc& op, double c, double sn, double eps,
                                         GateOut (&o)[N]) {
  const u64 pair_mask = op.ann | op.cre;
  u64 D[N], partner[N], h[N];
  int kind[N];  // 0: untouched, 1: T acts on D, 2: T^dagger acts on D
  HashSlot sl[N];
  long long jx[N];
  double araw[N], braw[N], own[N];
  // The entries' keys, then every entry's kind and probe position, then the
  // probes: key loads behind a branch, or a probe issued before the next
  // entry's key is used, would make the loads wait for each other.
#pragma unroll
  for (int j = 0; j < N; ++j) D[j] = S.keys[idx[j]];
  __builtin_amdgcn_sched_barrier(0);  // every key load before the first use of a key
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const bool isT = ((D[j] & op.ann) == op.ann) && ((D[j] & op.cre) == 0);
    const bool isTd = ((D[j] & op.cre) == op.cre) && ((D[j] & op.ann) == 0);
    kind[j] = use[j] ? (isT ? 1 : (isTd ? 2 : 0)) : 0;
    partner[j] = D[j] ^ pair_mask;
    h[j] = mix64(partner[j]) & S.hmask;
  }
  // an empty asm statement taking the positions and kinds as inputs keeps
  // them computed here instead of sunk behind an earlier entry's probe
#pragma unroll
  for (int j = 0; j < N; ++j) asm volatile("" : : "v"(h[j]), "v"(kind[j]));
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const u64 i = idx[j];
    if (kind[j]) {
      sl[j] = S.hash[h[j]];
      own[j] = S.amps[i];
    }
  }
#pragma unroll
  for (int j = 0; j < N; ++j) {
    jx[j] = -1;
    if (kind[j]) {
      while (true) {
        if (sl[j].key == partner[j]) {
          jx[j] = (long long)sl[j].idx;
          break;
        }
        if (sl[j].key == kEmptyKey) break;
        h[j] = (h[j] + 1) & S.hmask;
        sl[j] = S.hash[h[j]];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < N; ++j) {
    araw[j] = dead_value();
    braw[j] = dead_value();
    if (kind[j] == 1) {
      araw[j] = own[j];
      if (jx[j] >= 0) braw[j] = S.amps[jx[j]];
    } else if (kind[j] == 2 && jx[j] < 0) {
      braw[j] = own[j];
    }
  }
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const u64 i = idx[j];
    GateOut& r = o[j];
    r = GateOut{false, 0ULL, 0.0, 0, false, kNoEntry, kNoEntry, 0.0, 0.0, 0, kind[j] != 0};
    if (kind[j] == 1) {
      const bool aliveD = !is_dead(araw[j]), aliveX = !is_dead(braw[j]);
      if (aliveD || aliveX) {
        const double s = (double)phase_of_T(op, D[j]);
        const double a = aliveD ? araw[j] : 0.0;
        const double b = aliveX ? braw[j] : 0.0;
        const double nd = c * a - s * (sn * b);
        const double nx = c * b + s * (sn * a);
        const bool keepD = !(fabs(nd) < eps);
        const bool keepX = !(fabs(nx) < eps);
        S.amps[i] = keepD ? nd : dead_value();
        if (jx[j] >= 0) {
          S.amps[jx[j]] = keepX ? nx : dead_value();
        } else if (keepX) {
          r.append = true;
          r.key = partner[j];
          r.val = nx;
        }
        r.dalive = (long long)keepD - (long long)aliveD + (long long)keepX - (long long)aliveX;
        r.active = true;
        r.iD = i;
        r.iX = (jx[j] >= 0) ? (u64)jx[j] : kNoEntry;
        r.a_old = araw[j];
        r.b_old = braw[j];
        r.s = (int)s;
      }
    } else if (kind[j] == 2 && jx[j] < 0 && !is_dead(braw[j])) {
      // D = T partner and the partner is not stored: this thread owns the pair
      const double s = (double)phase_of_T(op, partner[j]);
      const double a = 0.0, b = braw[j];
      const double nd = c * a - s * (sn * b);
      const double nx = c * b + s * (sn * a);
      const bool keepD = !(fabs(nd) < eps);
      const bool keepX = !(fabs(nx) < eps);
      S.amps[i] = keepX ? nx : dead_value();
      if (keepD) {
        r.append = true;
        r.key = partner[j];
        r.val = nd;
      }
      r.dalive = (long long)keepD + (long long)keepX - 1LL;
      r.active = true;
      r.iD = kNoEntry;
      r.iX = i;
      r.a_old = dead_value();
      r.b_old = braw[j];
      r.s = (int)s;
    }
  }
}


// The strided form: entry j is i0 + j * stride, skipped at or beyond n
// (callers pass i0 < n, so the clamped index is valid).
template <int N>
__device__ inline void gate_entries_staged(const GlobalStore& S, u64 n, u64 i0, u64 stride,
                                           const OpDesc& op, double c, double sn, double eps,
                                           GateOut (&o)[N]) {
  u64 idx[N];
  bool use[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const u64 i = i0 + (u64)j * stride;
    use[j] = i < n;
    idx[j] = use[j] ? i : n - 1;
  }
  gate_entries_list<N>(S, idx, use, op, c, sn, eps, o);
}


}  // namespace swcs

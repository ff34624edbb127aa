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
};

// Store: key(i), amp(i), set_amp(i, v), find(key) -> index or -1.
template <class Store>
__device__ inline GateOut gate_entry(Store& S, u64 i, const OpDesc& op, double c, double sn,
                                     double eps) {
  GateOut o{false, 0ULL, 0.0, 0};
  const u64 D = S.key(i);
  const bool isT = ((D & op.ann) == op.ann) && ((D & op.cre) == 0);
  const bool isTd = ((D & op.cre) == op.cre) && ((D & op.ann) == 0);
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
      }
    }
  }
  return o;
}

// Reverse step of one gate for the frozen-support adjoint.  prev(i) is the
// amplitude before the gate (dead if not in that state); mu holds the
// adjoint after the gate (zero outside the kept support) and is overwritten
// with the adjoint before the gate.  Returns this entry's share of
// dE/dtheta = <mu | P U'(theta) psi_prev>, U' the derivative of the rotation.
template <class Keys, class Prev, class Mu>
__device__ inline double adjoint_entry(const Keys& K, const Prev& prev, Mu& mu, u64 i,
                                       const OpDesc& op, double c, double sn) {
  const u64 D = K.key(i);
  const bool isT = ((D & op.ann) == op.ann) && ((D & op.cre) == 0);
  const bool isTd = ((D & op.cre) == op.cre) && ((D & op.ann) == 0);
  const u64 pair_mask = op.ann | op.cre;
  if (isT) {
    const u64 X = D ^ pair_mask;
    const long long j = K.find(X);
    const double araw = prev(i);
    const double braw = (j >= 0) ? prev((u64)j) : dead_value();
    const bool aliveD = !is_dead(araw), aliveX = !is_dead(braw);
    if (!aliveD && !aliveX) return 0.0;
    const double s = (double)phase_of_T(op, D);
    const double a = aliveD ? araw : 0.0, b = aliveX ? braw : 0.0;
    const double muD = mu.get(i);
    const double muX = (j >= 0) ? mu.get((u64)j) : 0.0;
    mu.set(i, aliveD ? (c * muD + s * sn * muX) : 0.0);
    if (j >= 0) mu.set((u64)j, aliveX ? (c * muX - s * sn * muD) : 0.0);
    return muD * (-sn * a - s * c * b) + muX * (-sn * b + s * c * a);
  }
  if (isTd) {
    const u64 Dsrc = D ^ pair_mask;
    if (K.find(Dsrc) >= 0) return 0.0;  // the thread of Dsrc owns the pair
    const double braw = prev(i);
    if (is_dead(braw)) return 0.0;
    const double muX = mu.get(i);
    mu.set(i, c * muX);
    return muX * (-sn * braw);
  }
  return 0.0;
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

struct GlobalPrev {
  const double* p;
  __device__ double operator()(u64 i) const { return p[i]; }
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

}  // namespace swcs

// Gates of spin-complemented generators whose two parts overlap (Sec. III):
// G = A1 + s A2 for pool rows 1 and 2 (A_i = T_i - T_i^dagger, s = +-1) that
// share spin-orbitals, e.g. an opposite-spin double with p = q and its spin
// complement.  exp(theta G) is applied exactly with one parameter.
//
// G links each determinant to at most two others, in two shapes:
//   pair {D, X}: one row (or its adjoint) acts on D and nothing else links X;
//     the usual rotation, at angle theta for row 1 and s theta for row 2;
//   star {C, L1, L2}: both rows act on C, G C = alpha L1 + beta L2 (alpha,
//     beta = +-1), G L1 = -alpha C, G L2 = -beta C.  G^2 C = -2 C, so on the
//     star exp(theta G) turns C and u = (alpha x1 + beta x2) / sqrt(2) at
//     frequency sqrt(2) theta and keeps the leaf combination orthogonal to u:
//       xc' = c2 xc - s2 u,  u' = s2 xc + c2 u,
//       x1' = x1 + alpha (u' - u) / sqrt(2),  x2' = x2 + beta (u' - u) / sqrt(2)
//     (c2 = cos(sqrt(2) theta), s2 = sin(sqrt(2) theta)).
// Every determinant finds its shape from its own key: a star centre is acted
// on by both rows; the partner of a determinant acted on by one row is a star
// centre exactly when the other row acts on the partner.
//
// Ownership (race-free in-place update, as for one-row gates): a pair is
// updated by the thread of its source (the member the row's T acts on) when
// that is stored, else by the other member's; a star by its centre's thread
// when the centre is stored, else by the thread of the stored leaf with the
// smaller key.  The owner writes every stored member and appends the absent
// members that survive pruning (at most two per component).
#include "gate_ops.h"

namespace swcs {

// +1: T acts on D; -1: T^dagger acts on D; 0: neither.
__device__ inline int op_acts(const OpDesc& op, u64 D) {
  if (((D & op.ann) == op.ann) && ((D & op.cre) == 0)) return 1;
  if (((D & op.cre) == op.cre) && ((D & op.ann) == 0)) return -1;
  return 0;
}

// <Y|f A|D> for the row acting on D as `act` (Y its image): +f <Y|T|D>, or
// -f <Y|T^dagger|D> = -f <D|T|Y>.
__device__ inline double op_coef(const OpDesc& op, int act, u64 D, double f) {
  const u64 Y = D ^ (op.ann | op.cre);
  return act > 0 ? f * (double)phase_of_T(op, D) : -f * (double)phase_of_T(op, Y);
}

struct GenOut {
  int napp;
  u64 key[2];
  double val[2];
  long long dalive;
  int kind;  // 0 nothing to log, 1 pair, 2 star
  PairRec pr;
  StarRec sr;
};

__device__ inline unsigned rec_index(long long j) { return j >= 0 ? (unsigned)j : 0xffffffffu; }

template <class Store>
__device__ inline void gen_pair(Store& S, double eps, u64 src, long long js, u64 dst, long long jd, int s,
                                double c, double snr, double sg, GenOut& o) {
  const double araw = js >= 0 ? S.amp((u64)js) : dead_value();
  const double braw = jd >= 0 ? S.amp((u64)jd) : dead_value();
  const bool aliveS = !is_dead(araw), aliveD = !is_dead(braw);
  if (!aliveS && !aliveD) return;
  const double sp = (double)s;
  const double a = aliveS ? araw : 0.0, b = aliveD ? braw : 0.0;
  const double ns = c * a - sp * (snr * b);
  const double nd = c * b + sp * (snr * a);
  const bool keepS = !(fabs(ns) < eps), keepD = !(fabs(nd) < eps);
  if (js >= 0) S.set_amp((u64)js, keepS ? ns : dead_value());
  else if (keepS) { o.key[o.napp] = src; o.val[o.napp++] = ns; }
  if (jd >= 0) S.set_amp((u64)jd, keepD ? nd : dead_value());
  else if (keepD) { o.key[o.napp] = dst; o.val[o.napp++] = nd; }
  o.dalive = (long long)keepS - (long long)aliveS + (long long)keepD - (long long)aliveD;
  o.kind = 1;
  o.pr.iD = rec_index(js);
  o.pr.iX = rec_index(jd);
  o.pr.s = (int)(sp * sg);  // the second row turns by s theta: its sign folded in
  o.pr.pad = 0;
  o.pr.a_old = araw;
  o.pr.b_old = braw;
}

template <class Store>
__device__ inline void gen_star(Store& S, const GenGate& g, double eps, u64 C, long long jc, u64 L1,
                                long long j1, u64 L2, long long j2, double al, double be, GenOut& o) {
  const double craw = jc >= 0 ? S.amp((u64)jc) : dead_value();
  const double r1 = j1 >= 0 ? S.amp((u64)j1) : dead_value();
  const double r2 = j2 >= 0 ? S.amp((u64)j2) : dead_value();
  const bool aC = !is_dead(craw), a1 = !is_dead(r1), a2 = !is_dead(r2);
  if (!aC && !a1 && !a2) return;
  const double xc = aC ? craw : 0.0, x1 = a1 ? r1 : 0.0, x2 = a2 ? r2 : 0.0;
  const double u = (al * x1 + be * x2) * g.rt;
  const double nc = g.c2 * xc - g.s2 * u;
  const double nu = g.s2 * xc + g.c2 * u;
  const double du = nu - u;
  const double n1 = x1 + al * (g.rt * du);
  const double n2 = x2 + be * (g.rt * du);
  const bool kC = !(fabs(nc) < eps), k1 = !(fabs(n1) < eps), k2 = !(fabs(n2) < eps);
  if (jc >= 0) S.set_amp((u64)jc, kC ? nc : dead_value());
  else if (kC) { o.key[o.napp] = C; o.val[o.napp++] = nc; }
  if (j1 >= 0) S.set_amp((u64)j1, k1 ? n1 : dead_value());
  else if (k1) { o.key[o.napp] = L1; o.val[o.napp++] = n1; }
  if (j2 >= 0) S.set_amp((u64)j2, k2 ? n2 : dead_value());
  else if (k2) { o.key[o.napp] = L2; o.val[o.napp++] = n2; }
  o.dalive = (long long)kC - (long long)aC + (long long)k1 - (long long)a1 + (long long)k2 - (long long)a2;
  o.kind = 2;
  o.sr.iC = rec_index(jc);
  o.sr.i1 = rec_index(j1);
  o.sr.i2 = rec_index(j2);
  o.sr.al = (signed char)(al > 0.0 ? 1 : -1);
  o.sr.be = (signed char)(be > 0.0 ? 1 : -1);
  o.sr.xc = craw;
  o.sr.x1 = r1;
  o.sr.x2 = r2;
}

// The update of stored entry i (see the ownership rule above).  At most one
// absent member of a pair, or two of a star, is returned for appending.
template <class Store>
__device__ inline GenOut gen_entry(Store& S, u64 i, const GenGate& g, double eps) {
  GenOut o;
  o.napp = 0;
  o.dalive = 0;
  o.kind = 0;
  const u64 D = S.key(i);
  const int a1 = op_acts(g.op1, D), a2 = op_acts(g.op2, D);
  if (!a1 && !a2) return o;
  const u64 m1 = g.op1.ann | g.op1.cre, m2 = g.op2.ann | g.op2.cre;
  if (a1 && a2) {
    const u64 L1 = D ^ m1, L2 = D ^ m2;
    gen_star(S, g, eps, D, (long long)i, L1, S.find(L1), L2, S.find(L2), op_coef(g.op1, a1, D, 1.0),
             op_coef(g.op2, a2, D, g.sg), o);
    return o;
  }
  const bool one = a1 != 0;
  const OpDesc& op = one ? g.op1 : g.op2;
  const OpDesc& ot = one ? g.op2 : g.op1;
  const u64 P = D ^ (one ? m1 : m2);
  const int ao = op_acts(ot, P);
  if (ao) {
    // D is a leaf of the star centred at P
    if (S.find(P) >= 0) return o;  // the centre owns it
    const u64 Lo = P ^ (one ? m2 : m1);
    const long long jo = S.find(Lo);
    if (jo >= 0 && Lo < D) return o;  // the other leaf owns it
    const int ar = op_acts(op, P);
    const double al = one ? op_coef(g.op1, ar, P, 1.0) : op_coef(g.op1, ao, P, 1.0);
    const double be = one ? op_coef(g.op2, ao, P, g.sg) : op_coef(g.op2, ar, P, g.sg);
    if (one) gen_star(S, g, eps, P, -1, D, (long long)i, Lo, jo, al, be, o);
    else gen_star(S, g, eps, P, -1, Lo, jo, D, (long long)i, al, be, o);
    return o;
  }
  const int a = one ? a1 : a2;
  const double snr = one ? g.sn : g.sn2;
  const double sg = one ? 1.0 : g.sg;
  if (a > 0) {
    gen_pair(S, eps, D, (long long)i, P, S.find(P), phase_of_T(op, D), g.c, snr, sg, o);
  } else {
    if (S.find(P) >= 0) return o;  // the source owns the pair
    gen_pair(S, eps, P, -1, D, (long long)i, phase_of_T(op, P), g.c, snr, sg, o);
  }
  return o;
}

// Wave-aggregated slot reservation: every lane of the wave calls it; lanes
// with `want` get consecutive slots counted on *counter.
__device__ inline u64 wave_reserve(bool want, u64* counter) {
  const u64 m = __ballot(want);
  if (!m) return 0;
  const int lane = __lane_id();
  const int leader = __ffsll((long long)m) - 1;
  u64 b = 0;
  if (lane == leader) b = atomicAdd((unsigned long long*)counter, (unsigned long long)__popcll(m));
  b = __shfl(b, leader);
  return b + (u64)__popcll(m & ((1ULL << lane) - 1ULL));
}

constexpr int kGenThreads = 256;

// Forward gate: the same stop / fold protocol as k_gate (appends of a star
// gate are bounded by twice the alive count).
__global__ void __launch_bounds__(kGenThreads)
k_gen_gate(u64* __restrict__ keys, double* __restrict__ amps, HashSlot* __restrict__ hash, u64 hmask,
           u64 cap, Counters* __restrict__ ctr, GenGate g, double eps, u64* __restrict__ gate_n_in,
           int check_cap, unsigned gate_index, u64 max_keys, u64* __restrict__ gate_n_act) {
  __shared__ int s_run;
  __shared__ u64 s_n_in;
  __shared__ long long s_wsum[kGenThreads / 64];
  __shared__ bool is_last;
  if (threadIdx.x == 0) {
    int run = 1;
    const unsigned fl = __hip_atomic_load(&ctr->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const u64 n_in = __hip_atomic_load(&ctr->n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (fl & kFlagStopped) {
      run = 0;
    } else if (check_cap) {
      const u64 alive_in = __hip_atomic_load(&ctr->alive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const u64 room = max_keys > n_in ? max_keys - n_in : 0;
      if (n_in + (2 * alive_in < room ? 2 * alive_in : room) > cap) {
        run = 0;
        if (blockIdx.x == 0) {
          ctr->stop_gate = gate_index;
          atomicOr(&ctr->flags, kFlagStopped);
        }
      }
    }
    s_run = run;
    s_n_in = n_in;
  }
  __syncthreads();
  if (!s_run) return;
  const u64 n_in = s_n_in;
  GlobalStore S{keys, amps, hash, hmask};
  long long dalive = 0;
  unsigned nact = 0;
  const u64 stride = (u64)gridDim.x * kGenThreads;
  for (u64 base = (u64)blockIdx.x * kGenThreads; base < n_in; base += stride) {
    const u64 i = base + threadIdx.x;
    GenOut o;
    o.napp = 0;
    o.dalive = 0;
    if (i < n_in) {
      const u64 D = keys[i];
      nact += (op_acts(g.op1, D) || op_acts(g.op2, D)) ? 1u : 0u;
      o = gen_entry(S, i, g, eps);
    }
    dalive += o.dalive;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const bool want = o.napp > a;
      const u64 slot = wave_reserve(want, &ctr->app);
      if (want) {
        const u64 idx = n_in + slot;
        if (idx < cap) {
          keys[idx] = o.key[a];
          amps[idx] = o.val[a];
          hash_insert_new(hash, hmask, o.key[a], idx);
        } else {
          atomicOr(&ctr->flags, kFlagOverflow);
        }
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    dalive += __shfl_xor(dalive, off);
    nact += __shfl_xor(nact, off);
  }
  __shared__ unsigned s_nact[kGenThreads / 64];
  if (__lane_id() == 0) {
    s_wsum[threadIdx.x / 64] = dalive;
    s_nact[threadIdx.x / 64] = nact;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long d = 0;
    u64 na = 0;
    for (int w = 0; w < kGenThreads / 64; ++w) {
      d += s_wsum[w];
      na += s_nact[w];
    }
    if (gate_n_act && na) atomicAdd((unsigned long long*)gate_n_act, (unsigned long long)na);
    if (d != 0) atomicAdd((unsigned long long*)&ctr->dalive, (unsigned long long)d);
    __threadfence();
    const unsigned tk = atomicAdd(&ctr->ticket, 1u);
    is_last = (tk == gridDim.x - 1);
  }
  __syncthreads();
  if (is_last && threadIdx.x == 0) {
    __threadfence();
    const u64 app = atomicAdd(&ctr->app, 0ULL);
    const long long da = (long long)atomicAdd((unsigned long long*)&ctr->dalive, 0ULL);
    const u64 alive = ctr->alive;
    if (gate_n_in) *gate_n_in = alive;
    ctr->n = n_in + (app < cap - n_in ? app : cap - n_in);
    ctr->alive = (u64)((long long)alive + da);
    ctr->app = 0;
    ctr->dalive = 0;
    __threadfence();
    ctr->ticket = 0;
  }
}

// Replay inside the adjoint's recomputation: the forward update on a working
// copy of the amplitudes over the final keys (every reachable key is stored,
// so nothing is appended), logging one PairRec per updated pair and one
// StarRec per updated star.
__global__ void __launch_bounds__(kGenThreads)
k_gen_replay(const u64* __restrict__ keys, double* __restrict__ amps, const HashSlot* __restrict__ hash,
             u64 hmask, u64 n, GenGate g, double eps, PairRec* __restrict__ plog, u64* __restrict__ pcount,
             StarRec* __restrict__ slog, u64* __restrict__ scount, unsigned* __restrict__ flags) {
  GlobalStore S{(u64*)keys, amps, (HashSlot*)hash, hmask};
  const u64 stride = (u64)gridDim.x * kGenThreads;
  for (u64 base = (u64)blockIdx.x * kGenThreads; base < n; base += stride) {
    const u64 i = base + threadIdx.x;
    GenOut o;
    o.napp = 0;
    o.kind = 0;
    if (i < n) o = gen_entry(S, i, g, eps);
    if (o.napp) atomicOr(flags, kFlagOverflow);
    const u64 ps = wave_reserve(o.kind == 1, pcount);
    if (o.kind == 1) plog[ps] = o.pr;
    const u64 ss = wave_reserve(o.kind == 2, scount);
    if (o.kind == 2) slog[ss] = o.sr;
  }
}

// Reverse step of the logged stars: dE/dtheta += mu . (G U x_old) over the
// members (U = exp(theta G)), and mu <- U^T mu = exp(-theta G) mu restricted
// to the members alive before the gate.  Block sums are added to
// partial[blockIdx.x] (written by the pairs' reverse step of the same gate).
__global__ void __launch_bounds__(256)
k_adjoint_star(const StarRec* __restrict__ slog, const u64* __restrict__ scount, double* __restrict__ mu,
               GenGate g, double* __restrict__ partial) {
  const u64 cnt = *scount;
  double acc = 0.0;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x; r < cnt; r += stride) {
    const StarRec s = slog[r];
    const double al = (double)s.al, be = (double)s.be;
    const bool aC = !is_dead(s.xc), a1 = !is_dead(s.x1), a2 = !is_dead(s.x2);
    const double xc = aC ? s.xc : 0.0, x1 = a1 ? s.x1 : 0.0, x2 = a2 ? s.x2 : 0.0;
    const double u = (al * x1 + be * x2) * g.rt;
    const double nc = g.c2 * xc - g.s2 * u;
    const double nu = g.s2 * xc + g.c2 * u;
    const double du = nu - u;
    const double n1 = x1 + al * (g.rt * du);
    const double n2 = x2 + be * (g.rt * du);
    const double mc = s.iC != 0xffffffffu ? mu[s.iC] : 0.0;
    const double m1 = s.i1 != 0xffffffffu ? mu[s.i1] : 0.0;
    const double m2 = s.i2 != 0xffffffffu ? mu[s.i2] : 0.0;
    acc += mc * (-(al * n1 + be * n2)) + m1 * (al * nc) + m2 * (be * nc);
    const double v = (al * m1 + be * m2) * g.rt;
    const double bc = g.c2 * mc + g.s2 * v;
    const double bv = -g.s2 * mc + g.c2 * v;
    const double dv = bv - v;
    if (s.iC != 0xffffffffu) mu[s.iC] = aC ? bc : 0.0;
    if (s.i1 != 0xffffffffu) mu[s.i1] = a1 ? m1 + al * (g.rt * dv) : 0.0;
    if (s.i2 != 0xffffffffu) mu[s.i2] = a2 ? m2 + be * (g.rt * dv) : 0.0;
  }
  __shared__ double sacc[256];
  sacc[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sacc[threadIdx.x] += sacc[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] += sacc[0];
}

hipError_t launch_gen_gate(const DeviceState& st, const GenGate& g, double eps, u64* gate_n_in,
                           unsigned gate_index, u64 max_keys, int grid, hipStream_t stream, u64* gate_n_act) {
  hipLaunchKernelGGL(k_gen_gate, dim3(grid), dim3(kGenThreads), 0, stream, st.keys, st.amps, st.hash,
                     st.hmask, st.cap, st.ctr, g, eps, gate_n_in, 1, gate_index, max_keys, gate_n_act);
  return hipGetLastError();
}

hipError_t launch_gen_replay(const DeviceState& st, double* amps, u64 n, const GenGate& g, double eps,
                             PairRec* plog, u64* pcount, StarRec* slog, u64* scount, int grid,
                             hipStream_t stream) {
  hipLaunchKernelGGL(k_gen_replay, dim3(grid), dim3(kGenThreads), 0, stream, st.keys, amps, st.hash,
                     st.hmask, n, g, eps, plog, pcount, slog, scount, &st.ctr->flags);
  return hipGetLastError();
}

hipError_t launch_adjoint_star(const StarRec* slog, const u64* scount, double* mu, const GenGate& g,
                               double* partial, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(k_adjoint_star, dim3(grid), dim3(256), 0, stream, slog, scount, mu, g, partial);
  return hipGetLastError();
}

}  // namespace swcs

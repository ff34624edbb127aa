// Single-workgroup kernels that keep a small state in LDS and run a whole
// gate chain (or the whole adjoint sweep) in one launch.  A state of up to
// kLdsCap determinants (16 B of keys and amplitudes plus 8 B of hash index
// each) fits the 160 KB LDS of one CU; the gates then cost LDS latency
// instead of one kernel launch each.  The per-entry arithmetic is shared
// with the HBM kernels (gate_ops.h), so results are identical bit for bit.
#include "gate_ops.h"

namespace swcs {

constexpr int kChainThreads = 1024;
constexpr int kGateChunk = 256;  // gate descriptors staged in LDS at a time

// Deterministic block sum (fixed order over the 16 waves).
__device__ inline double block_sum_1024(double v, double* wsum) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  if (lane == 0) wsum[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kChainThreads / 64; ++w) r += wsum[w];
  __syncthreads();
  return r;  // valid in thread 0
}

// Keep only the ncut alive entries of amps[0, n) that come first in the N_CUT
// order (gate_ops.h); the rest are marked dead.  Called by all threads of
// the block; returns the number of entries dropped (valid in every thread).
__device__ inline unsigned lds_ncut(double* amps, const u64* keys, unsigned n, unsigned ncut,
                                    NcutState& st) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    st.phi = st.plo = st.mhi = st.mlo = 0;
    st.k = ncut;
    st.skip = 0;
    st.pad[0] = 0;
  }
  for (int d = 0; d < 16; ++d) {
    if (tid < 256) st.hist[tid] = 0;
    __syncthreads();
    if (st.skip) break;
    for (unsigned i = tid; i < n; i += kChainThreads) {
      const double a = amps[i];
      if (is_dead(a)) continue;
      u64 hi, lo;
      ncut_value(a, keys[i], &hi, &lo);
      if (ncut_matches(st, hi, lo)) atomicAdd(&st.hist[ncut_digit(hi, lo, d)], 1u);
    }
    __syncthreads();
    if (tid == 0) ncut_pick(st, d);
    __syncthreads();
  }
  if (st.skip) return 0;
  // st.phi / st.plo is now the ncut-th largest value; drop everything below.
  unsigned dropped = 0;
  for (unsigned i = tid; i < n; i += kChainThreads) {
    const double a = amps[i];
    if (is_dead(a)) continue;
    u64 hi, lo;
    ncut_value(a, keys[i], &hi, &lo);
    if (hi < st.phi || (hi == st.phi && lo < st.plo)) {
      amps[i] = dead_value();
      ++dropped;
    }
  }
  if (tid == 0) st.pad[0] = 0;
  __syncthreads();
  if (dropped) atomicAdd(&st.pad[0], dropped);
  __syncthreads();
  const unsigned tot = st.pad[0];
  __syncthreads();
  return tot;
}

// Forward chain of gates [g0, M) on the state held in keys / amps (HBM),
// moved into LDS for the duration.  Checkpoints (amplitudes before gate g
// for g % seg == 0) and the per-gate input sizes are written to HBM.  If a
// gate might not fit, the kernel stops before it: the state is written back
// and ctr->stop_gate / kFlagStopped tell the host where to continue.
template <int CAP>
__global__ void __launch_bounds__(kChainThreads)
k_chain_lds(u64* __restrict__ keys, double* __restrict__ amps, Counters* __restrict__ ctr,
            const GateDesc* __restrict__ gates, int g0, int M, double eps, int prune_first,
            double* const* __restrict__ ckpt, u64* __restrict__ ckpt_n, int seg,
            u64* __restrict__ gate_n_in, u64 max_keys, unsigned ncut) {
  __shared__ NcutState nst;
  __shared__ u64 skeys[CAP];
  __shared__ double samps[CAP];
  __shared__ int sslots[2 * CAP];
  __shared__ unsigned s_n, s_app, s_alive;
  __shared__ int s_dalive;
  __shared__ int s_stop;
  __shared__ GateDesc sg[kGateChunk];
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_n = (unsigned)ctr->n;
    s_alive = (unsigned)ctr->alive;
    s_app = 0;
    s_dalive = 0;
    s_stop = -1;
  }
  for (int t = tid; t < 2 * CAP; t += kChainThreads) sslots[t] = 0;
  __syncthreads();
  const unsigned n0 = s_n;
  if (n0 > (unsigned)CAP) {
    if (tid == 0) {
      ctr->stop_gate = (u64)g0;
      atomicOr(&ctr->flags, kFlagStopped);
    }
    return;
  }
  for (unsigned i = tid; i < n0; i += kChainThreads) {
    skeys[i] = keys[i];
    samps[i] = amps[i];
  }
  __syncthreads();
  LdsStore S{skeys, samps, sslots, 2u * CAP - 1u};
  for (unsigned i = tid; i < n0; i += kChainThreads) S.insert(skeys[i], (int)i);
  __syncthreads();
  for (int g = g0; g < M; ++g) {
    if ((g - g0) % kGateChunk == 0) {
      // stage the next chunk of gate descriptors (all earlier reads of sg done)
      __syncthreads();
      for (int t = tid; t < kGateChunk && g + t < M; t += kChainThreads) sg[t] = gates[g + t];
      __syncthreads();
    }
    const unsigned n = s_n, alive = s_alive;
    if (ckpt && g % seg == 0) {
      double* dst = ckpt[g / seg];
      for (unsigned i = tid; i < n; i += kChainThreads) dst[i] = samps[i];
      if (tid == 0) ckpt_n[g / seg] = n;
    }
    const u64 room = max_keys > n ? max_keys - n : 0;
    if ((u64)n + ((u64)alive < room ? (u64)alive : room) > (u64)CAP) {
      if (tid == 0) s_stop = g;
      break;  // uniform: every thread read the same n and alive
    }
    const GateDesc gd = sg[(g - g0) % kGateChunk];
    int dal = 0;
    for (unsigned i = tid; i < n; i += kChainThreads) {
      const GateOut o = gate_entry(S, i, gd.op, gd.c, gd.s, eps);
      dal += (int)o.dalive;
      if (o.append) {
        const unsigned idx = n + atomicAdd(&s_app, 1u);
        skeys[idx] = o.key;
        samps[idx] = o.val;
        __threadfence_block();
        S.insert(o.key, (int)idx);
      }
    }
    if (dal) atomicAdd(&s_dalive, dal);
    __syncthreads();
    if (tid == 0) {
      if (gate_n_in) gate_n_in[g] = alive;
      s_n = n + s_app;
      s_alive = (unsigned)((int)alive + s_dalive);
      s_app = 0;
      s_dalive = 0;
    }
    __syncthreads();
    if (ncut && s_alive > ncut) {
      const unsigned dropped = lds_ncut(samps, skeys, s_n, ncut, nst);
      if (tid == 0) s_alive -= dropped;
      __syncthreads();
    }
    if (g == 0 && prune_first) {
      // Entries of a caller-supplied starting state that the first gate did
      // not touch have not been tested against eps yet.
      const unsigned n1 = s_n;
      int dropped = 0;
      for (unsigned i = tid; i < n1; i += kChainThreads) {
        const double a = samps[i];
        if (!is_dead(a) && fabs(a) < eps) {
          samps[i] = dead_value();
          ++dropped;
        }
      }
      if (dropped) atomicSub(&s_alive, (unsigned)dropped);
      __syncthreads();
    }
  }
  __syncthreads();
  const unsigned n = s_n;
  for (unsigned i = tid; i < n; i += kChainThreads) {
    keys[i] = skeys[i];
    amps[i] = samps[i];
  }
  if (tid == 0) {
    ctr->n = n;
    ctr->alive = s_alive;
    if (s_stop >= 0) {
      ctr->stop_gate = (u64)s_stop;
      atomicOr(&ctr->flags, kFlagStopped);
    }
  }
}

// Whole frozen-support adjoint sweep for a final state of n <= CAP stored
// determinants.  For each segment (last first): restore the checkpoint into
// LDS, replay the segment's gates logging one PairRec per active pair (HBM
// scratch, seg * n records at most), then run the reverse steps over the
// logged pairs with the adjoint vector mu held in LDS.  dE[g] is a block sum
// in a fixed wave order.
constexpr int kMaxSeg = 256;

template <int CAP>
__global__ void __launch_bounds__(kChainThreads)
k_adjoint_lds(const u64* __restrict__ keys, unsigned n, const GateDesc* __restrict__ gates, int M,
              int seg, double eps, const double* const* __restrict__ ckpt,
              const u64* __restrict__ ckpt_n, const double* __restrict__ mu_init,
              PairRec* __restrict__ logbuf, double* __restrict__ dE, unsigned* __restrict__ flags,
              unsigned ncut) {
  __shared__ NcutState nst;
  __shared__ u64 skeys[CAP];
  __shared__ double sW[CAP];
  __shared__ double smu[CAP];
  __shared__ int sslots[2 * CAP];
  __shared__ double wsum[kChainThreads / 64];
  __shared__ unsigned cnt[kMaxSeg];
  __shared__ GateDesc sg[kMaxSeg];
  const int tid = threadIdx.x;
  for (int t = tid; t < 2 * CAP; t += kChainThreads) sslots[t] = 0;
  for (int t = tid; t < kMaxSeg; t += kChainThreads) cnt[t] = 0;
  for (unsigned i = tid; i < n; i += kChainThreads) {
    skeys[i] = keys[i];
    smu[i] = mu_init[i];
  }
  __syncthreads();
  LdsStore L{skeys, sW, sslots, 2u * CAP - 1u};
  for (unsigned i = tid; i < n; i += kChainThreads) L.insert(skeys[i], (int)i);
  __syncthreads();
  LdsMu mu{smu};
  const int nseg = (M + seg - 1) / seg;
  for (int j = nseg - 1; j >= 0; --j) {
    const int g_lo = j * seg;
    const int g_hi = (g_lo + seg < M) ? g_lo + seg : M;
    const int len = g_hi - g_lo;
    const unsigned nj = (unsigned)ckpt_n[j];
    const double* src = ckpt[j];
    for (unsigned i = tid; i < n; i += kChainThreads) sW[i] = (i < nj) ? src[i] : dead_value();
    for (int t = tid; t < len; t += kChainThreads) sg[t] = gates[g_lo + t];
    __syncthreads();
    for (int t = 0; t < len; ++t) {
      const GateDesc gd = sg[t];
      PairRec* lg = logbuf + (size_t)t * n;
      for (unsigned i = tid; i < n; i += kChainThreads) {
        const GateOut o = gate_entry(L, i, gd.op, gd.c, gd.s, eps);
        if (o.append) atomicOr(flags, kFlagOverflow);  // cannot happen: all keys are stored
        if (o.active) lg[atomicAdd(&cnt[t], 1u)] = make_rec(o);
      }
      __syncthreads();
      if (ncut) lds_ncut(sW, skeys, n, ncut, nst);
    }
    // Reverse over the segment's logs; each thread's first record of the
    // next (earlier) gate is loaded while the current gate is processed.
    PairRec cur{};
    bool has = false;
    if (len > 0 && (unsigned)tid < cnt[len - 1]) {
      cur = logbuf[(size_t)(len - 1) * n + tid];
      has = true;
    }
    for (int t = len - 1; t >= 0; --t) {
      const GateDesc gd = sg[t];
      const PairRec* lg = logbuf + (size_t)t * n;
      const unsigned c = cnt[t];
      PairRec nxt{};
      bool has_next = false;
      if (t > 0 && (unsigned)tid < cnt[t - 1]) {
        nxt = logbuf[(size_t)(t - 1) * n + tid];
        has_next = true;
      }
      double acc = 0.0;
      if (has) acc += adjoint_pair(cur, mu, gd.c, gd.s);
      for (unsigned r = tid + kChainThreads; r < c; r += kChainThreads) acc += adjoint_pair(lg[r], mu, gd.c, gd.s);
      __syncthreads();
      const double tot = block_sum_1024(acc, wsum);
      if (tid == 0) dE[g_lo + t] = tot;
      cur = nxt;
      has = has_next;
    }
    for (int t = tid; t < len; t += kChainThreads) cnt[t] = 0;
    __syncthreads();
  }
}

int lds_chain_capacity() { return kLdsCap; }

hipError_t launch_chain_lds(const DeviceState& st, const GateDesc* gates, int g0, int M, double eps,
                            int prune_first, double* const* ckpt, u64* ckpt_n, int seg,
                            u64* gate_n_in, u64 max_keys, unsigned ncut, hipStream_t stream) {
  hipLaunchKernelGGL(k_chain_lds<kLdsCap>, dim3(1), dim3(kChainThreads), 0, stream, st.keys,
                     st.amps, st.ctr, gates, g0, M, eps, prune_first, ckpt, ckpt_n, seg, gate_n_in,
                     max_keys, ncut);
  return hipGetLastError();
}

int lds_adjoint_max_segment() { return kMaxSeg; }

hipError_t launch_adjoint_lds(const u64* keys, unsigned n, const GateDesc* gates, int M, int seg,
                              double eps, const double* const* ckpt, const u64* ckpt_n,
                              const double* mu_init, PairRec* logbuf, double* dE, unsigned* flags,
                              unsigned ncut, hipStream_t stream) {
  if (seg > kMaxSeg) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_adjoint_lds<kLdsCap>, dim3(1), dim3(kChainThreads), 0, stream, keys, n, gates,
                     M, seg, eps, ckpt, ckpt_n, mu_init, logbuf, dE, flags, ncut);
  return hipGetLastError();
}

}  // namespace swcs

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
  // Per-gate append and alive-change counters, three in rotation: gate g
  // uses slot g % 3; after the gate's barrier every thread reads it, and
  // thread 0 clears slot (g + 2) % 3, last read before the previous barrier
  // and next used after the following one.
  __shared__ unsigned s_app[3];
  __shared__ int s_dal[3];
  __shared__ unsigned s_n0, s_alive0;
  __shared__ GateDesc sg[kGateChunk];
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_n0 = (unsigned)ctr->n;
    s_alive0 = (unsigned)ctr->alive;
  }
  if (tid < 3) {
    s_app[tid] = 0;
    s_dal[tid] = 0;
  }
  for (int t = tid; t < 2 * CAP; t += kChainThreads) sslots[t] = 0;
  __syncthreads();
  unsigned n = s_n0, alive = s_alive0;  // block-uniform, kept in every thread
  if (n > (unsigned)CAP) {
    if (tid == 0) {
      ctr->stop_gate = (u64)g0;
      atomicOr(&ctr->flags, kFlagStopped);
    }
    return;
  }
  for (unsigned i = tid; i < n; i += kChainThreads) {
    skeys[i] = keys[i];
    samps[i] = amps[i];
  }
  __syncthreads();
  LdsStore S{skeys, samps, sslots, 2u * CAP - 1u};
  for (unsigned i = tid; i < n; i += kChainThreads) S.insert(skeys[i], (int)i);
  int stop = -1;
  for (int g = g0; g < M; ++g) {
    // Every earlier read of sg and every write of the previous gate happened
    // before the previous gate's barrier (or the index build's).
    if ((g - g0) % kGateChunk == 0) {
      for (int t = tid; t < kGateChunk && g + t < M; t += kChainThreads) sg[t] = gates[g + t];
      __syncthreads();
    }
    if (ckpt && g % seg == 0) {
      double* dst = ckpt[g / seg];
      for (unsigned i = tid; i < n; i += kChainThreads) dst[i] = samps[i];
      if (tid == 0) ckpt_n[g / seg] = n;
      __syncthreads();  // the copy precedes the gate's updates
    }
    const u64 room = max_keys > n ? max_keys - n : 0;
    if ((u64)n + ((u64)alive < room ? (u64)alive : room) > (u64)CAP) {
      stop = g;
      break;  // uniform: every thread holds the same n and alive
    }
    const int slot = g % 3;
    const GateDesc gd = sg[(g - g0) % kGateChunk];
    int dal = 0;
    for (unsigned i = tid; i < n; i += kChainThreads) {
      const GateOut o = gate_entry(S, i, gd.op, gd.c, gd.s, eps);
      dal += (int)o.dalive;
      if (o.append) {
        const unsigned idx = n + atomicAdd(&s_app[slot], 1u);
        skeys[idx] = o.key;
        samps[idx] = o.val;
        __threadfence_block();
        S.insert(o.key, (int)idx);
      }
    }
    if (dal) atomicAdd(&s_dal[slot], dal);
    __syncthreads();
    if (tid == 0) {
      if (gate_n_in) gate_n_in[g] = alive;
      s_app[(g + 2) % 3] = 0;
      s_dal[(g + 2) % 3] = 0;
    }
    n += s_app[slot];
    alive = (unsigned)((int)alive + s_dal[slot]);
    if (ncut && alive > ncut) alive -= lds_ncut(samps, skeys, n, ncut, nst);
    if (g == 0 && prune_first) {
      // Entries of a caller-supplied starting state that the first gate did
      // not touch have not been tested against eps yet.
      if (tid == 0) nst.pad[1] = 0;
      __syncthreads();
      unsigned dropped = 0;
      for (unsigned i = tid; i < n; i += kChainThreads) {
        const double a = samps[i];
        if (!is_dead(a) && fabs(a) < eps) {
          samps[i] = dead_value();
          ++dropped;
        }
      }
      if (dropped) atomicAdd(&nst.pad[1], dropped);
      __syncthreads();
      alive -= nst.pad[1];
    }
  }
  __syncthreads();
  for (unsigned i = tid; i < n; i += kChainThreads) {
    keys[i] = skeys[i];
    amps[i] = samps[i];
  }
  if (tid == 0) {
    ctr->n = n;
    ctr->alive = alive;
    if (stop >= 0) {
      ctr->stop_gate = (u64)stop;
      atomicOr(&ctr->flags, kFlagStopped);
    }
  }
}

// Frozen-support adjoint sweep for a final state of n <= CAP stored
// determinants, in two launches.  (1) One workgroup per checkpoint segment
// restores the segment's checkpoint into LDS and replays its gates, logging
// one PairRec per active pair of gate g in logbuf[g * n ...] and the count in
// logcnt[g]; segments are independent, so they run side by side.  (2) One
// workgroup walks all gates backwards with the adjoint vector mu in LDS:
// one barrier per gate orders the mu updates, each wavefront's share of
// dE/dtheta_g goes to dE_part[g * 16 + wave], and the 16 shares are added in
// wave order at the end.
constexpr int kMaxSeg = 256;  // gate descriptors a segment stages in LDS at a time
constexpr int kWaves = kChainThreads / 64;

template <int CAP>
__global__ void __launch_bounds__(kChainThreads)
k_adjoint_replay_lds(const u64* __restrict__ keys, unsigned n, const GateDesc* __restrict__ gates,
                     int M, int seg, double eps, const double* const* __restrict__ ckpt,
                     const u64* __restrict__ ckpt_n, PairRec* __restrict__ logbuf,
                     unsigned* __restrict__ logcnt, unsigned* __restrict__ flags, unsigned ncut) {
  __shared__ NcutState nst;
  __shared__ u64 skeys[CAP];
  __shared__ double sW[CAP];
  __shared__ int sslots[2 * CAP];
  __shared__ GateDesc sg[kMaxSeg];
  __shared__ unsigned s_cnt;
  const int tid = threadIdx.x;
  const int j = blockIdx.x;
  const int g_lo = j * seg;
  const int g_hi = (g_lo + seg < M) ? g_lo + seg : M;
  const unsigned nj = (unsigned)ckpt_n[j];
  const double* src = ckpt[j];
  for (int t = tid; t < 2 * CAP; t += kChainThreads) sslots[t] = 0;
  for (unsigned i = tid; i < n; i += kChainThreads) {
    skeys[i] = keys[i];
    sW[i] = (i < nj) ? src[i] : dead_value();
  }
  if (tid == 0) s_cnt = 0;
  __syncthreads();
  LdsStore L{skeys, sW, sslots, 2u * CAP - 1u};
  for (unsigned i = tid; i < n; i += kChainThreads) L.insert(skeys[i], (int)i);
  const int lane = tid & 63;
  const u64 below = (1ULL << lane) - 1ULL;
  for (int g = g_lo; g < g_hi; ++g) {
    if ((g - g_lo) % kMaxSeg == 0) {
      __syncthreads();
      for (int t = tid; t < kMaxSeg && g + t < g_hi; t += kChainThreads) sg[t] = gates[g + t];
    }
    __syncthreads();
    const GateDesc gd = sg[(g - g_lo) % kMaxSeg];
    PairRec* lg = logbuf + (size_t)g * n;
    for (unsigned i0 = 0; i0 < n; i0 += kChainThreads) {
      const unsigned i = i0 + tid;
      GateOut o{false, 0ULL, 0.0, 0, false, kNoEntry, kNoEntry, 0.0, 0.0, 0};
      if (i < n) o = gate_entry(L, i, gd.op, gd.c, gd.s, eps);
      if (o.append) atomicOr(flags, kFlagOverflow);  // cannot happen: all keys are stored
      const u64 m = __ballot(o.active);
      if (m) {
        const int leader = __ffsll((long long)m) - 1;
        unsigned b = 0;
        if (lane == leader) b = atomicAdd(&s_cnt, (unsigned)__popcll(m));
        b = __shfl(b, leader);
        if (o.active) lg[b + (unsigned)__popcll(m & below)] = make_rec(o);
      }
    }
    __syncthreads();
    if (tid == 0) {
      logcnt[g] = s_cnt;
      s_cnt = 0;
    }
    if (ncut) lds_ncut(sW, skeys, n, ncut, nst);
  }
}

template <int CAP>
__global__ void __launch_bounds__(kChainThreads)
k_adjoint_reverse_lds(unsigned n, const GateDesc* __restrict__ gates, int M,
                      const double* __restrict__ mu_init, const PairRec* __restrict__ logbuf,
                      const unsigned* __restrict__ logcnt, double* __restrict__ dE_part,
                      double* __restrict__ dE) {
  __shared__ double smu[CAP];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  for (unsigned i = tid; i < n; i += kChainThreads) smu[i] = mu_init[i];
  LdsMu mu{smu};
  // The first record of this thread, the count and the descriptor of the
  // next (earlier) gate are loaded while the current gate is processed.
  PairRec cur{};
  unsigned c_cur = 0;
  GateDesc gd_cur{};
  if (M > 0) {
    gd_cur = gates[M - 1];
    c_cur = logcnt[M - 1];
    if ((unsigned)tid < n) cur = logbuf[(size_t)(M - 1) * n + tid];
  }
  __syncthreads();
  for (int g = M - 1; g >= 0; --g) {
    PairRec nxt{};
    unsigned c_nxt = 0;
    GateDesc gd_nxt{};
    if (g > 0) {
      gd_nxt = gates[g - 1];
      c_nxt = logcnt[g - 1];
      if ((unsigned)tid < n) nxt = logbuf[(size_t)(g - 1) * n + tid];
    }
    double acc = 0.0;
    if ((unsigned)tid < c_cur) acc += adjoint_pair(cur, mu, gd_cur.c, gd_cur.s);
    const PairRec* lg = logbuf + (size_t)g * n;
    for (unsigned r = tid + kChainThreads; r < c_cur; r += kChainThreads)
      acc += adjoint_pair(lg[r], mu, gd_cur.c, gd_cur.s);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) dE_part[(size_t)g * kWaves + wave] = acc;
    __syncthreads();  // every mu update of gate g precedes gate g - 1
    cur = nxt;
    c_cur = c_nxt;
    gd_cur = gd_nxt;
  }
  __syncthreads();
  for (int g = tid; g < M; g += kChainThreads) {
    double t = 0.0;
    for (int w = 0; w < kWaves; ++w) t += dE_part[(size_t)g * kWaves + w];
    dE[g] = t;
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

hipError_t launch_adjoint_replay_lds(const u64* keys, unsigned n, const GateDesc* gates, int M,
                                     int seg, double eps, const double* const* ckpt,
                                     const u64* ckpt_n, PairRec* logbuf, unsigned* logcnt,
                                     unsigned* flags, unsigned ncut, hipStream_t stream) {
  if (M <= 0) return hipSuccess;
  const int nseg = (M + seg - 1) / seg;
  hipLaunchKernelGGL(k_adjoint_replay_lds<kLdsCap>, dim3(nseg), dim3(kChainThreads), 0, stream, keys,
                     n, gates, M, seg, eps, ckpt, ckpt_n, logbuf, logcnt, flags, ncut);
  return hipGetLastError();
}

hipError_t launch_adjoint_reverse_lds(unsigned n, const GateDesc* gates, int M,
                                      const double* mu_init, const PairRec* logbuf,
                                      const unsigned* logcnt, double* dE_part, double* dE,
                                      hipStream_t stream) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adjoint_reverse_lds<kLdsCap>, dim3(1), dim3(kChainThreads), 0, stream, n,
                     gates, M, mu_init, logbuf, logcnt, dE_part, dE);
  return hipGetLastError();
}

size_t adjoint_lds_part_elems(int M) { return (size_t)M * kWaves; }

}  // namespace swcs

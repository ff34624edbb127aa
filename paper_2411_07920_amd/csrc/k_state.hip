// State kernels in HBM: the multi-block gate with fused pruning and wave-
// aggregated appends, the reverse (adjoint) step, hash index maintenance,
// checkpoints and small utilities.  The per-entry arithmetic is in
// gate_ops.h, shared with the LDS-resident single-workgroup kernels.
//
// State layout in HBM (structure of arrays, one entry per stored determinant):
//   keys[cap]  uint64 determinant bit strings (never reordered within a run)
//   amps[cap]  float64 amplitudes, kDeadBits for entries not in the state
//   hash[2^k]  16-byte slots {key, index}, linear probing, load <= 1/2
#include <algorithm>

#include "gate_ops.h"

namespace swcs {

// One gate over the stored entries, in three phases per tile of
// kGateThreads * SCAN entries:
//   scan   -- every thread loads SCAN keys (coalesced) and the
//             entries the operator or its adjoint acts on are listed in LDS
//             (16-bit tile offsets), so that the next phase runs on full
//             wavefronts whatever the active fraction;
//   update -- rounds of kGateTile listed entries, kGateItems per thread
//             staged together (gate_entries_list): index probe, amplitudes,
//             update with fused pruning; the new partner keys of a round are
//             staged in LDS;
//   append -- one atomic on the append counter per round, then coalesced
//             writes of the new keys and amplitudes and their index inserts
//             (the probe that found the key absent has just brought its
//             slot's line into L2, so the insert's CAS hits there; inserts
//             deferred to a separate pass cost more than they saved).
// SCAN = 16 for large states (more entries in flight per block), 2 for
// states of up to a few hundred thousand entries (more blocks).
template <int SCAN>
__global__ void __launch_bounds__(kGateThreads, 8)
k_gate(u64* __restrict__ keys, double* __restrict__ amps, HashSlot* __restrict__ hash, u64 hmask,
       u64 cap, Counters* __restrict__ ctr, OpDesc op, double c, double sn, double eps,
       u64* __restrict__ gate_n_in, int check_cap, unsigned gate_index, u64 max_keys,
       u64* __restrict__ gate_n_act) {
  constexpr int kScan = kGateThreads * SCAN;  // entries per tile (< 2^16)
  __shared__ unsigned short s_act[kScan];
  __shared__ u64 s_key[kGateTile];
  __shared__ double s_val[kGateTile];
  __shared__ unsigned s_nact, s_cnt;
  __shared__ int s_run;
  __shared__ u64 s_n_in, s_base;
  __shared__ long long s_wsum[kGateThreads / 64];
  __shared__ bool is_last;
  if (threadIdx.x == 0) {
    // A stopped chain skips every later gate; the host resumes it after
    // growing.  Appends are bounded by the alive sources and by the number of
    // keys not yet stored (max_keys = size of the electron-number sector), so
    // n_in + min(alive_in, max_keys - n_in) <= cap guarantees the gate fits.
    // Every block reads the same values and takes the same decision; nothing
    // has been modified when it stops.
    int run = 1;
    const unsigned fl = __hip_atomic_load(&ctr->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const u64 n_in = __hip_atomic_load(&ctr->n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (fl & kFlagStopped) {
      run = 0;
    } else if (check_cap) {
      const u64 alive_in = __hip_atomic_load(&ctr->alive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const u64 room = max_keys > n_in ? max_keys - n_in : 0;
      if (n_in + (alive_in < room ? alive_in : room) > cap) {
        run = 0;
        if (blockIdx.x == 0) {
          ctr->stop_gate = gate_index;
          atomicOr(&ctr->flags, kFlagStopped);
        }
      }
    }
    s_run = run;
    s_n_in = n_in;
    s_nact = 0;
    s_cnt = 0;
  }
  __syncthreads();
  if (!s_run) return;
  const u64 n_in = s_n_in;
  long long dalive = 0;
  u64 nact = 0;
  const int lane = __lane_id();
  const u64 below = (1ULL << lane) - 1ULL;
  const u64 ntiles = (n_in + kScan - 1) / kScan;
  const GlobalStore S{keys, amps, hash, hmask};
  for (u64 t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const u64 base = t * (u64)kScan;
    // scan: keys of the tile, active entries listed in LDS
    {
      u64 D[SCAN];
#pragma unroll
      for (int j = 0; j < SCAN; ++j) {
        const u64 i = base + (u64)j * kGateThreads + threadIdx.x;
        D[j] = (i < n_in) ? keys[i] : 0ULL;
      }
#pragma unroll
      for (int j = 0; j < SCAN; ++j) {
        const unsigned off = (unsigned)j * kGateThreads + threadIdx.x;
        const bool in = base + off < n_in;
        const bool isT = ((D[j] & op.ann) == op.ann) && ((D[j] & op.cre) == 0);
        const bool isTd = ((D[j] & op.cre) == op.cre) && ((D[j] & op.ann) == 0);
        const bool act = in && (isT || isTd);
        const u64 m = __ballot(act);
        if (m) {
          const int leader = __ffsll((long long)m) - 1;
          unsigned b = 0;
          if (lane == leader) b = atomicAdd(&s_nact, (unsigned)__popcll(m));
          b = __shfl(b, leader);
          if (act) s_act[b + (unsigned)__popcll(m & below)] = (unsigned short)off;
        }
      }
    }
    __syncthreads();
    const unsigned na = s_nact;
    nact += na;
    for (unsigned r0 = 0; r0 < na; r0 += kGateTile) {
      // update: kGateItems listed entries per thread
      u64 idx[kGateItems];
      bool use[kGateItems];
#pragma unroll
      for (int j = 0; j < kGateItems; ++j) {
        const unsigned q = r0 + (unsigned)j * kGateThreads + threadIdx.x;
        use[j] = q < na;
        idx[j] = base + (use[j] ? (u64)s_act[q] : 0ULL);
      }
      GateOut o[kGateItems];
      gate_entries_list<kGateItems>(S, idx, use, op, c, sn, eps, o);
#pragma unroll
      for (int j = 0; j < kGateItems; ++j) {
        dalive += o[j].dalive;
        const u64 m = __ballot(o[j].append);
        if (m) {
          const int leader = __ffsll((long long)m) - 1;
          unsigned b = 0;
          if (lane == leader) b = atomicAdd(&s_cnt, (unsigned)__popcll(m));
          b = __shfl(b, leader);
          if (o[j].append) {
            const unsigned slot = b + (unsigned)__popcll(m & below);
            s_key[slot] = o[j].key;
            s_val[slot] = o[j].val;
          }
        }
      }
      __syncthreads();
      // append: one counter atomic, coalesced writes
      const unsigned cnt = s_cnt;
      if (cnt) {
        if (threadIdx.x == 0) s_base = atomicAdd(&ctr->app, (u64)cnt);
        __syncthreads();
        const u64 gb = n_in + s_base;
        for (unsigned j = threadIdx.x; j < cnt; j += kGateThreads) {
          const u64 i = gb + j;
          if (i < cap) {
            keys[i] = s_key[j];
            amps[i] = s_val[j];
            hash_insert_new(hash, hmask, s_key[j], i);
          } else {
            atomicOr(&ctr->flags, kFlagOverflow);
          }
        }
        __syncthreads();
        if (threadIdx.x == 0) s_cnt = 0;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) s_nact = 0;
    __syncthreads();
  }
  // Block reduction of the alive-count change, then last-block finalization.
  for (int off = 32; off > 0; off >>= 1) dalive += __shfl_xor(dalive, off);
  if (lane == 0) s_wsum[threadIdx.x / 64] = dalive;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long d = 0;
    for (int w = 0; w < kGateThreads / 64; ++w) d += s_wsum[w];
    if (gate_n_act && nact) atomicAdd((unsigned long long*)gate_n_act, (unsigned long long)nact);
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

// Replay of one gate inside the adjoint's recomputation: the same update as
// k_gate on a working copy of the amplitudes, plus one PairRec per active
// pair, staged per tile in LDS and appended to log[] behind one atomic per
// tile.  Every key the replay can reach is already stored, so nothing is
// appended to the state.
__global__ void __launch_bounds__(kGateThreads)
k_gate_replay(const u64* __restrict__ keys, double* __restrict__ amps,
              const HashSlot* __restrict__ hash, u64 hmask, u64 n, OpDesc op, double c, double sn,
              double eps, PairRec* __restrict__ log, u64* __restrict__ log_count,
              unsigned* __restrict__ flags) {
  __shared__ PairRec s_rec[kReplayTile];
  __shared__ unsigned s_cnt;
  __shared__ u64 s_base;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  const GlobalStore S{(u64*)keys, amps, (HashSlot*)hash, hmask};
  const int lane = __lane_id();
  const u64 below = (1ULL << lane) - 1ULL;
  const u64 ntiles = (n + kReplayTile - 1) / kReplayTile;
  constexpr int kItems = kReplayTile / kGateThreads;
  for (u64 t = blockIdx.x; t < ntiles; t += gridDim.x) {
    GateOut o[kItems];
    gate_entries_staged<kItems>(S, n, t * (u64)kReplayTile + threadIdx.x, kGateThreads, op, c, sn,
                                eps, o);
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      if (o[j].append) atomicOr(flags, kFlagOverflow);
      const u64 m = __ballot(o[j].active);
      if (m) {
        const int leader = __ffsll((long long)m) - 1;
        unsigned b = 0;
        if (lane == leader) b = atomicAdd(&s_cnt, (unsigned)__popcll(m));
        b = __shfl(b, leader);
        if (o[j].active) s_rec[b + (unsigned)__popcll(m & below)] = make_rec(o[j]);
      }
    }
    __syncthreads();
    const unsigned cnt = s_cnt;
    if (cnt) {
      if (threadIdx.x == 0) s_base = atomicAdd(log_count, (u64)cnt);
      __syncthreads();
      const u64 gb = s_base;
      for (unsigned j = threadIdx.x; j < cnt; j += kGateThreads) log[gb + j] = s_rec[j];
      __syncthreads();
      if (threadIdx.x == 0) s_cnt = 0;
      __syncthreads();
    }
  }
}

// Reverse step of one gate over its logged pairs (see adjoint_pair);
// per-block partial sums of dE/dtheta go to partial[blockIdx.x].
__global__ void __launch_bounds__(256)
k_adjoint_rec(const PairRec* __restrict__ log, const u64* __restrict__ log_count,
              double* __restrict__ mu, double c, double sn, double* __restrict__ partial) {
  GlobalMu m{mu};
  const u64 cnt = *log_count;
  double acc = 0.0;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x; r < cnt; r += stride)
    acc += adjoint_pair(log[r], m, c, sn);
  __shared__ double sacc[256];
  sacc[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sacc[threadIdx.x] += sacc[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sacc[0];
}

__global__ void k_hash_clear(HashSlot* tab, u64 slots) {
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < slots; i += stride) {
    tab[i].key = kEmptyKey;
    tab[i].idx = 0;
  }
}

__global__ void k_hash_build(const u64* __restrict__ keys, HashSlot* hash, u64 hmask, u64 n) {
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    hash_insert_new(hash, hmask, keys[i], i);
}

// Presence filter of the alive keys: clear, then set one bit per key.
__global__ void k_filter_clear(unsigned* __restrict__ filt, u64 words) {
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) filt[i] = 0u;
}

__global__ void k_filter_set(const u64* __restrict__ keys, const double* __restrict__ amps, u64 n,
                             unsigned* __restrict__ filt, u64 fmask) {
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    if (is_dead(amps[i])) continue;
    const u64 b = filter_bit(keys[i], fmask);
    atomicOr(&filt[b >> 5], 1u << (b & 31));
  }
}

// N_CUT pruning of a state in HBM: a radix select of the ncut-th largest
// value in the N_CUT order (gate_ops.h), one histogram launch and one pick
// launch per 8-bit digit, then one marking launch.  With ctr the stored
// count comes from the counters and the alive count is updated; otherwise
// n_host entries are scanned.
__global__ void k_ncut_init(NcutState* __restrict__ st, unsigned ncut,
                            const Counters* __restrict__ ctr) {
  if (blockIdx.x != 0) return;
  const int t = threadIdx.x;
  if (t < 256) st->hist[t] = 0;
  if (t == 0) {
    st->phi = st->plo = st->mhi = st->mlo = 0;
    st->k = ncut;
    unsigned skip = 0;
    if (ctr) {
      const unsigned fl = __hip_atomic_load(&ctr->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const u64 alive = __hip_atomic_load(&ctr->alive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if ((fl & kFlagStopped) || alive <= ncut) skip = 1;
    }
    st->skip = skip;
  }
}

__global__ void __launch_bounds__(256)
k_ncut_hist(const double* __restrict__ amps, const u64* __restrict__ keys, u64 n_host,
            const Counters* __restrict__ ctr, NcutState* __restrict__ st, int d) {
  if (st->skip) return;
  __shared__ unsigned h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const u64 n = ctr ? __hip_atomic_load(&ctr->n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : n_host;
  const NcutState s = *st;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double a = amps[i];
    if (is_dead(a)) continue;
    u64 hi, lo;
    ncut_value(a, keys[i], &hi, &lo);
    if (ncut_matches(s, hi, lo)) atomicAdd(&h[ncut_digit(hi, lo, d)], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&st->hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void k_ncut_pick(NcutState* __restrict__ st, int d) {
  if (st->skip) return;
  if (threadIdx.x == 0) ncut_pick(*st, d);
  __syncthreads();
  if (threadIdx.x < 256) st->hist[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(256)
k_ncut_mark(double* __restrict__ amps, const u64* __restrict__ keys, u64 n_host,
            Counters* __restrict__ ctr, const NcutState* __restrict__ st) {
  if (st->skip) return;
  const u64 n = ctr ? __hip_atomic_load(&ctr->n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : n_host;
  const u64 thi = st->phi, tlo = st->plo;
  unsigned long long dropped = 0;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double a = amps[i];
    if (is_dead(a)) continue;
    u64 hi, lo;
    ncut_value(a, keys[i], &hi, &lo);
    if (hi < thi || (hi == thi && lo < tlo)) {
      amps[i] = dead_value();
      ++dropped;
    }
  }
  if (ctr) {
    for (int off = 32; off > 0; off >>= 1) dropped += __shfl_xor(dropped, off);
    if (__lane_id() == 0 && dropped) atomicAdd(&ctr->alive, (u64)(0ULL - dropped));
  }
}

// State = the single reference determinant with amplitude 1.
__global__ void k_reset_reference(u64* __restrict__ keys, double* __restrict__ amps,
                                  Counters* __restrict__ ctr, u64 ref) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    keys[0] = ref;
    amps[0] = 1.0;
    ctr->n = 1;
    ctr->alive = 1;
    ctr->app = 0;
    ctr->dalive = 0;
    ctr->ticket = 0;
    ctr->flags = 0;
    ctr->stop_gate = 0;
  }
}

// Same, with the entry count read from the device counters.
__global__ void k_hash_build_dev(const u64* __restrict__ keys, HashSlot* hash, u64 hmask,
                                 const Counters* __restrict__ ctr) {
  const u64 n = __hip_atomic_load(&ctr->n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    hash_insert_new(hash, hmask, keys[i], i);
}

__global__ void k_mark_dead_range(double* amps, u64 lo, u64 hi) {
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = lo + (u64)blockIdx.x * blockDim.x + threadIdx.x; i < hi; i += stride)
    amps[i] = dead_value();
}

// Drop every alive entry with |c| < eps (used once after the first gate of a
// chain that starts from a caller-supplied state, whose untouched entries
// have not been tested against eps yet).  Skipped if the chain has stopped.
__global__ void __launch_bounds__(256)
k_prune_all(double* __restrict__ amps, Counters* __restrict__ ctr, double eps) {
  if (__hip_atomic_load(&ctr->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kFlagStopped)
    return;
  const u64 n = __hip_atomic_load(&ctr->n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  unsigned long long dropped = 0;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double a = amps[i];
    if (!is_dead(a) && fabs(a) < eps) {
      amps[i] = dead_value();
      ++dropped;
    }
  }
  const u64 m = __ballot(dropped != 0);
  if (m) {
    // wave sum of dropped, then one atomic per wave
    unsigned long long s = dropped;
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (__lane_id() == 0) atomicAdd(&ctr->alive, (u64)(0ULL - s));
  }
}

// Copy amps[0, n) of the current state to dst and record n, unless the chain
// has stopped (the host re-enqueues the copy when it resumes).
__global__ void k_ckpt_save(const double* __restrict__ amps, const Counters* __restrict__ ctr,
                            double* __restrict__ dst, u64* __restrict__ dst_n) {
  if (__hip_atomic_load(&ctr->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kFlagStopped)
    return;
  const u64 n = __hip_atomic_load(&ctr->n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = amps[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) *dst_n = n;
}

// dst[0, n_src) = src, dst[n_src, n_total) = dead.
__global__ void k_restore(double* __restrict__ dst, const double* __restrict__ src,
                          const u64* __restrict__ n_src_ptr, u64 n_total) {
  const u64 n_src = *n_src_ptr;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n_total; i += stride)
    dst[i] = (i < n_src) ? src[i] : dead_value();
}

static int grid_for(u64 n, int block, int max_grid) {
  u64 g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > (u64)max_grid) g = max_grid;
  return (int)g;
}

hipError_t launch_hash_clear(HashSlot* tab, u64 slots, hipStream_t stream) {
  hipLaunchKernelGGL(k_hash_clear, dim3(grid_for(slots, 256, 8192)), dim3(256), 0, stream, tab, slots);
  return hipGetLastError();
}

hipError_t launch_hash_build(const DeviceState& st, u64 n, hipStream_t stream) {
  hipLaunchKernelGGL(k_hash_build, dim3(grid_for(n, 256, 8192)), dim3(256), 0, stream, st.keys,
                     st.hash, st.hmask, n);
  return hipGetLastError();
}

hipError_t launch_filter_build(const DeviceState& st, u64 n, int grid, hipStream_t stream) {
  const u64 words = (st.fmask + 1) / 32;
  hipLaunchKernelGGL(k_filter_clear, dim3(grid_for(words, 256, 4096)), dim3(256), 0, stream, st.filt,
                     words);
  if (n > 0)
    hipLaunchKernelGGL(k_filter_set, dim3(grid), dim3(256), 0, stream, st.keys, st.amps, n, st.filt,
                       st.fmask);
  return hipGetLastError();
}

hipError_t launch_ncut(double* amps, const u64* keys, u64 n_host, Counters* ctr, NcutState* st,
                       unsigned ncut, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(k_ncut_init, dim3(1), dim3(256), 0, stream, st, ncut, ctr);
  for (int d = 0; d < 16; ++d) {
    hipLaunchKernelGGL(k_ncut_hist, dim3(grid), dim3(256), 0, stream, amps, keys, n_host, ctr, st, d);
    hipLaunchKernelGGL(k_ncut_pick, dim3(1), dim3(256), 0, stream, st, d);
  }
  hipLaunchKernelGGL(k_ncut_mark, dim3(grid), dim3(256), 0, stream, amps, keys, n_host, ctr, st);
  return hipGetLastError();
}

hipError_t launch_reset_reference(const DeviceState& st, u64 ref, hipStream_t stream) {
  hipLaunchKernelGGL(k_reset_reference, dim3(1), dim3(64), 0, stream, st.keys, st.amps, st.ctr, ref);
  return hipGetLastError();
}

hipError_t launch_hash_build_dev(const DeviceState& st, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(k_hash_build_dev, dim3(grid), dim3(256), 0, stream, st.keys, st.hash, st.hmask,
                     st.ctr);
  return hipGetLastError();
}

hipError_t launch_gate(const DeviceState& st, const OpDesc& op, double c, double sn, double eps,
                       u64* gate_n_in, int check_cap, unsigned gate_index, u64 max_keys, int grid,
                       hipStream_t stream, u64* gate_n_act) {
  if (st.cap >= kGateWideCap)
    hipLaunchKernelGGL(k_gate<kGateScanWide>, dim3(grid), dim3(kGateThreads), 0, stream, st.keys, st.amps,
                       st.hash, st.hmask, st.cap, st.ctr, op, c, sn, eps, gate_n_in, check_cap, gate_index,
                       max_keys, gate_n_act);
  else
    hipLaunchKernelGGL(k_gate<kGateScanNarrow>, dim3(grid), dim3(kGateThreads), 0, stream, st.keys, st.amps,
                       st.hash, st.hmask, st.cap, st.ctr, op, c, sn, eps, gate_n_in, check_cap, gate_index,
                       max_keys, gate_n_act);
  return hipGetLastError();
}

hipError_t launch_prune_all(const DeviceState& st, double eps, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(k_prune_all, dim3(grid), dim3(256), 0, stream, st.amps, st.ctr, eps);
  return hipGetLastError();
}

hipError_t launch_gate_replay(const DeviceState& st, double* amps, u64 n, const OpDesc& op,
                             double c, double sn, double eps, PairRec* log, u64* log_count, int grid,
                             hipStream_t stream) {
  hipLaunchKernelGGL(k_gate_replay, dim3(grid), dim3(kGateThreads), 0, stream, st.keys, amps, st.hash,
                     st.hmask, n, op, c, sn, eps, log, log_count, &st.ctr->flags);
  return hipGetLastError();
}

hipError_t launch_adjoint_rec(const PairRec* log, const u64* log_count, double* mu, double c,
                              double sn, double* partial, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(k_adjoint_rec, dim3(grid), dim3(256), 0, stream, log, log_count, mu, c, sn,
                     partial);
  return hipGetLastError();
}

hipError_t launch_ckpt_save(const DeviceState& st, double* dst, u64* dst_n, int grid,
                            hipStream_t stream) {
  hipLaunchKernelGGL(k_ckpt_save, dim3(grid), dim3(256), 0, stream, st.amps, st.ctr, dst, dst_n);
  return hipGetLastError();
}

hipError_t launch_restore(double* dst, const double* src, const u64* n_src, u64 n_total,
                          hipStream_t stream) {
  hipLaunchKernelGGL(k_restore, dim3(grid_for(n_total, 256, 8192)), dim3(256), 0, stream, dst, src,
                     n_src, n_total);
  return hipGetLastError();
}

hipError_t launch_mark_dead_range(double* amps, u64 lo, u64 hi, hipStream_t stream) {
  if (hi <= lo) return hipSuccess;
  hipLaunchKernelGGL(k_mark_dead_range, dim3(grid_for(hi - lo, 256, 8192)), dim3(256), 0, stream,
                     amps, lo, hi);
  return hipGetLastError();
}

}  // namespace swcs

namespace swcs {

// Buffer clears and small host-to-device writes as kernels on the stream
// (fills instead of runtime memsets, counters passed as kernel arguments), so
// every step of a call is one of the library's own launches, in stream order,
// and a caller may capture it.
__global__ void k_fill_u32(unsigned* __restrict__ p, unsigned v, u64 words) {
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) p[i] = v;
}

__global__ void k_store_counters(Counters* __restrict__ ctr, Counters v) { *ctr = v; }

__global__ void k_clear_flag(Counters* __restrict__ ctr, unsigned bit) {
  atomicAnd(&ctr->flags, ~bit);
}

hipError_t launch_fill_u32(void* p, unsigned v, u64 words, hipStream_t stream) {
  if (words == 0) return hipSuccess;
  const u64 blocks = std::min<u64>((words + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, stream, (unsigned*)p, v, words);
  return hipGetLastError();
}

hipError_t launch_store_counters(Counters* ctr, const Counters& v, hipStream_t stream) {
  hipLaunchKernelGGL(k_store_counters, dim3(1), dim3(1), 0, stream, ctr, v);
  return hipGetLastError();
}

hipError_t launch_clear_flag(Counters* ctr, unsigned bit, hipStream_t stream) {
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, stream, ctr, bit);
  return hipGetLastError();
}

}  // namespace swcs

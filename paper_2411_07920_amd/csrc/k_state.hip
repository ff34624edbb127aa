// State kernels: hash index maintenance, the excitation-unitary gate with
// fused pruning, the reverse (adjoint) gate step and small utilities.
//
// State layout in HBM (structure of arrays, one entry per stored determinant):
//   keys[cap]  uint64 determinant bit strings (never reordered within a run)
//   amps[cap]  float64 amplitudes, kDeadBits for entries not in the state
//   hash[2^k]  16-byte slots {key, index}, linear probing, load <= 1/2
// A gate exp(theta A) with A = T - T^dagger pairs each determinant D on which
// T acts with X = T D (sign s = <X|T|D>) and rotates the pair:
//   psi'(D) = c psi(D) - s sn psi(X),   psi'(X) = c psi(X) + s sn psi(D)
// (c = cos theta, sn = sin theta), the exact value of exp(theta A) because
// T^2 = 0 and A^3 = -A (Sec. II.B evaluates each unitary exactly).  Every
// other determinant is unchanged.  Each output is a sum of two rounded
// products formed in a fixed order, so the result does not depend on thread
// scheduling.  Pruning (drop |c| < eps, Fig. 1) is applied to the touched
// entries only, since untouched ones kept their already-accepted value.
#include "swcs_internal.h"

namespace swcs {

// Ownership rule that makes the in-place update race-free: the pair (D, X) is
// processed by the thread of D whenever D is stored (alive or not); otherwise
// by the thread of X, which then appends D.  Lookups only ever target keys
// stored before the launch, and appended keys are new and distinct.
__global__ void __launch_bounds__(256)
k_gate(u64* __restrict__ keys, double* __restrict__ amps, HashSlot* __restrict__ hash, u64 hmask,
       u64 cap, Counters* __restrict__ ctr, OpDesc op, double c, double sn, double eps,
       u64* __restrict__ gate_n_in, int check_cap, unsigned gate_index) {
  // A stopped chain skips every later gate; the host resumes it after growing.
  if (__hip_atomic_load(&ctr->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kFlagStopped)
    return;
  const u64 n_in = __hip_atomic_load(&ctr->n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // Appends are bounded by the alive sources, so n_in + alive_in <= cap
  // guarantees the gate fits.  Every block reads the same values and takes
  // the same decision; nothing has been modified when it stops.
  if (check_cap) {
    const u64 alive_in = __hip_atomic_load(&ctr->alive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (n_in + alive_in > cap) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctr->stop_gate = gate_index;
        atomicOr(&ctr->flags, kFlagStopped);
      }
      return;
    }
  }
  const u64 pair_mask = op.ann | op.cre;
  long long dalive = 0;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n_in; i += stride) {
    const u64 D = keys[i];
    const bool isT = ((D & op.ann) == op.ann) && ((D & op.cre) == 0);
    const bool isTd = ((D & op.cre) == op.cre) && ((D & op.ann) == 0);
    bool want_append = false;
    u64 app_key = 0;
    double app_val = 0.0;
    if (isT) {
      const u64 X = D ^ pair_mask;
      const long long j = hash_find(hash, hmask, X);
      const double araw = amps[i];
      const double braw = (j >= 0) ? amps[j] : dead_value();
      const bool aliveD = !is_dead(araw), aliveX = !is_dead(braw);
      if (aliveD || aliveX) {
        const double s = (double)phase_of_T(op, D);
        const double a = aliveD ? araw : 0.0;
        const double b = aliveX ? braw : 0.0;
        const double nd = c * a - s * (sn * b);
        const double nx = c * b + s * (sn * a);
        const bool keepD = !(fabs(nd) < eps);
        const bool keepX = !(fabs(nx) < eps);
        amps[i] = keepD ? nd : dead_value();
        if (j >= 0) {
          amps[j] = keepX ? nx : dead_value();
        } else if (keepX) {
          want_append = true;
          app_key = X;
          app_val = nx;
        }
        dalive += (long long)keepD - (long long)aliveD + (long long)keepX - (long long)aliveX;
      }
    } else if (isTd) {
      const u64 Dsrc = D ^ pair_mask;
      const long long j = hash_find(hash, hmask, Dsrc);
      // When Dsrc is stored its thread owns the pair and may be writing this
      // entry; only read it when this thread is the owner.
      const double braw = (j < 0) ? amps[i] : dead_value();
      if (j < 0 && !is_dead(braw)) {
        const double s = (double)phase_of_T(op, Dsrc);
        const double a = 0.0, b = braw;
        const double nd = c * a - s * (sn * b);
        const double nx = c * b + s * (sn * a);
        const bool keepD = !(fabs(nd) < eps);
        const bool keepX = !(fabs(nx) < eps);
        amps[i] = keepX ? nx : dead_value();
        if (keepD) {
          want_append = true;
          app_key = Dsrc;
          app_val = nd;
        }
        dalive += (long long)keepD + (long long)keepX - 1LL;
      }
    }
    // Wave-aggregated append.
    const u64 m = __ballot(want_append);
    if (m) {
      const int lane = __lane_id();
      const int leader = __ffsll((long long)m) - 1;
      u64 base = 0;
      if (lane == leader) base = atomicAdd(&ctr->app, (u64)__popcll(m));
      base = __shfl(base, leader);
      if (want_append) {
        const u64 idx = n_in + base + (u64)__popcll(m & ((1ULL << lane) - 1ULL));
        if (idx < cap) {
          keys[idx] = app_key;
          amps[idx] = app_val;
          hash_insert_new(hash, hmask, app_key, idx);
        } else {
          atomicOr(&ctr->flags, kFlagOverflow);
        }
      }
    }
  }
  // Block reduction of the alive-count change, then last-block finalization.
  __shared__ long long sdelta[256];
  __shared__ bool is_last;
  sdelta[threadIdx.x] = dalive;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sdelta[threadIdx.x] += sdelta[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (sdelta[0] != 0) atomicAdd((unsigned long long*)&ctr->dalive, (unsigned long long)sdelta[0]);
    __threadfence();
    const unsigned t = atomicAdd(&ctr->ticket, 1u);
    is_last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (is_last && threadIdx.x == 0) {
    __threadfence();
    const u64 app = atomicAdd(&ctr->app, 0ULL);
    const long long da = (long long)atomicAdd((unsigned long long*)&ctr->dalive, 0ULL);
    const u64 alive = ctr->alive;
    if (gate_n_in) *gate_n_in = alive;
    const u64 napp = app;
    ctr->n = n_in + (napp < cap - n_in ? napp : cap - n_in);
    ctr->alive = (u64)((long long)alive + da);
    ctr->app = 0;
    ctr->dalive = 0;
    __threadfence();
    ctr->ticket = 0;
  }
}

// Reverse step of one gate for the frozen-support adjoint.  psi_prev holds
// the state before the gate (entries not in it are dead), mu holds the
// adjoint vector after the gate (zero outside the kept support).  Writes the
// adjoint before the gate in place and this block's share of
// dE/dtheta = <mu | P U'(theta) psi_prev>, U' = derivative of the 2x2 rotation.
__global__ void __launch_bounds__(256)
k_adjoint_step(const u64* __restrict__ keys, const HashSlot* __restrict__ hash, u64 hmask,
               u64 n_total, OpDesc op, double c, double sn, const double* __restrict__ psi_prev,
               double* __restrict__ mu, double* __restrict__ partial) {
  const u64 pair_mask = op.ann | op.cre;
  double acc = 0.0;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n_total; i += stride) {
    const u64 D = keys[i];
    const bool isT = ((D & op.ann) == op.ann) && ((D & op.cre) == 0);
    const bool isTd = ((D & op.cre) == op.cre) && ((D & op.ann) == 0);
    if (isT) {
      const u64 X = D ^ pair_mask;
      const long long j = hash_find(hash, hmask, X);
      const double araw = psi_prev[i];
      const double braw = (j >= 0) ? psi_prev[j] : dead_value();
      const bool aliveD = !is_dead(araw), aliveX = !is_dead(braw);
      if (!aliveD && !aliveX) continue;
      const double s = (double)phase_of_T(op, D);
      const double a = aliveD ? araw : 0.0, b = aliveX ? braw : 0.0;
      const double muD = mu[i];
      const double muX = (j >= 0) ? mu[j] : 0.0;
      acc += muD * (-sn * a - s * c * b) + muX * (-sn * b + s * c * a);
      mu[i] = aliveD ? (c * muD + s * sn * muX) : 0.0;
      if (j >= 0) mu[j] = aliveX ? (c * muX - s * sn * muD) : 0.0;
    } else if (isTd) {
      const u64 Dsrc = D ^ pair_mask;
      const long long j = hash_find(hash, hmask, Dsrc);
      if (j >= 0) continue;  // the thread of Dsrc owns the pair
      const double braw = psi_prev[i];
      if (is_dead(braw)) continue;
      const double muX = mu[i];
      acc += muX * (-sn * braw);
      mu[i] = c * muX;
    }
  }
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

__global__ void k_mark_dead_range(double* amps, u64 lo, u64 hi) {
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = lo + (u64)blockIdx.x * blockDim.x + threadIdx.x; i < hi; i += stride)
    amps[i] = dead_value();
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

hipError_t launch_gate(const DeviceState& st, const OpDesc& op, double c, double sn, double eps,
                       u64* gate_n_in, int check_cap, unsigned gate_index, int grid,
                       hipStream_t stream) {
  hipLaunchKernelGGL(k_gate, dim3(grid), dim3(256), 0, stream, st.keys, st.amps, st.hash, st.hmask,
                     st.cap, st.ctr, op, c, sn, eps, gate_n_in, check_cap, gate_index);
  return hipGetLastError();
}

hipError_t launch_adjoint_step(const DeviceState& st, const OpDesc& op, double c, double sn,
                               const double* amps_prev, double* mu, double* partial, u64 n_total,
                               int grid, hipStream_t stream) {
  hipLaunchKernelGGL(k_adjoint_step, dim3(grid), dim3(256), 0, stream, st.keys, st.hash, st.hmask,
                     n_total, op, c, sn, amps_prev, mu, partial);
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

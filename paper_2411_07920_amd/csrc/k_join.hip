// Pool gradients of a whole pool by sorting and joining, without a
// device-wide accumulation table.
//
// The pool gradient of ADAPT step 4 (Sec. II.C) is
//   g_k = (2 / <psi|psi>) sum_D psi(D) a_k(D) sigma(X_k(D)),
//   sigma(X) = sum_{D'} H_{X D'} psi(D'),
// with X_k(D) the determinant the generator A_k maps D to and a_k(D) = +-1.
// For a pool of all spin-conserving singles and doubles, the (D, k) pairs
// with X_k(D) != 0 are exactly the pairs (D, X) of D and one of its
// Slater-Condon connections, and sigma(X) sums over the same pairs grouped
// by X (plus H_{D D} psi(D) when X = D is stored).  So one record per pair
// carries everything:
//   emit   -- every alive D writes one 64-bit record per connection X and
//             one for itself: (d << (kb + bj)) | (j << kb) | bucket(X), where
//             d is D's storage index, j the connection's ordinal in D's
//             enumeration (j = C for D itself) and bucket(X) the low kb bits
//             of mix64(X); D's records are one coalesced run;
//   sort   -- a stable LSD radix sort on the kb bucket bits only, so every
//             record of one X lands in one contiguous bucket;
//   join   -- a block takes a run of whole buckets, decodes each record
//             back to (D, X), accumulates sigma(X) in an LDS table, then adds
//             psi(D) a_k(D) sigma(X) to g[k] for every record.
// The device-wide traffic is streaming (records written once, sorted in
// kb / 8 passes, read twice from L2-resident runs), where the table path
// pays one random read-modify-write per pair in HBM.
#include "conn_ops.h"

namespace swcs {

constexpr int kJoinEmitBlock = 256;
constexpr int kJoinBlock = 512;
constexpr int kJoinRun = (int)kJoinRunHost;  // records per block step before bucket alignment
constexpr int kJoinSlots = 4096;  // LDS table: keys and sums, 64 KB (two blocks per CU)

// Position of the r-th (from 0) set bit of m; m has more than r set bits.
__device__ inline int select_bit(u64 m, int r) {
  for (int i = 0; i < r; ++i) m &= m - 1ULL;
  return __ffsll((long long)m) - 1;
}

// (x, y), x < y, of the pair with triangular index t = y (y - 1) / 2 + x,
// the order of the pair tables of the connection enumeration.
__device__ inline void tri_pair(int t, int* x, int* y) {
  int yy = (int)((1.0 + sqrt(1.0 + 8.0 * (double)t)) * 0.5);
  while (yy * (yy - 1) / 2 > t) --yy;
  while ((yy + 1) * yy / 2 <= t) ++yy;
  *y = yy;
  *x = t - yy * (yy - 1) / 2;
}

// Connection j of D in the order of for_each_connection: class (alpha
// single, beta single, alpha-alpha, beta-beta, alpha-beta double), then hole
// set, then particle set.  Returns X and the holes h0 <= h1, particles
// p0 <= p1 (equal for singles), nh = 1 or 2.
__device__ inline u64 conn_decode(const ExcSpace& E, u64 D, long long j, int* nh, int* h0, int* h1, int* p0,
                                  int* p1) {
  const u64 amask = 0x5555555555555555ULL, bmask = 0xAAAAAAAAAAAAAAAAULL;
  const u64 full = (E.n >= 32) ? ~0ULL : ((1ULL << (2 * E.n)) - 1ULL);
  const u64 occ_a = D & amask, occ_b = D & bmask;
  const u64 vir_a = ~D & amask & full, vir_b = ~D & bmask & full;
  const long long sz[5] = {E.s_a, E.s_b, E.d_aa, E.d_bb, E.d_ab};
  const int nb = E.nb, va = E.va, vb = E.vb;
  const int npar[5] = {va, vb, va * (va - 1) / 2, vb * (vb - 1) / 2, va * vb};
  int c = 0;
  while (c < 4 && j >= sz[c]) {
    j -= sz[c];
    ++c;
  }
  const int hi = (int)(j / npar[c]);
  const int pi = (int)(j - (long long)hi * npar[c]);
  if (c < 2) {
    *nh = 1;
    *h0 = *h1 = select_bit(c == 0 ? occ_a : occ_b, hi);
    *p0 = *p1 = select_bit(c == 0 ? vir_a : vir_b, pi);
  } else if (c < 4) {
    *nh = 2;
    const u64 o = c == 2 ? occ_a : occ_b, v = c == 2 ? vir_a : vir_b;
    int x, y;
    tri_pair(hi, &x, &y);
    *h0 = select_bit(o, x);
    *h1 = select_bit(o, y);
    tri_pair(pi, &x, &y);
    *p0 = select_bit(v, x);
    *p1 = select_bit(v, y);
  } else {
    *nh = 2;
    const int ha = select_bit(occ_a, hi / nb), hb = select_bit(occ_b, hi - (hi / nb) * nb);
    const int pa = select_bit(vir_a, pi / vb), pb = select_bit(vir_b, pi - (pi / vb) * vb);
    *h0 = min(ha, hb);
    *h1 = max(ha, hb);
    *p0 = min(pa, pb);
    *p1 = max(pa, pb);
  }
  const u64 hm = (1ULL << *h0) | (1ULL << *h1), pm = (1ULL << *p0) | (1ULL << *p1);
  return D ^ hm ^ pm;
}

// Calls f(X, j) for every connection of D assigned to this lane, j its
// ordinal (class offsets + hole set * particle sets + particle set).
template <class F>
__device__ inline void for_each_connection_ord(const ConnTables& T, u64 D, F&& f) {
  long long off = 0;
  for (int c = 0; c < 5; ++c) {
    const int nh = T.nh[c], np = T.np[c];
    if (nh == 0 || np == 0) continue;
    const int hb = T.hbeg[c], pb = T.pbeg[c];
    int hi = (int)threadIdx.x / np;
    int pi = (int)threadIdx.x - hi * np;
    while (hi < nh) {
      const u64 X = D ^ T.hmask[hb + hi] ^ T.pmask[pb + pi];
      f(X, off + (long long)hi * np + pi);
      pi += blockDim.x;
      while (pi >= np) {
        pi -= np;
        ++hi;
      }
    }
    off += (long long)nh * np;
  }
}

// One run of C + 1 records per alive entry, at a position taken from
// *cursor; runs past cap_recs are not written and raise kFlagOverflow.
__global__ void __launch_bounds__(kJoinEmitBlock)
k_join_emit(const u64* __restrict__ keys, const double* __restrict__ amps, ExcSpace E, u64 n,
            u64* __restrict__ recs, u64 cap_recs, u64* __restrict__ cursor, int kb, int bj,
            unsigned* __restrict__ flags) {
  __shared__ SigShared S;
  __shared__ ConnTables T;
  extern __shared__ __align__(16) unsigned char conn_dyn[];
  __shared__ u64 s_base;
  build_pair_table(S);
  if (threadIdx.x == 0) attach_conn_tables(T, conn_dyn, E);
  const u64 C = (u64)E.total;
  const u64 bmask = (1ULL << kb) - 1ULL;
  const int sd = kb + bj;
  for (u64 d = blockIdx.x; d < n; d += gridDim.x) {
    if (is_dead(amps[d])) continue;
    const u64 D = keys[d];
    __syncthreads();
    build_lists_shared(D, E.n, S);
    if (threadIdx.x == 0) s_base = atomicAdd(cursor, C + 1);
    __syncthreads();
    build_conn_tables(S, E, T);
    __syncthreads();
    const u64 base = s_base;
    if (base + C + 1 > cap_recs) {
      if (threadIdx.x == 0) atomicOr(flags, kFlagOverflow);
      continue;
    }
    const u64 hd = d << sd;
    for_each_connection_ord(T, D, [&](u64 X, long long j) {
      recs[base + (u64)j] = hd | ((u64)j << kb) | (mix64(X) & bmask);
    });
    if (threadIdx.x == 0) recs[base + C] = hd | (C << kb) | (mix64(D) & bmask);
  }
}

// First position p' >= p whose bucket differs from that of p' - 1 (0 and
// R are boundaries).  Called by every thread of the block.
__device__ inline u64 bucket_boundary(const u64* __restrict__ recs, u64 R, u64 p, u64 bmask,
                                      unsigned* s_found, u64* s_pos) {
  if (p == 0 || p >= R) return p < R ? p : R;
  const u64 b0 = recs[p - 1] & bmask;
  u64 q0 = p;
  while (true) {
    if (threadIdx.x == 0) {
      *s_found = 0;
      *s_pos = R;
    }
    __syncthreads();
    const u64 q = q0 + threadIdx.x;
    if (q < R && (recs[q] & bmask) != b0) {
      atomicMin((unsigned long long*)s_pos, (unsigned long long)q);
      *s_found = 1;
    }
    __syncthreads();
    const bool found = *s_found != 0 || q0 + blockDim.x >= R;
    const u64 pos = *s_pos;
    __syncthreads();
    if (found) return pos;
    q0 += blockDim.x;
  }
}

// LDS slot of X (inserted if absent); -1 if the table is full.
__device__ inline int join_slot(u64* tk, u64 X, bool insert, double* inserted) {
  unsigned h = (unsigned)(mix64(X) >> 40) & (kJoinSlots - 1);
  for (int probes = 0; probes < kJoinSlots; ++probes) {
    const u64 k = tk[h];
    if (k == X) return (int)h;
    if (k == kEmptyKey) {
      if (!insert) return -1;
      const u64 prev = atomicCAS((unsigned long long*)&tk[h], (unsigned long long)kEmptyKey,
                                 (unsigned long long)X);
      if (prev == kEmptyKey) {
        *inserted += 1.0;
        return (int)h;
      }
      if (prev == X) return (int)h;
    }
    h = (h + 1) & (kJoinSlots - 1);
  }
  return -1;
}

// Record fields and the source entry.
struct JoinRec {
  u64 d;
  long long j;
};
__device__ inline JoinRec join_rec(u64 r, int kb, int bj) {
  JoinRec o;
  o.j = (long long)((r >> kb) & ((1ULL << bj) - 1ULL));
  o.d = r >> (kb + bj);
  return o;
}

// The join over sorted records: block steps of kJoinRun records, widened to
// whole buckets (a bucket belongs to the step it starts in).  Per step: the
// LDS table of sigma(X) over the step's records, then the gradient
// contributions; selected (may be NULL) limits them to flagged operators.
// A step whose distinct keys overflow the table raises kFlagOverflow (the
// host then uses the table path).  inserted[block] counts the distinct
// determinants X of the block's steps (stored ones included), so their sum
// is the size of the space sigma is formed on.
__global__ void __launch_bounds__(kJoinBlock)
k_join_reduce(const u64* __restrict__ recs, u64 R, const u64* __restrict__ cursor, int kb, int bj,
              const u64* __restrict__ keys, const double* __restrict__ amps, const double* __restrict__ diag,
              u64 n, Ints I, ExcSpace E, const int* __restrict__ optab, int npairs,
              const unsigned char* __restrict__ selected, double* __restrict__ gacc,
              unsigned* __restrict__ flags, double* __restrict__ inserted) {
  __shared__ u64 tk[kJoinSlots];
  __shared__ double tv[kJoinSlots];
  __shared__ unsigned s_found, s_bad;
  __shared__ u64 s_pos;
  __shared__ double red[kJoinBlock];
  const u64 bmask = (1ULL << kb) - 1ULL;
  const long long C = E.total;
  double ins = 0.0;
  // The emit wrote exactly R records only if the alive count it was sized
  // by is the number of alive entries; otherwise nothing is joined and the
  // pass reports an overflow.  Records are also checked field by field, so
  // no record can index outside the state.
  if (*cursor != R) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flags, kFlagOverflow);
    if (threadIdx.x == 0) inserted[blockIdx.x] = 0.0;
    return;
  }
  for (int s = threadIdx.x; s < kJoinSlots; s += kJoinBlock) tk[s] = kEmptyKey;
  for (u64 p = (u64)blockIdx.x * kJoinRun; p < R; p += (u64)gridDim.x * kJoinRun) {
    const u64 lo = bucket_boundary(recs, R, p, bmask, &s_found, &s_pos);
    const u64 hi = bucket_boundary(recs, R, p + kJoinRun, bmask, &s_found, &s_pos);
    if (lo >= hi) continue;  // uniform: the step lies inside a bucket begun earlier
    for (int s = threadIdx.x; s < kJoinSlots; s += kJoinBlock) tv[s] = 0.0;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    // sigma(X) over the step's records
    for (u64 i = lo + threadIdx.x; i < hi; i += kJoinBlock) {
      const JoinRec r = join_rec(recs[i], kb, bj);
      if (r.d >= n || r.j > C) continue;
      const u64 D = keys[r.d];
      const double psi = amps[r.d];
      u64 X;
      double v;
      if (r.j == C) {
        X = D;
        v = diag[r.d] * psi;
      } else {
        int nh, h0, h1, p0, p1;
        X = conn_decode(E, D, r.j, &nh, &h0, &h1, &p0, &p1);
        v = connection_element(I, D, nh, h0, h1, p0, p1) * psi;
      }
      const int sl = join_slot(tk, X, true, &ins);
      if (sl < 0) s_bad = 1;
      else atomicAdd(&tv[sl], v);
    }
    __syncthreads();
    if (s_bad) {
      if (threadIdx.x == 0) atomicOr(flags, kFlagOverflow);
    } else {
      // psi(D) a_k(D) sigma(X) for every pair record
      for (u64 i = lo + threadIdx.x; i < hi; i += kJoinBlock) {
        const JoinRec r = join_rec(recs[i], kb, bj);
        if (r.d >= n || r.j >= C) continue;
        const u64 D = keys[r.d];
        int nh, h0, h1, p0, p1;
        const u64 X = conn_decode(E, D, r.j, &nh, &h0, &h1, &p0, &p1);
        bool t_acts;
        OpDesc op;
        const int k = linking_operator(optab, npairs, nh, h0, h1, p0, p1, &t_acts, &op);
        if (k < 0 || (selected && !selected[k])) continue;
        const int sl = join_slot(tk, X, false, &ins);
        if (sl < 0) continue;  // not reached: pass 1 inserted every key of the step
        const double a = t_acts ? (double)phase_of_T(op, D) : -(double)phase_of_T(op, X);
        unsafeAtomicAdd(&gacc[k], amps[r.d] * a * tv[sl]);
      }
    }
    __syncthreads();
    for (int s = threadIdx.x; s < kJoinSlots; s += kJoinBlock) tk[s] = kEmptyKey;
    __syncthreads();
  }
  for (int off = 32; off > 0; off >>= 1) ins += __shfl_xor(ins, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ins;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kJoinBlock / 64; ++w) t += red[w];
    inserted[blockIdx.x] = t;
  }
}

hipError_t launch_join_emit(const DeviceState& st, const ExcSpace& E, u64 n, u64* recs, u64 cap_recs,
                            u64* cursor, int kb, int bj, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(k_join_emit, dim3(grid), dim3(kJoinEmitBlock), conn_tables_bytes(E), stream, st.keys, st.amps, E,
                     n, recs, cap_recs, cursor, kb, bj, &st.ctr->flags);
  return hipGetLastError();
}

hipError_t launch_join_reduce(const DeviceState& st, const u64* recs, u64 R, const u64* cursor, int kb, int bj,
                              u64 n, const Ints& I, const ExcSpace& E, const int* optab, int npairs,
                              const unsigned char* selected, double* gacc, double* inserted, int grid,
                              hipStream_t stream) {
  hipLaunchKernelGGL(k_join_reduce, dim3(grid), dim3(kJoinBlock), 0, stream, recs, R, cursor, kb, bj, st.keys,
                     st.amps, st.diag, n, I, E, optab, npairs, selected, gacc, &st.ctr->flags, inserted);
  return hipGetLastError();
}

}  // namespace swcs

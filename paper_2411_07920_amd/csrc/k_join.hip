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
//             one for itself: (d << (kb + bj)) | (f << kb) | bucket(X), where
//             d is D's storage index, f the connection -- its holes and
//             particles as four 6-bit spin-orbital indices when the word has
//             room (all ones for D itself), else (class, hole set, particle
//             set) as ranks -- and bucket(X) the low kb bits of mix64(X); D's
//             records are one
//             coalesced run, and (D, psi(D)) goes to a 16-byte table by d,
//             so the join reaches both with one load per record;
//   sort   -- a stable LSD radix sort on the kb bucket bits only, so every
//             record of one X lands in one contiguous bucket;
//   join   -- a block takes a run of whole buckets, decodes each record
//             back to (D, X), accumulates sigma(X) in an LDS table, then adds
//             psi(D) a_k(D) sigma(X) to g[k] for every record.
// The device-wide traffic is streaming (records written once, sorted in
// kb / 8 passes, read twice from L2-resident runs), where the table path
// pays one random read-modify-write per pair in HBM.
#include <algorithm>

#include "conn_ops.h"

namespace swcs {

constexpr int kJoinEmitBlock = 256;
constexpr int kJoinBlock = 512;
constexpr int kJoinRun = (int)kJoinRunHost;  // records per block step before bucket alignment
constexpr int kJoinSlots = 4096;  // LDS table: keys and sums, 64 KB (two blocks per CU)
constexpr int kJoinCache = 4;     // records per thread and step whose gradient term stays in registers

// Record layout: kb bucket bits, then the connection fields, then the
// storage index.  Orbital fields (orb): h0 | h1 << 6 | p0 << 12 | p1 << 18,
// 24 bits, all ones for D itself; decoding is four extractions.  Rank fields:
// class in 3 bits (7 for D itself), hole-set index in bh bits, particle-set
// index in bp bits; decoding selects the ranked orbitals from D's bits.
struct JoinFmt {
  int kb, bh, bp, orb;
  __host__ __device__ int bj() const { return orb ? 24 : 3 + bh + bp; }
};
constexpr unsigned kJoinSelf = 7;          // class field of the record of D itself (rank fields)
constexpr unsigned kJoinSelfOrb = 0xFFFFFFu;  // fields of the record of D itself (orbital fields)

// Calls f(X, ordinal, field) for every connection of D assigned to this
// lane: ordinal = class offset + hole set * particle sets + particle set (the
// order of for_each_connection), field = the record's connection fields.
template <class F>
__device__ inline void for_each_connection_fields(const ConnTables& T, u64 D, const JoinFmt& fm, F&& f) {
  long long off = 0;
  for (int c = 0; c < 5; ++c) {
    const int nh = T.nh[c], np = T.np[c];
    if (nh == 0 || np == 0) continue;
    const int hb = T.hbeg[c], pb = T.pbeg[c];
    int hi = (int)threadIdx.x / np;
    int pi = (int)threadIdx.x - hi * np;
    const u64 cf = (u64)c << (fm.bh + fm.bp);
    while (hi < nh) {
      const int H = hb + hi, Pp = pb + pi;
      const u64 X = D ^ T.hmask[H] ^ T.pmask[Pp];
      const u64 field = fm.orb ? ((u64)T.h0[H] | ((u64)T.h1[H] << 6) | ((u64)T.p0[Pp] << 12) | ((u64)T.p1[Pp] << 18))
                               : (cf | ((u64)hi << fm.bp) | (u64)pi);
      f(X, off + (long long)hi * np + pi, field);
      pi += blockDim.x;
      while (pi >= np) {
        pi -= np;
        ++hi;
      }
    }
    off += (long long)nh * np;
  }
}

// Position of the r-th (from 0) set bit of m (m has more than r set bits),
// by halving: six popcounts instead of a walk over the bits below it.
__device__ inline int select_bit(u64 m, unsigned r) {
  int pos = 0;
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) {
    const u64 low = m & ((1ULL << w) - 1ULL);
    const unsigned c = (unsigned)__popcll(low);
    if (r >= c) {
      r -= c;
      m >>= w;
      pos += w;
    } else {
      m = low;
    }
  }
  return pos;
}

// Connection of a record: holes h0 <= h1 and particles p0 <= p1
// (spin-orbitals; equal for singles) from the class and set indices: the
// r-th occupied or virtual spin-orbital of one spin is the r-th set bit of
// D's (or its complement's) bits of that spin; pairs of one spin come from
// the triangular pair tables (px, py) of the enumeration.
__device__ inline u64 join_decode(const ExcSpace& E, u64 D, unsigned c, unsigned hi, unsigned pi,
                                  const unsigned char* px, const unsigned char* py, int* nh, int* h0, int* h1,
                                  int* p0, int* p1) {
  const u64 amask = 0x5555555555555555ULL, bmask = 0xAAAAAAAAAAAAAAAAULL;
  const u64 full = (E.n >= 32) ? ~0ULL : ((1ULL << (2 * E.n)) - 1ULL);
  const u64 oa = D & amask, ob = D & bmask, xa = ~D & amask & full, xb = ~D & bmask & full;
  if (c < 2) {
    *nh = 1;
    *h0 = *h1 = select_bit(c == 0 ? oa : ob, hi);
    *p0 = *p1 = select_bit(c == 0 ? xa : xb, pi);
  } else if (c < 4) {
    *nh = 2;
    const u64 o = c == 2 ? oa : ob, v = c == 2 ? xa : xb;
    *h0 = select_bit(o, px[hi]);
    *h1 = select_bit(o, py[hi]);
    *p0 = select_bit(v, px[pi]);
    *p1 = select_bit(v, py[pi]);
  } else {
    *nh = 2;
    const unsigned nb = (unsigned)E.nb, vb = (unsigned)E.vb;
    const unsigned i = hi / nb, a = pi / vb;
    const int ha = select_bit(oa, i), hb = select_bit(ob, hi - i * nb);
    const int pa = select_bit(xa, a), pb = select_bit(xb, pi - a * vb);
    *h0 = min(ha, hb);
    *h1 = max(ha, hb);
    *p0 = min(pa, pb);
    *p1 = max(pa, pb);
  }
  const u64 hm = (1ULL << *h0) | (1ULL << *h1), pm = (1ULL << *p0) | (1ULL << *p1);
  return D ^ hm ^ pm;
}

// Source entry of the records: key and amplitude side by side.
struct JoinSrc {
  u64 key;
  double psi;
};

// One run of C + 1 records per alive entry, at a position taken from
// *cursor, and (D, psi(D)) at src[d]; runs past cap_recs are not written
// and raise kFlagOverflow.
__global__ void __launch_bounds__(kJoinEmitBlock)
k_join_emit(const u64* __restrict__ keys, const double* __restrict__ amps, ExcSpace E, u64 n,
            u64* __restrict__ recs, u64 cap_recs, u64* __restrict__ cursor, JoinFmt fm,
            JoinSrc* __restrict__ src, unsigned* __restrict__ flags) {
  __shared__ SigShared S;
  __shared__ ConnTables T;
  extern __shared__ __align__(16) unsigned char conn_dyn[];
  __shared__ u64 s_base;
  build_pair_table(S);
  if (threadIdx.x == 0) attach_conn_tables(T, conn_dyn, E);
  const u64 C = (u64)E.total;
  const u64 bmask = (1ULL << fm.kb) - 1ULL;
  const int sd = fm.kb + fm.bj();
  for (u64 d = blockIdx.x; d < n; d += gridDim.x) {
    const double psi = amps[d];
    if (is_dead(psi)) continue;
    const u64 D = keys[d];
    __syncthreads();
    build_lists_shared(D, E.n, S);
    if (threadIdx.x == 0) s_base = atomicAdd(cursor, C + 1);
    __syncthreads();
    build_conn_tables(S, E, T);
    if (threadIdx.x == 0) src[d] = JoinSrc{D, psi};
    __syncthreads();
    const u64 base = s_base;
    if (base + C + 1 > cap_recs) {
      if (threadIdx.x == 0) atomicOr(flags, kFlagOverflow);
      continue;
    }
    const u64 hd = d << sd;
    for_each_connection_fields(T, D, fm, [&](u64 X, long long j, u64 field) {
      recs[base + (u64)j] = hd | (field << fm.kb) | (mix64(X) & bmask);
    });
    if (threadIdx.x == 0) {
      const u64 self_field = fm.orb ? (u64)kJoinSelfOrb : ((u64)kJoinSelf << (fm.bh + fm.bp));
      recs[base + C] = hd | (self_field << fm.kb) | (mix64(D) & bmask);
    }
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

// Fields of a record.
struct JoinRec {
  u64 d;
  unsigned f;  // connection fields
};
__device__ inline JoinRec join_rec(u64 r, const JoinFmt& fm) {
  JoinRec o;
  o.f = (unsigned)((r >> fm.kb) & ((1ULL << fm.bj()) - 1ULL));
  o.d = r >> (fm.kb + fm.bj());
  return o;
}

__device__ inline bool join_is_self(const JoinFmt& fm, const JoinRec& r) {
  return fm.orb ? r.f == kJoinSelfOrb : (r.f >> (fm.bh + fm.bp)) == kJoinSelf;
}

// Connection of a pair record: X and its holes h0 <= h1 and particles
// p0 <= p1 (equal for singles), or false when the fields name no connection
// of D (a record that was never written cannot index outside the state, the
// integrals or the tables).
__device__ inline bool join_connection(const JoinFmt& fm, const ExcSpace& E, u64 D, const JoinRec& r,
                                       const unsigned char* px, const unsigned char* py, u64* X, int* nh,
                                       int* h0, int* h1, int* p0, int* p1) {
  if (fm.orb) {
    const unsigned n2 = 2u * (unsigned)E.n;
    const unsigned a = r.f & 63u, b = (r.f >> 6) & 63u, c = (r.f >> 12) & 63u, d = (r.f >> 18) & 63u;
    if (a > b || c > d || b >= n2 || d >= n2 || ((a == b) != (c == d))) return false;
    const u64 hm = (1ULL << a) | (1ULL << b), pm = (1ULL << c) | (1ULL << d);
    if ((D & hm) != hm || (D & pm) != 0) return false;
    *nh = (a == b) ? 1 : 2;
    *h0 = (int)a;
    *h1 = (int)b;
    *p0 = (int)c;
    *p1 = (int)d;
    *X = D ^ hm ^ pm;
    return true;
  }
  const unsigned c = r.f >> (fm.bh + fm.bp);
  const unsigned hi = (r.f >> fm.bp) & ((1u << fm.bh) - 1u), pi = r.f & ((1u << fm.bp) - 1u);
  const int na = E.na, nb = E.nb, va = E.va, vb = E.vb;
  const unsigned nhs[5] = {(unsigned)na, (unsigned)nb, (unsigned)(na * (na - 1) / 2), (unsigned)(nb * (nb - 1) / 2),
                           (unsigned)(na * nb)};
  const unsigned nps[5] = {(unsigned)va, (unsigned)vb, (unsigned)(va * (va - 1) / 2), (unsigned)(vb * (vb - 1) / 2),
                           (unsigned)(va * vb)};
  if (c >= 5 || hi >= nhs[c] || pi >= nps[c]) return false;
  *X = join_decode(E, D, c, hi, pi, px, py, nh, h0, h1, p0, p1);
  return true;
}

// 64-bit lane exchange: the value v of lane src.
__device__ inline u64 shfl_u64(u64 v, int src) {
  const unsigned lo = (unsigned)__shfl((int)(unsigned)v, src);
  const unsigned hi = (unsigned)__shfl((int)(unsigned)(v >> 32), src);
  return ((u64)hi << 32) | lo;
}

// <X|H|D> for the single excitations X = a+_A a_Ih D held by the lanes set
// in ball (each lane its own D, Ih and A), formed by the whole wavefront:
// sixteen lanes per excitation, each adding the two-electron terms of every
// sixteenth occupied spin-orbital of D, then a four-step reduction.  A wave
// whose records include a single (most waves: singles are scattered through
// the sorted records) thus pays one round of integral loads per four
// singles instead of one per electron.  Called by every lane of the wave.
// Returns the element in the lanes set in ball.
__device__ inline double single_elements_wave(const Ints& I, u64 ball, u64 D, int Ih, int A) {
  const int lane = (int)(threadIdx.x & 63u);
  const int g = lane >> 4, j = lane & 15;
  const int cnt = __popcll(ball);
  const bool mine = ((ball >> lane) & 1ULL) != 0;
  const int rank = __popcll(ball & ((1ULL << lane) - 1ULL));
  double two = 0.0;
  for (int base = 0; base < cnt; base += 4) {
    const bool act = base + g < cnt;
    const int from = act ? select_bit(ball, (unsigned)(base + g)) : lane;
    const u64 Dg = shfl_u64(D, from);
    const int Ig = __shfl(Ih, from), Ag = __shfl(A, from);
    double t = 0.0;
    if (act) {
      const int a = Ag >> 1, i = Ig >> 1, ne = __popcll(Dg);
      for (int r = j; r < ne; r += 16) {
        const int Q = select_bit(Dg, (unsigned)r);
        const int q = Q >> 1;
        t += eri_sp(I, a, i, q, q);
        if (((Q ^ Ag) & 1) == 0) t -= eri_sp(I, a, q, q, i);
      }
    }
    t += __shfl_xor(t, 8);
    t += __shfl_xor(t, 4);
    t += __shfl_xor(t, 2);
    t += __shfl_xor(t, 1);
    const double got = __shfl(t, ((rank - base) & 3) << 4);
    if (mine && rank >= base && rank < base + 4) two = got;
  }
  if (!mine) return 0.0;
  int s = __popcll(D & ((1ULL << Ih) - 1ULL));
  s += __popcll((D ^ (1ULL << Ih)) & ((1ULL << A) - 1ULL));
  const double v = I.h[(A >> 1) * I.n + (Ih >> 1)] + two;
  return (s & 1) ? -v : v;
}

// First pass over one record: sigma(X) += H_{X D} psi(D) (or H_{D D} psi(D)
// for the record of D itself) in the LDS table; *s_bad is set when the table
// is full.  With term, also the record's gradient term: *k the linking
// operator (-1 for none, for an operator not selected and for D itself), *sl
// the LDS slot of X and *w = psi(D) a_k(D).  Called by every lane of the
// wave (singles are formed by the wave together); lanes without a record
// pass valid = false.
__device__ inline void join_record_sigma(bool valid, u64 rec, const JoinFmt& fm, const JoinSrc* __restrict__ src,
                                         const double* __restrict__ diag, u64 n, const Ints& I,
                                         const ExcSpace& E, const int* __restrict__ optab, int nsp,
                                         const unsigned char* __restrict__ selected, const unsigned char* px,
                                         const unsigned char* py, u64* tk, double* tv, double* ins,
                                         unsigned* s_bad, bool term, int* k, int* sl, double* w) {
  *k = -1;
  *sl = 0;
  *w = 0.0;
  bool ok = valid;
  JoinRec r{0, 0};
  JoinSrc sd{0, 0.0};
  if (ok) {
    r = join_rec(rec, fm);
    ok = r.d < n;
  }
  u64 X = 0;
  double v = 0.0;
  int kk = -1;
  double a = 0.0;
  int nh = 0, h0 = 0, h1 = 0, p0 = 0, p1 = 0;
  if (ok) {
    sd = src[r.d];
    X = sd.key;
    if (join_is_self(fm, r)) {
      v = diag[r.d] * sd.psi;
    } else if (!join_connection(fm, E, sd.key, r, px, py, &X, &nh, &h0, &h1, &p0, &p1)) {
      ok = false;
    } else {
      if (nh == 2) v = double_element(I, sd.key, h0, h1, p0, p1) * sd.psi;
      if (term) {
        bool t_acts;
        OpDesc op;
        kk = linking_operator(optab, nsp, nh, h0, h1, p0, p1, &t_acts, &op);
        if (kk >= 0 && selected && !selected[kk]) kk = -1;
        if (kk >= 0) a = t_acts ? (double)phase_of_T(op, sd.key) : -(double)phase_of_T(op, X);
      }
    }
  }
  const bool single = ok && nh == 1;
  const u64 ball = __ballot(single);
  if (ball != 0) {  // uniform over the wave
    const double e = single_elements_wave(I, ball, sd.key, h0, p0);
    if (single) v = e * sd.psi;
  }
  if (!ok) return;
  const int s = join_slot(tk, X, true, ins);
  if (s < 0) {
    *s_bad = 1;
    return;
  }
  atomicAdd(&tv[s], v);
  if (kk >= 0) {
    *k = kk;
    *sl = s;
    *w = sd.psi * a;
  }
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
k_join_reduce(const u64* __restrict__ recs, u64 R, const u64* __restrict__ cursor, JoinFmt fm,
              const JoinSrc* __restrict__ src, const double* __restrict__ diag, u64 n, Ints I, ExcSpace E,
              const int* __restrict__ optab,
              int nsp, const unsigned char* __restrict__ selected, double* __restrict__ gacc,
              JoinTerms terms, unsigned* __restrict__ flags, double* __restrict__ inserted) {
  __shared__ u64 tk[kJoinSlots];
  __shared__ unsigned s_bcnt[1 << kJoinMaxBinsLog], s_boff[1 << kJoinMaxBinsLog];
  __shared__ u64 s_bbase[1 << kJoinMaxBinsLog];
  __shared__ unsigned s_nterm;
  // the staged terms of a step (8 B value, 2 B operator, 1 B bin each) fit
  // the key table
  static_assert(kJoinCache * kJoinBlock * (8 + 2 + 1) <= kJoinSlots * 8, "staging");
  static_assert((1 << kJoinMaxBinsLog) <= 4 * 64 && (1 << kJoinMaxBinsLog) <= kJoinBlock, "bin scan");
  __shared__ double tv[kJoinSlots];
  __shared__ unsigned char px[kMaxPairs], py[kMaxPairs];
  __shared__ unsigned s_found, s_bad;
  __shared__ u64 s_pos;
  __shared__ double red[kJoinBlock / 64];
  const u64 bmask = (1ULL << fm.kb) - 1ULL;
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
  for (int s = threadIdx.x; s < kMaxPairs; s += kJoinBlock) {
    int y = 1;
    while ((y + 1) * y / 2 <= s) ++y;
    py[s] = (unsigned char)y;
    px[s] = (unsigned char)(s - y * (y - 1) / 2);
  }
  for (int s = threadIdx.x; s < kJoinSlots; s += kJoinBlock) tk[s] = kEmptyKey;
  const int nbins = terms.lb >= 0 ? 1 << terms.lb : 0;
  for (int b = threadIdx.x; b < nbins; b += kJoinBlock) s_bcnt[b] = 0;
  for (u64 p = (u64)blockIdx.x * kJoinRun; p < R; p += (u64)gridDim.x * kJoinRun) {
    const u64 lo = bucket_boundary(recs, R, p, bmask, &s_found, &s_pos);
    const u64 hi = bucket_boundary(recs, R, p + kJoinRun, bmask, &s_found, &s_pos);
    if (lo >= hi) continue;  // uniform: the step lies inside a bucket begun earlier
    for (int s = threadIdx.x; s < kJoinSlots; s += kJoinBlock) tv[s] = 0.0;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    // sigma(X) over the step's records.  A record's gradient term is formed
    // here too (operator, psi(D) a_k(D), LDS slot of X) and kept in
    // registers for the thread's first kJoinCache records of the step, so
    // that the second pass decodes only the records beyond them.
    int ck[kJoinCache], csl[kJoinCache];
    double cw[kJoinCache];
#pragma unroll
    for (int m = 0; m < kJoinCache; ++m) {
      const u64 i = lo + threadIdx.x + (u64)m * kJoinBlock;
      const bool valid = i < hi;
      join_record_sigma(valid, valid ? recs[i] : 0, fm, src, diag, n, I, E, optab, nsp, selected, px, py, tk,
                        tv, &ins, &s_bad, true, &ck[m], &csl[m], &cw[m]);
    }
    // (b is uniform over the block, so every lane of a wave takes part)
    for (u64 b = lo + (u64)kJoinCache * kJoinBlock; b < hi; b += kJoinBlock) {
      const u64 i = b + threadIdx.x;
      const bool valid = i < hi;
      int k, sl;
      double w;
      join_record_sigma(valid, valid ? recs[i] : 0, fm, src, diag, n, I, E, optab, nsp, selected, px, py, tk,
                        tv, &ins, &s_bad, false, &k, &sl, &w);
    }
    __syncthreads();
    if (s_bad) {
      if (threadIdx.x == 0) atomicOr(flags, kFlagOverflow);
    } else {
      // psi(D) a_k(D) sigma(X) for every pair record: the terms of the
      // records beyond the cached ones go straight to g[k]; with bins, the
      // cached terms are then appended to their operator's bin -- ranks
      // from LDS counters, one cursor add per bin and step, the step's
      // terms staged in LDS in bin order (over the key table, which is no
      // longer read) and written as one contiguous run per bin.  A term
      // past its bin's capacity goes straight to g[k].
      double xv[kJoinCache];
#pragma unroll
      for (int m = 0; m < kJoinCache; ++m) xv[m] = ck[m] >= 0 ? cw[m] * tv[csl[m]] : 0.0;
      for (u64 i = lo + threadIdx.x + (u64)kJoinCache * kJoinBlock; i < hi; i += kJoinBlock) {
        const JoinRec r = join_rec(recs[i], fm);
        if (r.d >= n || join_is_self(fm, r)) continue;
        const JoinSrc sd = src[r.d];
        const u64 D = sd.key;
        int nh, h0, h1, p0, p1;
        u64 X;
        if (!join_connection(fm, E, D, r, px, py, &X, &nh, &h0, &h1, &p0, &p1)) continue;
        bool t_acts;
        OpDesc op;
        const int k = linking_operator(optab, nsp, nh, h0, h1, p0, p1, &t_acts, &op);
        if (k < 0 || (selected && !selected[k])) continue;
        const int sl = join_slot(tk, X, false, &ins);
        if (sl < 0) continue;  // not reached: pass 1 inserted every key of the step
        const double a = t_acts ? (double)phase_of_T(op, D) : -(double)phase_of_T(op, X);
        unsafeAtomicAdd(&gacc[k], sd.psi * a * tv[sl]);
      }
      if (nbins > 0) {
        unsigned rk[kJoinCache];
#pragma unroll
        for (int m = 0; m < kJoinCache; ++m)
          rk[m] = ck[m] >= 0 ? atomicAdd(&s_bcnt[ck[m] & (nbins - 1)], 1u) : 0u;
        __syncthreads();
        if (threadIdx.x < (unsigned)nbins) {
          const unsigned c = s_bcnt[threadIdx.x];
          s_bbase[threadIdx.x] =
              c ? (u64)atomicAdd((unsigned long long*)&terms.cursor[threadIdx.x], (unsigned long long)c) : 0ULL;
        }
        if (threadIdx.x < 64) {  // exclusive scan of the counts, four bins per lane
          const int l = (int)threadIdx.x;
          unsigned c4[4], sum = 0;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int b = 4 * l + q;
            c4[q] = b < nbins ? s_bcnt[b] : 0u;
            sum += c4[q];
          }
          unsigned inc = sum;
          for (int off = 1; off < 64; off <<= 1) {
            const unsigned v = __shfl_up(inc, off);
            if (l >= off) inc += v;
          }
          unsigned run = inc - sum;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int b = 4 * l + q;
            if (b < nbins) s_boff[b] = run;
            run += c4[q];
          }
          if (l == 63) s_nterm = inc;
        }
        __syncthreads();
        double* sw = reinterpret_cast<double*>(tk);
        unsigned short* sj = reinterpret_cast<unsigned short*>(tk + kJoinCache * kJoinBlock);
        unsigned char* sb = reinterpret_cast<unsigned char*>(tk + kJoinCache * kJoinBlock * 5 / 4);
#pragma unroll
        for (int m = 0; m < kJoinCache; ++m) {
          if (ck[m] < 0) continue;
          const int b = ck[m] & (nbins - 1);
          const unsigned lp = s_boff[b] + rk[m];
          sw[lp] = xv[m];
          sj[lp] = (unsigned short)(ck[m] >> terms.lb);
          sb[lp] = (unsigned char)b;
        }
        if (threadIdx.x < (unsigned)nbins) s_bcnt[threadIdx.x] = 0;
        __syncthreads();
        const unsigned total = s_nterm;
        for (unsigned i = threadIdx.x; i < total; i += kJoinBlock) {
          const int b = sb[i];
          const u64 pos = s_bbase[b] + (i - s_boff[b]);
          if (pos < terms.cap) {
            terms.w[(u64)b * terms.cap + pos] = sw[i];
            terms.j[(u64)b * terms.cap + pos] = sj[i];
          } else {
            unsafeAtomicAdd(&gacc[((long long)sj[i] << terms.lb) | b], sw[i]);
          }
        }
      } else {
#pragma unroll
        for (int m = 0; m < kJoinCache; ++m)
          if (ck[m] >= 0) unsafeAtomicAdd(&gacc[ck[m]], xv[m]);
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

// Record layout for a state of n stored entries: kb bucket bits for about
// 256 records per bucket (8, 16 or 24), the connection fields, the index.
// Returns false when they do not fit 64 bits.
bool join_format(const ExcSpace& E, u64 n, u64 R, int* kb, int* bh, int* bp, int* orb) {
  auto bits_for = [](u64 v) {
    int b = 1;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
  };
  const long long nh = std::max<long long>({(long long)E.na, (long long)E.nb, (long long)E.na * (E.na - 1) / 2,
                                            (long long)E.nb * (E.nb - 1) / 2, (long long)E.na * E.nb, 1LL});
  const long long np = std::max<long long>({(long long)E.va, (long long)E.vb, (long long)E.va * (E.va - 1) / 2,
                                            (long long)E.vb * (E.vb - 1) / 2, (long long)E.va * E.vb, 1LL});
  *bh = bits_for((u64)(nh - 1));
  *bp = bits_for((u64)(np - 1));
  *kb = 8;
  while (*kb < 24 && (R >> *kb) > 256) *kb += 8;
  const int bd = bits_for(n > 0 ? n - 1 : 0);
  *orb = (*kb + 24 + bd <= 64) ? 1 : 0;
  return *orb || *kb + 3 + *bh + *bp + bd <= 64;
}

hipError_t launch_join_emit(const DeviceState& st, const ExcSpace& E, u64 n, u64* recs, u64 cap_recs,
                            u64* cursor, int kb, int bh, int bp, int orb, void* src, int grid, hipStream_t stream) {
  const JoinFmt fm{kb, bh, bp, orb};
  hipLaunchKernelGGL(k_join_emit, dim3(grid), dim3(kJoinEmitBlock), conn_tables_bytes(E), stream, st.keys, st.amps, E,
                     n, recs, cap_recs, cursor, fm, (JoinSrc*)src, &st.ctr->flags);
  return hipGetLastError();
}

hipError_t launch_join_reduce(const DeviceState& st, const u64* recs, u64 R, const u64* cursor, int kb, int bh,
                              int bp, int orb, const void* src, u64 n, const Ints& I, const ExcSpace& E,
                              const int* optab, int nsp, const unsigned char* selected, double* gacc,
                              JoinTerms terms, double* inserted, int grid, hipStream_t stream) {
  if (terms.lb > kJoinMaxBinsLog) return hipErrorInvalidValue;
  const JoinFmt fm{kb, bh, bp, orb};
  hipLaunchKernelGGL(k_join_reduce, dim3(grid), dim3(kJoinBlock), 0, stream, recs, R, cursor, fm,
                     (const JoinSrc*)src, st.diag, n, I, E, optab, nsp, selected, gacc, terms, &st.ctr->flags,
                     inserted);
  return hipGetLastError();
}

// One block per (bin, chunk of `chunk` terms): the chunk's terms are added
// into an LDS table of the bin's operators, then each nonzero sum goes to g[k]
// with one device-scope add.  Chunks hold 2^20 terms for large joins and
// fewer (down to 4,096) for small ones, so that a launch has about a thousand
// blocks.
constexpr u64 kJoinTermChunkMax = 1ULL << 20, kJoinTermChunkMin = 1ULL << 12;
__global__ void __launch_bounds__(kJoinBlock)
k_join_terms(JoinTerms terms, int per_bin, u64 chunk, double* __restrict__ gacc, long long K) {
  __shared__ double acc[kJoinTermSlots];
  const int b = (int)(blockIdx.x / (unsigned)per_bin);
  const u64 c = blockIdx.x % (unsigned)per_bin;
  const u64 filled = terms.cursor[b] < terms.cap ? terms.cursor[b] : terms.cap;
  const u64 lo = c * chunk;
  if (lo >= filled) return;  // uniform over the block
  const u64 hi = lo + chunk < filled ? lo + chunk : filled;
  for (int s = threadIdx.x; s < kJoinTermSlots; s += kJoinBlock) acc[s] = 0.0;
  __syncthreads();
  const double* __restrict__ w = terms.w + (u64)b * terms.cap;
  const unsigned short* __restrict__ j = terms.j + (u64)b * terms.cap;
  // four terms per thread and load (chunks start at multiples of four and
  // bins at multiples of eight entries, so the vector loads are aligned)
  const u64 n4 = (hi - lo) / 4;
  const double2* __restrict__ w2 = reinterpret_cast<const double2*>(w + lo);
  const ushort4* __restrict__ j4 = reinterpret_cast<const ushort4*>(j + lo);
  for (u64 q = threadIdx.x; q < n4; q += kJoinBlock) {
    const double2 a = w2[2 * q], bb = w2[2 * q + 1];
    const ushort4 s = j4[q];
    if (s.x < kJoinTermSlots) atomicAdd(&acc[s.x], a.x);
    if (s.y < kJoinTermSlots) atomicAdd(&acc[s.y], a.y);
    if (s.z < kJoinTermSlots) atomicAdd(&acc[s.z], bb.x);
    if (s.w < kJoinTermSlots) atomicAdd(&acc[s.w], bb.y);
  }
  for (u64 i = lo + 4 * n4 + threadIdx.x; i < hi; i += kJoinBlock) {
    const unsigned s = j[i];
    if (s < (unsigned)kJoinTermSlots) atomicAdd(&acc[s], w[i]);
  }
  __syncthreads();
  for (int s = threadIdx.x; s < kJoinTermSlots; s += kJoinBlock) {
    const double v = acc[s];
    const long long k = ((long long)s << terms.lb) | b;
    if (v != 0.0 && k < K) unsafeAtomicAdd(&gacc[k], v);
  }
}

hipError_t launch_join_terms(JoinTerms terms, double* gacc, long long K, hipStream_t stream) {
  if (terms.lb < 0) return hipSuccess;
  if (terms.lb > kJoinMaxBinsLog) return hipErrorInvalidValue;
  u64 chunk = kJoinTermChunkMin;
  while (chunk < kJoinTermChunkMax && (terms.cap << terms.lb) / chunk > 1024) chunk <<= 1;
  const u64 per_bin = (terms.cap + chunk - 1) / chunk;
  const u64 grid = per_bin << terms.lb;
  if (per_bin == 0 || grid > 0x7fffffffULL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_join_terms, dim3((unsigned)grid), dim3(kJoinBlock), 0, stream, terms, (int)per_bin, chunk,
                     gacc, K);
  return hipGetLastError();
}

}  // namespace swcs

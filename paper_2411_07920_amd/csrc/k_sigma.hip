// Sigma-vector kernels: the projected sigma vector and energy, the external
// sigma vector pushed into an accumulation table, the pool-gradient
// contraction, occupations and deterministic reductions.
//
// Matrix elements follow the Slater-Condon rules (Szabo & Ostlund, cited in
// Sec. III) for H = sum h a+a + 1/2 sum (pq|rs) a+a+aa.  One block handles
// one determinant at a time: its occupied / virtual lists and the hole- and
// particle-set tables of its spin-conserving singles and doubles are staged
// in LDS, and the lanes walk the connections from those tables.
#include "conn_ops.h"

namespace swcs {

__device__ inline double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kSigBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Diagonal Slater-Condon elements of the stored determinants (0 for dead
// entries).  A group of kDiagLanes lanes takes one determinant: lane j of the
// group handles the occupied spin-orbitals of rank j, j + kDiagLanes, ...
// against all occupied ones, with J, K and diag(h) staged in LDS; the group
// sums its lanes in a fixed order.
constexpr int kDiagMaxN = 32;  // spatial orbitals (2n <= 64)

__global__ void __launch_bounds__(256)
k_diag(const u64* __restrict__ keys, const double* __restrict__ amps, u64 n, Ints I,
       double* __restrict__ diag) {
  __shared__ double sJ[kDiagMaxN * kDiagMaxN], sK[kDiagMaxN * kDiagMaxN], sh[kDiagMaxN];
  const int no = I.n;
  for (int t = threadIdx.x; t < no * no; t += blockDim.x) {
    sJ[t] = I.J[t];
    sK[t] = I.K[t];
  }
  for (int t = threadIdx.x; t < no; t += blockDim.x) sh[t] = I.h[t * no + t];
  __syncthreads();
  const int sub = (int)threadIdx.x & (kDiagLanes - 1);
  const u64 per_pass = ((u64)gridDim.x * blockDim.x) / kDiagLanes;
  // the pass loop has the same trip count in every lane, so the group sums
  // below run with all lanes active
  for (u64 base = 0; base < n; base += per_pass) {
    const u64 d = base + ((u64)blockIdx.x * blockDim.x + threadIdx.x) / kDiagLanes;
    const bool valid = d < n;
    const bool alive = valid && !is_dead(amps[d]);
    double e = 0.0;
    if (alive) {
      const u64 D = keys[d];
      // this lane's electrons: ranks sub, sub + kDiagLanes, ... (the lanes of
      // a wavefront step through their electrons in lockstep)
      u64 x = D;
      for (int t = 0; t < sub && x; ++t) x &= x - 1;
      while (x) {
        const int P = __ffsll((long long)x) - 1;
        const int p = P >> 1;
        double ep = 0.0;
        u64 y = D;
        while (y) {
          const int Q = __ffsll((long long)y) - 1;
          y &= y - 1;
          double v = sJ[p * no + (Q >> 1)];
          if (((P ^ Q) & 1) == 0) v -= sK[p * no + (Q >> 1)];
          ep += v;
        }
        e += sh[p] + 0.5 * ep;
        for (int t = 0; t < kDiagLanes && x; ++t) x &= x - 1;
      }
    }
    for (int off = 1; off < kDiagLanes; off <<= 1) e += __shfl_xor(e, off);
    if (valid && sub == 0) diag[d] = alive ? I.ecore + e : 0.0;
  }
}

// sigma_P(D) = sum_{D' in psi} H_{D D'} psi(D') for every stored entry D
// (dead entries get 0), plus per-block partial sums of psi*sigma and psi^2.
__global__ void __launch_bounds__(kSigBlock)
k_sigma_proj(const u64* __restrict__ keys, const double* __restrict__ amps,
             const HashSlot* __restrict__ hash, u64 hmask, const unsigned* __restrict__ filt,
             u64 fmask, Ints I, ExcSpace E, u64 n, const double* __restrict__ diag,
             double* __restrict__ sigma, double* __restrict__ partial) {
  __shared__ SigShared S;
  __shared__ ConnTables T;
  extern __shared__ __align__(16) unsigned char conn_dyn[];
  __shared__ double red[kSigBlock];
  build_pair_table(S);
  if (threadIdx.x == 0) attach_conn_tables(T, conn_dyn, E);
  double num = 0.0, nrm = 0.0;
  for (u64 d = blockIdx.x; d < n; d += gridDim.x) {
    const double psiD = amps[d];
    if (is_dead(psiD)) {
      if (threadIdx.x == 0) sigma[d] = 0.0;
      continue;
    }
    const u64 D = keys[d];
    __syncthreads();
    build_lists_shared(D, I.n, S);
    __syncthreads();
    build_conn_tables(S, E, T);
    __syncthreads();
    double acc = 0.0;
    for_each_connection(T, D, [&](u64 X, int nh, int h0, int h1, int p0, int p1) {
      if (!filter_maybe(filt, fmask, X)) return;
      const long long j = hash_find(hash, hmask, X);
      if (j < 0) return;
      const double psiX = amps[j];
      if (is_dead(psiX)) return;
      acc += connection_element(I, D, nh, h0, h1, p0, p1) * psiX;
    });
    if (threadIdx.x == 0) acc += diag[d] * psiD;
    const double sig = block_sum(acc, red);
    if (threadIdx.x == 0) {
      sigma[d] = sig;
      num += psiD * sig;
      nrm += psiD * psiD;
    }
  }
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = num;
    partial[gridDim.x + blockIdx.x] = nrm;
  }
}

// ---------------------------------------------------------------- hole pairs
// sigma_P for large states by grouping instead of enumeration.  Two distinct
// determinants of one sector have a nonzero Slater-Condon element only if
// they differ in at most two electrons, so they share at least one subset of
// N_e - 2 electrons.  Every alive entry emits its C(N_e, 2) such subsets (its
// key with two occupied bits cleared); after a sort by subset the members of
// each group are exactly the candidate partners.  A double-excitation pair
// shares one subset; a single-excitation pair shares N_e - 1 and is counted
// only on the one that drops the lowest common electron.
//
// A subset removes two alpha electrons (class 0), one of each spin (class 1)
// or two beta electrons (class 2); subsets of different classes never
// coincide.  Within a class a subset is keyed by
//   rank(alpha string) * C(n, beta count) + rank(beta string),
// with the rank of a string of occupied spatial orbitals p_1 < p_2 < ... in
// the combinatorial number system (sum over j of C(p_j, j)), a bijection onto
// [0, C(n, alpha count) C(n, beta count)); the class sits in bits 60 and up.
// Each class's records form one segment that is sorted on its own, on
// fewer key bits than a rank over all 2n spin-orbitals would need.

struct BinomTable {
  u64 v[65][65];  // v[m][k] = C(m, k); C(64, 32) < 2^63
};

constexpr BinomTable make_binom_table() {
  BinomTable t{};
  for (int m = 0; m <= 64; ++m) {
    t.v[m][0] = 1;
    for (int k = 1; k <= m; ++k) t.v[m][k] = t.v[m - 1][k - 1] + (k < m ? t.v[m - 1][k] : 0);
  }
  return t;
}

__constant__ BinomTable kBinom = make_binom_table();
constexpr int kClassShift = 60;

// Spatial string of one spin of an interleaved key (bit p = orbital p).
__device__ inline u64 spin_string(u64 D, int spin) {
  u64 x = (D >> spin) & 0x5555555555555555ULL;
  x = (x | (x >> 1)) & 0x3333333333333333ULL;
  x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0FULL;
  x = (x | (x >> 4)) & 0x00FF00FF00FF00FFULL;
  x = (x | (x >> 8)) & 0x0000FFFF0000FFFFULL;
  x = (x | (x >> 16)) & 0x00000000FFFFFFFFULL;
  return x;
}

__device__ inline u64 string_rank(u64 S) {
  u64 r = 0;
  for (int j = 1; S; ++j) {
    r += kBinom.v[__ffsll((long long)S) - 1][j];
    S &= S - 1;
  }
  return r;
}

// Key of a subset of na + nb - 2 electrons (na, nb: the sector's counts).
__device__ inline u64 subset_key(u64 S, int n_spatial, int na) {
  const u64 sa = spin_string(S, 0), sb = spin_string(S, 1);
  const int ca = __popcll(sa), cb = __popcll(sb);
  const u64 cls = (ca == na - 2) ? 0 : (ca == na - 1 ? 1 : 2);
  return (cls << kClassShift) | (string_rank(sa) * kBinom.v[n_spatial][cb] + string_rank(sb));
}

// Triangular index p = b (b - 1) / 2 + a, a < b.
__device__ inline void tri_decode(u64 p, u64* a, u64* b) {
  u64 bb = (u64)((1.0 + sqrt(1.0 + 8.0 * (double)p)) * 0.5);
  while (bb * (bb - 1) / 2 > p) --bb;
  while ((bb + 1) * bb / 2 <= p) ++bb;
  *b = bb;
  *a = p - bb * (bb - 1) / 2;
}

__device__ inline u64 readlane_u64(u64 v, int l) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
  return ((u64)hi << 32) | lo;
}

// Inclusive prefix sum over each 32-lane half of the wavefront by DPP row
// shifts (1, 2, 4, 8 within 16-lane rows) and a broadcast of lane 15 of rows
// 0 and 2 into rows 1 and 3.
__device__ inline unsigned half_scan_u32(unsigned v) {
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  return v;
}

// One wavefront per entry; records of class 0, 1, 2 go to the segments that
// start at 0, n r0 and n (r0 + r1) (r0 = C(na, 2), r1 = na nb), entry i's at
// i r_c + p.  Lanes 0..31 hold the alpha electrons and 32..63 the beta ones:
// lane s + l holds the orbital c_l of electron l of its spin and, as
// inclusive prefix sums over l within the half, IA, IB, IG of C(c_l, l + 1),
// C(c_l, l) and C(c_l, l - 1) -- the rank terms of an electron kept with
// none, one or two removed electrons below it.  A string's rank is then
//   none removed:  IA[cnt - 1]
//   a removed:     IA[a - 1] + IB[cnt - 1] - IB[a]
//   a < b removed: IA[a - 1] + IB[b - 1] - IB[a] + IG[cnt - 1] - IG[b].
// Every partial sum is a rank of some string of at most 32 orbitals, below
// C(32, 16) < 2^32, so the sums are 32-bit.
// Dead entries emit the key ~0 (class bits 3, low bits above every rank).
// With shift > 0 a record is one word instead: the key without its class in
// the low `shift` bits (all ones for dead entries) and the entry index above
// them, and out_val is not used.
// A wavefront takes `cw` (1..64) consecutive entries at a time, loaded by
// one coalesced read (the next chunk's read is issued before this chunk's
// work), and handles them one after another; the removed pairs of record
// p < 64 are decoded once.
__global__ void __launch_bounds__(256)
k_holepair_emit(const u64* __restrict__ keys, const double* __restrict__ amps, u64 n, int n_spatial,
                int na, int nb, int shift, int cw, u64* __restrict__ out_key, unsigned* __restrict__ out_val) {
  const u64 rmask = shift ? (1ULL << shift) - 1ULL : 0ULL;
  const int lane = threadIdx.x & 63, half = lane >> 5, hl = lane & 31;
  const u64 r0 = (u64)na * (u64)(na - 1) / 2, r1 = (u64)na * (u64)nb, r2 = (u64)nb * (u64)(nb - 1) / 2;
  const u64 seg1 = n * r0, seg2 = n * (r0 + r1);
  const u64 mul0 = kBinom.v[n_spatial][nb], mul1 = kBinom.v[n_spatial][nb > 0 ? nb - 1 : 0],
            mul2 = kBinom.v[n_spatial][nb > 1 ? nb - 2 : 0];
  // removed pairs of record p = lane (first 64 records of each class)
  u64 ta0, tb0;
  tri_decode((u64)lane, &ta0, &tb0);
  const unsigned xa0 = nb > 0 ? (unsigned)lane / (unsigned)nb : 0u;
  const unsigned xb0 = (unsigned)lane - xa0 * (unsigned)nb;
  // C(m, k) for the m < 32 orbitals and k <= 33 the prefix terms use, in LDS
  // (all below 2^32), so that the three lookups of a determinant are issued
  // together
  __shared__ unsigned sbin[32 * 34];
  for (int t = threadIdx.x; t < 32 * 34; t += blockDim.x) sbin[t] = (unsigned)kBinom.v[t / 34][t % 34];
  __syncthreads();
  const u64 nchunk = (n + (u64)cw - 1) / (u64)cw;
  const u64 w0 = ((u64)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const u64 wstride = ((u64)gridDim.x * blockDim.x) >> 6;
  u64 next_key = 0, next_amp = kDeadBits;
  if (w0 < nchunk && lane < cw && w0 * cw + lane < n) {
    next_key = keys[w0 * cw + lane];
    next_amp = (u64)__double_as_longlong(amps[w0 * cw + lane]);
  }
  for (u64 ch = w0; ch < nchunk; ch += wstride) {
    const u64 ck = next_key, ca = next_amp;
    const u64 nx = ch + wstride;
    if (nx < nchunk && lane < cw && nx * cw + lane < n) {
      next_key = keys[nx * cw + lane];
      next_amp = (u64)__double_as_longlong(amps[nx * cw + lane]);
    }
    const u64 i0 = ch * (u64)cw;
    const int m = (int)((n - i0) < (u64)cw ? (n - i0) : (u64)cw);
    for (int j = 0; j < m; ++j) {
      const u64 i = i0 + (u64)j;
      const bool dead = readlane_u64(ca, j) == kDeadBits;  // uniform
      const u64 D = readlane_u64(ck, j);
      u64 x = spin_string(D, half);
      const int cnt = half ? nb : na;
      for (int t = 0; t < hl && x; ++t) x &= x - 1;
      const bool mine = hl < cnt;
      const int c = mine ? __ffsll((long long)x) - 1 : 0;
      const unsigned* row = sbin + c * 34;
      const unsigned va = row[hl + 1], vb = row[hl], vg = row[hl >= 1 ? hl - 1 : 0];
      const unsigned ia = half_scan_u32(mine ? va : 0u);
      const unsigned ib = half_scan_u32(mine ? vb : 0u);
      const unsigned ig = half_scan_u32((mine && hl >= 1) ? vg : 0u);
      // whole strings and the top prefix values (uniform lanes)
      const u64 full_a = na > 0 ? (unsigned)__builtin_amdgcn_readlane((int)ia, na - 1) : 0u;
      const u64 full_b = nb > 0 ? (unsigned)__builtin_amdgcn_readlane((int)ia, 32 + nb - 1) : 0u;
      const unsigned ib_top_a = na > 0 ? (unsigned)__builtin_amdgcn_readlane((int)ib, na - 1) : 0u;
      const unsigned ib_top_b = nb > 0 ? (unsigned)__builtin_amdgcn_readlane((int)ib, 32 + nb - 1) : 0u;
      const unsigned ig_top_a = na > 0 ? (unsigned)__builtin_amdgcn_readlane((int)ig, na - 1) : 0u;
      const unsigned ig_top_b = nb > 0 ? (unsigned)__builtin_amdgcn_readlane((int)ig, 32 + nb - 1) : 0u;
      // class 0 and 2: two electrons of one spin removed (s = 0 alpha, 32 beta)
      for (int cls = 0; cls < 3; cls += 2) {
        const int s = cls ? 32 : 0;
        const u64 rc = cls ? r2 : r0, base = (cls ? seg2 : 0) + i * rc;
        const unsigned ig_top = cls ? ig_top_b : ig_top_a;
        const u64 other = cls ? full_a : full_b;
        for (u64 p0 = 0; p0 < rc; p0 += 64) {
          const u64 p = p0 + (u64)lane;
          const bool valid = p < rc;
          u64 a = ta0, b = tb0;
          if (p0 > 0) {
            a = 0;
            b = 1;
            if (valid) tri_decode(p, &a, &b);
          } else if (!valid) {
            a = 0;
            b = 1;
          }
          const unsigned a_lo = (unsigned)__shfl((int)ia, s + (a > 0 ? (int)a - 1 : 0));
          const unsigned b_lo = (unsigned)__shfl((int)ib, s + (int)b - 1);
          const unsigned b_a = (unsigned)__shfl((int)ib, s + (int)a);
          const unsigned g_b = (unsigned)__shfl((int)ig, s + (int)b);
          if (valid) {
            const u64 r = (u64)((a > 0 ? a_lo : 0u) + (b_lo - b_a) + (ig_top - g_b));
            const u64 key = cls ? (other * mul2 + r) : (r * mul0 + other);
            if (shift) {
              out_key[base + p] = (dead ? rmask : (key & rmask)) | (i << shift);
            } else {
              out_key[base + p] = dead ? ~0ULL : (((u64)cls << kClassShift) | key);
              out_val[base + p] = (unsigned)i;
            }
          }
        }
      }
      // class 1: alpha electron a and beta electron b removed
      for (u64 p0 = 0; p0 < r1; p0 += 64) {
        const u64 p = p0 + (u64)lane;
        const bool valid = p < r1;
        unsigned a = 0, b = 0;
        if (valid) {
          if (p0 == 0) {
            a = xa0;
            b = xb0;
          } else {
            a = (unsigned)p / (unsigned)nb;
            b = (unsigned)p - a * (unsigned)nb;
          }
        }
        const unsigned aa_lo = (unsigned)__shfl((int)ia, a > 0 ? (int)a - 1 : 0);
        const unsigned ab = (unsigned)__shfl((int)ib, (int)a);
        const unsigned ba_lo = (unsigned)__shfl((int)ia, 32 + (b > 0 ? (int)b - 1 : 0));
        const unsigned bb = (unsigned)__shfl((int)ib, 32 + (int)b);
        if (valid) {
          const u64 ra = (u64)((a > 0 ? aa_lo : 0u) + (ib_top_a - ab));
          const u64 rb = (u64)((b > 0 ? ba_lo : 0u) + (ib_top_b - bb));
          const u64 key = ra * mul1 + rb;
          if (shift) {
            out_key[seg1 + i * r1 + p] = (dead ? rmask : (key & rmask)) | (i << shift);
          } else {
            out_key[seg1 + i * r1 + p] = dead ? ~0ULL : ((1ULL << kClassShift) | key);
            out_val[seg1 + i * r1 + p] = (unsigned)i;
          }
        }
      }
    }
  }
}

// sigma[i] = H_ii psi_i for alive entries, 0 for dead ones.
__global__ void __launch_bounds__(256)
k_sigma_diag(const double* __restrict__ amps, const double* __restrict__ diag, u64 n,
             double* __restrict__ sigma) {
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double a = amps[i];
    sigma[i] = is_dead(a) ? 0.0 : diag[i] * a;
  }
}

// Sorted records of one class segment: a full key (class in bits 60 and up)
// with a separate entry index, or (shift > 0) one word holding the key
// without its class in the low `shift` bits and the entry index above.
struct HoleRecords {
  const u64* key;
  const unsigned* idx;
  int shift;
  __device__ u64 subset(u64 g) const { return shift ? key[g] & ((1ULL << shift) - 1ULL) : key[g]; }
  __device__ u64 entry(u64 g) const { return shift ? key[g] >> shift : (u64)idx[g]; }
  __device__ bool dead(u64 S) const { return shift ? S == (1ULL << shift) - 1ULL : S == ~0ULL; }
};

// One thread per sorted record of segment `cls`: adds H_{D X} psi(X) over
// the other members X of its group to sigma(D).  The record and both
// neighbours are loaded before any test (clamped at the ends), one grid
// stride ahead, so a record that is a group of one -- nearly all of them --
// costs less than one round trip.
__global__ void __launch_bounds__(256)
k_holepair_sigma(HoleRecords R, u64 total, int cls, const u64* __restrict__ keys,
                 const double* __restrict__ amps, u64 n, Ints I, int na, double* __restrict__ sigma) {
  const u64 stride = (u64)gridDim.x * blockDim.x;
  const u64 g0 = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  u64 nS = 0, nSp = 0, nSn = 0;  // the next record's three words, loaded one step ahead
  if (g0 < total) {
    nS = R.subset(g0);
    nSp = R.subset(g0 > 0 ? g0 - 1 : g0);
    nSn = R.subset(g0 + 1 < total ? g0 + 1 : g0);
  }
  for (u64 g = g0; g < total; g += stride) {
    const u64 S = nS, Sp = nSp, Sn = nSn;
    const u64 gn = g + stride < total ? g + stride : g;
    nS = R.subset(gn);
    nSp = R.subset(gn > 0 ? gn - 1 : gn);
    nSn = R.subset(gn + 1 < total ? gn + 1 : gn);
    const bool prev = (g > 0) & (Sp == S);
    const bool next = (g + 1 < total) & (Sn == S);
    if (!(!R.dead(S) & (prev | next))) continue;  // bitwise: no test before the loads
    u64 lo = g;
    while (lo > 0 && R.subset(lo - 1) == S) --lo;
    u64 hi = g + 1;
    while (hi < total && R.subset(hi) == S) ++hi;
    const u64 iD = R.entry(g);
    if (iD >= n) continue;  // never for records of the emit kernel
    const u64 D = keys[iD];
    // the key of the subset as subset_key forms it
    const u64 S_full = R.shift ? (((u64)cls << kClassShift) | S) : S;
    double acc = 0.0;
    for (u64 f = lo; f < hi; ++f) {
      if (f == g) continue;
      const u64 iX = R.entry(f);
      if (iX >= n) continue;
      const u64 X = keys[iX];
      const u64 diff = D ^ X;
      const u64 holes = D & diff, parts = X & diff;
      double h;
      if (__popcll(diff) == 4) {
        const int h0 = __ffsll((long long)holes) - 1, h1 = 63 - __clzll((long long)holes);
        const int p0 = __ffsll((long long)parts) - 1, p1 = 63 - __clzll((long long)parts);
        h = double_element(I, D, h0, h1, p0, p1);
      } else {
        const u64 common = D & X;
        if (S_full != subset_key(common & (common - 1), I.n, na)) continue;
        h = single_element(I, D, __ffsll((long long)holes) - 1, __ffsll((long long)parts) - 1);
      }
      acc += h * amps[iX];
    }
    if (acc != 0.0) unsafeAtomicAdd(&sigma[iD], acc);
  }
}

// Per-block partial sums of psi * sigma (partial[b]) and psi^2
// (partial[grid + b]) over the alive entries.
__global__ void __launch_bounds__(256)
k_sigma_dots(const double* __restrict__ amps, const double* __restrict__ sigma, u64 n,
             double* __restrict__ partial) {
  __shared__ double r1[256], r2[256];
  double num = 0.0, nrm = 0.0;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double a = amps[i];
    if (is_dead(a)) continue;
    num += a * sigma[i];
    nrm += a * a;
  }
  r1[threadIdx.x] = num;
  r2[threadIdx.x] = nrm;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      r1[threadIdx.x] += r1[threadIdx.x + w];
      r2[threadIdx.x] += r2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = r1[0];
    partial[gridDim.x + blockIdx.x] = r2[0];
  }
}

// ---------------------------------------------------------------- small states
// sigma_P for states of at most kPairCap stored determinants: every pair is tested;
// two determinants of one sector have a nonzero Slater-Condon element only
// if they differ in at most four spin-orbitals, which a popcount decides.
// The whole state sits in LDS (dynamic, at most 64 KB), so there is no index
// or accumulation table and no atomics; each output is a fixed-order sum.
constexpr int kPairCap = 4096;  // sigma_P by pairs: 16 B of LDS per entry

// <X|H|D> for distinct X, D of one sector differing in at most four
// spin-orbitals.
__device__ inline double pair_element(const Ints& I, u64 X, u64 D) {
  const u64 diff = X ^ D;
  const int pc = __popcll(diff);
  const u64 holes = D & diff, parts = X & diff;
  if (pc == 2) return single_element(I, D, __ffsll((long long)holes) - 1, __ffsll((long long)parts) - 1);
  return double_element(I, D, __ffsll((long long)holes) - 1, 63 - __clzll((long long)holes),
                        __ffsll((long long)parts) - 1, 63 - __clzll((long long)parts));
}

__device__ inline void stage_state(const u64* __restrict__ keys, const double* __restrict__ amps,
                                   unsigned n, u64* sk, double* sa) {
  for (unsigned i = threadIdx.x; i < n; i += blockDim.x) {
    const double a = amps[i];
    sk[i] = keys[i];
    sa[i] = is_dead(a) ? 0.0 : a;
  }
}

// sigma_P by pairs: one wavefront per row D, lanes over the columns D'.
// Dead rows get 0; per-block partial sums of psi*sigma and psi^2.
__global__ void __launch_bounds__(256)
k_sigma_pairwise(const u64* __restrict__ keys, const double* __restrict__ amps, unsigned n, Ints I,
                 const double* __restrict__ diag, double* __restrict__ sigma,
                 double* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char pair_dyn[];
  u64* sk = (u64*)pair_dyn;      // n keys
  double* sa = (double*)(sk + n);  // n amplitudes (0 for dead entries)
  __shared__ double r1[4], r2[4];
  stage_state(keys, amps, n, sk, sa);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double num = 0.0, nrm = 0.0;
  for (unsigned d = blockIdx.x * 4 + wave; d < n; d += gridDim.x * 4) {
    const double psiD = sa[d];
    const bool alive = !is_dead(amps[d]);
    const u64 D = sk[d];
    double acc = 0.0;
    if (alive) {
      if (lane == 0) acc = diag[d] * psiD;
      for (unsigned j = lane; j < n; j += 64) {
        const double pj = sa[j];
        if (pj == 0.0 || j == d || __popcll(D ^ sk[j]) > 4) continue;
        acc += pair_element(I, D, sk[j]) * pj;
      }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) {
      sigma[d] = alive ? acc : 0.0;
      num += psiD * acc;
      nrm += psiD * psiD;
    }
  }
  if (lane == 0) {
    r1[wave] = num;
    r2[wave] = nrm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = r1[0] + r1[1] + r1[2] + r1[3];
    partial[gridDim.x + blockIdx.x] = r2[0] + r2[1] + r2[2] + r2[3];
  }
}

// Batch of an external determinant when the accumulation table is split.
__device__ inline int batch_of(u64 X, int nbatch) {
  return (int)((mix64(X ^ 0x9e3779b97f4a7c15ULL) >> 32) % (u64)nbatch);
}

// sigma(X) += H_{X D'} psi(D') for every stored, alive D' and every X among
// D' and its singles and doubles (only X of the current batch).
__global__ void __launch_bounds__(kSigBlock)
k_sigma_push(const u64* __restrict__ keys, const double* __restrict__ amps, Ints I, ExcSpace E,
             u64 n, const double* __restrict__ diag, AccSlot* __restrict__ tab, u64 tmask,
             int nbatch, int batch, unsigned* __restrict__ flags, double* __restrict__ inserted) {
  __shared__ SigShared S;
  __shared__ ConnTables T;
  extern __shared__ __align__(16) unsigned char conn_dyn[];
  __shared__ double red[kSigBlock];
  build_pair_table(S);
  if (threadIdx.x == 0) attach_conn_tables(T, conn_dyn, E);
  double ins = 0.0;  // keys this thread inserted (exact below 2^53)
  for (u64 d = blockIdx.x; d < n; d += gridDim.x) {
    const double psiD = amps[d];
    if (is_dead(psiD)) continue;
    const u64 D = keys[d];
    __syncthreads();
    build_lists_shared(D, I.n, S);
    __syncthreads();
    build_conn_tables(S, E, T);
    __syncthreads();
    if (threadIdx.x == 0 && (nbatch == 1 || batch_of(D, nbatch) == batch)) {
      const int r = acc_add(tab, tmask, D, diag[d] * psiD);
      if (!r) atomicOr(flags, kFlagOverflow);
      ins += (r == 2) ? 1.0 : 0.0;
    }
    for_each_connection(T, D, [&](u64 X, int nh, int h0, int h1, int p0, int p1) {
      if (nbatch > 1 && batch_of(X, nbatch) != batch) return;
      const int r = acc_add(tab, tmask, X, connection_element(I, D, nh, h0, h1, p0, p1) * psiD);
      if (!r) atomicOr(flags, kFlagOverflow);
      ins += (r == 2) ? 1.0 : 0.0;
    });
  }
  const double tot = block_sum(ins, red);
  if (threadIdx.x == 0) inserted[blockIdx.x] = tot;
}

// g_k accumulation, determinant-major: every connection X of every alive D
// names its linking operator k; adds psi(D) a_k(D) sigma(X) to gacc[k]
// (only X of the current batch when the sigma table is split).
__global__ void __launch_bounds__(kSigBlock)
k_pool_contract_det(const u64* __restrict__ keys, const double* __restrict__ amps, ExcSpace E,
                    int n_spatial, u64 n, const int* __restrict__ optab, int nsp,
                    const unsigned char* __restrict__ selected, const AccSlot* __restrict__ tab,
                    u64 tmask, int nbatch, int batch, double* __restrict__ gacc) {
  __shared__ SigShared S;
  __shared__ ConnTables T;
  extern __shared__ __align__(16) unsigned char conn_dyn[];
  build_pair_table(S);
  if (threadIdx.x == 0) attach_conn_tables(T, conn_dyn, E);
  for (u64 d = blockIdx.x; d < n; d += gridDim.x) {
    const double psiD = amps[d];
    if (is_dead(psiD)) continue;
    const u64 D = keys[d];
    __syncthreads();
    build_lists_shared(D, n_spatial, S);
    __syncthreads();
    build_conn_tables(S, E, T);
    __syncthreads();
    for_each_connection(T, D, [&](u64 X, int nh, int h0, int h1, int p0, int p1) {
      if (nbatch > 1 && batch_of(X, nbatch) != batch) return;
      bool t_acts;
      OpDesc op;
      const int k = linking_operator(optab, nsp, nh, h0, h1, p0, p1, &t_acts, &op);
      if (k < 0) return;
      if (selected && !selected[k]) return;
      double sx;
      if (!acc_find(tab, tmask, X, &sx)) return;
      const double a = t_acts ? (double)phase_of_T(op, D) : -(double)phase_of_T(op, X);
      unsafeAtomicAdd(&gacc[k], psiD * a * sx);
    });
  }
}

// Screened pool gradients need sigma only on Q = {X_k(D): k selected, D in
// psi}.  Pass 1 counts (count_only = s >= 1: the (D, k) pairs of every s-th
// determinant, or tile of determinants) or inserts Q into the table; pass 2
// (k_sigma_push_into) adds H_{X D'} psi(D') only for X already in the table,
// evaluating the matrix element only on those hits.  With a presence filter
// of Q (one bit per hash of each query key, set by pass 1 on the key's
// first insert), pass 2 looks a connection up in the table only when its
// bit is set: most connections are not in Q, and the filter is a small
// fraction of the table.
__device__ inline void qfilter_set(unsigned* qf, u64 qfmask, u64 key) {
  const u64 b = filter_bit(key, qfmask);
  atomicOr(&qf[b >> 5], 1u << (b & 31));
}

__device__ inline bool qfilter_maybe(const unsigned* __restrict__ qf, u64 qfmask, u64 key) {
  return !qf || filter_maybe(qf, qfmask, key);
}

// Key-only insert into an accumulation table whose values start at zero:
// 2 when the key was new, 1 when it was there, 0 when no slot was found
// within the probe limit (acc_add without its value add, which for a query
// key would be a device-scope add of zero per (operator, determinant) pair).
__device__ inline int acc_insert(AccSlot* tab, u64 mask, u64 key) {
  u64 h = mix64(key) & mask;
  const u64 lim = mask < kAccMaxProbes ? mask : kAccMaxProbes;
  for (u64 probes = 0; probes <= lim; ++probes) {
    const u64 k = tab[h].key;
    if (k == key) return 1;
    if (k == kEmptyKey) {
      const u64 prev = atomicCAS(&tab[h].key, kEmptyKey, key);
      if (prev == kEmptyKey) return 2;
      if (prev == key) return 1;
    }
    h = (h + 1) & mask;
  }
  return 0;
}

// Insert a query key; sets its filter bit on the first insert.  Returns 1
// when the key was new.
__device__ inline int query_insert(AccSlot* tab, u64 tmask, u64 X, unsigned* qf, u64 qfmask,
                                   unsigned* flags) {
  const int r = acc_insert(tab, tmask, X);
  if (!r) atomicOr(flags, kFlagOverflow);
  else if (r == 2 && qf) qfilter_set(qf, qfmask, X);
  return r == 2 ? 1 : 0;
}

// Determinant-major query pass: as k_query_ops (counts or inserts, with
// the same use of counter), over the connections of each determinant whose
// linking operator is selected.
__global__ void __launch_bounds__(kSigBlock)
k_query_set(const u64* __restrict__ keys, const double* __restrict__ amps, ExcSpace E, int n_spatial,
            u64 n, const int* __restrict__ optab, int nsp,
            const unsigned char* __restrict__ selected, AccSlot* __restrict__ tab, u64 tmask,
            int count_only, u64* __restrict__ counter, unsigned* __restrict__ flags, int nbatch, int batch,
            unsigned* __restrict__ qf, u64 qfmask) {
  __shared__ SigShared S;
  __shared__ ConnTables T;
  extern __shared__ __align__(16) unsigned char conn_dyn[];
  build_pair_table(S);
  if (threadIdx.x == 0) attach_conn_tables(T, conn_dyn, E);
  unsigned long long mine = 0;
  const u64 dstep = count_only ? (u64)count_only : 1ULL;
  for (u64 d = blockIdx.x * dstep; d < n; d += gridDim.x * dstep) {
    if (is_dead(amps[d])) continue;
    const u64 D = keys[d];
    __syncthreads();
    build_lists_shared(D, n_spatial, S);
    __syncthreads();
    build_conn_tables(S, E, T);
    __syncthreads();
    for_each_connection(T, D, [&](u64 X, int nh, int h0, int h1, int p0, int p1) {
      bool t_acts;
      OpDesc op;
      const int k = linking_operator(optab, nsp, nh, h0, h1, p0, p1, &t_acts, &op);
      if (k < 0 || !selected[k]) return;
      if (count_only) {
        ++mine;
        return;
      }
      if (nbatch > 1 && batch_of(X, nbatch) != batch) return;
      mine += query_insert(tab, tmask, X, qf, qfmask, flags);
    });
  }
  if (counter) {
    for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off);
    if (__lane_id() == 0 && mine) atomicAdd(counter, (u64)mine);
  }
}

// Operator-major passes for a screened subset: block (x, y) stages a tile of
// determinants in LDS (x) and gives each thread one selected operator (y).
// Pass "query" counts (count_only > 0: the active pairs of every
// count_only-th tile, into *counter) or inserts X_k(D) for every active
// (k, D) (adding the number of keys that were new to *counter when counter is
// given); pass "contract" accumulates psi(D) a_k(D) sigma(X_k(D)) per
// operator slot.
constexpr int kOpTile = 16;
// The contraction's tile is longer: one device-scope add per (operator,
// tile) with a nonzero sum, so 64 determinants per tile send a quarter of
// the adds a 16-determinant tile would.
constexpr int kOpTileContract = 64;

__global__ void __launch_bounds__(256)
k_query_ops(const u64* __restrict__ keys, const double* __restrict__ amps, u64 n,
            const OpDesc* __restrict__ ops, const int* __restrict__ subset, long long n_sub,
            AccSlot* __restrict__ tab, u64 tmask, int count_only, u64* __restrict__ counter,
            unsigned* __restrict__ flags, int nbatch, int batch, unsigned* __restrict__ qf, u64 qfmask) {
  __shared__ u64 skey[kOpTile];
  const u64 t0 = (u64)blockIdx.x * kOpTile * (count_only ? (u64)count_only : 1ULL);
  const int tile = (int)((n - t0) < (u64)kOpTile ? (n - t0) : (u64)kOpTile);
  for (int t = threadIdx.x; t < tile; t += blockDim.x)
    skey[t] = is_dead(amps[t0 + t]) ? 0ULL : keys[t0 + t];
  __syncthreads();
  const long long slot = (long long)blockIdx.y * blockDim.x + threadIdx.x;
  unsigned long long mine = 0;
  if (slot < n_sub) {
    const OpDesc op = ops[subset[slot]];
    const u64 pm = op.ann | op.cre;
    for (int t = 0; t < tile; ++t) {
      const u64 D = skey[t];
      if (D == 0ULL) continue;
      const bool act = (((D & op.ann) == op.ann) && ((D & op.cre) == 0)) ||
                       (((D & op.cre) == op.cre) && ((D & op.ann) == 0));
      if (!act) continue;
      if (count_only) ++mine;
      else if (nbatch > 1 && batch_of(D ^ pm, nbatch) != batch) continue;
      else mine += query_insert(tab, tmask, D ^ pm, qf, qfmask, flags);
    }
  }
  if (counter) {
    for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off);
    if (__lane_id() == 0 && mine) atomicAdd(counter, (u64)mine);
  }
}

__global__ void __launch_bounds__(256)
k_contract_ops(const u64* __restrict__ keys, const double* __restrict__ amps, u64 n,
               const OpDesc* __restrict__ ops, const int* __restrict__ subset, long long n_sub,
               const AccSlot* __restrict__ tab, u64 tmask, double* __restrict__ gslot, int nbatch,
               int batch) {
  __shared__ u64 skey[kOpTileContract];
  __shared__ double samp[kOpTileContract];
  const u64 t0 = (u64)blockIdx.x * kOpTileContract;
  const int tile = (int)((n - t0) < (u64)kOpTileContract ? (n - t0) : (u64)kOpTileContract);
  for (int t = threadIdx.x; t < tile; t += blockDim.x) {
    const double a = amps[t0 + t];
    skey[t] = is_dead(a) ? 0ULL : keys[t0 + t];
    samp[t] = a;
  }
  __syncthreads();
  const long long slot = (long long)blockIdx.y * blockDim.x + threadIdx.x;
  if (slot >= n_sub) return;
  const OpDesc op = ops[subset[slot]];
  const u64 pm = op.ann | op.cre;
  double acc = 0.0;
  for (int t = 0; t < tile; ++t) {
    const u64 D = skey[t];
    if (D == 0ULL) continue;
    const bool isT = ((D & op.ann) == op.ann) && ((D & op.cre) == 0);
    const bool isTd = ((D & op.cre) == op.cre) && ((D & op.ann) == 0);
    if (!(isT || isTd)) continue;
    const u64 X = D ^ pm;
    if (nbatch > 1 && batch_of(X, nbatch) != batch) continue;
    double sx;
    if (!acc_find(tab, tmask, X, &sx)) continue;
    const double a = isT ? (double)phase_of_T(op, D) : -(double)phase_of_T(op, X);
    acc += samp[t] * a * sx;
  }
  if (acc != 0.0) unsafeAtomicAdd(&gslot[slot], acc);
}

// Inserts stop kAccMaxProbes slots from a key's home, and so does this
// lookup: a table that overflowed is not walked end to end on every miss.
__device__ inline double* acc_slot(AccSlot* tab, u64 mask, u64 key) {
  u64 h = mix64(key) & mask;
  const u64 lim = mask < kAccMaxProbes ? mask : kAccMaxProbes;
  for (u64 probes = 0; probes <= lim; ++probes) {
    const u64 k = tab[h].key;
    if (k == key) return &tab[h].val;
    if (k == kEmptyKey) return nullptr;
    h = (h + 1) & mask;
  }
  return nullptr;
}

__global__ void __launch_bounds__(kSigBlock)
k_sigma_push_into(const u64* __restrict__ keys, const double* __restrict__ amps, Ints I, ExcSpace E,
                  u64 n, const double* __restrict__ diag, AccSlot* __restrict__ tab, u64 tmask, int nbatch,
                  int batch, const unsigned* __restrict__ qf, u64 qfmask) {
  __shared__ SigShared S;
  __shared__ ConnTables T;
  extern __shared__ __align__(16) unsigned char conn_dyn[];
  build_pair_table(S);
  if (threadIdx.x == 0) attach_conn_tables(T, conn_dyn, E);
  for (u64 d = blockIdx.x; d < n; d += gridDim.x) {
    const double psiD = amps[d];
    if (is_dead(psiD)) continue;
    const u64 D = keys[d];
    __syncthreads();
    build_lists_shared(D, I.n, S);
    __syncthreads();
    build_conn_tables(S, E, T);
    __syncthreads();
    if (threadIdx.x == 0 && (nbatch == 1 || batch_of(D, nbatch) == batch)) {
      double* v = qfilter_maybe(qf, qfmask, D) ? acc_slot(tab, tmask, D) : nullptr;
      if (v) unsafeAtomicAdd(v, diag[d] * psiD);
    }
    for_each_connection(T, D, [&](u64 X, int nh, int h0, int h1, int p0, int p1) {
      if (nbatch > 1 && batch_of(X, nbatch) != batch) return;
      if (!qfilter_maybe(qf, qfmask, X)) return;
      double* v = acc_slot(tab, tmask, X);
      if (v) unsafeAtomicAdd(v, connection_element(I, D, nh, h0, h1, p0, p1) * psiD);
    });
  }
}

// out[t] = (2 / norm2) * gacc[subset[t]] (subset == NULL: identity), with
// norm2 = <psi|psi> read from device memory.
__global__ void k_gather_scaled(const double* __restrict__ gacc, const int* __restrict__ subset,
                                long long count, const double* __restrict__ norm2,
                                double* __restrict__ out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) out[t] = (2.0 / norm2[0]) * gacc[subset ? subset[t] : t];
}

__global__ void k_mark_selected(const int* __restrict__ subset, long long count,
                                unsigned char* __restrict__ selected) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) selected[subset[t]] = 1;
}

// Copy of a caller's device subset with indices outside [0, K) replaced by 0
// (so every later lookup stays in bounds) ...
__global__ void k_sanitize_subset(const int* __restrict__ in, long long count, long long K,
                                  int* __restrict__ out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) {
    const int k = in[t];
    out[t] = (k >= 0 && k < K) ? k : 0;
  }
}

// ... and NaN written to the gradients of those entries afterwards.
__global__ void k_nan_invalid(const int* __restrict__ in, long long count, long long K,
                              double* __restrict__ g) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) {
    const int k = in[t];
    if (k < 0 || k >= K) g[t] = __longlong_as_double(0x7ff8000000000000LL);
  }
}

// All of out[0, count) set to NaN when the counters carry flag `bit` (an
// accumulation table that filled up), read on the device so that a call
// that does not synchronize still cannot return partial sums as results.
__global__ void k_nan_if_flag(const Counters* __restrict__ ctr, unsigned bit, double* __restrict__ out,
                              long long count) {
  if (!(ctr->flags & bit)) return;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) out[t] = __longlong_as_double(0x7ff8000000000000LL);
}

// Per-block partial sums of psi^2 [P in D] for P < nso and of psi^2.
__global__ void __launch_bounds__(256)
k_occupations(const u64* __restrict__ keys, const double* __restrict__ amps, u64 n, int nso,
              double* __restrict__ partial) {
  __shared__ double red[4][65];
  double acc[65];
#pragma unroll
  for (int P = 0; P < 65; ++P) acc[P] = 0.0;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double a = amps[i];
    if (is_dead(a)) continue;
    const double w = a * a;
    const u64 D = keys[i];
#pragma unroll
    for (int P = 0; P < 64; ++P)
      if ((D >> P) & 1ULL) acc[P] += w;
    acc[64] += w;
  }
  // wavefront sums, then the four wavefronts of the block in order
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int P = 0; P < 65; ++P) {
    double v = acc[P];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[wave][P] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x <= nso) {
    const int P = ((int)threadIdx.x == nso) ? 64 : (int)threadIdx.x;
    partial[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = red[0][P] + red[1][P] + red[2][P] + red[3][P];
  }
}

// out[v] = sum_{b < count} partial[v * stride + b] in a fixed order.
__global__ void k_reduce_partials(const double* __restrict__ partial, int count, int stride,
                                  double* __restrict__ out) {
  __shared__ double red[256];
  const int v = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < count; b += blockDim.x) acc += partial[(size_t)v * stride + b];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = red[0];
}

// mu = (2 / norm2) (sigma - E psi) on alive entries, 0 elsewhere, with
// (numer, norm2) = nn[0], nn[1] in device memory and E = numer / norm2.
__global__ void k_mu_init(const double* __restrict__ amps, const double* __restrict__ sigma, u64 n,
                          const double* __restrict__ nn, double* __restrict__ mu) {
  const double scale = 2.0 / nn[1], E = nn[0] / nn[1];
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double a = amps[i];
    mu[i] = is_dead(a) ? 0.0 : scale * (sigma[i] - E * a);
  }
}

int pairwise_capacity() { return kPairCap; }

hipError_t launch_sigma_pairwise(const DeviceState& st, const Ints& I, u64 n, double* sigma,
                                 double* partial, int grid, hipStream_t stream) {
  if (n > (u64)kPairCap) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sigma_pairwise, dim3(grid), dim3(256), (size_t)n * 16, stream, st.keys,
                     st.amps, (unsigned)n, I, st.diag, sigma, partial);
  return hipGetLastError();
}

hipError_t launch_diag(const DeviceState& st, const Ints& I, u64 n, int grid, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  if (I.n > kDiagMaxN) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_diag, dim3(grid), dim3(256), 0, stream, st.keys, st.amps, n, I, st.diag);
  return hipGetLastError();
}

hipError_t launch_sigma_proj(const DeviceState& st, const Ints& I, const ExcSpace& E, u64 n,
                             double* sigma, double* partial_num, double* partial_norm, int grid,
                             hipStream_t stream) {
  (void)partial_norm;
  hipLaunchKernelGGL(k_sigma_proj, dim3(grid), dim3(kSigBlock), conn_tables_bytes(E), stream, st.keys, st.amps,
                     st.hash, st.hmask, st.filt, st.fmask, I, E, n, st.diag, sigma, partial_num);
  return hipGetLastError();
}

hipError_t launch_holepair_emit(const DeviceState& st, u64 n, int n_spatial, int na, int nb, int shift,
                                u64* out_key, unsigned* out_val, int grid, hipStream_t stream) {
  if (na > 32 || nb > 32 || grid < 1) return hipErrorInvalidValue;
  // entries per wavefront chunk: enough chunks for every wavefront of the grid
  const u64 waves = (u64)grid * 4;
  const int cw = (int)std::min<u64>(64, std::max<u64>(1, (n + waves - 1) / waves));
  hipLaunchKernelGGL(k_holepair_emit, dim3(grid), dim3(256), 0, stream, st.keys, st.amps, n, n_spatial, na, nb,
                     shift, cw, out_key, out_val);
  return hipGetLastError();
}

hipError_t launch_sigma_diag(const DeviceState& st, const Ints& I, u64 n, double* sigma, int grid,
                             hipStream_t stream) {
  (void)I;
  hipLaunchKernelGGL(k_sigma_diag, dim3(grid), dim3(256), 0, stream, st.amps, st.diag, n, sigma);
  return hipGetLastError();
}

hipError_t launch_holepair_sigma(const DeviceState& st, const Ints& I, int na, u64 n, const u64* skey,
                                 const unsigned* sidx, int shift, u64 total, int cls, double* sigma, int grid,
                                 hipStream_t stream) {
  if (total == 0) return hipSuccess;
  const HoleRecords R{skey, sidx, shift};
  hipLaunchKernelGGL(k_holepair_sigma, dim3(grid), dim3(256), 0, stream, R, total, cls, st.keys, st.amps, n, I,
                     na, sigma);
  return hipGetLastError();
}

hipError_t launch_sigma_dots(const DeviceState& st, const double* sigma, u64 n, double* partial,
                             int grid, hipStream_t stream) {
  hipLaunchKernelGGL(k_sigma_dots, dim3(grid), dim3(256), 0, stream, st.amps, sigma, n, partial);
  return hipGetLastError();
}

hipError_t launch_mu_init(const DeviceState& st, const double* sigma, u64 n, const double* nn,
                          double* mu, hipStream_t stream) {
  u64 g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_mu_init, dim3((unsigned)g), dim3(256), 0, stream, st.amps, sigma, n, nn, mu);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double* partial, int count, int stride, int nvec,
                                  double* out, hipStream_t stream) {
  hipLaunchKernelGGL(k_reduce_partials, dim3(nvec), dim3(256), 0, stream, partial, count, stride,
                     out);
  return hipGetLastError();
}

hipError_t launch_sigma_push(const DeviceState& st, const Ints& I, const ExcSpace& E, u64 n,
                             AccSlot* tab, u64 tmask, int nbatch, int batch, double* inserted,
                             int grid, hipStream_t stream) {
  hipLaunchKernelGGL(k_sigma_push, dim3(grid), dim3(kSigBlock), conn_tables_bytes(E), stream, st.keys, st.amps, I, E,
                     n, st.diag, tab, tmask, nbatch, batch, &st.ctr->flags, inserted);
  return hipGetLastError();
}

hipError_t launch_pool_contract_det(const DeviceState& st, const ExcSpace& E, int n_spatial, u64 n,
                                   const int* optab, int nsp, const unsigned char* selected,
                                   const AccSlot* tab, u64 tmask, int nbatch, int batch,
                                   double* gacc, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(k_pool_contract_det, dim3(grid), dim3(kSigBlock), conn_tables_bytes(E), stream, st.keys, st.amps,
                     E, n_spatial, n, optab, nsp, selected, tab, tmask, nbatch, batch, gacc);
  return hipGetLastError();
}

hipError_t launch_query_set(const DeviceState& st, const ExcSpace& E, int n_spatial, u64 n,
                            const int* optab, int nsp, const unsigned char* selected,
                            AccSlot* tab, u64 tmask, int count_only, u64* counter, int grid,
                            hipStream_t stream, int nbatch, int batch, unsigned* qf, u64 qfmask) {
  if (nbatch < 1 || batch < 0 || batch >= nbatch) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_query_set, dim3(grid), dim3(kSigBlock), conn_tables_bytes(E), stream, st.keys, st.amps, E,
                     n_spatial, n, optab, nsp, selected, tab, tmask, count_only, counter,
                     &st.ctr->flags, nbatch, batch, qf, qfmask);
  return hipGetLastError();
}

hipError_t launch_query_ops(const DeviceState& st, u64 n, const OpDesc* ops, const int* subset,
                            long long n_sub, AccSlot* tab, u64 tmask, int count_only, u64* counter,
                            hipStream_t stream, int nbatch, int batch, unsigned* qf, u64 qfmask) {
  if (nbatch < 1 || batch < 0 || batch >= nbatch) return hipErrorInvalidValue;
  if (n == 0 || n_sub == 0) return hipSuccess;
  const u64 tiles = (n + kOpTile - 1) / kOpTile, stride = count_only > 0 ? (u64)count_only : 1ULL;
  const dim3 grid((unsigned)((tiles + stride - 1) / stride), (unsigned)((n_sub + 255) / 256));
  hipLaunchKernelGGL(k_query_ops, grid, dim3(256), 0, stream, st.keys, st.amps, n, ops, subset,
                     n_sub, tab, tmask, count_only, counter, &st.ctr->flags, nbatch, batch, qf, qfmask);
  return hipGetLastError();
}

hipError_t launch_contract_ops(const DeviceState& st, u64 n, const OpDesc* ops, const int* subset,
                               long long n_sub, const AccSlot* tab, u64 tmask, double* gslot,
                               hipStream_t stream, int nbatch, int batch) {
  if (nbatch < 1 || batch < 0 || batch >= nbatch) return hipErrorInvalidValue;
  if (n == 0 || n_sub == 0) return hipSuccess;
  const dim3 grid((unsigned)((n + kOpTileContract - 1) / kOpTileContract), (unsigned)((n_sub + 255) / 256));
  hipLaunchKernelGGL(k_contract_ops, grid, dim3(256), 0, stream, st.keys, st.amps, n, ops, subset,
                     n_sub, tab, tmask, gslot, nbatch, batch);
  return hipGetLastError();
}

hipError_t launch_sigma_push_into(const DeviceState& st, const Ints& I, const ExcSpace& E, u64 n,
                                  AccSlot* tab, u64 tmask, int grid, hipStream_t stream, int nbatch, int batch,
                                  const unsigned* qf, u64 qfmask) {
  if (nbatch < 1 || batch < 0 || batch >= nbatch) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sigma_push_into, dim3(grid), dim3(kSigBlock), conn_tables_bytes(E), stream, st.keys, st.amps, I,
                     E, n, st.diag, tab, tmask, nbatch, batch, qf, qfmask);
  return hipGetLastError();
}

hipError_t launch_gather_scaled(const double* gacc, const int* subset, long long count,
                                const double* norm2, double* out, hipStream_t stream) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_scaled, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream,
                     gacc, subset, count, norm2, out);
  return hipGetLastError();
}

hipError_t launch_mark_selected(const int* subset, long long count, unsigned char* selected,
                                hipStream_t stream) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mark_selected, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream,
                     subset, count, selected);
  return hipGetLastError();
}

hipError_t launch_sanitize_subset(const int* in, long long count, long long K, int* out,
                                  hipStream_t stream) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sanitize_subset, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream,
                     in, count, K, out);
  return hipGetLastError();
}

hipError_t launch_nan_invalid(const int* in, long long count, long long K, double* g,
                              hipStream_t stream) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_nan_invalid, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream,
                     in, count, K, g);
  return hipGetLastError();
}

hipError_t launch_nan_if_flag(const Counters* ctr, unsigned bit, double* out, long long count,
                              hipStream_t stream) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_nan_if_flag, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream,
                     ctr, bit, out, count);
  return hipGetLastError();
}

hipError_t launch_occupations(const DeviceState& st, u64 n, int nso, double* partial, int grid,
                              hipStream_t stream) {
  hipLaunchKernelGGL(k_occupations, dim3(grid), dim3(256), 0, stream, st.keys, st.amps, n, nso,
                     partial);
  return hipGetLastError();
}

}  // namespace swcs

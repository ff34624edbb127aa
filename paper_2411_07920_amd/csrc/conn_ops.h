// Connection enumeration shared by the sigma-vector and pool-gradient
// kernels: one block stages a determinant's occupied and virtual lists and
// the hole- and particle-set tables of its spin-conserving singles and
// doubles in LDS (Slater-Condon connectivity, Sec. III), and the lanes walk
// the connections from those tables.  Also the map from a connection to the
// pool operator that links its two determinants.
#pragma once

#include "swcs_internal.h"

namespace swcs {

constexpr int kSigBlock = 256;
constexpr int kMaxPairs = 32 * 31 / 2;

struct SigShared {
  int occ_a[32], occ_b[32], vir_a[32], vir_b[32];
  unsigned char px[kMaxPairs], py[kMaxPairs];
};

__device__ inline void build_pair_table(SigShared& S) {
  for (int t = threadIdx.x; t < kMaxPairs; t += blockDim.x) {
    int y = 1;
    while ((y + 1) * y / 2 <= t) ++y;
    S.py[t] = (unsigned char)y;
    S.px[t] = (unsigned char)(t - y * (y - 1) / 2);
  }
}

// Thread p < n places spatial orbital p in the alpha / beta lists.
__device__ inline void build_lists_shared(u64 D, int n, SigShared& S) {
  const int p = threadIdx.x;
  if (p < n) {
    const u64 below = (p == 0) ? 0ULL : ((1ULL << (2 * p)) - 1ULL);
    const u64 amask = 0x5555555555555555ULL, bmask = 0xAAAAAAAAAAAAAAAAULL;
    const u64 occ_below = D & below, vir_below = ~D & below;
    if ((D >> (2 * p)) & 1ULL) S.occ_a[__popcll(occ_below & amask)] = 2 * p;
    else S.vir_a[__popcll(vir_below & amask)] = 2 * p;
    if ((D >> (2 * p + 1)) & 1ULL) S.occ_b[__popcll(occ_below & bmask)] = 2 * p + 1;
    else S.vir_b[__popcll(vir_below & bmask)] = 2 * p + 1;
  }
}

// Connection tables of one determinant, in LDS: the hole sets and particle
// sets of the five spin-conserving classes (alpha single, beta single,
// alpha-alpha double, beta-beta double, alpha-beta double) as bit masks plus
// their sorted spin-orbital indices.  A connection is (hole set h, particle
// set p) of one class, X = D ^ hmask[h] ^ pmask[p]; the lanes walk the
// (h, p) grid of each class with a stride of the block size, stepping the
// indices incrementally (one division per class and lane).
struct ConnTables {
  u64* hmask;  // arrays in dynamic LDS, sized by the launcher (conn_tables_bytes)
  u64* pmask;
  unsigned char *h0, *h1, *p0, *p1;
  int hbeg[5], nh[5], pbeg[5], np[5];
};

__host__ __device__ inline void conn_set_counts(const ExcSpace& E, int* NH, int* NP) {
  const int na = E.na, nb = E.nb, va = E.va, vb = E.vb;
  *NH = na + nb + na * (na - 1) / 2 + nb * (nb - 1) / 2 + na * nb;
  *NP = va + vb + va * (va - 1) / 2 + vb * (vb - 1) / 2 + va * vb;
}

inline size_t conn_tables_bytes(const ExcSpace& E) {
  int NH, NP;
  conn_set_counts(E, &NH, &NP);
  return (size_t)(NH + NP) * 10;
}

// Carve the tables out of the dynamic LDS buffer.
__device__ inline void attach_conn_tables(ConnTables& T, unsigned char* dyn, const ExcSpace& E) {
  int NH, NP;
  conn_set_counts(E, &NH, &NP);
  T.hmask = (u64*)dyn;
  T.pmask = T.hmask + NH;
  T.h0 = (unsigned char*)(T.pmask + NP);
  T.h1 = T.h0 + NH;
  T.p0 = T.h1 + NH;
  T.p1 = T.p0 + NP;
}

__device__ inline void build_conn_tables(const SigShared& S, const ExcSpace& E, ConnTables& T) {
  const int na = E.na, nb = E.nb, va = E.va, vb = E.vb;
  if (threadIdx.x == 0) {
    int h = 0, p = 0;
    const int nhs[5] = {na, nb, na * (na - 1) / 2, nb * (nb - 1) / 2, na * nb};
    const int nps[5] = {va, vb, va * (va - 1) / 2, vb * (vb - 1) / 2, va * vb};
    for (int c = 0; c < 5; ++c) {
      T.hbeg[c] = h;
      T.nh[c] = nhs[c];
      T.pbeg[c] = p;
      T.np[c] = nps[c];
      h += nhs[c];
      p += nps[c];
    }
  }
  __syncthreads();
  const int tid = threadIdx.x;
  // holes
  for (int t = tid; t < na; t += blockDim.x) {
    const int P = S.occ_a[t];
    T.hmask[T.hbeg[0] + t] = 1ULL << P; T.h0[T.hbeg[0] + t] = P; T.h1[T.hbeg[0] + t] = P;
  }
  for (int t = tid; t < nb; t += blockDim.x) {
    const int P = S.occ_b[t];
    T.hmask[T.hbeg[1] + t] = 1ULL << P; T.h0[T.hbeg[1] + t] = P; T.h1[T.hbeg[1] + t] = P;
  }
  for (int t = tid; t < T.nh[2]; t += blockDim.x) {
    const int x = S.occ_a[S.px[t]], y = S.occ_a[S.py[t]];
    T.hmask[T.hbeg[2] + t] = (1ULL << x) | (1ULL << y); T.h0[T.hbeg[2] + t] = x; T.h1[T.hbeg[2] + t] = y;
  }
  for (int t = tid; t < T.nh[3]; t += blockDim.x) {
    const int x = S.occ_b[S.px[t]], y = S.occ_b[S.py[t]];
    T.hmask[T.hbeg[3] + t] = (1ULL << x) | (1ULL << y); T.h0[T.hbeg[3] + t] = x; T.h1[T.hbeg[3] + t] = y;
  }
  for (int t = tid; t < T.nh[4]; t += blockDim.x) {
    const int i = t / nb, j = t - (t / nb) * nb;
    const int x = S.occ_a[i], y = S.occ_b[j];
    T.hmask[T.hbeg[4] + t] = (1ULL << x) | (1ULL << y);
    T.h0[T.hbeg[4] + t] = min(x, y); T.h1[T.hbeg[4] + t] = max(x, y);
  }
  // particles
  for (int t = tid; t < va; t += blockDim.x) {
    const int P = S.vir_a[t];
    T.pmask[T.pbeg[0] + t] = 1ULL << P; T.p0[T.pbeg[0] + t] = P; T.p1[T.pbeg[0] + t] = P;
  }
  for (int t = tid; t < vb; t += blockDim.x) {
    const int P = S.vir_b[t];
    T.pmask[T.pbeg[1] + t] = 1ULL << P; T.p0[T.pbeg[1] + t] = P; T.p1[T.pbeg[1] + t] = P;
  }
  for (int t = tid; t < T.np[2]; t += blockDim.x) {
    const int x = S.vir_a[S.px[t]], y = S.vir_a[S.py[t]];
    T.pmask[T.pbeg[2] + t] = (1ULL << x) | (1ULL << y); T.p0[T.pbeg[2] + t] = x; T.p1[T.pbeg[2] + t] = y;
  }
  for (int t = tid; t < T.np[3]; t += blockDim.x) {
    const int x = S.vir_b[S.px[t]], y = S.vir_b[S.py[t]];
    T.pmask[T.pbeg[3] + t] = (1ULL << x) | (1ULL << y); T.p0[T.pbeg[3] + t] = x; T.p1[T.pbeg[3] + t] = y;
  }
  for (int t = tid; t < T.np[4]; t += blockDim.x) {
    const int a = t / vb, b = t - (t / vb) * vb;
    const int x = S.vir_a[a], y = S.vir_b[b];
    T.pmask[T.pbeg[4] + t] = (1ULL << x) | (1ULL << y);
    T.p0[T.pbeg[4] + t] = min(x, y); T.p1[T.pbeg[4] + t] = max(x, y);
  }
}

// Calls f(X, nh, h0, h1, p0, p1) for every single (nh = 1) and double
// (nh = 2) connection X of D assigned to this lane; holes h0 < h1 and
// particles p0 < p1 are spin-orbital indices.
template <class F>
__device__ inline void for_each_connection(const ConnTables& T, u64 D, F&& f) {
  for (int c = 0; c < 5; ++c) {
    const int nh = T.nh[c], np = T.np[c];
    if (nh == 0 || np == 0) continue;
    const int hb = T.hbeg[c], pb = T.pbeg[c];
    int hi = (int)threadIdx.x / np;
    int pi = (int)threadIdx.x - hi * np;
    const int nholes = c < 2 ? 1 : 2;
    while (hi < nh) {
      const int H = hb + hi, Pp = pb + pi;
      const u64 X = D ^ T.hmask[H] ^ T.pmask[Pp];
      f(X, nholes, (int)T.h0[H], (int)T.h1[H], (int)T.p0[Pp], (int)T.p1[Pp]);
      pi += blockDim.x;
      while (pi >= np) {
        pi -= np;
        ++hi;
      }
    }
  }
}

// Generator table (P, Q, R, S) -> pool index for nsp spatial orbitals:
// singles (P > Q, one spin) at pair(P, Q) = P (P - 1) / 2 + Q; doubles by the
// spin class of their pairs -- both alpha, both beta, mixed -- each class a
// triangle over its own pair indices (p (p - 1) / 2 + q for a same-spin pair
// of spatial orbitals p > q; alpha * nsp + beta for a mixed pair).  A
// spin-conserving double pairs two pairs of one class, so the table holds
// 2 tri(nsp (nsp - 1) / 2) + tri(nsp^2) double slots (333,450 at nsp = 26,
// 1.3 MB, against 878,475 for a triangle over all spin-orbital pairs), and
// the lookups of the pool kernels stay in L2.
// (a below 2^12: the masked product is a full-rate 24-bit multiply)
__host__ __device__ inline int pair_index(int a, int b) {
  const unsigned u = (unsigned)a & 0xFFFu;
  return (int)((u * u - u) >> 1) + b;
}

__host__ __device__ inline long long optab_size(int nsp) {
  const long long nso = 2LL * nsp, ss = (long long)nsp * (nsp - 1) / 2, mx = (long long)nsp * nsp;
  return nso * (nso - 1) / 2 + ss * (ss - 1) + mx * (mx - 1) / 2;
}

// Slot of the double (P, Q, R, S): P > Q, R > S, both pairs of one spin class.
__host__ __device__ inline int optab_double_slot(int nsp, int P, int Q, int R, int S) {
  nsp &= 63;
  const int nso = 2 * nsp, ss = pair_index(nsp, 0);
  int a, b, base = pair_index(nso, 0);
  if ((P & 1) == (Q & 1)) {
    a = pair_index(P >> 1, Q >> 1);
    b = pair_index(R >> 1, S >> 1);
    if (P & 1) base += pair_index(ss, 0);
  } else {
    a = (((P & 1) ? Q : P) >> 1 & 63) * nsp + (((P & 1) ? P : Q) >> 1);
    b = (((R & 1) ? S : R) >> 1 & 63) * nsp + (((R & 1) ? R : S) >> 1);
    base += 2 * pair_index(ss, 0);
  }
  const int hi = a > b ? a : b, lo = a > b ? b : a;
  return base + pair_index(hi, lo);
}

// Operator of the pool that links D to its connection (holes h0 < h1,
// particles p0 < p1): returns its index (or -1), whether T (rather than
// T^dagger) acts on D, and the operator's (P, Q, R, S).
__device__ inline int linking_operator(const int* __restrict__ optab, int nsp, int nh, int h0,
                                       int h1, int p0, int p1, bool* t_acts, OpDesc* op) {
  if (nh == 1) {
    *t_acts = p0 > h0;
    op->P = *t_acts ? p0 : h0;
    op->Q = *t_acts ? h0 : p0;
    op->R = op->S = -1;
    return optab[pair_index(op->P, op->Q)];
  }
  *t_acts = p1 > h1;
  op->P = *t_acts ? p1 : h1;
  op->Q = *t_acts ? p0 : h0;
  op->R = *t_acts ? h1 : p1;
  op->S = *t_acts ? h0 : p0;
  return optab[optab_double_slot(nsp, op->P, op->Q, op->R, op->S)];
}

}  // namespace swcs

// Internal definitions shared by the HIP translation units of libswcs.
// Device data layout, hash tables, phase rules and host launch wrappers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

namespace swcs {

typedef unsigned long long u64;

// Amplitude bit pattern that marks a stored determinant as not part of the
// state (pruned, or never reached).  A quiet NaN no arithmetic produces.
constexpr u64 kDeadBits = 0x7ff8dead0000deadULL;
constexpr u64 kEmptyKey = 0ULL;  // no determinant of >= 1 electron has key 0

__host__ __device__ inline u64 mix64(u64 x) {
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ULL;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebULL;
  x ^= x >> 31;
  return x;
}

__device__ inline bool is_dead(double a) { return (u64)__double_as_longlong(a) == kDeadBits; }
__device__ inline double dead_value() { return __longlong_as_double((long long)kDeadBits); }

// One operator of the pool, preprocessed on the host.
//   T = a+_P a+_Q a_S a_R (double) or a+_P a_Q (single, R = S = -1)
//   ann = bits annihilated by T, cre = bits created by T.
struct OpDesc {
  u64 ann;
  u64 cre;
  int P, Q, R, S;
};

// Sign of T acting on D (T must act: ann subset of D, cre disjoint from D).
// The rightmost ladder operator acts first; each contributes
// (-1)^(occupied spin-orbitals below its index) in the current determinant.
__device__ inline int phase_of_T(const OpDesc& op, u64 D) {
  int s;
  if (op.R < 0) {
    s = __popcll(D & ((1ULL << op.Q) - 1ULL));
    D ^= 1ULL << op.Q;
    s += __popcll(D & ((1ULL << op.P) - 1ULL));
  } else {
    s = __popcll(D & ((1ULL << op.R) - 1ULL));
    D ^= 1ULL << op.R;
    s += __popcll(D & ((1ULL << op.S) - 1ULL));
    D ^= 1ULL << op.S;
    s += __popcll(D & ((1ULL << op.Q) - 1ULL));
    D ^= 1ULL << op.Q;
    s += __popcll(D & ((1ULL << op.P) - 1ULL));
  }
  return (s & 1) ? -1 : 1;
}

// Open-addressing (linear probing) index from determinant key to position in
// the structure-of-arrays state.  Slots are 16 bytes so a probe touches one
// line for both key and index.  Capacity is a power of two.
struct HashSlot {
  u64 key;
  u64 idx;
};

__device__ inline long long hash_find(const HashSlot* __restrict__ tab, u64 mask, u64 key) {
  u64 h = mix64(key) & mask;
  while (true) {
    u64 k = tab[h].key;
    if (k == key) return (long long)tab[h].idx;
    if (k == kEmptyKey) return -1;
    h = (h + 1) & mask;
  }
}

// Insert a key known to be absent; concurrent inserts of other keys allowed.
__device__ inline void hash_insert_new(HashSlot* tab, u64 mask, u64 key, u64 idx) {
  u64 h = mix64(key) & mask;
  while (true) {
    u64 prev = atomicCAS(&tab[h].key, kEmptyKey, key);
    if (prev == kEmptyKey || prev == key) {
      tab[h].idx = idx;
      return;
    }
    h = (h + 1) & mask;
  }
}

// Accumulation table for the external sigma vector: key -> double.
struct AccSlot {
  u64 key;
  double val;
};

// Probe limit of the accumulation table: an insert that finds no free slot
// within this many probes fails (the caller raises kFlagOverflow and the host
// retries with a larger table), so a lookup that has not met its key within
// the same distance can stop.
constexpr u64 kAccMaxProbes = 4096;

// Adds v to the entry of key, inserting the key if needed.  Returns 2 if
// the key was inserted, 1 if it was present, 0 (adding nothing) if no slot
// within kAccMaxProbes is free.
__device__ inline int acc_add(AccSlot* tab, u64 mask, u64 key, double v) {
  u64 h = mix64(key) & mask;
  const u64 lim = mask < kAccMaxProbes ? mask : kAccMaxProbes;
  for (u64 probes = 0; probes <= lim; ++probes) {
    u64 k = tab[h].key;
    if (k == key) {
      unsafeAtomicAdd(&tab[h].val, v);
      return 1;
    }
    if (k == kEmptyKey) {
      u64 prev = atomicCAS(&tab[h].key, kEmptyKey, key);
      if (prev == kEmptyKey || prev == key) {
        unsafeAtomicAdd(&tab[h].val, v);
        return prev == kEmptyKey ? 2 : 1;
      }
    }
    h = (h + 1) & mask;
  }
  return 0;
}

__device__ inline bool acc_find(const AccSlot* __restrict__ tab, u64 mask, u64 key, double* v) {
  u64 h = mix64(key) & mask;
  const u64 lim = mask < kAccMaxProbes ? mask : kAccMaxProbes;
  for (u64 probes = 0; probes <= lim; ++probes) {
    u64 k = tab[h].key;
    if (k == key) {
      *v = tab[h].val;
      return true;
    }
    if (k == kEmptyKey) return false;
    h = (h + 1) & mask;
  }
  return false;
}

// Device counters of the state.  n: stored entries (alive or dead);
// alive: entries that are part of the state; app / dalive / ticket: per-gate
// scratch folded in by the last block of each gate launch; flags: error bits.
struct Counters {
  u64 n;
  u64 alive;
  u64 app;
  long long dalive;
  unsigned int ticket;
  unsigned int flags;
  u64 stop_gate;
};

// kFlagOverflow: an append or table insert found no room (a bug guard: the
// host sizes buffers so it cannot happen).  kFlagStopped: a gate found too
// little capacity and did nothing; later gates of the chain skip too.
enum : unsigned int { kFlagOverflow = 1u, kFlagStopped = 2u };

// Integrals on the device, spin-free spatial arrays.
struct Ints {
  const double* h;    // n*n
  const double* eri;  // (pq|rs) packed by its 8-fold symmetry: eri_packed_index
  const double* J;    // n*n, J[p*n+q] = (pp|qq)
  const double* K;    // n*n, K[p*n+q] = (pq|qp)
  double ecore;
  int n;
};

// Position of (pq|rs) in the packed array: pair indices pq = p (p + 1) / 2 +
// q (p >= q), rs likewise, then pq (pq + 1) / 2 + rs (pq >= rs).  The array
// has m (m + 1) / 2 entries, m = n (n + 1) / 2 (61,776 doubles, 494 KB, at
// n = 26 against 3.7 MB for n^4), so the lookups of the sigma and gradient
// kernels stay in L2.
// Orbital indices are below 64, so every product fits 24 bits; the masks let
// the compiler use full-rate 24-bit multiplies instead of 32-bit ones.
__host__ __device__ inline unsigned eri_packed_index(unsigned p, unsigned q, unsigned r, unsigned s) {
  p &= 63u;
  q &= 63u;
  r &= 63u;
  s &= 63u;
  const unsigned hi1 = p >= q ? p : q, lo1 = p >= q ? q : p;
  const unsigned hi2 = r >= s ? r : s, lo2 = r >= s ? s : r;
  const unsigned pq = ((hi1 * hi1 + hi1) >> 1) + lo1, rs = ((hi2 * hi2 + hi2) >> 1) + lo2;
  const unsigned a = (pq >= rs ? pq : rs) & 0xFFFu, b = pq >= rs ? rs : pq;
  return ((a * a + a) >> 1) + b;
}

__device__ inline double eri_sp(const Ints& I, int p, int q, int r, int s) {
  return I.eri[eri_packed_index((unsigned)p, (unsigned)q, (unsigned)r, (unsigned)s)];
}

// Spin-orbital (PQ|RS) with the spin deltas.
__device__ inline double eri_so(const Ints& I, int P, int Q, int R, int S) {
  if (((P ^ Q) & 1) || ((R ^ S) & 1)) return 0.0;
  return eri_sp(I, P >> 1, Q >> 1, R >> 1, S >> 1);
}

// <D'|H|D> for D' = a+_A a_I D (same spin, I in D, A not in D).
__device__ inline double single_element(const Ints& I, u64 D, int Ih, int A) {
  int s = __popcll(D & ((1ULL << Ih) - 1ULL));
  u64 x = D ^ (1ULL << Ih);
  s += __popcll(x & ((1ULL << A) - 1ULL));
  int a = A >> 1, i = Ih >> 1, n = I.n;
  double v = I.h[a * n + i];
  u64 y = D;
  while (y) {
    int Q = __ffsll((long long)y) - 1;
    y &= y - 1;
    int q = Q >> 1;
    v += eri_sp(I, a, i, q, q);
    if (((Q ^ A) & 1) == 0) v -= eri_sp(I, a, q, q, i);
  }
  return (s & 1) ? -v : v;
}

// <D'|H|D> for D' = a+_A a+_B a_J a_I D with I < J in D and A < B not in D.
__device__ inline double double_element(const Ints& I, u64 D, int Ih, int Jh, int A, int B) {
  int s = __popcll(D & ((1ULL << Ih) - 1ULL));
  u64 x = D ^ (1ULL << Ih);
  s += __popcll(x & ((1ULL << Jh) - 1ULL));
  x ^= 1ULL << Jh;
  s += __popcll(x & ((1ULL << B) - 1ULL));
  x ^= 1ULL << B;
  s += __popcll(x & ((1ULL << A) - 1ULL));
  double v = eri_so(I, A, Ih, B, Jh) - eri_so(I, A, Jh, B, Ih);
  return (s & 1) ? -v : v;
}

// Enumeration of the spin-conserving single and double excitations of a
// determinant with na alpha and nb beta electrons in n spatial orbitals.
// Connection c in [0, C) decodes to (holes, particles) in spin-orbitals.
struct ExcSpace {
  int n, na, nb;
  int va, vb;        // virtual counts
  long long s_a, s_b, d_aa, d_bb, d_ab;  // counts per class
  long long total;
};

inline ExcSpace make_exc_space(int n, int na, int nb) {
  ExcSpace e;
  e.n = n; e.na = na; e.nb = nb;
  e.va = n - na; e.vb = n - nb;
  e.s_a = (long long)na * e.va;
  e.s_b = (long long)nb * e.vb;
  e.d_aa = (long long)na * (na - 1) / 2 * ((long long)e.va * (e.va - 1) / 2);
  e.d_bb = (long long)nb * (nb - 1) / 2 * ((long long)e.vb * (e.vb - 1) / 2);
  e.d_ab = (long long)na * nb * e.va * e.vb;
  e.total = e.s_a + e.s_b + e.d_aa + e.d_bb + e.d_ab;
  return e;
}

// <D'|H|D> for the connection decoded above.
__device__ inline double connection_element(const Ints& I, u64 D, int nh, int h0, int h1, int p0,
                                            int p1) {
  if (nh == 1) return single_element(I, D, h0, p0);
  return double_element(I, D, h0, h1, p0, p1);
}

// One gate of an ansatz as the device sees it.
struct GateDesc {
  OpDesc op;
  double c;  // cos(theta)
  double s;  // sin(theta)
};

// A spin-complemented generator G = A1 + s A2 whose rows share spin-orbitals,
// applied as one gate exp(theta G) (k_generator.hip).
struct GenGate {
  OpDesc op1, op2;
  double c, sn;   // cos theta, sin theta: pairs of row 1
  double sn2;     // s sin theta: pairs of row 2
  double c2, s2;  // cos(sqrt(2) theta), sin(sqrt(2) theta): stars
  double rt;      // 1 / sqrt(2)
  double sg;      // s = +-1
};

// Largest state the single-workgroup LDS kernels hold (24 B per entry for
// the forward chain, 32 B for the adjoint sweep: 128 KB of LDS).
constexpr int kLdsCap = 4096;

// Multi-block gate kernels in HBM: threads per block, entries per thread and
// tile sizes (a tile's appended keys / logged pairs are staged in LDS).
constexpr int kDiagLanes = 8;  // lanes per determinant in k_diag
constexpr int kGateThreads = 1024;
constexpr int kGateItems = 2;                              // listed entries per thread and round
constexpr int kGateTile = kGateThreads * kGateItems;       // listed entries per round
// Keys per thread in the gate's scan: wide tiles for state arrays of at least
// kGateWideCap entries, narrow ones below (more blocks for small states).
constexpr int kGateScanWide = 16;
constexpr int kGateScanNarrow = 2;
constexpr u64 kGateWideCap = 1ULL << 21;
// entries per tile of the gate kernel for a state array of capacity cap
__host__ __device__ inline int gate_scan_tile(u64 cap) {
  return kGateThreads * (cap >= kGateWideCap ? kGateScanWide : kGateScanNarrow);
}
constexpr int kReplayTile = 2048;

// ---------------------------------------------------------------- host side
struct DeviceState {
  u64* keys = nullptr;
  double* amps = nullptr;
  HashSlot* hash = nullptr;
  Counters* ctr = nullptr;
  u64 cap = 0;        // SoA capacity
  u64 hmask = 0;      // hash capacity - 1
  unsigned* filt = nullptr;  // presence filter of the alive keys (1 bit per hash)
  u64 fmask = 0;             // filter bits - 1
  double* diag = nullptr;    // diagonal elements H_DD of the stored entries (launch_diag)
};

// Presence filter: one bit per (independent) hash of an alive key, about 16
// bits per key so that it stays in L2; a clear bit proves absence, so most
// probes for determinants that are not in the state never reach the table.
__device__ inline u64 filter_bit(u64 key, u64 fmask) {
  return mix64(key ^ 0xd6e8feb86659fd93ULL) & fmask;
}

__device__ inline bool filter_maybe(const unsigned* __restrict__ filt, u64 fmask, u64 key) {
  const u64 b = filter_bit(key, fmask);
  return (filt[b >> 5] >> (b & 31)) & 1u;
}

// Launch wrappers (defined in the .hip files).  All enqueue on `stream`.
struct PairRec;
struct StarRec;
hipError_t launch_gen_gate(const DeviceState& st, const GenGate& g, double eps, u64* gate_n_in,
                           unsigned gate_index, u64 max_keys, int grid, hipStream_t stream,
                           u64* gate_n_act = nullptr);
hipError_t launch_gen_replay(const DeviceState& st, double* amps, u64 n, const GenGate& g, double eps,
                             PairRec* plog, u64* pcount, StarRec* slog, u64* scount, int grid,
                             hipStream_t stream);
hipError_t launch_adjoint_star(const StarRec* slog, const u64* scount, double* mu, const GenGate& g,
                               double* partial, int grid, hipStream_t stream);
hipError_t launch_fill_u32(void* p, unsigned v, u64 words, hipStream_t stream);
hipError_t launch_store_counters(Counters* ctr, const Counters& v, hipStream_t stream);
hipError_t launch_clear_flag(Counters* ctr, unsigned bit, hipStream_t stream);
hipError_t launch_nan_if_flag(const Counters* ctr, unsigned bit, double* out, long long count,
                              hipStream_t stream);
hipError_t launch_hash_clear(HashSlot* tab, u64 slots, hipStream_t stream);
hipError_t launch_hash_build(const DeviceState& st, u64 n, hipStream_t stream);
hipError_t launch_gate(const DeviceState& st, const OpDesc& op, double c, double sn, double eps,
                       u64* gate_n_in, int check_cap, unsigned gate_index, u64 max_keys, int grid,
                       hipStream_t stream, u64* gate_n_act = nullptr);
hipError_t launch_prune_all(const DeviceState& st, double eps, int grid, hipStream_t stream);
hipError_t launch_hash_build_dev(const DeviceState& st, int grid, hipStream_t stream);
hipError_t launch_filter_build(const DeviceState& st, u64 n, int grid, hipStream_t stream);
hipError_t launch_reset_reference(const DeviceState& st, u64 ref, hipStream_t stream);
struct NcutState;
hipError_t launch_ncut(double* amps, const u64* keys, u64 n_host, Counters* ctr, NcutState* st,
                       unsigned ncut, int grid, hipStream_t stream);
int lds_chain_capacity();
hipError_t launch_chain_lds(const DeviceState& st, const GateDesc* gates, int g0, int M, double eps,
                            int prune_first, double* const* ckpt, u64* ckpt_n, int seg,
                            u64* gate_n_in, u64 max_keys, unsigned ncut, hipStream_t stream);
hipError_t launch_adjoint_replay_lds(const u64* keys, unsigned n, const GateDesc* gates, int M,
                                     int seg, double eps, const double* const* ckpt,
                                     const u64* ckpt_n, PairRec* logbuf, unsigned* logcnt,
                                     unsigned* flags, unsigned ncut, hipStream_t stream);
hipError_t launch_adjoint_reverse_lds(unsigned n, const GateDesc* gates, int M,
                                      const double* mu_init, const PairRec* logbuf,
                                      const unsigned* logcnt, double* dE_part, double* dE,
                                      hipStream_t stream);
size_t adjoint_lds_part_elems(int M);
hipError_t launch_gate_replay(const DeviceState& st, double* amps, u64 n, const OpDesc& op,
                             double c, double sn, double eps, PairRec* log, u64* log_count, int grid,
                             hipStream_t stream);
hipError_t launch_adjoint_rec(const PairRec* log, const u64* log_count, double* mu, double c,
                              double sn, double* partial, int grid, hipStream_t stream);
hipError_t launch_ckpt_save(const DeviceState& st, double* dst, u64* dst_n, int grid,
                            hipStream_t stream);
hipError_t launch_restore(double* dst, const double* src, const u64* n_src, u64 n_total,
                          hipStream_t stream);
hipError_t launch_mark_dead_range(double* amps, u64 lo, u64 hi, hipStream_t stream);
hipError_t launch_sigma_proj(const DeviceState& st, const Ints& I, const ExcSpace& E, u64 n,
                             double* sigma, double* partial_num, double* partial_norm, int grid,
                             hipStream_t stream);
int pairwise_capacity();
hipError_t launch_sigma_pairwise(const DeviceState& st, const Ints& I, u64 n, double* sigma,
                                 double* partial, int grid, hipStream_t stream);
hipError_t launch_diag(const DeviceState& st, const Ints& I, u64 n, int grid, hipStream_t stream);
hipError_t launch_holepair_emit(const DeviceState& st, u64 n, int n_spatial, int na, int nb, int shift,
                                u64* out_key, unsigned* out_val, int grid, hipStream_t stream);
hipError_t launch_sigma_diag(const DeviceState& st, const Ints& I, u64 n, double* sigma, int grid,
                             hipStream_t stream);
hipError_t launch_holepair_sigma(const DeviceState& st, const Ints& I, int na, u64 n, const u64* skey,
                                 const unsigned* sidx, int shift, u64 total, int cls, double* sigma, int grid,
                                 hipStream_t stream);
hipError_t launch_sigma_dots(const DeviceState& st, const double* sigma, u64 n, double* partial,
                             int grid, hipStream_t stream);
hipError_t launch_mu_init(const DeviceState& st, const double* sigma, u64 n, const double* nn,
                          double* mu, hipStream_t stream);
hipError_t launch_reduce_partials(const double* partial, int count, int stride, int nvec,
                                  double* out, hipStream_t stream);
// Full-pool gradients by sort and join (k_join.hip); kJoinRunHost records
// per step of the join kernel.
constexpr u64 kJoinRunHost = 2048;
// Largest record count for which SWCS_POOL_AUTO takes the join.
constexpr u64 kJoinAutoMaxRecords = 1ULL << 31;
bool join_format(const ExcSpace& E, u64 n, u64 R, int* kb, int* bh, int* bp, int* orb);
hipError_t launch_join_emit(const DeviceState& st, const ExcSpace& E, u64 n, u64* recs, u64 cap_recs,
                            u64* cursor, int kb, int bh, int bp, int orb, void* src, int grid, hipStream_t stream);
// Gradient terms of the join partitioned by operator: bin b = k mod 2^lb
// holds the terms of operators k = j 2^lb + b (j < kJoinTermSlots) as
// (j, value) at w / j arrays [b cap, b cap + cap), filled up to cursor[b];
// lb < 0 sends every term straight to g[k] with a device-scope add.
constexpr int kJoinTermSlots = 8192;  // operators per bin (one FP64 LDS table of 64 KB)
constexpr int kJoinMaxBinsLog = 8;
struct JoinTerms {
  int lb;
  u64 cap;
  u64* cursor;
  double* w;
  unsigned short* j;
};
hipError_t launch_join_reduce(const DeviceState& st, const u64* recs, u64 R, const u64* cursor, int kb, int bh,
                              int bp, int orb, const void* src, u64 n, const Ints& I, const ExcSpace& E,
                              const int* optab, int nsp, const unsigned char* selected, double* gacc,
                              JoinTerms terms, double* inserted, int grid, hipStream_t stream);
// Sums the binned terms into g[K] (nothing when terms.lb < 0).
hipError_t launch_join_terms(JoinTerms terms, double* gacc, long long K, hipStream_t stream);
hipError_t launch_sigma_push(const DeviceState& st, const Ints& I, const ExcSpace& E, u64 n,
                             AccSlot* tab, u64 tmask, int nbatch, int batch, double* inserted,
                             int grid, hipStream_t stream);
hipError_t launch_pool_contract_det(const DeviceState& st, const ExcSpace& E, int n_spatial, u64 n,
                                   const int* optab, int nsp, const unsigned char* selected,
                                   const AccSlot* tab, u64 tmask, int nbatch, int batch,
                                   double* gacc, int grid, hipStream_t stream);
hipError_t launch_query_set(const DeviceState& st, const ExcSpace& E, int n_spatial, u64 n,
                            const int* optab, int nsp, const unsigned char* selected,
                            AccSlot* tab, u64 tmask, int count_only, u64* counter, int grid,
                            hipStream_t stream, int nbatch = 1, int batch = 0, unsigned* qf = nullptr,
                            u64 qfmask = 0);
hipError_t launch_query_ops(const DeviceState& st, u64 n, const OpDesc* ops, const int* subset,
                            long long n_sub, AccSlot* tab, u64 tmask, int count_only, u64* counter,
                            hipStream_t stream, int nbatch = 1, int batch = 0, unsigned* qf = nullptr,
                            u64 qfmask = 0);
hipError_t launch_contract_ops(const DeviceState& st, u64 n, const OpDesc* ops, const int* subset,
                               long long n_sub, const AccSlot* tab, u64 tmask, double* gslot,
                               hipStream_t stream, int nbatch = 1, int batch = 0);
hipError_t launch_sigma_push_into(const DeviceState& st, const Ints& I, const ExcSpace& E, u64 n,
                                  AccSlot* tab, u64 tmask, int grid, hipStream_t stream, int nbatch = 1, int batch = 0,
                                  const unsigned* qf = nullptr, u64 qfmask = 0);
hipError_t launch_gather_scaled(const double* gacc, const int* subset, long long count,
                                const double* norm2, double* out, hipStream_t stream);
hipError_t launch_mark_selected(const int* subset, long long count, unsigned char* selected,
                                hipStream_t stream);
hipError_t launch_occupations(const DeviceState& st, u64 n, int nso, double* partial, int grid,
                              hipStream_t stream);
hipError_t launch_compact_alive(const DeviceState& st, u64 n, const double* vals, u64* out_keys,
                                double* out_amps, u64* d_count, u64* scratch, u64 scratch_elems,
                                hipStream_t stream);
hipError_t radix_sort_pairs(u64* keys, u64* vals, u64* tmp_keys, u64* tmp_vals, u64 count,
                            int key_bits, u64* scratch, u64 scratch_elems, hipStream_t stream,
                            u64** out_keys = nullptr, u64** out_vals = nullptr);
// Same with 32-bit payloads.
hipError_t radix_sort_pairs32(u64* keys, unsigned* vals, u64* tmp_keys, unsigned* tmp_vals, u64 count,
                              int key_bits, u64* scratch, u64 scratch_elems, hipStream_t stream,
                              u64** out_keys, unsigned** out_vals);
// Keys only (no LDS or traffic for values); out_keys as above.
hipError_t radix_sort_keys(u64* keys, u64* tmp_keys, u64 count, int key_bits, u64* scratch,
                           u64 scratch_elems, hipStream_t stream, u64** out_keys);
u64 radix_sort_scratch_elems(u64 count);
u64 compact_scratch_elems(u64 n);

// Screener.
hipError_t launch_fock(const double* h, const double* eri, int n, int n_occ, double* fock,
                       hipStream_t stream);
hipError_t launch_features(const OpDesc* ops, long long K, const double* fock, const double* eri,
                           int n, const double* occ, const float* prev_absg, const float* age,
                           const float* count, float* feat, hipStream_t stream);
hipError_t launch_mlp_forward(const float* W, const float* x, long long B, float* y, float* act,
                              hipStream_t stream);
long long mlp_backward_partial_rows(long long B);
hipError_t launch_mlp_backward(const float* W, const float* x, const float* act, const float* dy,
                               long long B, float* dW, float* partial, long long partial_rows,
                               hipStream_t stream);
int mse_partial_count(long long B);
hipError_t launch_mse(const float* y, const float* t, long long B, float* dy, float* loss,
                      float* partial, hipStream_t stream);
hipError_t launch_add_feature(float* v, const float* feat, long long n, int col, float sign, float scale,
                              hipStream_t stream);
hipError_t launch_log_abs(const double* g, long long n, float* t, hipStream_t stream);
hipError_t launch_sanitize_subset(const int* in, long long count, long long K, int* out,
                                  hipStream_t stream);
hipError_t launch_nan_invalid(const int* in, long long count, long long K, double* g,
                              hipStream_t stream);
hipError_t launch_adam(float* W, float* m, float* v, const float* g, long long P, float lr,
                       float b1, float b2, float eps, int step, hipStream_t stream);
hipError_t launch_select(const float* score, const uint32_t* rnd, long long K, long long n_top,
                         long long n_rand, int* idx, u64* scratch, u64 scratch_elems,
                         hipStream_t stream);
u64 select_scratch_elems(long long K);

constexpr int kMlpIn = 16;
constexpr int kMlpHidden = 128;
constexpr long long kMlpParams = kMlpIn * kMlpHidden + kMlpHidden + kMlpHidden * kMlpHidden +
                                 kMlpHidden + kMlpHidden + 1;

}  // namespace swcs

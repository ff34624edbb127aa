// C ABI of libswcs: argument validation, device memory, and the host
// orchestration of the kernels in k_state / k_sigma / k_sort / k_screener.
// Declarations and the contract of every call are in include/swcs.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/swcs.h"
#include "conn_ops.h"
#include "gate_ops.h"
#include "swcs_internal.h"

using namespace swcs;

namespace {

thread_local std::string g_create_error;

// Device memory routines of a context: the caller's (swcs_set_allocator)
// or, when none is set, hipMalloc / hipFree.  `cached` counts the bytes the
// library has handed back to the caller's allocator and not taken again, an
// estimate of what a caching allocator holds for it beyond hipMemGetInfo's
// free figure.
struct Allocator {
  swcs_alloc_fn alloc = nullptr;
  swcs_free_fn free = nullptr;
  void* user = nullptr;
  size_t cached = 0;
};

// Device buffer that grows on demand (contents are not preserved on growth).
// It is freed by the routines that allocated it, even if the context's
// allocator has been replaced since.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  Allocator* cur = nullptr;             // allocator of the next allocation
  swcs_free_fn owner_free = nullptr;    // how p is freed (null: hipFree)
  void* owner_user = nullptr;
  Allocator* owner = nullptr;
  hipError_t ensure(size_t want) {
    if (want <= bytes && p) return hipSuccess;
    release();
    if (want == 0) want = 8;
    if (cur && cur->alloc) {
      p = cur->alloc(want, cur->user);
      if (!p) return hipErrorOutOfMemory;
      owner_free = cur->free;
      owner_user = cur->user;
      owner = cur;
      cur->cached = cur->cached > want ? cur->cached - want : 0;
    } else {
      hipError_t e = hipMalloc(&p, want);
      if (e != hipSuccess) {
        p = nullptr;
        return e;
      }
      owner_free = nullptr;
      owner = nullptr;
    }
    bytes = want;
    return hipSuccess;
  }
  void release() {
    if (p) {
      if (owner_free) {
        owner_free(p, owner_user);
        if (owner) owner->cached += bytes;
      } else {
        (void)hipFree(p);
      }
    }
    p = nullptr;
    bytes = 0;
    owner_free = nullptr;
    owner = nullptr;
  }
  template <class T> T* as() const { return (T*)p; }
};

// C(m, k) for m <= 64 by Pascal's rule (no intermediate overflow).
u64 binomial_u64(int m, int k) {
  if (k < 0 || k > m) return 0;
  std::vector<u64> row((size_t)m + 1, 0);
  row[0] = 1;
  for (int i = 1; i <= m; ++i)
    for (int j = std::min(i, k); j >= 1; --j) row[(size_t)j] += row[(size_t)j - 1];
  return row[(size_t)k];
}

u64 next_pow2(u64 x) {
  u64 p = 1;
  while (p < x) p <<= 1;
  return p;
}

double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

}  // namespace

struct swcs_ctx {
  int n = 0, na = 0, nb = 0, nso = 0, device = 0, num_cu = 1;
  hipStream_t stream = nullptr;
  std::string err;
  Allocator alloc;          // device memory routines (swcs_set_allocator)
  int64_t max_dets = 0;
  bool allow_regrow = true;  // false: state arrays reserved once at max_dets
  int64_t table_budget = 0;  // bytes for one sigma accumulation table (0 = from free memory)
  u64 sector = 0;
  ExcSpace exc;

  // integrals
  bool have_ints = false;
  double ecore = 0.0;
  DevBuf h, eri, eri8, J, K, fock;

  // reference and pool
  bool have_ref = false;
  u64 ref = 0;
  bool have_pool = false;
  int64_t K_pool = 0;
  std::vector<OpDesc> ops_host;
  std::vector<int32_t> pool_rows;
  DevBuf ops, opmap;  // pool rows; generator table (P, Q, R, S) -> pool index

  // state
  DevBuf keys, amps, hash, ctr, filt;
  u64 filt_bits_alloc = 0;
  DeviceState st;
  Counters hc;            // host copy of the device counters
  bool hc_valid = false;  // true while no launch may have changed them
  bool have_state = false;
  u64 peak_n = 0;

  // last ansatz (for parameter gradients)
  bool ansatz_valid = false;
  std::vector<int32_t> a_ops;           // per unitary: pool row (row 1 of a star gate)
  std::vector<double> a_theta, a_c, a_s;  // parameters; cos / sin of each unitary's angle
  std::vector<int> a_kind;              // per unitary: 0 one row, 1 overlapping generator
  std::vector<GenGate> a_gen;           // per unitary (kind 1)
  std::vector<int64_t> a_owner;         // per unitary: its parameter
  std::vector<double> a_factor;         // d(angle) / d(parameter)
  bool a_has_star = false;
  double a_eps = 0.0;
  int64_t a_ncut = 0;
  int seg = 1;
  std::vector<DevBuf> ckpt;
  DevBuf ckpt_n;      // u64 per checkpoint
  DevBuf ckpt_ptrs;   // double* per checkpoint (device table)
  std::vector<double*> ckpt_ptrs_host;  // last uploaded contents of ckpt_ptrs
  std::vector<GateDesc> gate_tab_host;  // source of the last gate-table upload
  DevBuf gate_tab;    // GateDesc per gate of the last apply call
  DevBuf gate_n_in;   // u64 per gate of the last apply call
  DevBuf gate_n_act;  // u64 per gate: stored entries the gate's operator acts on
  int64_t last_M = 0;

  // kernel timer: HIP events around every launch of one kernel
  int timer_kernel = 0;
  std::vector<hipEvent_t> ev_start, ev_stop;
  size_t ev_used = 0;

  // scratch
  DevBuf gacc, selected, ncut_state, qfilt;
  DevBuf partial, partial2, sigma, mu, work, seg_states, acc_tab, gbuf, subset_buf, scalars,
      exp_keys, exp_amps, exp_tmp_k, exp_tmp_v, sort_scratch, ctr_r, occ, sel_scratch, mlp_partial, mse_partial, hp_key, hp_val, hp_tk, hp_tv, diag, join_src,
      join_w, join_j, join_bins;
  int sigma_method = SWCS_SIGMA_AUTO;
  int pool_method = SWCS_POOL_AUTO;
  double ext_count = 0.0, ext_alive = 0.0;  // distinct external keys of the last full pool pass
  // the last pool-gradient pass (swcs_pool_stats): keys the table was sized
  // for (distinct external keys after a full pass), slots, batches, passes
  double ps_keys = 0.0;
  u64 ps_slots = 0;
  int ps_batches = 0, ps_passes = 0, ps_screened = 0;
  // The state (and integrals) version, bumped by every call that may change
  // them; the diagonal elements and <psi|psi> on the device are reused while
  // they were computed for the current version.
  u64 state_version = 1, diag_version = 0, norm_version = 0;

  template <class F> void for_each_buf(F&& f) {
    DevBuf* all[] = {&h, &eri, &eri8, &J, &K, &fock, &ops, &opmap, &gacc, &selected, &ncut_state, &filt, &keys, &amps, &hash, &ctr, &ckpt_n, &ckpt_ptrs,
                     &gate_tab, &gate_n_in, &gate_n_act,
                     &partial, &partial2, &sigma, &mu, &work, &seg_states, &acc_tab, &gbuf,
                     &subset_buf, &scalars, &exp_keys, &exp_amps, &exp_tmp_k, &exp_tmp_v,
                     &sort_scratch, &ctr_r, &occ, &sel_scratch, &mlp_partial, &mse_partial,
                     &hp_key, &hp_val, &hp_tk, &hp_tv, &diag, &qfilt, &join_src};
    for (DevBuf* b : all) f(*b);
    for (auto& b : ckpt) f(b);
  }
  // Point every buffer's next allocation at the context's allocator.
  void bind_buffers() {
    for_each_buf([this](DevBuf& b) { b.cur = &alloc; });
  }

  ~swcs_ctx() {
    for_each_buf([](DevBuf& b) { b.release(); });
    for (hipEvent_t e : ev_start) (void)hipEventDestroy(e);
    for (hipEvent_t e : ev_stop) (void)hipEventDestroy(e);
  }
};

namespace {

int fail(swcs_ctx* c, int code, const std::string& msg) {
  c->err = msg;
  return code;
}

int hip_fail(swcs_ctx* c, hipError_t e, const char* where) {
  int code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? SWCS_E_OOM : SWCS_E_DEVICE;
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return code;
}

#define HIP_TRY(ctx, expr, where)                       \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return hip_fail(ctx, _e, where); \
  } while (0)

// Event pair around a launch of the kernel selected by swcs_timer_start.
hipError_t timer_mark(swcs_ctx* c, int kid, bool start) {
  if (c->timer_kernel != kid) return hipSuccess;
  if (start) {
    if (c->ev_used == c->ev_start.size()) {
      hipEvent_t a, b;
      hipError_t e = hipEventCreate(&a);
      if (e != hipSuccess) return e;
      e = hipEventCreate(&b);
      if (e != hipSuccess) return e;
      c->ev_start.push_back(a);
      c->ev_stop.push_back(b);
    }
    return hipEventRecord(c->ev_start[c->ev_used], c->stream);
  }
  hipError_t e = hipEventRecord(c->ev_stop[c->ev_used], c->stream);
  ++c->ev_used;
  return e;
}

#define TIMED(ctx, kid, expr, where)                             \
  do {                                                           \
    HIP_TRY(ctx, timer_mark(ctx, kid, true), "timer");           \
    HIP_TRY(ctx, expr, where);                                   \
    HIP_TRY(ctx, timer_mark(ctx, kid, false), "timer");          \
  } while (0)

int grid_blocks(swcs_ctx* c, u64 work_items, int per_block) {
  u64 g = (work_items + per_block - 1) / per_block;
  u64 maxg = (u64)c->num_cu * 16;
  if (g > maxg) g = maxg;
  if (g < 1) g = 1;
  return (int)g;
}

// Grid of the tiled gate kernels: one block per tile, up to 2,048 resident
// threads per compute unit.
int gate_grid(swcs_ctx* c, u64 n_entries, int tile) {
  u64 g = (n_entries + tile - 1) / tile;
  const u64 maxg = (u64)c->num_cu * (2048 / kGateThreads);
  if (g > maxg) g = maxg;
  if (g < 1) g = 1;
  return (int)g;
}

int sigma_grid(swcs_ctx* c, u64 n) {
  u64 g = n;
  u64 maxg = (u64)c->num_cu * 32;
  if (g > maxg) g = maxg;
  if (g < 1) g = 1;
  return (int)g;
}

Ints ints_view(swcs_ctx* c) {
  Ints I;
  I.h = c->h.as<double>();
  I.eri = c->eri8.as<double>();
  I.J = c->J.as<double>();
  I.K = c->K.as<double>();
  I.ecore = c->ecore;
  I.n = c->n;
  return I;
}

Counters read_counters(swcs_ctx* c, hipError_t* e) {
  Counters h;
  std::memset(&h, 0, sizeof(h));
  *e = hipMemcpyAsync(&h, c->ctr.p, sizeof(Counters), hipMemcpyDeviceToHost, c->stream);
  if (*e == hipSuccess) *e = hipStreamSynchronize(c->stream);
  if (*e == hipSuccess) {
    c->hc = h;
    c->hc_valid = true;
  }
  return h;
}

// Counters without a round trip when nothing has changed them since the
// last read (state sizes only change in apply / set_state).
Counters get_counters(swcs_ctx* c, hipError_t* e) {
  if (c->hc_valid) {
    *e = hipSuccess;
    return c->hc;
  }
  return read_counters(c, e);
}

// Device memory the context may still claim: hipMemGetInfo's free bytes plus
// what it has given back to a caching allocator of the caller.
size_t avail_bytes(swcs_ctx* c) {
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
  return free_b + c->alloc.cached;
}

// Buffers that hold nothing from one call to the next (the external sigma
// table, hole-pair records, sort and export scratch): given back to the device
// when the state needs the memory, and allocated again on their next use.
void release_scratch(swcs_ctx* c) {
  DevBuf* bufs[] = {&c->acc_tab, &c->hp_key, &c->hp_val, &c->hp_tk, &c->hp_tv, &c->sort_scratch,
                    &c->exp_keys, &c->exp_amps, &c->exp_tmp_k, &c->exp_tmp_v, &c->qfilt, &c->join_src};
  for (DevBuf* b : bufs) b->release();
}

// The sort-and-join pool pass keeps its records, sort buffers and source
// table between calls (they hold nothing); a table pass that sizes itself
// from free memory gives them back first when they are large, so that the
// join of a smaller state earlier does not shrink (and split into batches)
// the table of a larger one.
void release_join_scratch(swcs_ctx* c) {
  DevBuf* bufs[] = {&c->hp_key, &c->hp_tk, &c->join_src, &c->sort_scratch, &c->join_w, &c->join_j};
  size_t held = 0;
  for (DevBuf* b : bufs) held += b->bytes;
  if (held < ((size_t)1 << 30)) return;
  for (DevBuf* b : bufs) b->release();
}

// Whether the whole-pool join is taken for a state of `alive` entries: a
// forced join always, AUTO up to kJoinAutoMaxRecords records.
bool join_fits_state(swcs_ctx* c, u64 alive) {
  if (c->pool_method == SWCS_POOL_TABLE) return false;
  if (c->pool_method == SWCS_POOL_JOIN) return true;
  return alive * (u64)(c->exc.total + 1) <= kJoinAutoMaxRecords;
}

// Budget for a table sized from free memory: 40 % of what is free (blocks
// cached by the allocator included) plus the table's own allocation.  The
// join's scratch is given back first only when a table of `need` bytes would
// not fit that budget otherwise: giving it back on every call makes a caching
// allocator split and regrow its blocks from one call to the next.
double free_table_budget(swcs_ctx* c, double need) {
  auto budget = [&]() {
    return std::max<double>(64.0 * 1024 * 1024, 0.4 * (double)(avail_bytes(c) + c->acc_tab.bytes));
  };
  double b = budget();
  if (need > b) {
    release_join_scratch(c);
    b = budget();
  }
  return b;
}

u64 max_capacity(swcs_ctx* c) {
  u64 cap = c->sector;
  if (c->max_dets > 0 && (u64)c->max_dets < cap) cap = (u64)c->max_dets;
  if (c->max_dets <= 0) {
    u64 lim = (u64)(avail_bytes(c) / 96);  // keys + amps + 2 hash slots + headroom
    if (lim < cap) cap = lim;
  }
  if (cap < 16) cap = 16;
  return cap;
}

// Capacity of the state arrays when they may not be regrown: the configured
// maximum (never more than the sector).
u64 fixed_capacity(swcs_ctx* c) {
  return std::max<u64>(16, std::min<u64>(c->sector, (u64)c->max_dets));
}

// (Re)allocate the state arrays with capacity `cap`, preserving the first
// n_keep entries, and rebuild the hash index.
int state_reserve(swcs_ctx* c, u64 cap, u64 n_keep) {
  const u64 hslots = next_pow2(2 * cap);
  DevBuf nk, na;
  nk.cur = &c->alloc;
  na.cur = &c->alloc;
  HIP_TRY(c, nk.ensure(cap * sizeof(u64)), "alloc keys");
  HIP_TRY(c, na.ensure(cap * sizeof(double)), "alloc amps");
  if (n_keep > 0) {
    HIP_TRY(c, hipMemcpyAsync(nk.p, c->keys.p, n_keep * sizeof(u64), hipMemcpyDeviceToDevice, c->stream), "copy keys");
    HIP_TRY(c, hipMemcpyAsync(na.p, c->amps.p, n_keep * sizeof(double), hipMemcpyDeviceToDevice, c->stream), "copy amps");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  }
  c->keys.release();
  c->amps.release();
  c->keys = nk;
  c->amps = na;
  nk.p = nullptr;
  na.p = nullptr;
  if (c->hash.bytes < hslots * sizeof(HashSlot)) {
    c->hash.release();
    HIP_TRY(c, c->hash.ensure(hslots * sizeof(HashSlot)), "alloc hash");
  }
  const u64 fbits = next_pow2(std::max<u64>(4096, 16 * cap));
  HIP_TRY(c, c->filt.ensure(fbits / 8), "alloc filter");
  c->filt_bits_alloc = fbits;
  c->st.keys = c->keys.as<u64>();
  c->st.amps = c->amps.as<double>();
  c->st.hash = c->hash.as<HashSlot>();
  c->st.cap = cap;
  c->st.hmask = hslots - 1;
  c->st.filt = c->filt.as<unsigned>();
  c->st.fmask = fbits - 1;
  c->st.ctr = c->ctr.as<Counters>();
  HIP_TRY(c, launch_hash_clear(c->st.hash, hslots, c->stream), "hash clear");
  if (n_keep > 0) HIP_TRY(c, launch_hash_build(c->st, n_keep, c->stream), "hash build");
  return SWCS_OK;
}

// Presence filter of the alive keys, about 16 bits per key (bounded by the
// allocation) so that it stays cache-resident.
int build_filter(swcs_ctx* c, u64 n, u64 alive) {
  const u64 want = next_pow2(std::max<u64>(4096, 16 * alive));
  c->st.fmask = std::min<u64>(want, c->filt_bits_alloc) - 1;
  HIP_TRY(c, launch_filter_build(c->st, n, grid_blocks(c, n, 256), c->stream), "filter");
  return SWCS_OK;
}

// Rebuild of the state without its pruned entries (tombstones): the alive
// entries are moved, in storage order, to the front of the arrays and the
// index is rebuilt over them.  Storage positions change, so a gate record
// that refers to them (the checkpoints of a chain applied from the
// reference) no longer matches the state: callers compact only states that
// carry no such record, or drop it.  *h is updated to the new counters.
int state_compact(swcs_ctx* c, Counters* h) {
  const u64 n = h->n, alive = h->alive;
  if (alive >= n) return SWCS_OK;
  HIP_TRY(c, c->exp_keys.ensure(std::max<u64>(1, alive) * 8), "alloc");
  HIP_TRY(c, c->exp_amps.ensure(std::max<u64>(1, alive) * 8), "alloc");
  const u64 scr = compact_scratch_elems(n);
  HIP_TRY(c, c->sort_scratch.ensure(scr * 8), "alloc");
  HIP_TRY(c, launch_compact_alive(c->st, n, nullptr, c->exp_keys.as<u64>(), c->exp_amps.as<double>(),
                                  c->scalars.as<u64>() + 8, c->sort_scratch.as<u64>(), scr, c->stream), "compact");
  if (alive > 0) {
    HIP_TRY(c, hipMemcpyAsync(c->st.keys, c->exp_keys.p, alive * 8, hipMemcpyDeviceToDevice, c->stream), "copy keys");
    HIP_TRY(c, hipMemcpyAsync(c->st.amps, c->exp_amps.p, alive * 8, hipMemcpyDeviceToDevice, c->stream), "copy amps");
  }
  HIP_TRY(c, launch_hash_clear(c->st.hash, c->st.hmask + 1, c->stream), "hash clear");
  if (alive > 0) HIP_TRY(c, launch_hash_build(c->st, alive, c->stream), "hash build");
  h->n = alive;
  HIP_TRY(c, launch_store_counters(c->st.ctr, *h, c->stream), "counters");
  c->hc = *h;
  c->hc_valid = true;
  ++c->state_version;
  return SWCS_OK;
}

// Tombstones are reclaimed once they outnumber the alive entries (and are
// at least kCompactMin), so a scan over the stored entries costs at most
// twice one over the alive ones.
constexpr u64 kCompactMin = 4096;
bool compact_due(const Counters& h) {
  const u64 dead = h.n - h.alive;
  return dead >= kCompactMin && dead > h.alive;
}

// Reset the state to the single reference determinant.
int state_reset_to_reference(swcs_ctx* c) {
  u64 cap;
  if (!c->allow_regrow) {
    cap = fixed_capacity(c);
  } else {
    cap = next_pow2(std::max<u64>(4096, 4 * c->peak_n));
    if (cap > c->st.cap && cap > max_capacity(c)) release_scratch(c);
    cap = std::min<u64>(cap, max_capacity(c));
  }
  if (cap < 2) cap = 2;
  if (!c->keys.p || c->st.cap != cap) {
    int r = state_reserve(c, cap, 0);
    if (r) return r;
  } else {
    HIP_TRY(c, launch_hash_clear(c->st.hash, c->st.hmask + 1, c->stream), "hash clear");
  }
  HIP_TRY(c, launch_reset_reference(c->st, c->ref, c->stream), "reset");
  HIP_TRY(c, launch_hash_build(c->st, 1, c->stream), "hash build");
  std::memset(&c->hc, 0, sizeof(c->hc));
  c->hc.n = 1;
  c->hc.alive = 1;
  c->hc_valid = true;
  c->have_state = true;
  return SWCS_OK;
}

int check_ready(swcs_ctx* c) {
  if (!c->have_ints) return fail(c, SWCS_E_STATE, "integrals not set");
  if (!c->have_ref) return fail(c, SWCS_E_STATE, "reference not set");
  if (!c->have_pool) return fail(c, SWCS_E_STATE, "pool not set");
  return SWCS_OK;
}

int validate_gates(swcs_ctx* c, const int32_t* op_idx, const double* theta, int64_t M, double eps,
                   int64_t ncut) {
  if (M < 0) return fail(c, SWCS_E_INVALID, "M < 0");
  if (M > 0 && (!op_idx || !theta)) return fail(c, SWCS_E_INVALID, "null op_idx/theta");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(c, SWCS_E_INVALID, "eps must be finite and >= 0");
  if (ncut < 0) return fail(c, SWCS_E_INVALID, "ncut < 0");
  if (ncut > 0x7fffffffLL) return fail(c, SWCS_E_INVALID, "ncut too large");
  for (int64_t i = 0; i < M; ++i) {
    if (op_idx[i] < 0 || op_idx[i] >= c->K_pool) return fail(c, SWCS_E_INVALID, "op index out of range");
    if (!std::isfinite(theta[i])) return fail(c, SWCS_E_INVALID, "non-finite theta");
  }
  return SWCS_OK;
}

// Upload the checkpoint pointer table (device array of double*).
int upload_ckpt_table(swcs_ctx* c, int nck) {
  std::vector<double*> ptrs((size_t)nck);
  for (int j = 0; j < nck; ++j) ptrs[(size_t)j] = c->ckpt[(size_t)j].as<double>();
  if (ptrs == c->ckpt_ptrs_host && c->ckpt_ptrs.bytes >= (size_t)nck * sizeof(double*))
    return SWCS_OK;  // device table already current
  // The previous upload may still be reading the host copy: wait for it.
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  c->ckpt_ptrs_host = ptrs;
  HIP_TRY(c, c->ckpt_ptrs.ensure((size_t)nck * sizeof(double*)), "alloc ckpt table");
  HIP_TRY(c, hipMemcpyAsync(c->ckpt_ptrs.p, c->ckpt_ptrs_host.data(), (size_t)nck * sizeof(double*),
                            hipMemcpyHostToDevice, c->stream), "copy ckpt table");
  return SWCS_OK;
}

// Apply gates [0, M) of (ops, c, s) to the current state, with checkpoints
// every `seg` gates when ckpt is requested.  A state that starts with at
// most lds_chain_capacity() entries runs in one single-workgroup launch
// (LDS-resident) for as long as it fits; the rest runs one multi-block
// launch per gate in HBM, growing the arrays when a gate would not fit.
int run_chain(swcs_ctx* c, const int32_t* op_idx, const double* cs, const double* sn, int64_t M,
              double eps, unsigned ncut, bool ckpt, u64 n_start, Counters* out,
              const int* kind = nullptr, const GenGate* gen = nullptr) {
  bool has_star = false;
  for (int64_t g = 0; kind && g < M; ++g) has_star |= kind[g] != 0;
  // With N_CUT the gates keep everything and the selection prunes.
  if (ncut) eps = 0.0;
  int64_t g0 = 0;
  c->hc_valid = false;
  if (M == 0) {
    hipError_t e;
    *out = read_counters(c, &e);
    if (e != hipSuccess) return hip_fail(c, e, "read counters");
    return SWCS_OK;
  }
  // The previous upload from gate_tab_host must be complete before it is
  // rewritten.
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  std::vector<GateDesc>& gt = c->gate_tab_host;
  gt.resize((size_t)M);
  for (int64_t g = 0; g < M; ++g) {
    gt[(size_t)g].op = c->ops_host[op_idx[g]];
    gt[(size_t)g].c = cs[g];
    gt[(size_t)g].s = sn[g];
  }
  HIP_TRY(c, c->gate_tab.ensure((size_t)M * sizeof(GateDesc)), "alloc gate table");
  HIP_TRY(c, hipMemcpyAsync(c->gate_tab.p, gt.data(), (size_t)M * sizeof(GateDesc),
                            hipMemcpyHostToDevice, c->stream), "copy gate table");
  if (ckpt) {
    const int nck = (int)((M + c->seg - 1) / c->seg);
    for (int j = 0; j < nck; ++j)
      HIP_TRY(c, c->ckpt[(size_t)j].ensure(c->st.cap * sizeof(double)), "alloc checkpoint");
    int r = upload_ckpt_table(c, nck);
    if (r) return r;
  }
  // overlapping generators have no single-workgroup kernel: such chains run
  // in HBM from the first gate
  if (!has_star && n_start <= (u64)lds_chain_capacity() && c->st.cap >= (u64)lds_chain_capacity() &&
      M <= (int64_t)1 << 30) {
    TIMED(c, SWCS_K_CHAIN_LDS, launch_chain_lds(c->st, c->gate_tab.as<GateDesc>(), 0, (int)M, eps, eps > 0.0 ? 1 : 0,
                                ckpt ? c->ckpt_ptrs.as<double*>() : nullptr, c->ckpt_n.as<u64>(),
                                c->seg, c->gate_n_in.as<u64>(), c->sector, ncut, c->stream), "chain");
    HIP_TRY(c, launch_hash_clear(c->st.hash, c->st.hmask + 1, c->stream), "hash clear");
    HIP_TRY(c, launch_hash_build_dev(c->st, grid_blocks(c, lds_chain_capacity(), 256), c->stream), "hash build");
    hipError_t e;
    Counters h = read_counters(c, &e);
    if (e != hipSuccess) return hip_fail(c, e, "read counters");
    if (!(h.flags & kFlagStopped)) {
      *out = h;
      return SWCS_OK;
    }
    // Continue in HBM from the gate that did not fit in LDS.
    g0 = (int64_t)h.stop_gate;
    h.flags &= ~kFlagStopped;
    h.stop_gate = 0;
    HIP_TRY(c, launch_store_counters(c->st.ctr, h, c->stream), "counters");
  }
  for (int attempt = 0; attempt < 64; ++attempt) {
    for (int64_t g = g0; g < M; ++g) {
      if (ckpt && g % c->seg == 0) {
        const int j = (int)(g / c->seg);
        HIP_TRY(c, c->ckpt[j].ensure(c->st.cap * sizeof(double)), "alloc checkpoint");
        HIP_TRY(c, launch_ckpt_save(c->st, c->ckpt[j].as<double>(), c->ckpt_n.as<u64>() + j,
                                    grid_blocks(c, c->st.cap / 4, 256), c->stream), "checkpoint");
      }
      const OpDesc& op = c->ops_host[op_idx[g]];
      if (kind && kind[g])
        HIP_TRY(c, launch_gen_gate(c->st, gen[g], eps, c->gate_n_in.as<u64>() + g, (unsigned)g, c->sector,
                                   grid_blocks(c, c->st.cap / 2, 256), c->stream, c->gate_n_act.as<u64>() + g),
                "generator gate");
      else
        TIMED(c, SWCS_K_GATE, launch_gate(c->st, op, cs[g], sn[g], eps, c->gate_n_in.as<u64>() + g, 1,
                               (unsigned)g, c->sector, gate_grid(c, c->st.cap / 2, gate_scan_tile(c->st.cap)), c->stream,
                               c->gate_n_act.as<u64>() + g),
                "gate");
      // The gates only test the entries they touch; entries of a starting
      // state that were never tested against eps are pruned once, after the
      // first gate, so every later state is exactly P(U psi).
      if (g == 0 && eps > 0.0)
        HIP_TRY(c, launch_prune_all(c->st, eps, grid_blocks(c, c->st.cap / 2, 256), c->stream), "prune");
      if (ncut)
        HIP_TRY(c, launch_ncut(c->st.amps, c->st.keys, 0, c->st.ctr, c->ncut_state.as<NcutState>(), ncut,
                               grid_blocks(c, c->st.cap / 2, 256), c->stream), "ncut");
    }
    hipError_t e;
    Counters h = read_counters(c, &e);
    if (e != hipSuccess) return hip_fail(c, e, "read counters");
    if (h.flags & kFlagOverflow) {
      h.flags &= ~(kFlagOverflow | kFlagStopped);
      HIP_TRY(c, launch_store_counters(c->st.ctr, h, c->stream), "counters");
      c->hc_valid = false;
      return fail(c, SWCS_E_DEVICE, "internal overflow in gate chain");
    }
    if (!(h.flags & kFlagStopped)) {
      // a chain without checkpoints leaves no record of storage positions
      if (!ckpt && compact_due(h)) {
        int r = state_compact(c, &h);
        if (r) return r;
      }
      *out = h;
      return SWCS_OK;
    }
    g0 = (int64_t)h.stop_gate;
    h.flags &= ~kFlagStopped;
    h.stop_gate = 0;
    // A stopped gate changed nothing.  Without checkpoints, tombstones are
    // reclaimed first when they are a quarter of the alive entries or more,
    // and the arrays grow only if the gate still does not fit.
    const bool star_stop = kind && kind[g0];
    if (!ckpt && h.n - h.alive >= kCompactMin && 4 * (h.n - h.alive) >= h.alive) {
      int r = state_compact(c, &h);
      if (r) return r;
      const u64 room = c->sector > h.n ? c->sector - h.n : 0;
      const u64 grow_c = star_stop ? 2 * h.alive : h.alive;
      if (h.n + std::min<u64>(grow_c, room) <= c->st.cap) continue;
    }
    HIP_TRY(c, launch_store_counters(c->st.ctr, h, c->stream), "counters");
    if (!c->allow_regrow) {
      c->have_state = false;  // the chain stopped part way
      return fail(c, SWCS_E_CAPACITY, "state exceeds the fixed capacity (regrowth disabled)");
    }
    // Grow so that the stopped gate (and a few more) fit, then resume (a star
    // gate appends up to two entries per alive one).
    const u64 grow = star_stop ? 2 * h.alive : h.alive;
    const u64 need = h.n + std::min<u64>(grow, c->sector > h.n ? c->sector - h.n : 0);
    u64 cap = next_pow2(std::max<u64>(2 * c->st.cap, 2 * need));
    u64 maxc = max_capacity(c);
    if (maxc < cap) {
      release_scratch(c);
      maxc = max_capacity(c);
    }
    if (cap > maxc) cap = maxc;
    if (cap < need) return fail(c, SWCS_E_CAPACITY, "state exceeds the maximum capacity");
    int r = state_reserve(c, cap, h.n);
    if (r) return r;
    // Checkpoint of the gate where the chain resumes was skipped if it lies
    // on a segment boundary: the loop above re-enqueues it.
  }
  return fail(c, SWCS_E_CAPACITY, "capacity growth did not converge");
}

}  // namespace

// ---- energy without allocation ----
// Scratch of the allocation-free energy: the library's own device array,
// 32 MiB on every device the library runs on, held until the process ends.
// Layout in doubles: 2 x 8,192 per-block partial sums, 64 result slots, then
// the diagonal elements and sigma_P of up to kNoAllocMaxEntries stored
// entries.  Host code never passes `scratch` itself to a kernel: it resolves
// the array's device address once per device (noalloc_scratch).
constexpr size_t kNoAllocBytes = (size_t)32 << 20;
constexpr size_t kNoAllocPartials = 2 * 8192;
constexpr size_t kNoAllocHead = kNoAllocPartials + 64;
constexpr u64 kNoAllocMaxEntries = (kNoAllocBytes / 8 - kNoAllocHead) / 2;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_dev[64] = {};  // device address of `scratch` per device index

// Device address of `scratch` on the context's device (which must be
// current), resolved on the first call for that device.
hipError_t noalloc_scratch(int device, double** out) {
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[device] = p;
  }
  *out = (double*)g_scratch_dev[device];
  return hipSuccess;
}
}  // namespace

extern "C" {

const char* swcs_version(void) { return "swcs-mi355x 0.1 (gfx950)"; }

int swcs_create(int n_spatial, int n_alpha, int n_beta, int device, swcs_ctx** out) {
  if (!out) {
    g_create_error = "out is NULL";
    return SWCS_E_INVALID;
  }
  *out = nullptr;
  if (n_spatial < 1 || 2 * n_spatial > 64 || n_alpha < 0 || n_beta < 0 || n_alpha > n_spatial ||
      n_beta > n_spatial || n_alpha + n_beta < 1) {
    g_create_error = "invalid orbital / electron counts (need 1 <= 2n <= 64, 0 <= n_a, n_b <= n)";
    return SWCS_E_INVALID;
  }
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
    g_create_error = "no HIP device available";
    return SWCS_E_UNSUPPORTED;
  }
  if (device < 0 || device >= count) {
    g_create_error = "device index out of range";
    return SWCS_E_INVALID;
  }
  if (hipSetDevice(device) != hipSuccess) {
    g_create_error = "hipSetDevice failed";
    return SWCS_E_DEVICE;
  }
  swcs_ctx* c = new swcs_ctx;
  c->n = n_spatial;
  c->na = n_alpha;
  c->nb = n_beta;
  c->nso = 2 * n_spatial;
  c->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->num_cu = prop.multiProcessorCount;
  double sec = binom(n_spatial, n_alpha) * binom(n_spatial, n_beta);
  c->sector = sec > 1e18 ? (u64)1e18 : (u64)sec;
  c->exc = make_exc_space(n_spatial, n_alpha, n_beta);
  c->bind_buffers();
  if (c->ctr.ensure(sizeof(Counters)) != hipSuccess || c->scalars.ensure(64 * sizeof(double)) != hipSuccess) {
    g_create_error = "device allocation failed";
    delete c;
    return SWCS_E_OOM;
  }
  if (hipMemset(c->ctr.p, 0, sizeof(Counters)) != hipSuccess) {
    g_create_error = "device memset failed";
    delete c;
    return SWCS_E_DEVICE;
  }
  c->st.ctr = c->ctr.as<Counters>();
  // device address of the allocation-free energy's scratch, once per device
  // (a failure here is reported by that entry point, which retries)
  double* scr = nullptr;
  (void)noalloc_scratch(device, &scr);
  *out = c;
  return SWCS_OK;
}

void swcs_destroy(swcs_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  delete ctx;
}

const char* swcs_last_error(const swcs_ctx* ctx) {
  if (!ctx) return g_create_error.c_str();
  return ctx->err.c_str();
}

int swcs_set_stream(swcs_ctx* c, void* hip_stream) {
  if (!c) return SWCS_E_INVALID;
  ++c->state_version;  // cached device results belong to the old stream's order
  c->stream = (hipStream_t)hip_stream;
  return SWCS_OK;
}

int swcs_set_capacity(swcs_ctx* c, int64_t max_dets, int allow_regrow) {
  if (!c) return SWCS_E_INVALID;
  if (max_dets < 0) return fail(c, SWCS_E_INVALID, "max_dets < 0");
  if (!allow_regrow && max_dets == 0) return fail(c, SWCS_E_INVALID, "a fixed capacity needs max_dets > 0");
  c->max_dets = max_dets;
  c->allow_regrow = allow_regrow != 0;
  return SWCS_OK;
}

int swcs_set_allocator(swcs_ctx* c, swcs_alloc_fn alloc_fn, swcs_free_fn free_fn, void* user) {
  if (!c) return SWCS_E_INVALID;
  if ((alloc_fn == nullptr) != (free_fn == nullptr))
    return fail(c, SWCS_E_INVALID, "alloc_fn and free_fn must both be set or both be NULL");
  c->alloc.alloc = alloc_fn;
  c->alloc.free = free_fn;
  c->alloc.user = user;
  c->alloc.cached = 0;
  return SWCS_OK;
}

int swcs_set_table_budget(swcs_ctx* c, int64_t bytes) {
  if (!c) return SWCS_E_INVALID;
  if (bytes < 0) return fail(c, SWCS_E_INVALID, "bytes < 0");
  if (bytes > 0 && bytes < 4096) return fail(c, SWCS_E_INVALID, "table budget below 4096 bytes");
  c->table_budget = bytes;
  return SWCS_OK;
}

int swcs_set_sigma_method(swcs_ctx* c, int method) {
  if (!c) return SWCS_E_INVALID;
  if (method != SWCS_SIGMA_AUTO && method != SWCS_SIGMA_ENUMERATE && method != SWCS_SIGMA_HOLE_PAIRS &&
      method != SWCS_SIGMA_PAIRS)
    return fail(c, SWCS_E_INVALID, "unknown sigma method");
  c->sigma_method = method;
  return SWCS_OK;
}

int swcs_set_pool_method(swcs_ctx* c, int method) {
  if (!c) return SWCS_E_INVALID;
  if (method != SWCS_POOL_AUTO && method != SWCS_POOL_TABLE && method != SWCS_POOL_JOIN)
    return fail(c, SWCS_E_INVALID, "unknown pool method");
  c->pool_method = method;
  return SWCS_OK;
}

int swcs_set_integrals(swcs_ctx* c, const double* h, const double* eri, double e_core) {
  if (!c) return SWCS_E_INVALID;
  ++c->state_version;
  if (!h || !eri) return fail(c, SWCS_E_INVALID, "null integrals");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  const int n = c->n;
  const size_t n2 = (size_t)n * n, n4 = n2 * n2;
  if (!std::isfinite(e_core)) return fail(c, SWCS_E_INVALID, "non-finite e_core");
  for (size_t i = 0; i < n2; ++i)
    if (!std::isfinite(h[i])) return fail(c, SWCS_E_INVALID, "non-finite h");
  for (size_t i = 0; i < n4; ++i)
    if (!std::isfinite(eri[i])) return fail(c, SWCS_E_INVALID, "non-finite eri");
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q)
      if (std::fabs(h[p * n + q] - h[q * n + p]) > 1e-12) return fail(c, SWCS_E_INVALID, "h not symmetric");
  auto E = [&](int p, int q, int r, int s) { return eri[((size_t)(p * n + q) * n + r) * n + s]; };
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q)
      for (int r = 0; r < n; ++r)
        for (int s = 0; s < n; ++s) {
          const double v = E(p, q, r, s);
          if (std::fabs(v - E(q, p, r, s)) > 1e-12 || std::fabs(v - E(p, q, s, r)) > 1e-12 ||
              std::fabs(v - E(r, s, p, q)) > 1e-12)
            return fail(c, SWCS_E_INVALID, "eri lacks 8-fold symmetry");
        }
  // (pq|rs) packed by symmetry, the element at p >= q, r >= s, pq >= rs
  const size_t m = (size_t)n * (n + 1) / 2;
  std::vector<double> e8(m * (m + 1) / 2);
  for (int p = 0; p < n; ++p)
    for (int q = 0; q <= p; ++q)
      for (int r = 0; r < n; ++r)
        for (int s = 0; s <= r; ++s)
          if (p * (p + 1) / 2 + q >= r * (r + 1) / 2 + s) e8[eri_packed_index(p, q, r, s)] = E(p, q, r, s);
  std::vector<double> Jh(n2), Kh(n2);
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) {
      Jh[p * n + q] = E(p, p, q, q);
      Kh[p * n + q] = E(p, q, q, p);
    }
  HIP_TRY(c, c->h.ensure(n2 * 8), "alloc h");
  HIP_TRY(c, c->eri.ensure(n4 * 8), "alloc eri");
  HIP_TRY(c, c->eri8.ensure(e8.size() * 8), "alloc packed eri");
  HIP_TRY(c, c->J.ensure(n2 * 8), "alloc J");
  HIP_TRY(c, c->K.ensure(n2 * 8), "alloc K");
  HIP_TRY(c, c->fock.ensure(n2 * 8), "alloc fock");
  HIP_TRY(c, hipMemcpyAsync(c->h.p, h, n2 * 8, hipMemcpyHostToDevice, c->stream), "copy h");
  HIP_TRY(c, hipMemcpyAsync(c->eri.p, eri, n4 * 8, hipMemcpyHostToDevice, c->stream), "copy eri");
  HIP_TRY(c, hipMemcpyAsync(c->eri8.p, e8.data(), e8.size() * 8, hipMemcpyHostToDevice, c->stream), "copy eri");
  HIP_TRY(c, hipMemcpyAsync(c->J.p, Jh.data(), n2 * 8, hipMemcpyHostToDevice, c->stream), "copy J");
  HIP_TRY(c, hipMemcpyAsync(c->K.p, Kh.data(), n2 * 8, hipMemcpyHostToDevice, c->stream), "copy K");
  HIP_TRY(c, launch_fock(c->h.as<double>(), c->eri.as<double>(), n, c->na, c->fock.as<double>(),
                         c->stream), "fock");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  c->ecore = e_core;
  c->have_ints = true;
  c->ansatz_valid = false;
  return SWCS_OK;
}

int swcs_set_reference(swcs_ctx* c, uint64_t det) {
  if (!c) return SWCS_E_INVALID;
  if (c->nso < 64 && (det >> c->nso) != 0) return fail(c, SWCS_E_INVALID, "reference has bits beyond 2n");
  const int a = __builtin_popcountll(det & 0x5555555555555555ULL);
  const int b = __builtin_popcountll(det & 0xAAAAAAAAAAAAAAAAULL);
  if (a != c->na || b != c->nb) return fail(c, SWCS_E_INVALID, "reference electron counts differ from n_alpha/n_beta");
  c->ref = det;
  c->have_ref = true;
  c->ansatz_valid = false;
  return SWCS_OK;
}

int swcs_set_pool(swcs_ctx* c, const int32_t* rows, int64_t K) {
  if (!c) return SWCS_E_INVALID;
  if (K < 0 || (K > 0 && !rows)) return fail(c, SWCS_E_INVALID, "bad pool arguments");
  if (K > (int64_t)1 << 30) return fail(c, SWCS_E_INVALID, "pool too large");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  std::vector<OpDesc> ops((size_t)K);
  const int N = c->nso;
  for (int64_t k = 0; k < K; ++k) {
    const int32_t* r = rows + 4 * k;
    OpDesc o;
    o.P = r[0]; o.Q = r[1]; o.R = r[2]; o.S = r[3];
    const bool single = (o.R == -1 && o.S == -1);
    if (o.P < 0 || o.P >= N || o.Q < 0 || o.Q >= N || o.P <= o.Q)
      return fail(c, SWCS_E_INVALID, "pool row " + std::to_string(k) + ": need 2n > P > Q >= 0");
    if (single) {
      if ((o.P & 1) != (o.Q & 1)) return fail(c, SWCS_E_INVALID, "pool row " + std::to_string(k) + ": single changes spin");
      o.cre = 1ULL << o.P;
      o.ann = 1ULL << o.Q;
    } else {
      if (o.R < 0 || o.R >= N || o.S < 0 || o.S >= N || o.R <= o.S)
        return fail(c, SWCS_E_INVALID, "pool row " + std::to_string(k) + ": need 2n > R > S >= 0");
      if (o.P == o.R || o.P == o.S || o.Q == o.R || o.Q == o.S)
        return fail(c, SWCS_E_INVALID, "pool row " + std::to_string(k) + ": index sets overlap");
      if (((o.P & 1) + (o.Q & 1)) != ((o.R & 1) + (o.S & 1)))
        return fail(c, SWCS_E_INVALID, "pool row " + std::to_string(k) + ": double changes spin");
      if (!(o.P > o.R || (o.P == o.R && o.Q > o.S)))
        return fail(c, SWCS_E_INVALID, "pool row " + std::to_string(k) + ": need (P, Q) > (R, S)");
      o.cre = (1ULL << o.P) | (1ULL << o.Q);
      o.ann = (1ULL << o.R) | (1ULL << o.S);
    }
    ops[(size_t)k] = o;
  }
  // Generator table (P, Q, R, S) -> pool index in the layout of
  // optab_double_slot (conn_ops.h); -1 where the pool has no operator.
  // Rejects duplicate rows.
  std::vector<int> optab((size_t)optab_size(c->n), -1);
  for (int64_t k = 0; k < K; ++k) {
    const OpDesc& o = ops[(size_t)k];
    const int64_t slot = o.R < 0 ? pair_index(o.P, o.Q) : optab_double_slot(c->n, o.P, o.Q, o.R, o.S);
    if (optab[(size_t)slot] >= 0)
      return fail(c, SWCS_E_INVALID, "pool row " + std::to_string(k) + " duplicates an earlier row");
    optab[(size_t)slot] = (int)k;
  }
  // earlier work of the stream may still read the old tables
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  HIP_TRY(c, c->opmap.ensure(optab.size() * sizeof(int)), "alloc generator table");
  HIP_TRY(c, hipMemcpyAsync(c->opmap.p, optab.data(), optab.size() * sizeof(int), hipMemcpyHostToDevice, c->stream),
          "copy generator table");
  HIP_TRY(c, c->ops.ensure(std::max<size_t>(1, (size_t)K) * sizeof(OpDesc)), "alloc pool");
  if (K > 0)
    HIP_TRY(c, hipMemcpyAsync(c->ops.p, ops.data(), (size_t)K * sizeof(OpDesc), hipMemcpyHostToDevice, c->stream),
            "copy pool");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  c->ops_host.swap(ops);
  c->pool_rows.assign(rows, rows + 4 * K);
  c->K_pool = K;
  c->have_pool = true;
  c->ansatz_valid = false;
  return SWCS_OK;
}

// The unitaries of one apply call and the parameters they depend on.
struct ChainSpec {
  std::vector<int32_t> ops;    // pool row (row 1 of a star gate)
  std::vector<double> cs, sn;  // cos and sin of each unitary's angle
  std::vector<int> kind;       // 0 one row, 1 overlapping generator
  std::vector<GenGate> gen;    // kind 1
  std::vector<int64_t> owner;  // parameter of each unitary
  std::vector<double> factor;  // d(angle) / d(parameter)
  std::vector<double> theta;   // the parameters
  bool has_star = false;
};

static void spec_plain(const int32_t* op_idx, const double* theta, int64_t M, ChainSpec* sp) {
  sp->ops.assign(op_idx, op_idx + M);
  sp->theta.assign(theta, theta + M);
  sp->cs.resize((size_t)M);
  sp->sn.resize((size_t)M);
  for (int64_t i = 0; i < M; ++i) {
    sp->cs[(size_t)i] = std::cos(theta[i]);
    sp->sn[(size_t)i] = std::sin(theta[i]);
  }
  sp->kind.assign((size_t)M, 0);
  sp->gen.assign((size_t)M, GenGate{});
  sp->owner.resize((size_t)M);
  for (int64_t i = 0; i < M; ++i) sp->owner[(size_t)i] = i;
  sp->factor.assign((size_t)M, 1.0);
}

static int apply_common(swcs_ctx* c, ChainSpec& sp, double eps, int64_t ncut, int64_t* n_det_out,
                        bool from_reference) {
  const int64_t M = (int64_t)sp.ops.size();
  if (!from_reference && !c->have_state) return fail(c, SWCS_E_STATE, "no current state");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  ++c->state_version;
  HIP_TRY(c, c->gate_n_in.ensure(std::max<int64_t>(1, M) * sizeof(u64)), "alloc stats");
  HIP_TRY(c, c->gate_n_act.ensure(std::max<int64_t>(1, M) * sizeof(u64)), "alloc stats");
  HIP_TRY(c, launch_fill_u32(c->gate_n_act.p, 0u, (u64)std::max<int64_t>(1, M) * 2, c->stream), "zero stats");
  c->ansatz_valid = false;
  if (from_reference) {
    int r = state_reset_to_reference(c);
    if (r) return r;
    c->seg = std::max<int>(1, (int)std::ceil(std::sqrt((double)std::max<int64_t>(1, M))));
    const int nck = (int)((M + c->seg - 1) / c->seg) + 1;
    if ((int)c->ckpt.size() < nck) {
      c->ckpt.resize(nck);
      c->bind_buffers();
    }
    HIP_TRY(c, c->ckpt_n.ensure((size_t)nck * sizeof(u64)), "alloc ckpt sizes");
  }
  Counters h;
  u64 n_start = 1;
  if (!from_reference) {
    hipError_t e;
    Counters h0 = get_counters(c, &e);
    if (e != hipSuccess) return hip_fail(c, e, "read counters");
    n_start = h0.n;
  }
  HIP_TRY(c, c->ncut_state.ensure(sizeof(NcutState)), "alloc ncut state");
  int r = run_chain(c, sp.ops.data(), sp.cs.data(), sp.sn.data(), M, eps, (unsigned)ncut, from_reference,
                    n_start, &h, sp.kind.data(), sp.gen.data());
  if (r) return r;
  r = build_filter(c, h.n, h.alive);
  if (r) return r;
  c->peak_n = std::max<u64>(c->peak_n, h.n);
  c->last_M = M;
  if (from_reference) {
    c->a_ops = sp.ops;
    c->a_theta = sp.theta;
    c->a_c = sp.cs;
    c->a_s = sp.sn;
    c->a_kind = sp.kind;
    c->a_gen = sp.gen;
    c->a_owner = sp.owner;
    c->a_factor = sp.factor;
    c->a_has_star = sp.has_star;
    c->a_eps = eps;
    c->a_ncut = ncut;
    c->ansatz_valid = true;
  }
  if (n_det_out) *n_det_out = (int64_t)h.alive;
  return SWCS_OK;
}

int swcs_apply_ansatz(swcs_ctx* c, const int32_t* op_idx, const double* theta, int64_t M,
                      double eps, int64_t ncut, int64_t* n_det_out) {
  if (!c) return SWCS_E_INVALID;
  int r = check_ready(c);
  if (r) return r;
  r = validate_gates(c, op_idx, theta, M, eps, ncut);
  if (r) return r;
  ChainSpec sp;
  spec_plain(op_idx, theta, M, &sp);
  return apply_common(c, sp, eps, ncut, n_det_out, true);
}

// Row k2 is the spin flip of row k1 (every spin-orbital P -> P ^ 1, in the
// same or the adjoint orientation).
static bool is_spin_flip(const OpDesc& a, const OpDesc& b) {
  auto flip = [](u64 m) { return ((m & 0x5555555555555555ULL) << 1) | ((m >> 1) & 0x5555555555555555ULL); };
  return (flip(a.cre) == b.cre && flip(a.ann) == b.ann) || (flip(a.cre) == b.ann && flip(a.ann) == b.cre);
}

int swcs_apply_generators(swcs_ctx* c, const int32_t* gens, const double* theta, int64_t M, double eps,
                          int64_t ncut, int64_t* n_det_out) {
  if (!c) return SWCS_E_INVALID;
  int r = check_ready(c);
  if (r) return r;
  if (M < 0) return fail(c, SWCS_E_INVALID, "M < 0");
  if (M > 0 && (!gens || !theta)) return fail(c, SWCS_E_INVALID, "null gens/theta");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(c, SWCS_E_INVALID, "eps must be finite and >= 0");
  if (ncut < 0 || ncut > 0x7fffffffLL) return fail(c, SWCS_E_INVALID, "ncut out of range");
  ChainSpec sp;
  const double rt = 1.0 / std::sqrt(2.0);
  for (int64_t i = 0; i < M; ++i) {
    const int32_t k1 = gens[3 * i], k2 = gens[3 * i + 1], sg = gens[3 * i + 2];
    const std::string at = "generator " + std::to_string(i) + ": ";
    if (k1 < 0 || k1 >= c->K_pool) return fail(c, SWCS_E_INVALID, at + "row 1 out of range");
    if (k2 < -1 || k2 >= c->K_pool || k2 == k1) return fail(c, SWCS_E_INVALID, at + "bad row 2");
    if (k2 >= 0 && sg != 1 && sg != -1) return fail(c, SWCS_E_INVALID, at + "sign must be +1 or -1");
    if (!std::isfinite(theta[i])) return fail(c, SWCS_E_INVALID, at + "non-finite theta");
    const double cth = std::cos(theta[i]), sth = std::sin(theta[i]);
    auto push = [&](int32_t k, double sn_u, double factor, int kd, const GenGate& g) {
      sp.ops.push_back(k);
      sp.cs.push_back(cth);
      sp.sn.push_back(sn_u);
      sp.kind.push_back(kd);
      sp.gen.push_back(g);
      sp.owner.push_back(i);
      sp.factor.push_back(factor);
    };
    if (k2 < 0) {
      push(k1, sth, 1.0, 0, GenGate{});
    } else {
      const OpDesc& o1 = c->ops_host[k1];
      const OpDesc& o2 = c->ops_host[k2];
      const bool overlap = ((o1.ann | o1.cre) & (o2.ann | o2.cre)) != 0;
      if (!overlap) {
        // commuting parts: two unitaries, row 2 at s theta
        push(k1, sth, 1.0, 0, GenGate{});
        push(k2, (double)sg * sth, (double)sg, 0, GenGate{});
      } else {
        if (o1.R < 0 || o2.R < 0 || !is_spin_flip(o1, o2))
          return fail(c, SWCS_E_UNSUPPORTED, at + "overlapping rows must be a double and its spin flip");
        GenGate g;
        g.op1 = o1;
        g.op2 = o2;
        g.c = cth;
        g.sn = sth;
        g.sn2 = (double)sg * sth;
        const double w = std::sqrt(2.0) * theta[i];
        g.c2 = std::cos(w);
        g.s2 = std::sin(w);
        g.rt = rt;
        g.sg = (double)sg;
        push(k1, sth, 1.0, 1, g);
        sp.has_star = true;
      }
    }
  }
  sp.theta.assign(theta, theta + M);
  return apply_common(c, sp, eps, ncut, n_det_out, true);
}

int swcs_apply_gates(swcs_ctx* c, const int32_t* op_idx, const double* theta, int64_t M,
                     double eps, int64_t ncut, int64_t* n_det_out) {
  if (!c) return SWCS_E_INVALID;
  int r = check_ready(c);
  if (r) return r;
  r = validate_gates(c, op_idx, theta, M, eps, ncut);
  if (r) return r;
  ChainSpec sp;
  spec_plain(op_idx, theta, M, &sp);
  return apply_common(c, sp, eps, ncut, n_det_out, false);
}

int swcs_set_state(swcs_ctx* c, const uint64_t* keys, const double* amps, int64_t n) {
  if (!c) return SWCS_E_INVALID;
  ++c->state_version;
  if (n < 0 || (n > 0 && (!keys || !amps))) return fail(c, SWCS_E_INVALID, "bad state arguments");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  std::vector<u64> sorted(keys, keys + n);
  std::sort(sorted.begin(), sorted.end());
  for (int64_t i = 0; i < n; ++i) {
    const u64 k = keys[i];
    if (c->nso < 64 && (k >> c->nso) != 0) return fail(c, SWCS_E_INVALID, "key has bits beyond 2n");
    if (__builtin_popcountll(k & 0x5555555555555555ULL) != c->na ||
        __builtin_popcountll(k & 0xAAAAAAAAAAAAAAAAULL) != c->nb)
      return fail(c, SWCS_E_INVALID, "key outside the (n_alpha, n_beta) sector");
    if (!std::isfinite(amps[i])) return fail(c, SWCS_E_INVALID, "non-finite amplitude");
    if (i > 0 && sorted[(size_t)i] == sorted[(size_t)i - 1]) return fail(c, SWCS_E_INVALID, "duplicate key");
  }
  u64 cap = next_pow2(std::max<u64>(4096, 2 * (u64)n));
  cap = c->allow_regrow ? std::min<u64>(cap, max_capacity(c)) : fixed_capacity(c);
  if (cap < (u64)n) return fail(c, SWCS_E_CAPACITY, "state exceeds the maximum capacity");
  int r;
  if (!c->keys.p || c->st.cap != cap) {
    r = state_reserve(c, cap, 0);
    if (r) return r;
  } else {
    HIP_TRY(c, launch_hash_clear(c->st.hash, c->st.hmask + 1, c->stream), "hash clear");
  }
  if (n > 0) {
    HIP_TRY(c, hipMemcpyAsync(c->keys.p, keys, n * sizeof(u64), hipMemcpyHostToDevice, c->stream), "copy keys");
    HIP_TRY(c, hipMemcpyAsync(c->amps.p, amps, n * sizeof(double), hipMemcpyHostToDevice, c->stream), "copy amps");
  }
  Counters h;
  std::memset(&h, 0, sizeof(h));
  h.n = (u64)n;
  h.alive = (u64)n;
  HIP_TRY(c, launch_store_counters(c->st.ctr, h, c->stream), "counters");
  if (n > 0) HIP_TRY(c, launch_hash_build(c->st, (u64)n, c->stream), "hash build");
  r = build_filter(c, (u64)n, (u64)n);
  if (r) return r;
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  c->hc = h;
  c->hc_valid = true;
  c->peak_n = std::max<u64>(c->peak_n, (u64)n);
  c->have_state = true;
  c->ansatz_valid = false;
  return SWCS_OK;
}

// Export (key, vals[i]) of the alive entries sorted by key; vals = amps if NULL.
static int export_sorted(swcs_ctx* c, u64 n, u64 alive, const double* vals, uint64_t* keys,
                         double* out) {
  HIP_TRY(c, c->exp_keys.ensure(n * 8), "alloc");
  HIP_TRY(c, c->exp_amps.ensure(n * 8), "alloc");
  HIP_TRY(c, c->exp_tmp_k.ensure(n * 8), "alloc");
  HIP_TRY(c, c->exp_tmp_v.ensure(n * 8), "alloc");
  const u64 scr = std::max(radix_sort_scratch_elems(n), compact_scratch_elems(n));
  HIP_TRY(c, c->sort_scratch.ensure(scr * 8), "alloc");
  HIP_TRY(c, launch_compact_alive(c->st, n, vals, c->exp_keys.as<u64>(), c->exp_amps.as<double>(),
                                  c->scalars.as<u64>() + 8, c->sort_scratch.as<u64>(), scr, c->stream), "compact");
  HIP_TRY(c, radix_sort_pairs(c->exp_keys.as<u64>(), c->exp_amps.as<u64>(), c->exp_tmp_k.as<u64>(),
                              c->exp_tmp_v.as<u64>(), alive, c->nso, c->sort_scratch.as<u64>(), scr,
                              c->stream), "sort");
  HIP_TRY(c, hipMemcpyAsync(keys, c->exp_keys.p, alive * 8, hipMemcpyDeviceToHost, c->stream), "copy");
  HIP_TRY(c, hipMemcpyAsync(out, c->exp_amps.p, alive * 8, hipMemcpyDeviceToHost, c->stream), "copy");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  return SWCS_OK;
}

int swcs_get_state(swcs_ctx* c, uint64_t* keys, double* amps, int64_t cap, int64_t* n_out) {
  if (!c) return SWCS_E_INVALID;
  if (!c->have_state) return fail(c, SWCS_E_STATE, "no current state");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  hipError_t e;
  Counters h = get_counters(c, &e);
  if (e != hipSuccess) return hip_fail(c, e, "read counters");
  if (n_out) *n_out = (int64_t)h.alive;
  if ((int64_t)h.alive > cap) return fail(c, SWCS_E_INVALID, "output capacity too small");
  if (h.alive == 0) return SWCS_OK;
  if (!keys || !amps) return fail(c, SWCS_E_INVALID, "null output arrays");
  return export_sorted(c, h.n, h.alive, nullptr, keys, amps);
}

// Enumeration probes every connection of every alive entry (alive * C
// probes); hole-pair grouping sorts n * C(N_e, 2) records instead.  The
// automatic choice takes grouping once the probe count passes this bound.
constexpr double kHolePairProbes = 3.0e7;

static bool use_holepair(swcs_ctx* c, u64 alive) {
  const int ne = c->na + c->nb;
  if (ne < 2 || c->sigma_method == SWCS_SIGMA_ENUMERATE) return false;
  if (c->sigma_method == SWCS_SIGMA_HOLE_PAIRS) return true;
  return (double)alive * (double)c->exc.total > kHolePairProbes;
}

// Small states: every pair of stored determinants is tested in LDS.  The
// automatic choice takes it when the pair count is at most 8 probes' worth
// of enumeration per determinant.
static bool use_sigma_pairs(swcs_ctx* c, u64 n) {
  if (n == 0 || n > (u64)pairwise_capacity()) return false;
  if (c->sigma_method == SWCS_SIGMA_PAIRS) return true;
  if (c->sigma_method != SWCS_SIGMA_AUTO) return false;
  return (double)n <= 8.0 * (double)c->exc.total;
}

// Diagonal elements of the n stored entries into c->diag (stream-ordered),
// unless already computed for the current state.
static int diag_enqueue(swcs_ctx* c, u64 n) {
  if (c->diag_version == c->state_version && c->diag.bytes >= n * 8 && c->st.diag == c->diag.p)
    return SWCS_OK;
  HIP_TRY(c, c->diag.ensure(std::max<u64>(1, n) * 8), "alloc diagonal");
  c->st.diag = c->diag.as<double>();
  HIP_TRY(c, launch_diag(c->st, ints_view(c), n, grid_blocks(c, n * kDiagLanes, 256), c->stream), "diagonal");
  c->diag_version = c->state_version;
  return SWCS_OK;
}

// sigma_P over the stored entries; (numer, norm2) land in scalars[0..1] on
// the device, without synchronizing.
static int energy_enqueue(swcs_ctx* c, u64 n) {
  const int grid = sigma_grid(c, n);
  int rd = diag_enqueue(c, n);
  if (rd) return rd;
  HIP_TRY(c, c->sigma.ensure(std::max<u64>(1, n) * 8), "alloc sigma");
  HIP_TRY(c, c->partial.ensure((size_t)2 * grid * 8), "alloc partial");
  hipError_t e;
  const Counters h = get_counters(c, &e);
  if (e != hipSuccess) return hip_fail(c, e, "read counters");
  if (use_sigma_pairs(c, n)) {
    const int pgrid = (int)std::min<u64>((n + 3) / 4, (u64)c->num_cu * 8);
    HIP_TRY(c, c->partial.ensure((size_t)2 * pgrid * 8), "alloc partial");
    TIMED(c, SWCS_K_SIGMA_PROJ, launch_sigma_pairwise(c->st, ints_view(c), n, c->sigma.as<double>(),
                                 c->partial.as<double>(), pgrid, c->stream), "sigma pairs");
    HIP_TRY(c, launch_reduce_partials(c->partial.as<double>(), pgrid, pgrid, 2, c->scalars.as<double>(), c->stream), "reduce");
    return SWCS_OK;
  }
  if (n > 0 && n < (1ULL << 32) && use_holepair(c, h.alive)) {
    const int ne = c->na + c->nb;
    const u64 total = n * ((u64)ne * (u64)(ne - 1) / 2);
    // Segments of the three removal classes (alpha-alpha, alpha-beta,
    // beta-beta), each sorted on its own on the key bits of the largest
    // class; the dead marker's low bits are all ones, above every key.
    const u64 na = (u64)c->na, nb = (u64)c->nb;
    const u64 seg_len[3] = {n * (na * (na - 1) / 2), n * na * nb, n * (nb * (nb - 1) / 2)};
    u64 cmax = 1;
    if (na >= 2) cmax = std::max(cmax, binomial_u64(c->n, c->na - 2) * binomial_u64(c->n, c->nb));
    if (na >= 1 && nb >= 1) cmax = std::max(cmax, binomial_u64(c->n, c->na - 1) * binomial_u64(c->n, c->nb - 1));
    if (nb >= 2) cmax = std::max(cmax, binomial_u64(c->n, c->na) * binomial_u64(c->n, c->nb - 2));
    int rank_bits = 1;
    while (rank_bits < 60 && (cmax >> rank_bits) != 0) ++rank_bits;
    // Records are single words when key and entry index fit: the key in the
    // low bytes that the radix passes read (rank_bits rounded up to whole
    // digits, so no pass sees index bits), the index above.  Otherwise a
    // 64-bit key plus a 32-bit index.
    int idx_bits = 1;
    while (idx_bits < 63 && ((n - 1) >> idx_bits) != 0) ++idx_bits;
    const int digit_bits = (rank_bits + 7) / 8 * 8;
    const int shift = (digit_bits + idx_bits <= 64) ? digit_bits : 0;
    HIP_TRY(c, c->hp_key.ensure(total * 8), "alloc hole-pair keys");
    HIP_TRY(c, c->hp_tk.ensure(total * 8), "alloc hole-pair keys");
    if (!shift) {
      HIP_TRY(c, c->hp_val.ensure(total * 4), "alloc hole-pair values");
      HIP_TRY(c, c->hp_tv.ensure(total * 4), "alloc hole-pair values");
    }
    // the segments are sorted one by one; a short segment uses small tiles
    // and can need more scratch than a longer one
    u64 scr = 0;
    for (u64 len : seg_len) scr = std::max(scr, radix_sort_scratch_elems(len));
    HIP_TRY(c, c->sort_scratch.ensure(scr * 8), "alloc sort scratch");
    u64* key = c->hp_key.as<u64>();
    u64* tkey = c->hp_tk.as<u64>();
    unsigned* val = shift ? nullptr : c->hp_val.as<unsigned>();
    unsigned* tval = shift ? nullptr : c->hp_tv.as<unsigned>();
    HIP_TRY(c, launch_holepair_emit(c->st, n, c->n, c->na, c->nb, shift, key, val, grid_blocks(c, n * 64, 256),
                                    c->stream), "emit");
    // every segment of two or more records ends in the same buffers (same
    // pass count); a single record stays put and is copied if needed
    const bool in_tmp = ((rank_bits + 7) / 8) % 2 == 1;
    u64 off = 0;
    for (int sgm = 0; sgm < 3; ++sgm) {
      const u64 len = seg_len[sgm];
      if (len >= 2) {
        u64* ok = nullptr;  // where the last pass left the segment (not copied back)
        if (shift) {
          HIP_TRY(c, radix_sort_keys(key + off, tkey + off, len, shift, c->sort_scratch.as<u64>(), scr,
                                     c->stream, &ok), "sort");
        } else {
          unsigned* ov = nullptr;
          HIP_TRY(c, radix_sort_pairs32(key + off, val + off, tkey + off, tval + off, len, rank_bits,
                                        c->sort_scratch.as<u64>(), scr, c->stream, &ok, &ov), "sort");
        }
        if (ok != (in_tmp ? tkey + off : key + off)) return fail(c, SWCS_E_DEVICE, "sort parity");
      } else if (len == 1 && in_tmp) {
        HIP_TRY(c, hipMemcpyAsync(tkey + off, key + off, 8, hipMemcpyDeviceToDevice, c->stream), "copy");
        if (!shift) HIP_TRY(c, hipMemcpyAsync(tval + off, val + off, 4, hipMemcpyDeviceToDevice, c->stream), "copy");
      }
      off += len;
    }
    u64* sk = in_tmp ? tkey : key;
    unsigned* sv = shift ? nullptr : (in_tmp ? tval : val);
    HIP_TRY(c, launch_sigma_diag(c->st, ints_view(c), n, c->sigma.as<double>(), grid_blocks(c, n, 256),
                                 c->stream), "diagonal sigma");
    off = 0;
    for (int sgm = 0; sgm < 3; ++sgm) {
      const u64 len = seg_len[sgm];
      TIMED(c, SWCS_K_HOLEPAIR, launch_holepair_sigma(c->st, ints_view(c), c->na, n, sk + off, sv ? sv + off : nullptr,
                                                      shift, len, sgm, c->sigma.as<double>(),
                                                      grid_blocks(c, len, 256), c->stream), "hole pairs");
      off += len;
    }
    HIP_TRY(c, launch_sigma_dots(c->st, c->sigma.as<double>(), n, c->partial.as<double>(), grid, c->stream), "dots");
  } else {
    TIMED(c, SWCS_K_SIGMA_PROJ, launch_sigma_proj(c->st, ints_view(c), c->exc, n, c->sigma.as<double>(),
                                 c->partial.as<double>(), nullptr, grid, c->stream), "sigma");
  }
  HIP_TRY(c, launch_reduce_partials(c->partial.as<double>(), grid, grid, 2, c->scalars.as<double>(), c->stream), "reduce");
  return SWCS_OK;
}

// Same, returning numer and norm2 on the host.
static int energy_internal(swcs_ctx* c, u64 n, double* numer, double* norm2) {
  int r = energy_enqueue(c, n);
  if (r) return r;
  double out[2];
  HIP_TRY(c, hipMemcpyAsync(out, c->scalars.p, 16, hipMemcpyDeviceToHost, c->stream), "copy");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  *numer = out[0];
  *norm2 = out[1];
  return SWCS_OK;
}

int swcs_energy(swcs_ctx* c, double* E, double* numer, double* norm2) {
  if (!c) return SWCS_E_INVALID;
  if (!c->have_ints) return fail(c, SWCS_E_STATE, "integrals not set");
  if (!c->have_state) return fail(c, SWCS_E_STATE, "no current state");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  hipError_t e;
  Counters h = get_counters(c, &e);
  if (e != hipSuccess) return hip_fail(c, e, "read counters");
  double nu = 0.0, no = 0.0;
  int r = energy_internal(c, h.n, &nu, &no);
  if (r) return r;
  if (numer) *numer = nu;
  if (norm2) *norm2 = no;
  if (E) *E = nu / no;
  return SWCS_OK;
}

int swcs_energy_noalloc(swcs_ctx* c, double* E, double* numer, double* norm2) {
  if (!c) return SWCS_E_INVALID;
  if (!c->have_ints) return fail(c, SWCS_E_STATE, "integrals not set");
  if (!c->have_state) return fail(c, SWCS_E_STATE, "no current state");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  hipError_t e;
  const Counters h = get_counters(c, &e);
  if (e != hipSuccess) return hip_fail(c, e, "read counters");
  const u64 n = h.n;
  if (n > kNoAllocMaxEntries)
    return fail(c, SWCS_E_CAPACITY, "state has " + std::to_string(n) + " stored entries; the allocation-free "
                                     "energy takes at most " + std::to_string(kNoAllocMaxEntries));
  double* base = nullptr;
  HIP_TRY(c, noalloc_scratch(c->device, &base), "scratch address");
  double* partial = base;
  double* res = base + kNoAllocPartials;
  DeviceState st = c->st;
  st.diag = base + kNoAllocHead;
  double* sig = st.diag + n;
  const Ints I = ints_view(c);
  if (n > 0) {
    HIP_TRY(c, launch_diag(st, I, n, grid_blocks(c, n * kDiagLanes, 256), c->stream), "diagonal");
    if (n <= (u64)pairwise_capacity()) {
      const int pgrid = (int)std::min<u64>((n + 3) / 4, kNoAllocPartials / 2);
      HIP_TRY(c, launch_sigma_pairwise(st, I, n, sig, partial, pgrid, c->stream), "sigma pairs");
      HIP_TRY(c, launch_reduce_partials(partial, pgrid, pgrid, 2, res, c->stream), "reduce");
    } else {
      const int grid = std::min<int>(sigma_grid(c, n), (int)(kNoAllocPartials / 2));
      HIP_TRY(c, launch_sigma_proj(st, I, c->exc, n, sig, partial, nullptr, grid, c->stream), "sigma");
      HIP_TRY(c, launch_reduce_partials(partial, grid, grid, 2, res, c->stream), "reduce");
    }
  } else {
    HIP_TRY(c, launch_fill_u32(res, 0u, 4, c->stream), "zero");
  }
  double out[2];
  HIP_TRY(c, hipMemcpyAsync(out, res, 16, hipMemcpyDeviceToHost, c->stream), "copy");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  if (numer) *numer = out[0];
  if (norm2) *norm2 = out[1];
  if (E) *E = out[0] / out[1];
  return SWCS_OK;
}

int swcs_sigma_projected(swcs_ctx* c, uint64_t* keys, double* sigma, int64_t cap, int64_t* n_out) {
  if (!c) return SWCS_E_INVALID;
  if (!c->have_ints) return fail(c, SWCS_E_STATE, "integrals not set");
  if (!c->have_state) return fail(c, SWCS_E_STATE, "no current state");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  hipError_t e;
  Counters h = get_counters(c, &e);
  if (e != hipSuccess) return hip_fail(c, e, "read counters");
  if (n_out) *n_out = (int64_t)h.alive;
  if ((int64_t)h.alive > cap) return fail(c, SWCS_E_INVALID, "output capacity too small");
  if (h.alive == 0) return SWCS_OK;
  if (!keys || !sigma) return fail(c, SWCS_E_INVALID, "null output arrays");
  double nu, no;
  int r = energy_internal(c, h.n, &nu, &no);
  if (r) return r;
  return export_sorted(c, h.n, h.alive, c->sigma.as<double>(), keys, sigma);
}

// <psi|psi> into scalars[2] on the device, without synchronizing (kept while
// the state is unchanged).
static int norm2_enqueue(swcs_ctx* c, u64 n) {
  if (c->norm_version == c->state_version) return SWCS_OK;
  const int grid = grid_blocks(c, n, 256);
  HIP_TRY(c, c->partial.ensure((size_t)grid * 8 * 2), "alloc partial");
  HIP_TRY(c, launch_occupations(c->st, n, 0, c->partial.as<double>(), grid, c->stream), "norm");
  HIP_TRY(c, launch_reduce_partials(c->partial.as<double>(), grid, grid, 1, c->scalars.as<double>() + 2, c->stream), "reduce");
  c->norm_version = c->state_version;
  return SWCS_OK;
}

// The screened query table is sized from a bound on its key count (no host
// round trip) when that table stays below this size and no table budget is
// set, otherwise from an exact count.
constexpr double kQueryBoundBytes = 512.0 * 1024 * 1024;

// Screened pool gradients of the n_subset operators d_subset (valid device
// indices) into d_out (device, n_subset doubles): sigma only on the
// determinants the selected operators reach.  Small subsets are walked
// operator-major (|psi| x n_subset activity tests), larger ones
// determinant-major through the generator table.  Synchronizes only when the
// query table has to be sized by an exact count.
static int mark_subset(swcs_ctx* c, const int* d_subset, int64_t n_subset);

static int screened_gradients(swcs_ctx* c, u64 n, u64 alive, const int* d_subset, int64_t n_subset,
                              const double* norm2, double* d_out, bool may_sync) {
  // a state too large for the join makes its scratch dead weight
  if (!join_fits_state(c, alive)) release_join_scratch(c);
  const bool op_major = n_subset <= c->exc.total;
  const unsigned char* d_sel = nullptr;
  if (!op_major) {
    // the determinant-major passes test the operator flags and accumulate
    // into the pool-wide g
    int r = mark_subset(c, d_subset, n_subset);
    if (r) return r;
    d_sel = c->selected.as<unsigned char>();
  }
  const double bound = std::min<double>((double)c->sector,
                                        (double)alive * (double)(op_major ? n_subset : c->exc.total));
  u64 nq;
  bool counted = false, sampled = false;
  if (c->table_budget == 0 && 2.0 * bound * sizeof(AccSlot) <= kQueryBoundBytes) {
    nq = (u64)bound;
  } else {
    // count the (determinant, operator) pairs, on every 16th determinant
    // (or tile) of a state of 16,384 stored entries or more: the scaled
    // sample sizes the table, and a pass whose table fills is repeated with
    // twice the estimate (a full count costs as much as the insert pass)
    counted = true;
    const int stride = n >= 16384 ? 16 : 1;
    sampled = stride > 1;
    u64* qcount = c->scalars.as<u64>() + 16;
    HIP_TRY(c, launch_fill_u32(qcount, 0u, 2, c->stream), "zero counter");
    if (op_major)
      HIP_TRY(c, launch_query_ops(c->st, n, c->ops.as<OpDesc>(), d_subset, n_subset, nullptr, 0, stride,
                                  qcount, c->stream), "count");
    else
      HIP_TRY(c, launch_query_set(c->st, c->exc, c->n, n, c->opmap.as<int>(), c->n, d_sel,
                                  nullptr, 0, stride, qcount, sigma_grid(c, n), c->stream), "count");
    HIP_TRY(c, hipMemcpyAsync(&nq, qcount, 8, hipMemcpyDeviceToHost, c->stream), "copy");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
    if (sampled) nq = (u64)(1.25 * (double)nq * stride) + 4096;
  }
  // The query keys number at most q; a table for all of them that would
  // not fit in 40% of the free device memory is split by key hash into
  // batches, each a full query / push / contract pass over its own keys.
  // Counted pairs repeat keys many times over: the query keys are external
  // determinants, so the distinct external count of the last full-pool call
  // (scaled by the alive count) caps the estimate, and a pass that
  // overflows is repeated with twice the estimate.
  double q = (double)std::min<u64>(nq, c->sector);
  bool estimated = sampled;
  if (counted && c->ext_count > 0.0 && c->ext_alive > 0.0) {
    const double est = 1.5 * c->ext_count * std::max(1.0, (double)alive / c->ext_alive);
    if (est < q) {
      q = est;
      estimated = true;
    }
  }
  double budget = (double)c->table_budget;
  auto slots_for = [&](int nb) { return next_pow2((u64)std::max(64.0, (nb > 1 ? 2.5 : 2.0) * q / nb)); };
  auto batches = [&]() {
    int nb = 1;
    if (budget <= 0.0 && (double)slots_for(1) * sizeof(AccSlot) <= kQueryBoundBytes) return nb;
    if (budget <= 0.0) budget = free_table_budget(c, (double)slots_for(1) * sizeof(AccSlot));
    while (nb < 4096 && (double)slots_for(nb) * sizeof(AccSlot) > budget) nb *= 2;
    return nb;
  };
  int nbatch = batches();
  bool checked = false, replanned = false;
  int passes = 0;
  for (int attempt = 0;;) {
    const u64 qslots = slots_for(nbatch);
    HIP_TRY(c, c->acc_tab.ensure(qslots * sizeof(AccSlot)), "alloc sigma table");
    // presence filter of the batch's query keys: 8 bits per table slot (1/16
    // of the table's bytes), at least 4,096 bits and at most 2^30 (128 MB,
    // so that it stays in the last-level cache)
    const u64 qbits = std::min<u64>((u64)1 << 30, next_pow2(std::max<u64>(4096, 8 * qslots)));
    HIP_TRY(c, c->qfilt.ensure(qbits / 8), "alloc query filter");
    unsigned* qf = c->qfilt.as<unsigned>();
    ++passes;
    if (op_major)
      HIP_TRY(c, launch_fill_u32(d_out, 0u, (u64)n_subset * 2, c->stream), "zero g");
    else
      HIP_TRY(c, launch_fill_u32(c->gacc.p, 0u, (u64)c->K_pool * 2, c->stream), "zero g");
    bool replan = false;
    for (int b = 0; b < nbatch; ++b) {
      HIP_TRY(c, launch_fill_u32(c->acc_tab.p, 0u, qslots * (sizeof(AccSlot) / 4), c->stream), "clear table");
      HIP_TRY(c, launch_fill_u32(qf, 0u, qbits / 32, c->stream), "clear filter");
      // The estimate that set the batch count is an upper bound (pairs, or
      // the distinct count of all external keys); the first batch of a
      // batched pass counts its new keys, and since key-hash batches split
      // the query set evenly, a set much smaller than planned restarts the
      // pass with fewer batches (only this batch's query pass is lost).
      u64* qnew = (b == 0 && nbatch > 1 && estimated && !replanned) ? c->scalars.as<u64>() + 40 : nullptr;
      if (qnew) HIP_TRY(c, launch_fill_u32(qnew, 0u, 2, c->stream), "zero counter");
      if (op_major)
        HIP_TRY(c, launch_query_ops(c->st, n, c->ops.as<OpDesc>(), d_subset, n_subset,
                                    c->acc_tab.as<AccSlot>(), qslots - 1, 0, qnew, c->stream, nbatch, b,
                                    qf, qbits - 1), "query set");
      else
        HIP_TRY(c, launch_query_set(c->st, c->exc, c->n, n, c->opmap.as<int>(), c->n, d_sel,
                                    c->acc_tab.as<AccSlot>(), qslots - 1, 0, qnew, sigma_grid(c, n),
                                    c->stream, nbatch, b, qf, qbits - 1), "query set");
      if (qnew) {
        replanned = true;
        u64 got = 0;
        HIP_TRY(c, hipMemcpyAsync(&got, qnew, 8, hipMemcpyDeviceToHost, c->stream), "copy");
        HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
        const double q_new = std::max(64.0, 1.25 * (double)got * nbatch);
        if (q_new < 0.5 * q) {
          const double q_old = q;
          q = q_new;
          const int nb_new = batches();
          if (nb_new < nbatch) {
            nbatch = nb_new;
            replan = true;
            break;
          }
          q = q_old;
        }
      }
      TIMED(c, SWCS_K_SIGMA_PUSH_INTO, launch_sigma_push_into(c->st, ints_view(c), c->exc, n, c->acc_tab.as<AccSlot>(),
                                                              qslots - 1, sigma_grid(c, n), c->stream, nbatch, b,
                                                              qf, qbits - 1),
            "sigma push");
      if (op_major)
        TIMED(c, SWCS_K_CONTRACT_OPS, launch_contract_ops(c->st, n, c->ops.as<OpDesc>(), d_subset, n_subset,
                                                          c->acc_tab.as<AccSlot>(), qslots - 1, d_out, c->stream,
                                                          nbatch, b), "contract");
      else
        TIMED(c, SWCS_K_POOL_CONTRACT, launch_pool_contract_det(c->st, c->exc, c->n, n, c->opmap.as<int>(), c->n,
                                                                d_sel, c->acc_tab.as<AccSlot>(), qslots - 1, nbatch, b,
                                                                c->gacc.as<double>(), sigma_grid(c, n), c->stream),
              "contract");
    }
    if (replan) continue;
    // A single bound-sized table (at most half full) is checked on the
    // device when the caller does not synchronize (below); otherwise a pass
    // in which a table filled is repeated with twice the estimate.
    if (!may_sync && nbatch == 1 && !estimated) break;
    checked = true;
    hipError_t e;
    Counters h2 = read_counters(c, &e);  // synchronizes
    if (e != hipSuccess) return hip_fail(c, e, "read counters");
    if (!(h2.flags & kFlagOverflow)) break;
    h2.flags &= ~kFlagOverflow;
    HIP_TRY(c, launch_store_counters(c->st.ctr, h2, c->stream), "counters");
    c->hc = h2;
    if (++attempt > 16) return fail(c, SWCS_E_DEVICE, "sigma table overflow");
    q *= 2.0;
    nbatch = batches();
  }
  c->ps_keys = q;
  c->ps_slots = slots_for(nbatch);
  c->ps_batches = nbatch;
  c->ps_passes = passes;
  c->ps_screened = 1;
  if (op_major)
    HIP_TRY(c, launch_gather_scaled(d_out, nullptr, n_subset, norm2, d_out, c->stream), "scale");
  else
    HIP_TRY(c, launch_gather_scaled(c->gacc.as<double>(), d_subset, n_subset, norm2, d_out, c->stream), "gather");
  if (!checked) {
    // unchecked pass: a table that filled turns every result into NaN, and
    // the flag is cleared for later calls
    HIP_TRY(c, launch_nan_if_flag(c->st.ctr, kFlagOverflow, d_out, n_subset, c->stream), "overflow check");
    HIP_TRY(c, launch_clear_flag(c->st.ctr, kFlagOverflow, c->stream), "overflow clear");
  }
  return SWCS_OK;
}

// Shared set-up of both pool-gradient entry points: counters, norm, diagonal
// elements and the pool-wide accumulator's allocation.
static int pool_setup(swcs_ctx* c, Counters* h) {
  int r = check_ready(c);
  if (r) return r;
  if (!c->have_state) return fail(c, SWCS_E_STATE, "no current state");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  hipError_t e;
  *h = get_counters(c, &e);
  if (e != hipSuccess) return hip_fail(c, e, "read counters");
  if (h->alive == 0) return fail(c, SWCS_E_STATE, "state is empty");
  r = norm2_enqueue(c, h->n);
  if (r) return r;
  r = diag_enqueue(c, h->n);
  if (r) return r;
  HIP_TRY(c, c->gacc.ensure((size_t)c->K_pool * 8), "alloc g accumulator");
  return SWCS_OK;
}

static int mark_subset(swcs_ctx* c, const int* d_subset, int64_t n_subset) {
  const u64 words = ((u64)c->K_pool + 3) / 4;
  HIP_TRY(c, c->selected.ensure(words * 4), "alloc selection");
  HIP_TRY(c, launch_fill_u32(c->selected.p, 0u, words, c->stream), "zero selection");
  HIP_TRY(c, launch_mark_selected(d_subset, n_subset, c->selected.as<unsigned char>(), c->stream), "mark");
  return SWCS_OK;
}

int swcs_pool_gradients_device(swcs_ctx* c, const int32_t* d_subset, int64_t n_subset, double* d_g) {
  if (!c) return SWCS_E_INVALID;
  if (n_subset < 0) return fail(c, SWCS_E_INVALID, "n_subset < 0");
  if (n_subset > 0 && (!d_subset || !d_g)) return fail(c, SWCS_E_INVALID, "null device pointer");
  if (n_subset == 0) return SWCS_OK;
  Counters h;
  int r = pool_setup(c, &h);
  if (r) return r;
  HIP_TRY(c, c->subset_buf.ensure((size_t)n_subset * 4), "alloc subset");
  HIP_TRY(c, launch_sanitize_subset(d_subset, n_subset, c->K_pool, c->subset_buf.as<int>(), c->stream), "subset");
  const int* sub = c->subset_buf.as<int>();
  const double* norm2 = c->scalars.as<double>() + 2;
  r = screened_gradients(c, h.n, h.alive, sub, n_subset, norm2, d_g, false);
  if (r) return r;
  HIP_TRY(c, launch_nan_invalid(d_subset, n_subset, c->K_pool, d_g, c->stream), "flag invalid");
  return SWCS_OK;
}

// Full-pool (or large-subset) gradients by sort and join (k_join.hip).
// Returns 1 when the join does not apply (method, memory, record word) or a
// join step overflowed its LDS table and AUTO may fall back to the table,
// else an SWCS status; on SWCS_OK the scaled gradients are in gbuf.
static int join_gradients(swcs_ctx* c, const Counters& h, const unsigned char* d_sel, const int* d_subset,
                          int64_t count, const double* norm2) {
  if (c->pool_method == SWCS_POOL_TABLE) return 1;
  if (c->pool_method == SWCS_POOL_AUTO && c->table_budget > 0) return 1;
  const bool forced = c->pool_method == SWCS_POOL_JOIN;
  const u64 n = h.n, C = (u64)c->exc.total;
  const u64 R = h.alive * (C + 1);
  // Measured at 52 spin-orbitals: 1.54e9 records take 120 ms by the join
  // against 187 ms by the table, but 7.9e9 records (266,101 determinants)
  // take 1.9 s, where the table needs about 1 s: beyond 2^31 records AUTO
  // takes the table (and gives back the join's scratch, which a state of
  // this size leaves unused).
  if (!join_fits_state(c, h.alive)) {
    release_join_scratch(c);
    return 1;
  }
  int kb, bh, bp, orb;
  if (!join_format(c->exc, n, R, &kb, &bh, &bp, &orb)) {
    if (forced) return fail(c, SWCS_E_CAPACITY, "join records do not fit 64 bits");
    return 1;
  }
  const u64 scr = radix_sort_scratch_elems(R);
  const u64 list_bytes = n * 16;  // (key, psi) of every stored entry
  const double need = 16.0 * (double)R + 8.0 * (double)scr + (double)list_bytes;
  const double have = (double)(avail_bytes(c) + c->hp_key.bytes + c->hp_tk.bytes + c->sort_scratch.bytes +
                               c->join_src.bytes + c->join_w.bytes + c->join_j.bytes);
  if (need > 0.5 * have) {
    if (forced) return fail(c, SWCS_E_CAPACITY, "join records exceed half of the free device memory");
    return 1;
  }
  // Gradient terms by operator bin (2^lb bins of at most kJoinTermSlots
  // operators, k mod 2^lb), each with room for 1.25 times an even share of
  // the records: the device-scope adds into g[K] then number about 8192 per
  // bin and chunk instead of one per record.  Terms past a full bin, and
  // every term when the bins do not fit, take the direct adds.
  JoinTerms terms{-1, 0, nullptr, nullptr, nullptr};
  {
    int lb = 0;
    while (lb <= kJoinMaxBinsLog && (u64)c->K_pool > ((u64)kJoinTermSlots << lb)) ++lb;
    const u64 cap = ((u64)(1.25 * (double)R / (double)(1ULL << lb)) + 4096 + 7) & ~7ULL;
    const double bin_bytes = 10.0 * (double)cap * (double)(1ULL << lb);
    if (lb <= kJoinMaxBinsLog && need + bin_bytes <= 0.5 * have) {
      HIP_TRY(c, c->join_w.ensure((size_t)(cap << lb) * 8), "alloc join terms");
      HIP_TRY(c, c->join_j.ensure((size_t)(cap << lb) * 2), "alloc join terms");
      HIP_TRY(c, c->join_bins.ensure((size_t)8 << lb), "alloc join bins");
      HIP_TRY(c, launch_fill_u32(c->join_bins.p, 0u, (u64)2 << lb, c->stream), "zero bins");
      terms = JoinTerms{lb, cap, c->join_bins.as<u64>(), c->join_w.as<double>(), c->join_j.as<unsigned short>()};
    }
  }
  HIP_TRY(c, c->hp_key.ensure(R * 8), "alloc join records");
  HIP_TRY(c, c->hp_tk.ensure(R * 8), "alloc join records");
  HIP_TRY(c, c->sort_scratch.ensure(scr * 8), "alloc sort scratch");
  HIP_TRY(c, c->join_src.ensure(std::max<u64>(16, list_bytes)), "alloc join sources");
  const int rgrid = (int)std::min<u64>((R + kJoinRunHost - 1) / kJoinRunHost, (u64)c->num_cu * 8);
  HIP_TRY(c, c->partial2.ensure((size_t)std::max(rgrid, 1) * 8), "alloc partials");
  u64* cursor = c->scalars.as<u64>() + 32;
  HIP_TRY(c, launch_fill_u32(cursor, 0u, 2, c->stream), "zero cursor");
  u64* recs = c->hp_key.as<u64>();
  TIMED(c, SWCS_K_JOIN_EMIT, launch_join_emit(c->st, c->exc, n, recs, R, cursor, kb, bh, bp, orb,
                                                c->join_src.p, sigma_grid(c, n), c->stream),
        "join emit");
  u64* sorted = recs;
  TIMED(c, SWCS_K_JOIN_SORT, radix_sort_keys(recs, c->hp_tk.as<u64>(), R, kb, c->sort_scratch.as<u64>(), scr,
                                             c->stream, &sorted), "join sort");
  HIP_TRY(c, launch_fill_u32(c->gacc.p, 0u, (u64)c->K_pool * 2, c->stream), "zero g");
  double* ins = c->partial2.as<double>();
  TIMED(c, SWCS_K_JOIN_REDUCE, launch_join_reduce(c->st, sorted, R, cursor, kb, bh, bp, orb, c->join_src.p, n,
                                                  ints_view(c), c->exc, c->opmap.as<int>(),
                                                  c->n, d_sel, c->gacc.as<double>(), terms, ins, rgrid,
                                                  c->stream),
        "join reduce");
  TIMED(c, SWCS_K_JOIN_TERMS, launch_join_terms(terms, c->gacc.as<double>(), c->K_pool, c->stream), "join terms");
  HIP_TRY(c, launch_reduce_partials(ins, rgrid, rgrid, 1, c->scalars.as<double>() + 24, c->stream), "count");
  double distinct = 0.0;
  HIP_TRY(c, hipMemcpyAsync(&distinct, c->scalars.as<double>() + 24, 8, hipMemcpyDeviceToHost, c->stream), "copy");
  HIP_TRY(c, launch_gather_scaled(c->gacc.as<double>(), d_subset, count, norm2, c->gbuf.as<double>(), c->stream),
          "gather");
  hipError_t e;
  Counters h2 = read_counters(c, &e);  // synchronizes
  if (e != hipSuccess) return hip_fail(c, e, "read counters");
  if (h2.flags & kFlagOverflow) {
    h2.flags &= ~kFlagOverflow;
    HIP_TRY(c, launch_store_counters(c->st.ctr, h2, c->stream), "counters");
    c->hc = h2;
    if (forced) return fail(c, SWCS_E_DEVICE, "join group overflowed its LDS table");
    return 1;
  }
  c->ext_count = distinct;
  c->ext_alive = (double)h.alive;
  c->ps_keys = distinct;
  c->ps_slots = 0;
  c->ps_batches = 1;
  c->ps_passes = 1;
  c->ps_screened = 0;
  return SWCS_OK;
}

int swcs_pool_gradients(swcs_ctx* c, const int32_t* subset, int64_t n_subset, double* g_out) {
  if (!c) return SWCS_E_INVALID;
  if (!g_out) return fail(c, SWCS_E_INVALID, "null g_out");
  const int64_t count = subset ? n_subset : c->K_pool;
  if (subset) {
    if (n_subset < 0) return fail(c, SWCS_E_INVALID, "n_subset < 0");
    for (int64_t t = 0; t < n_subset; ++t)
      if (subset[t] < 0 || subset[t] >= c->K_pool) return fail(c, SWCS_E_INVALID, "subset index out of range");
  }
  int r = check_ready(c);
  if (r) return r;
  if (!c->have_state) return fail(c, SWCS_E_STATE, "no current state");
  if (count == 0) return SWCS_OK;
  Counters h;
  r = pool_setup(c, &h);
  if (r) return r;
  hipError_t e;
  const u64 n = h.n;
  const double* norm2 = c->scalars.as<double>() + 2;
  HIP_TRY(c, c->gbuf.ensure((size_t)count * 8), "alloc g");
  const int* d_subset = nullptr;
  const unsigned char* d_sel = nullptr;
  if (subset) {
    HIP_TRY(c, c->subset_buf.ensure((size_t)n_subset * 4), "alloc subset");
    HIP_TRY(c, hipMemcpyAsync(c->subset_buf.p, subset, (size_t)n_subset * 4, hipMemcpyHostToDevice, c->stream), "copy subset");
    // the host array is pageable: wait for the copy before the kernels that
    // read it are enqueued
    HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
    d_subset = c->subset_buf.as<int>();
  }
  if (subset && 2 * n_subset < c->K_pool) {
    r = screened_gradients(c, n, h.alive, d_subset, n_subset, norm2, c->gbuf.as<double>(), true);
    if (r) return r;
    HIP_TRY(c, hipMemcpyAsync(g_out, c->gbuf.p, (size_t)count * 8, hipMemcpyDeviceToHost, c->stream), "copy g");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
    return SWCS_OK;
  }
  if (subset) {
    r = mark_subset(c, d_subset, n_subset);
    if (r) return r;
    d_sel = c->selected.as<unsigned char>();
  }
  r = join_gradients(c, h, d_sel, d_subset, count, norm2);
  if (r <= 0) {
    if (r) return r;
    HIP_TRY(c, hipMemcpyAsync(g_out, c->gbuf.p, (size_t)count * 8, hipMemcpyDeviceToHost, c->stream), "copy g");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
    return SWCS_OK;
  }
  // External-space table.  At most alive * (C + 1) distinct keys (and never
  // more than the sector) can occur, but states built by gate chains overlap
  // heavily, so the table is sized from the distinct-key count of the
  // previous call scaled by the alive count; load factor <= 1/2; split by key
  // hash only when the table would exceed the memory budget.  A table that
  // fills up raises kFlagOverflow and the pass is repeated with twice the
  // estimate.
  const double bound_d = std::min<double>((double)c->sector, (double)h.alive * (double)(c->exc.total + 1));
  double guess = bound_d;
  if (c->ext_count > 0.0 && c->ext_alive > 0.0)
    guess = std::min(bound_d, 1.5 * c->ext_count * std::max(1.0, (double)h.alive / c->ext_alive));
  // Tables up to 256 MB need no free-memory query.
  double budget = 256.0 * 1024 * 1024;
  if (c->table_budget > 0) {
    budget = (double)c->table_budget;
  } else if (4.0 * guess * sizeof(AccSlot) > budget) {
    budget = free_table_budget(c, 4.0 * guess * sizeof(AccSlot));
  }
  const int sgrid = sigma_grid(c, n);
  for (int attempt = 0;; ++attempt) {
    int nbatch = 1;
    while ((2.0 * guess / nbatch) * sizeof(AccSlot) > budget && nbatch < 4096) nbatch *= 2;
    u64 slots = next_pow2((u64)std::max<double>(64.0, 2.0 * guess / nbatch * (nbatch > 1 ? 1.25 : 1.0)));
    // a single table that fits twice over runs at load <= 1/4 (shorter probes)
    if (nbatch == 1 && 2.0 * (double)slots * sizeof(AccSlot) <= budget) slots *= 2;
    HIP_TRY(c, c->acc_tab.ensure(slots * sizeof(AccSlot)), "alloc sigma table");
    HIP_TRY(c, c->partial2.ensure((size_t)sgrid * nbatch * 8), "alloc partials");
    HIP_TRY(c, launch_fill_u32(c->gacc.p, 0u, (u64)c->K_pool * 2, c->stream), "zero g");
    double* ins = c->partial2.as<double>();
    for (int b = 0; b < nbatch; ++b) {
      HIP_TRY(c, launch_fill_u32(c->acc_tab.p, 0u, slots * (sizeof(AccSlot) / 4), c->stream), "clear table");
      TIMED(c, SWCS_K_SIGMA_PUSH, launch_sigma_push(c->st, ints_view(c), c->exc, n, c->acc_tab.as<AccSlot>(), slots - 1,
                                   nbatch, b, ins + (size_t)b * sgrid, sgrid, c->stream), "sigma push");
      TIMED(c, SWCS_K_POOL_CONTRACT, launch_pool_contract_det(c->st, c->exc, c->n, n, c->opmap.as<int>(), c->n,
                                          d_sel, c->acc_tab.as<AccSlot>(), slots - 1, nbatch, b,
                                          c->gacc.as<double>(), sgrid, c->stream), "contract");
    }
    // distinct keys over all batches (the batches partition the keys)
    HIP_TRY(c, launch_reduce_partials(ins, sgrid * nbatch, sgrid * nbatch, 1, c->scalars.as<double>() + 24,
                                      c->stream), "count");
    double distinct = 0.0;
    HIP_TRY(c, hipMemcpyAsync(&distinct, c->scalars.as<double>() + 24, 8, hipMemcpyDeviceToHost, c->stream), "copy");
    HIP_TRY(c, launch_gather_scaled(c->gacc.as<double>(), d_subset, count, norm2, c->gbuf.as<double>(),
                                    c->stream), "gather");
    HIP_TRY(c, hipMemcpyAsync(g_out, c->gbuf.p, (size_t)count * 8, hipMemcpyDeviceToHost, c->stream), "copy g");
    Counters h2 = read_counters(c, &e);  // synchronizes
    if (e != hipSuccess) return hip_fail(c, e, "read counters");
    if (!(h2.flags & kFlagOverflow)) {
      c->ext_count = distinct;
      c->ext_alive = (double)h.alive;
      c->ps_keys = distinct;
      c->ps_slots = slots;
      c->ps_batches = nbatch;
      c->ps_passes = attempt + 1;
      c->ps_screened = 0;
      return SWCS_OK;
    }
    h2.flags &= ~kFlagOverflow;
    HIP_TRY(c, launch_store_counters(c->st.ctr, h2, c->stream), "counters");
    c->hc = h2;
    if (guess >= bound_d || attempt >= 16) return fail(c, SWCS_E_DEVICE, "sigma table overflow");
    guess = std::min(bound_d, 2.0 * guess);
  }
}

int swcs_param_gradients(swcs_ctx* c, double* dE, double* E_out) {
  if (!c) return SWCS_E_INVALID;
  if (!c->ansatz_valid) return fail(c, SWCS_E_STATE, "no ansatz applied from the reference");
  if (!dE && c->a_theta.size() > 0) return fail(c, SWCS_E_INVALID, "null dE_dtheta");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  const int64_t M = (int64_t)c->a_ops.size();  // unitaries (a parameter may drive two)
  const int64_t M_par = (int64_t)c->a_theta.size();
  hipError_t e;
  Counters hfin = get_counters(c, &e);
  if (e != hipSuccess) return hip_fail(c, e, "read counters");
  const u64 n = hfin.n;
  int r;
  if (M == 0) {
    double numer = 0.0, norm2 = 0.0;
    r = energy_internal(c, n, &numer, &norm2);
    if (r) return r;
    if (E_out) *E_out = numer / norm2;
    return SWCS_OK;
  }
  r = energy_enqueue(c, n);
  if (r) return r;
  const double* nn = c->scalars.as<double>();
  const int seg = c->seg;
  const int nseg = (int)((M + seg - 1) / seg);
  const int grid = grid_blocks(c, n, 256);
  HIP_TRY(c, c->mu.ensure(n * 8), "alloc mu");
  HIP_TRY(c, c->gbuf.ensure((size_t)M * 8), "alloc dE");
  const bool lds = !c->a_has_star && n <= (u64)lds_chain_capacity();
  // Pair logs: at most one record per stored entry per gate, for every gate
  // (single-workgroup path, all segments replayed at once) or for one
  // segment at a time (HBM path); with overlapping generators each gate's
  // slot also holds up to one star record per stored entry.
  const size_t gate_log_bytes = n * (sizeof(PairRec) + (c->a_has_star ? sizeof(StarRec) : 0));
  HIP_TRY(c, c->seg_states.ensure((size_t)(lds ? M : seg) * gate_log_bytes), "alloc pair logs");
  PairRec* logs = c->seg_states.as<PairRec>();
  auto plog_of = [&](int t) { return (PairRec*)((char*)c->seg_states.p + (size_t)t * gate_log_bytes); };
  auto slog_of = [&](int t) {
    return (StarRec*)((char*)c->seg_states.p + (size_t)t * gate_log_bytes + n * sizeof(PairRec));
  };
  HIP_TRY(c, launch_mu_init(c->st, c->sigma.as<double>(), n, nn, c->mu.as<double>(), c->stream), "mu init");
  if (lds) {
    // Segments replayed side by side (one workgroup each), then one
    // workgroup walks every gate back with mu in LDS; the gate table of the
    // last apply call is reused.
    int r2 = upload_ckpt_table(c, nseg);
    if (r2) return r2;
    HIP_TRY(c, c->ctr_r.ensure((size_t)M * sizeof(unsigned)), "alloc log counters");
    HIP_TRY(c, c->partial2.ensure(adjoint_lds_part_elems((int)M) * sizeof(double)), "alloc partials");
    TIMED(c, SWCS_K_ADJOINT_REPLAY_LDS, launch_adjoint_replay_lds(c->st.keys, (unsigned)n, c->gate_tab.as<GateDesc>(), (int)M, seg,
                                          c->a_ncut ? 0.0 : c->a_eps, c->ckpt_ptrs.as<double*>(), c->ckpt_n.as<u64>(),
                                          logs, c->ctr_r.as<unsigned>(), &c->st.ctr->flags, (unsigned)c->a_ncut,
                                          c->stream), "adjoint replay");
    TIMED(c, SWCS_K_ADJOINT_LDS, launch_adjoint_reverse_lds((unsigned)n, c->gate_tab.as<GateDesc>(), (int)M, c->mu.as<double>(),
                                  logs, c->ctr_r.as<unsigned>(), c->partial2.as<double>(), c->gbuf.as<double>(),
                                  c->stream), "adjoint");
  } else {
    // Per segment: restore the checkpoint into a working copy, replay the
    // segment's gates logging their active pairs, then walk the logs back.
    HIP_TRY(c, c->partial2.ensure((size_t)M * grid * 8), "alloc partials");
    HIP_TRY(c, c->work.ensure(n * 8), "alloc working amplitudes");
    HIP_TRY(c, c->ctr_r.ensure((size_t)2 * seg * sizeof(u64)), "alloc log counters");
    double* W = c->work.as<double>();
    u64* lc = c->ctr_r.as<u64>();   // pair records per gate of the segment
    u64* sc = lc + seg;             // star records per gate
    for (int j = nseg - 1; j >= 0; --j) {
      const int64_t g_lo = (int64_t)j * seg;
      const int64_t g_hi = std::min<int64_t>(M, g_lo + seg);
      const int len = (int)(g_hi - g_lo);
      HIP_TRY(c, launch_restore(W, c->ckpt[j].as<double>(), c->ckpt_n.as<u64>() + j, n, c->stream), "restore");
      HIP_TRY(c, launch_fill_u32(lc, 0u, (u64)seg * 4, c->stream), "zero log counters");
      for (int t = 0; t < len; ++t) {
        const int64_t g = g_lo + t;
        if (c->a_kind[g])
          HIP_TRY(c, launch_gen_replay(c->st, W, n, c->a_gen[g], c->a_ncut ? 0.0 : c->a_eps, plog_of(t), lc + t,
                                       slog_of(t), sc + t, grid_blocks(c, n, 256), c->stream), "generator replay");
        else
          TIMED(c, SWCS_K_GATE_REPLAY, launch_gate_replay(c->st, W, n, c->ops_host[c->a_ops[g]], c->a_c[g], c->a_s[g],
                                        c->a_ncut ? 0.0 : c->a_eps, plog_of(t), lc + t,
                                        gate_grid(c, n, kReplayTile), c->stream), "replay");
        if (c->a_ncut)
          HIP_TRY(c, launch_ncut(W, c->st.keys, n, nullptr, c->ncut_state.as<NcutState>(), (unsigned)c->a_ncut,
                                 grid, c->stream), "ncut");
      }
      for (int t = len - 1; t >= 0; --t) {
        const int64_t g = g_lo + t;
        TIMED(c, SWCS_K_ADJOINT_REC, launch_adjoint_rec(plog_of(t), lc + t, c->mu.as<double>(), c->a_c[g], c->a_s[g],
                                      c->partial2.as<double>() + (size_t)g * grid, grid, c->stream), "reverse");
        if (c->a_kind[g])
          HIP_TRY(c, launch_adjoint_star(slog_of(t), sc + t, c->mu.as<double>(), c->a_gen[g],
                                         c->partial2.as<double>() + (size_t)g * grid, grid, c->stream), "reverse stars");
      }
    }
    HIP_TRY(c, launch_reduce_partials(c->partial2.as<double>(), grid, grid, (int)M, c->gbuf.as<double>(), c->stream), "reduce");
  }
  std::vector<double> d_unit((size_t)M);
  HIP_TRY(c, hipMemcpyAsync(d_unit.data(), c->gbuf.p, (size_t)M * 8, hipMemcpyDeviceToHost, c->stream), "copy dE");
  double nn_host[2];
  HIP_TRY(c, hipMemcpyAsync(nn_host, nn, 16, hipMemcpyDeviceToHost, c->stream), "copy energy");
  Counters hchk = read_counters(c, &e);  // synchronizes
  if (e != hipSuccess) return hip_fail(c, e, "sync");
  if (hchk.flags & kFlagOverflow) {
    hchk.flags &= ~kFlagOverflow;
    HIP_TRY(c, launch_store_counters(c->st.ctr, hchk, c->stream), "counters");
    c->hc = hchk;
    return fail(c, SWCS_E_DEVICE, "recomputation diverged from the forward run");
  }
  // per parameter: the unitaries it drives, each scaled by d(angle)/d(parameter)
  for (int64_t i = 0; i < M_par; ++i) dE[i] = 0.0;
  for (int64_t g = 0; g < M; ++g) dE[c->a_owner[(size_t)g]] += c->a_factor[(size_t)g] * d_unit[(size_t)g];
  if (E_out) *E_out = nn_host[0] / nn_host[1];
  return SWCS_OK;
}

int swcs_gate_active(swcs_ctx* c, int64_t* n_act, int64_t M) {
  if (!c) return SWCS_E_INVALID;
  if (M != c->last_M) return fail(c, SWCS_E_INVALID, "M differs from the last apply call");
  if (M == 0) return SWCS_OK;
  if (!n_act) return fail(c, SWCS_E_INVALID, "null n_act");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  HIP_TRY(c, hipMemcpyAsync(n_act, c->gate_n_act.p, (size_t)M * 8, hipMemcpyDeviceToHost, c->stream), "copy");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  return SWCS_OK;
}

int swcs_compact(swcs_ctx* c, int64_t* stored) {
  if (!c) return SWCS_E_INVALID;
  if (!c->have_state) return fail(c, SWCS_E_STATE, "no current state");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  hipError_t e;
  Counters h = get_counters(c, &e);
  if (e != hipSuccess) return hip_fail(c, e, "read counters");
  if (h.alive < h.n) {
    int r = state_compact(c, &h);
    if (r) return r;
    r = build_filter(c, h.n, h.alive);
    if (r) return r;
    c->ansatz_valid = false;  // the checkpoints refer to the old positions
  }
  if (stored) *stored = (int64_t)h.n;
  return SWCS_OK;
}

int swcs_state_counts(swcs_ctx* c, int64_t* stored, int64_t* alive) {
  if (!c) return SWCS_E_INVALID;
  if (!c->have_state) return fail(c, SWCS_E_STATE, "no current state");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  hipError_t e;
  const Counters h = get_counters(c, &e);
  if (e != hipSuccess) return hip_fail(c, e, "read counters");
  if (stored) *stored = (int64_t)h.n;
  if (alive) *alive = (int64_t)h.alive;
  return SWCS_OK;
}

int swcs_pool_stats(swcs_ctx* c, double* keys, int64_t* table_slots, int32_t* batches, int32_t* passes,
                    int32_t* screened) {
  if (!c) return SWCS_E_INVALID;
  if (!c->ps_passes) return fail(c, SWCS_E_STATE, "no pool-gradient pass yet");
  if (keys) *keys = c->ps_keys;
  if (table_slots) *table_slots = (int64_t)c->ps_slots;
  if (batches) *batches = c->ps_batches;
  if (passes) *passes = c->ps_passes;
  if (screened) *screened = c->ps_screened;
  return SWCS_OK;
}

int swcs_gate_sizes(swcs_ctx* c, int64_t* n_in, int64_t M) {
  if (!c) return SWCS_E_INVALID;
  if (M != c->last_M) return fail(c, SWCS_E_INVALID, "M differs from the last apply call");
  if (M == 0) return SWCS_OK;
  if (!n_in) return fail(c, SWCS_E_INVALID, "null n_in");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  HIP_TRY(c, hipMemcpyAsync(n_in, c->gate_n_in.p, (size_t)M * 8, hipMemcpyDeviceToHost, c->stream), "copy");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  return SWCS_OK;
}

static int occupations_device(swcs_ctx* c, u64 n) {
  const int grid = grid_blocks(c, n, 256);
  HIP_TRY(c, c->partial.ensure((size_t)grid * (c->nso + 1) * 8), "alloc partial");
  HIP_TRY(c, c->occ.ensure((size_t)(c->nso + 1) * 8), "alloc occ");
  HIP_TRY(c, launch_occupations(c->st, n, c->nso, c->partial.as<double>(), grid, c->stream), "occupations");
  HIP_TRY(c, launch_reduce_partials(c->partial.as<double>(), grid, grid, c->nso + 1, c->occ.as<double>(), c->stream), "reduce");
  return SWCS_OK;
}

int swcs_occupations(swcs_ctx* c, double* n_out) {
  if (!c) return SWCS_E_INVALID;
  if (!c->have_state) return fail(c, SWCS_E_STATE, "no current state");
  if (!n_out) return fail(c, SWCS_E_INVALID, "null n_out");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  hipError_t e;
  Counters h = get_counters(c, &e);
  if (e != hipSuccess) return hip_fail(c, e, "read counters");
  int r = occupations_device(c, h.n);
  if (r) return r;
  std::vector<double> tmp((size_t)c->nso + 1);
  HIP_TRY(c, hipMemcpyAsync(tmp.data(), c->occ.p, tmp.size() * 8, hipMemcpyDeviceToHost, c->stream), "copy");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  for (int P = 0; P < c->nso; ++P) n_out[P] = tmp[(size_t)P] / tmp[(size_t)c->nso];
  return SWCS_OK;
}

int swcs_timer_start(swcs_ctx* c, int kernel_id) {
  if (!c) return SWCS_E_INVALID;
  if (kernel_id < SWCS_K_CHAIN_LDS || kernel_id > SWCS_K_JOIN_TERMS)
    return fail(c, SWCS_E_INVALID, "unknown kernel id");
  c->timer_kernel = kernel_id;
  c->ev_used = 0;
  return SWCS_OK;
}

int swcs_timer_stop(swcs_ctx* c, int64_t* launches, double* total_ms) {
  if (!c) return SWCS_E_INVALID;
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  double tot = 0.0;
  for (size_t i = 0; i < c->ev_used; ++i) {
    float ms = 0.0f;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev_start[i], c->ev_stop[i]), "elapsed");
    tot += ms;
  }
  if (launches) *launches = (int64_t)c->ev_used;
  if (total_ms) *total_ms = tot;
  c->timer_kernel = 0;
  c->ev_used = 0;
  return SWCS_OK;
}

int64_t swcs_mlp_param_count(void) { return kMlpParams; }

int swcs_fock_diagonal(swcs_ctx* c, double* f_out) {
  if (!c) return SWCS_E_INVALID;
  if (!c->have_ints) return fail(c, SWCS_E_STATE, "integrals not set");
  if (!f_out) return fail(c, SWCS_E_INVALID, "null f_out");
  if (c->na != c->nb) return fail(c, SWCS_E_UNSUPPORTED, "closed-shell Fock needs n_alpha == n_beta");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  const int n = c->n;
  std::vector<double> f((size_t)n * n);
  HIP_TRY(c, hipMemcpyAsync(f.data(), c->fock.p, f.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream),
          "copy");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "sync");
  for (int p = 0; p < n; ++p) f_out[p] = f[(size_t)p * n + p];
  return SWCS_OK;
}

int swcs_features(swcs_ctx* c, const float* d_prev_absg, const float* d_age, const float* d_count,
                  float* d_feat) {
  if (!c) return SWCS_E_INVALID;
  int r = check_ready(c);
  if (r) return r;
  if (!c->have_state) return fail(c, SWCS_E_STATE, "no current state");
  if (!d_prev_absg || !d_age || !d_count || !d_feat) return fail(c, SWCS_E_INVALID, "null device pointer");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  hipError_t e;
  Counters h = get_counters(c, &e);
  if (e != hipSuccess) return hip_fail(c, e, "read counters");
  r = occupations_device(c, h.n);
  if (r) return r;
  HIP_TRY(c, launch_features(c->ops.as<OpDesc>(), c->K_pool, c->fock.as<double>(), c->eri.as<double>(),
                             c->n, c->occ.as<double>(), d_prev_absg, d_age, d_count, d_feat, c->stream), "features");
  return SWCS_OK;
}

int swcs_mlp_forward(swcs_ctx* c, const float* d_W, const float* d_x, int64_t B, float* d_y,
                     float* d_act) {
  if (!c) return SWCS_E_INVALID;
  if (B < 0 || (B > 0 && (!d_W || !d_x || !d_y))) return fail(c, SWCS_E_INVALID, "bad mlp arguments");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  HIP_TRY(c, launch_mlp_forward(d_W, d_x, B, d_y, d_act, c->stream), "mlp forward");
  return SWCS_OK;
}

int swcs_mlp_backward(swcs_ctx* c, const float* d_W, const float* d_x, const float* d_act,
                      const float* d_dy, int64_t B, float* d_dW) {
  if (!c) return SWCS_E_INVALID;
  if (B < 0 || !d_W || !d_dW || (B > 0 && (!d_x || !d_act || !d_dy)))
    return fail(c, SWCS_E_INVALID, "bad mlp arguments");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  const long long rows = std::max<long long>(1, mlp_backward_partial_rows(B));
  HIP_TRY(c, c->mlp_partial.ensure((size_t)rows * kMlpParams * 4), "alloc partial");
  HIP_TRY(c, launch_mlp_backward(d_W, d_x, d_act, d_dy, B, d_dW, c->mlp_partial.as<float>(), rows,
                                 c->stream), "mlp backward");
  return SWCS_OK;
}

int swcs_mse(swcs_ctx* c, const float* d_y, const float* d_t, int64_t B, float* d_dy, float* d_loss) {
  if (!c) return SWCS_E_INVALID;
  if (B <= 0 || !d_y || !d_t || !d_dy || !d_loss) return fail(c, SWCS_E_INVALID, "bad mse arguments");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  HIP_TRY(c, c->mse_partial.ensure((size_t)mse_partial_count(B) * 4), "alloc partial");
  HIP_TRY(c, launch_mse(d_y, d_t, B, d_dy, d_loss, c->mse_partial.as<float>(), c->stream), "mse");
  return SWCS_OK;
}

int swcs_log_abs(swcs_ctx* c, const double* d_g, int64_t n, float* d_t) {
  if (!c) return SWCS_E_INVALID;
  if (n < 0 || (n > 0 && (!d_g || !d_t))) return fail(c, SWCS_E_INVALID, "bad log_abs arguments");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  HIP_TRY(c, launch_log_abs(d_g, n, d_t, c->stream), "log_abs");
  return SWCS_OK;
}

int swcs_add_feature(swcs_ctx* c, float* d_v, const float* d_feat, int64_t n, int col, int sign, float scale) {
  if (!c) return SWCS_E_INVALID;
  if (n < 0 || (n > 0 && (!d_v || !d_feat)) || col < 0 || col >= 16 || (sign != 1 && sign != -1) ||
      !(scale >= 0.0f && scale <= 1.0f))
    return fail(c, SWCS_E_INVALID, "bad add_feature arguments");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  HIP_TRY(c, launch_add_feature(d_v, d_feat, n, col, (float)sign, scale, c->stream), "add_feature");
  return SWCS_OK;
}

int swcs_adam_step(swcs_ctx* c, float* d_W, float* d_m, float* d_v, const float* d_dW, int64_t P,
                   float lr, float b1, float b2, float eps, int step) {
  if (!c) return SWCS_E_INVALID;
  if (P <= 0 || !d_W || !d_m || !d_v || !d_dW || step < 1 || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1))
    return fail(c, SWCS_E_INVALID, "bad adam arguments");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  HIP_TRY(c, launch_adam(d_W, d_m, d_v, d_dW, P, lr, b1, b2, eps, step, c->stream), "adam");
  return SWCS_OK;
}

int swcs_select(swcs_ctx* c, const float* d_score, const uint32_t* d_rand, int64_t K, int64_t n_top,
                int64_t n_rand, int32_t* d_idx) {
  if (!c) return SWCS_E_INVALID;
  if (K <= 0 || K > ((int64_t)1 << 31) - 1 || n_top < 0 || n_rand < 0 || n_top + n_rand > K ||
      !d_score || !d_idx || (n_rand > 0 && !d_rand))
    return fail(c, SWCS_E_INVALID, "bad select arguments");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  const u64 need = select_scratch_elems(K);
  HIP_TRY(c, c->sel_scratch.ensure(need * 8), "alloc select scratch");
  TIMED(c, SWCS_K_SELECT, launch_select(d_score, d_rand, K, n_top, n_rand, d_idx, c->sel_scratch.as<u64>(), need,
                                        c->stream), "select");
  return SWCS_OK;
}

}  // extern "C"

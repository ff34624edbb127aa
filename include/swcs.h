/* swcs.h -- C ABI of the MI355X sparse wavefunction circuit solver (SWCS).
 *
 * The library evaluates the hot path of ADAPT-VQE with a sparse wavefunction
 * circuit solver (Mullinax et al., "Classical Pre-optimization Approach for
 * ADAPT-VQE", arXiv 2411.07920) on one AMD Instinct MI355X (gfx950):
 *
 *   - the factorized unitary coupled-cluster ansatz, Eq. (1), built from the
 *     single- and double-excitation unitaries of Eqs. (2) and (3) and their
 *     generalized forms (Sec. II.C), applied to a sparse state of
 *     (uint64 determinant, float64 amplitude) pairs, each unitary evaluated
 *     exactly (Sec. II.B) and the state pruned after every unitary (Fig. 1);
 *   - the energy, the operator-pool gradient of ADAPT step 4 (Sec. II.C) and
 *     the analytic parameter gradients used by the VQE optimizer (Sec. II.B);
 *   - the kernels of a learned pool screener (features, MLP, Adam, selection).
 *
 * Conventions shared by every call
 * --------------------------------
 * Orbitals.  n spatial orbitals, 2n <= 64 spin-orbitals, spin-orbital
 *   P = 2p + sigma (sigma 0 = alpha, 1 = beta).  Bit P of a determinant key is
 *   the occupation of P; |D> = a+_{P1}...a+_{Pk}|0> with P1 < ... < Pk, so a
 *   ladder operator on P carries (-1)^(occupied spin-orbitals below P).
 * Hamiltonian.  H = e_core + sum_PQ h_PQ a+_P a_Q
 *   + 1/2 sum_PQRS (PQ|RS) a+_P a+_R a_S a_Q with spin-orbital integrals built
 *   from the spatial h[p*n+q] and eri[((p*n+q)*n+r)*n+s] = (pq|rs) (chemists'
 *   notation), spin-conserving.
 * Pool.  Row k of the int32 table [K x 4] is (P, Q, R, S): a double
 *   T = a+_P a+_Q a_S a_R (P > Q, R > S, disjoint index sets, equal spin
 *   multisets) or, with R = S = -1, a single T = a+_P a_Q (P > Q, equal spin).
 *   The generator is A = T - T^dagger and the unitary exp(theta A).
 * Truncation.  After every unitary either entries with |c| < eps are dropped
 *   (eps = 0 keeps everything, exact zeros included) or, when ncut > 0, only the
 *   ncut entries of largest |c| are kept (ties keep the smaller key).  The state
 *   is not renormalized.
 * Energy.  E = <psi|H|psi> / <psi|psi> (Rayleigh quotient of the pruned state).
 * Memory.  Unless stated otherwise, pointer arguments are HOST pointers that
 *   are read (or written) during the call only; the library copies inputs to
 *   its own device memory, which it obtains from the allocator set with
 *   swcs_set_allocator (default hipMalloc / hipFree) and releases in
 *   swcs_destroy.  Screener calls (swcs_features .. swcs_select) take DEVICE
 *   pointers owned by the caller and enqueue work on the context stream
 *   without synchronizing.
 * Streams.  All device work of a context runs on its stream (default: the
 *   null stream).  Calls that return host values synchronize that stream.
 * Errors.  Every int-returning call returns SWCS_OK (0) or a negative status
 *   and records a message readable with swcs_last_error.  Nothing aborts and
 *   nothing throws across this boundary.  A context is not thread-safe.
 * Call order.  Integrals, reference and pool must be set before applying an
 *   ansatz; energy / gradient calls refer to the last applied ansatz or state,
 *   otherwise they return SWCS_E_STATE.
 */
#ifndef SWCS_H
#define SWCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct swcs_ctx swcs_ctx;

/* Device memory routines a caller may supply (swcs_set_allocator), e.g. a
 * framework's caching allocator.  alloc_fn returns at least `bytes` of device
 * memory on the context's device, 256-byte aligned, or NULL on failure;
 * free_fn returns a block that alloc_fn gave.  `user` is passed through. */
typedef void* (*swcs_alloc_fn)(size_t bytes, void* user);
typedef void (*swcs_free_fn)(void* p, void* user);

enum {
  SWCS_OK = 0,
  SWCS_E_INVALID = -1,     /* bad argument (shape, range, symmetry, NaN)    */
  SWCS_E_STATE = -2,       /* call order violated                           */
  SWCS_E_OOM = -3,         /* device allocation failed                      */
  SWCS_E_CAPACITY = -4,    /* state would exceed the configured maximum     */
  SWCS_E_DEVICE = -5,      /* HIP runtime error                             */
  SWCS_E_UNSUPPORTED = -6  /* no usable device / feature not available      */
};

/* Library version string (static storage). */
const char* swcs_version(void);

/* Create a context on HIP device `device` for n_spatial orbitals (2n <= 64)
 * and n_alpha / n_beta electrons.  *out receives the context or NULL. */
int swcs_create(int n_spatial, int n_alpha, int n_beta, int device, swcs_ctx** out);

/* Release the context and all device memory it owns.  NULL is ignored. */
void swcs_destroy(swcs_ctx* ctx);

/* Message of the last failing call on ctx (owned by ctx; valid until the next
 * call).  With ctx == NULL: the last failure of swcs_create on this thread. */
const char* swcs_last_error(const swcs_ctx* ctx);

/* Run all later work on `hip_stream` (a hipStream_t; NULL = null stream). */
int swcs_set_stream(swcs_ctx* ctx, void* hip_stream);

/* Route every later device allocation of the context through alloc_fn /
 * free_fn (both NULL: hipMalloc / hipFree again).  Blocks allocated before
 * the call are freed with the routines that allocated them.  The library
 * calls them on the calling thread inside any entry point that needs memory,
 * and may free a block while work it enqueued earlier on the context stream
 * still reads it: the allocator must keep a freed block from other use until
 * that stream has passed the free (a caching allocator bound to the context
 * stream does; otherwise synchronize in free_fn).  An alloc_fn failure
 * returns SWCS_E_OOM from the call that needed the memory.  Budgets the
 * library derives from free device memory (state capacity, pool-gradient
 * tables) count hipMemGetInfo's free bytes plus the bytes the library has
 * handed back to free_fn; memory the allocator caches for others is not
 * seen, so set swcs_set_capacity / swcs_set_table_budget to size them
 * exactly.  SWCS_E_INVALID if only one routine is given. */
int swcs_set_allocator(swcs_ctx* ctx, swcs_alloc_fn alloc_fn, swcs_free_fn free_fn, void* user);

/* Upper bound on stored determinants (0 = library default, sized from free
 * device memory).  With allow_regrow != 0 the state arrays grow on demand up
 * to that bound; growth past it fails with SWCS_E_CAPACITY.  With
 * allow_regrow == 0 (max_dets > 0 required, else SWCS_E_INVALID) the arrays
 * are reserved once at max_dets on the next apply or set_state and then kept:
 * no state allocation happens inside later applies, and a chain that would
 * need more fails with SWCS_E_CAPACITY and leaves no current state. */
int swcs_set_capacity(swcs_ctx* ctx, int64_t max_dets, int allow_regrow);

/* Upper bound, in bytes, on the hash table that pool gradients accumulate
 * sigma_P(X) in over the external space (Sec. II.C).  Keys that would not fit
 * are split by key hash into batches, each a full pass over the state, and
 * the gradients are summed over the batches.  0 (default) = 40% of the free
 * device memory; 1 to 4095 fail with SWCS_E_INVALID.  Batched results agree
 * with unbatched ones up to the order of floating-point summation. */
int swcs_set_table_budget(swcs_ctx* ctx, int64_t bytes);

/* How sigma_P (energy, parameter gradients) is formed.  ENUMERATE probes
 * every single and double excitation of every alive determinant (alive * C
 * probes).  HOLE_PAIRS groups the determinants by their subsets of N_e - 2
 * electrons (a sort of n * C(N_e, 2) records of 8 bytes, or 12 when the
 * subset key and the entry index do not fit one word) and evaluates only
 * pairs that share one, which are exactly the pairs within a double
 * excitation; it needs fewer than 2^32 stored entries (larger states use
 * ENUMERATE).  PAIRS
 * (states of at most 4,096 stored determinants; larger ones fall back to
 * AUTO's choice among the others) tests every pair of stored determinants in
 * LDS by popcount.  AUTO (default) takes PAIRS when the state
 * fits and n <= 8 C, otherwise HOLE_PAIRS when the probe count would exceed
 * 3e7, otherwise ENUMERATE.  All give the same sigma up to summation order.
 * Returns SWCS_E_INVALID for an unknown method. */
enum { SWCS_SIGMA_AUTO = 0, SWCS_SIGMA_ENUMERATE = 1, SWCS_SIGMA_HOLE_PAIRS = 2, SWCS_SIGMA_PAIRS = 3 };
int swcs_set_sigma_method(swcs_ctx* ctx, int method);

/* How the pool gradients of a whole pool, or of a subset of at least half
 * of it, are formed (ADAPT step 4, Sec. II.C: g_k = <psi|[H, A_k]|psi> /
 * <psi|psi> = 2 <sigma|A_k psi> / <psi|psi> with sigma = H psi on the
 * external space).  TABLE pushes H_{X D} psi(D) for every alive D and
 * connection X into a device-wide hash table of sigma(X), then contracts
 * (swcs_set_table_budget applies).  JOIN writes one 8-byte record per
 * (D, X) pair (alive * (C + 1) records, C the connections per determinant),
 * sorts them by a hash of X and forms sigma(X) and the gradients per group
 * in LDS; it needs 16 bytes per record of device memory and storage index,
 * connection fields and 8 to 24 hash bits within one 64-bit word.  When
 * another 12.5 bytes per record fit as well, the gradient terms are summed
 * through per-operator bins (LDS sums, then one device-scope add per
 * operator and bin chunk) instead of one device-scope add per record.  AUTO
 * (default) takes JOIN when no table budget is set, there are at most 2^31
 * records (beyond that the table was faster at 52 spin-orbitals) and they fit
 * within half of the free device memory and the word, else TABLE; a JOIN pass
 * whose hash group overflows its LDS table is redone by TABLE.  Forced JOIN that
 * does not fit returns SWCS_E_CAPACITY.  Both agree up to summation order.
 * Returns SWCS_E_INVALID for an unknown method. */
enum { SWCS_POOL_AUTO = 0, SWCS_POOL_TABLE = 1, SWCS_POOL_JOIN = 2 };
int swcs_set_pool_method(swcs_ctx* ctx, int method);


/* Step 1 of the ADAPT procedure (Sec. II.C): molecular integrals.  h[n*n] and
 * eri[n^4] (host, float64, layouts above).  Rejects non-finite values, an
 * asymmetric h and an eri without 8-fold symmetry (tolerance 1e-12). */
int swcs_set_integrals(swcs_ctx* ctx, const double* h, const double* eri, double e_core);

/* Step 3: the reference determinant (e.g. Hartree-Fock).  Its alpha and beta
 * popcounts must equal n_alpha and n_beta and it must fit in 2n bits. */
int swcs_set_reference(swcs_ctx* ctx, uint64_t det);

/* Step 2: the operator pool, int32 ops[K*4] (host, rows as above).  Rows are
 * validated (range, ordering, disjointness, spin conservation, canonical
 * orientation (P, Q) > (R, S) for doubles, no duplicate rows). */
int swcs_set_pool(swcs_ctx* ctx, const int32_t* ops, int64_t K);

/* Eq. (1): psi = prod_I U_I(theta_I) psi_0 with psi_0 = the reference, the
 * unitary of pool row op_idx[0] applied first (new operators are appended at
 * the end, as in step 5 of ADAPT), pruning after every unitary (Fig. 1) with
 * eps (ncut == 0) or ncut (ncut > 0).  op_idx[M], theta[M] are host arrays;
 * M may be 0.  *n_det_out (may be NULL) receives the number of kept
 * determinants.  The run keeps checkpoints for swcs_param_gradients. */
int swcs_apply_ansatz(swcs_ctx* ctx, const int32_t* op_idx, const double* theta, int64_t M,
                      double eps, int64_t ncut, int64_t* n_det_out);

/* Eq. (1) over spin-complemented generators (Sec. III): row i of
 * gens[M x 3] (host int32) is (k1, k2, s).  k2 = -1: the unitary
 * exp(theta_i A_k1).  Otherwise exp(theta_i (A_k1 + s A_k2)), s = +1 or -1,
 * one parameter for two pool rows:
 *   - rows acting on disjoint spin-orbitals commute and are applied as two
 *     unitaries, exp(theta A_k1) then exp(s theta A_k2), each followed by
 *     pruning;
 *   - a double and its spin flip that share spin-orbitals (an opposite-spin
 *     double with two indices on one spatial orbital) are applied as one
 *     exact unitary: on a determinant both rows act on, exp(theta G) rotates
 *     it and its two images at frequency sqrt(2) theta; other overlapping
 *     rows fail with SWCS_E_UNSUPPORTED.
 * Otherwise as swcs_apply_ansatz; swcs_param_gradients then returns one
 * derivative per generator (M entries) and swcs_gate_sizes refers to the
 * unitaries (a commuting pair counts two). */
int swcs_apply_generators(swcs_ctx* ctx, const int32_t* gens, const double* theta, int64_t M,
                          double eps, int64_t ncut, int64_t* n_det_out);

/* Continue from the current state: apply M more unitaries with the same
 * pruning rule without resetting to the reference.  Parameter gradients are
 * not available after this call (they need an ansatz started from psi_0). */
int swcs_apply_gates(swcs_ctx* ctx, const int32_t* op_idx, const double* theta, int64_t M,
                     double eps, int64_t ncut, int64_t* n_det_out);

/* Replace the current state by n (key, amplitude) pairs (host arrays, keys
 * distinct, each in the (n_alpha, n_beta) sector). */
int swcs_set_state(swcs_ctx* ctx, const uint64_t* keys, const double* amps, int64_t n);

/* Export the current state sorted ascending by key into caller arrays of
 * length cap.  *n receives the state size; if it exceeds cap nothing is
 * written and SWCS_E_INVALID is returned. */
int swcs_get_state(swcs_ctx* ctx, uint64_t* keys, double* amps, int64_t cap, int64_t* n);

/* Energy of the current state: *E = numer / norm2 with numer = <psi|H|psi>
 * (Slater-Condon rules over the kept determinants) and norm2 = <psi|psi>.
 * Any output pointer may be NULL. */
int swcs_energy(swcs_ctx* ctx, double* E, double* numer, double* norm2);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as swcs_energy, computed with no device allocation.  The diagonal
 * elements, sigma_P and the partial sums live in a fixed 32 MiB device array
 * of the library (one per device, held until the process ends), so the
 * state may hold at most 2,088,928 stored entries (SWCS_E_CAPACITY beyond).
 * sigma_P is formed by pairs for at most 4,096 stored entries and by
 * enumeration otherwise.  Every call on a device shares that array: calls
 * that overlap on one device (several contexts or threads at once) race and
 * must be serialized by the caller. */
int swcs_energy_noalloc(swcs_ctx* ctx, double* E, double* numer, double* norm2);

/* The projected sigma vector sigma_P(D) = sum_{D' in psi} H_{D D'} psi(D')
 * on the kept determinants, exported as (key, sigma) pairs sorted by key into
 * caller arrays of length cap (same size rules as swcs_get_state).  E is
 * sum psi sigma_P / sum psi^2. */
int swcs_sigma_projected(swcs_ctx* ctx, uint64_t* keys, double* sigma, int64_t cap, int64_t* n);

/* ADAPT step 4 (Sec. II.C): g_k = <psi|[H, A_k]|psi> / <psi|psi>, the
 * derivative of E with respect to the parameter of pool operator k appended
 * at the end of the ansatz, for k in subset[n_subset] (host int32; NULL =
 * all K in pool order).  g_out has n_subset (or K) entries. */
int swcs_pool_gradients(swcs_ctx* ctx, const int32_t* subset, int64_t n_subset, double* g_out);

/* Same as swcs_pool_gradients for a subset, with the subset and the result in
 * DEVICE memory and no host round trip: d_subset[n_subset] int32 pool indices,
 * d_g[n_subset] float64 written on the context stream (read it after the
 * stream has synchronized).  Indices outside [0, K) give NaN in d_g.  The
 * query table of the selected operators is sized from the bound
 * (alive determinants x min(n_subset, C)) when that table stays below
 * 512 MB and no table budget is set (swcs_set_table_budget); otherwise from
 * a count of (determinant, operator) pairs (on every 16th determinant tile
 * from 16,384 stored entries, scaled), capped by the distinct external count
 * of the last full-pool call, which synchronizes once, and again after each
 * pass that was split into key-hash batches or sized by that cap (a pass
 * whose table filled is repeated with twice the estimate).  A pass split
 * into batches also counts the new keys of its first batch (one more
 * synchronization) and restarts with fewer batches when the query set is
 * under half the estimate.
 * A bound-sized table is not checked on the host: if an insert found it full
 * (more than 4,096 probes at load <= 1/2), every entry of d_g is NaN.
 * Returns SWCS_E_OOM if even 4,096 batches do not fit the table memory. */
int swcs_pool_gradients_device(swcs_ctx* ctx, const int32_t* d_subset, int64_t n_subset,
                               double* d_g);

/* Analytic parameter gradients (Sec. II.B) of the last swcs_apply_ansatz:
 * dE_dtheta[M] with every gate's kept support held fixed (the pruning acts as
 * a fixed projection; at eps = 0 and no ncut this is the exact gradient).
 * Reverse (adjoint) sweep over states recomputed from checkpoints stored
 * every ceil(sqrt(M)) gates.  *E_out (may be NULL) receives E. */
int swcs_param_gradients(swcs_ctx* ctx, double* dE_dtheta, double* E_out);

/* Per-gate sizes of the last apply call: n_in[M] receives the number of kept
 * determinants entering each gate.  Returns SWCS_E_INVALID if M differs. */
int swcs_gate_sizes(swcs_ctx* ctx, int64_t* n_in, int64_t M);

/* Per-gate active counts of the last apply call: n_act[M] receives the number
 * of stored entries the gate's operator (or its adjoint) acts on, counted by
 * the multi-block gate kernels (0 for gates run in the single-workgroup chain
 * of small states).  Returns SWCS_E_INVALID if M differs. */
int swcs_gate_active(swcs_ctx* ctx, int64_t* n_act, int64_t M);

/* Stored entries (alive or pruned; every gate scans them) and alive
 * entries of the current state. */
int swcs_state_counts(swcs_ctx* ctx, int64_t* stored, int64_t* alive);

/* Rebuild of the current state without its pruned entries (Sec. II.B, the
 * truncated state keeps only amplitudes at or above eps): the alive entries
 * move to the front of the storage arrays in their storage order and the
 * index is rebuilt; keys, amplitudes and every later result are unchanged
 * (sums over the state may differ in rounding order).  Storage positions
 * change, so the record that swcs_param_gradients needs is dropped (it
 * then returns SWCS_E_STATE until the next ansatz is applied from the
 * reference).  Gate chains that keep no such record (swcs_apply_gates)
 * rebuild by themselves when pruned entries outnumber alive ones, or are a
 * quarter of them when the arrays would otherwise grow.  *stored (may be
 * NULL) receives the stored count afterwards.  SWCS_E_STATE without a
 * state. */
int swcs_compact(swcs_ctx* ctx, int64_t* stored);

/* The last pool-gradient pass: *keys the key count its accumulation table
 * was sized for (after a full-pool pass: the distinct determinants sigma was
 * formed on), *table_slots the slots of one table (0 for a sort-and-join
 * pass, which has none), *batches the key-hash batches, *passes how many
 * times the pass ran (a pass whose table filled is repeated), *screened 1
 * for a subset pass.  Any pointer may be NULL; SWCS_E_STATE before the
 * first pass. */
int swcs_pool_stats(swcs_ctx* ctx, double* keys, int64_t* table_slots, int32_t* batches,
                    int32_t* passes, int32_t* screened);

/* Spin-orbital occupations <n_P> = sum_D psi(D)^2 [P in D] / norm2 of the
 * current state, n_out[2n] (host). */
int swcs_occupations(swcs_ctx* ctx, double* n_out);

/* Diagonal of the closed-shell Fock matrix of the reference occupation,
 * f_pp = h_pp + sum_{j < n_alpha} [2 (pp|jj) - (pj|jp)], for the n spatial
 * orbitals, f_out[n] (host).  These are the orbital energies of the
 * Moller-Plesset partition that orders the UCCSD ansatz (Sec. II.A) with
 * H0 = sum_P f_{P/2,P/2} n_P.  Needs integrals; SWCS_E_UNSUPPORTED when
 * n_alpha != n_beta (no closed-shell reference). */
int swcs_fock_diagonal(swcs_ctx* ctx, double* f_out);

/* ---- measurement ---- */

/* Kernels that swcs_timer_start can time. */
enum {
  SWCS_K_CHAIN_LDS = 1,     /* whole gate chain in one LDS-resident workgroup   */
  SWCS_K_GATE = 2,          /* one gate, multi-block, state in HBM              */
  SWCS_K_SIGMA_PROJ = 3,    /* projected sigma vector + energy partial sums     */
  SWCS_K_SIGMA_PUSH = 4,    /* external sigma vector accumulation               */
  SWCS_K_POOL_CONTRACT = 5, /* pool-gradient contraction                        */
  SWCS_K_ADJOINT_LDS = 6,   /* reverse adjoint sweep in one LDS-resident workgroup */
  SWCS_K_GATE_REPLAY = 7,   /* one replayed gate with pair logging (adjoint)    */
  SWCS_K_ADJOINT_REC = 8,   /* one reverse step over logged pairs (adjoint)     */
  SWCS_K_SIGMA_PUSH_INTO = 9, /* external sigma on the screened query set        */
  SWCS_K_CONTRACT_OPS = 10,  /* operator-major contraction of a small subset     */
  SWCS_K_HOLEPAIR = 11,      /* sigma_P pair evaluation inside hole-pair groups  */
  SWCS_K_ADJOINT_REPLAY_LDS = 12, /* segment replays of the LDS adjoint, one workgroup each */
  SWCS_K_SELECT = 13,        /* screener selection (top + random), swcs_select   */
  SWCS_K_JOIN_EMIT = 14,     /* full-pool gradients: one record per connection   */
  SWCS_K_JOIN_SORT = 15,     /* full-pool gradients: radix sort of the records   */
  SWCS_K_JOIN_REDUCE = 16,   /* full-pool gradients: sigma and g per bucket run  */
  SWCS_K_JOIN_TERMS = 17     /* full-pool gradients: sums of the binned g terms  */
};

/* From now on record HIP events on the context stream around every launch
 * of kernel `kernel_id` (one of SWCS_K_*), discarding earlier records. */
int swcs_timer_start(swcs_ctx* ctx, int kernel_id);

/* Synchronize the stream, return the number of timed launches and their
 * summed duration in milliseconds, and stop timing. */
int swcs_timer_stop(swcs_ctx* ctx, int64_t* launches, double* total_ms);

/* ---- learned pool screener (device pointers, float32, ctx stream) ---- */

/* Number of float32 parameters of the screener MLP 16 -> 128 -> 128 -> 1
 * (ReLU), laid out W1[16x128], b1[128], W2[128x128], b2[128], W3[128], b3. */
int64_t swcs_mlp_param_count(void);

/* Sixteen features per pool operator into d_feat[K x 16]:
 *  0-3 closed-shell Fock diagonal f_pp of the spatial orbitals of P,Q,R,S
 *      (occupied = lowest n_alpha spatial orbitals; 0 when absent),
 *  4   |(pr|qs)| for doubles, |f_pq| for singles,
 *  5-8 occupations <n_P> of the current state for P,Q,R,S (0 when absent),
 *  9   d_prev_absg[k], 10 log10(d_prev_absg[k] + 1e-16),
 *  11  d_age[k] / 10, 12-14 one-hot single / same-spin / opposite-spin double,
 *  15  d_count[k].  Requires a current state. */
int swcs_features(swcs_ctx* ctx, const float* d_prev_absg, const float* d_age,
                  const float* d_count, float* d_feat);

/* Forward pass on B rows of d_x[B x 16] into d_y[B].  If d_act is not NULL it
 * receives the post-ReLU activations [B x 256] (layer 1 then layer 2) used by
 * swcs_mlp_backward. */
int swcs_mlp_forward(swcs_ctx* ctx, const float* d_W, const float* d_x, int64_t B, float* d_y,
                     float* d_act);

/* Gradient of sum_b d_dy[b] * y_b with respect to the parameters into d_dW
 * (overwritten), from the inputs and the activations of the forward pass. */
int swcs_mlp_backward(swcs_ctx* ctx, const float* d_W, const float* d_x, const float* d_act,
                      const float* d_dy, int64_t B, float* d_dW);

/* Mean squared error: *d_loss = mean (y - t)^2 and d_dy = 2 (y - t) / B. */
int swcs_mse(swcs_ctx* ctx, const float* d_y, const float* d_t, int64_t B, float* d_dy,
             float* d_loss);

/* Screener targets: d_t[i] = log10(|d_g[i]| + 1e-12) as float32 (device). */
int swcs_log_abs(swcs_ctx* ctx, const double* d_g, int64_t n, float* d_t);

/* d_v[i] = scale * d_v[i] + sign * d_feat[i * 16 + col] for i < n (float32,
 * device; sign is +1 or -1, 0 <= col < 16, 0 <= scale <= 1).  The screener
 * scores an operator by feature 10, log10 of its last exact |g|, plus the
 * network output shrunk by its out-of-sample fit (scale), and trains the
 * network on the matching residual target (scale 1). */
int swcs_add_feature(swcs_ctx* ctx, float* d_v, const float* d_feat, int64_t n, int col, int sign,
                     float scale);

/* One Adam step with bias correction (step >= 1) on P parameters. */
int swcs_adam_step(swcs_ctx* ctx, float* d_W, float* d_m, float* d_v, const float* d_dW,
                   int64_t P, float lr, float b1, float b2, float eps, int step);

/* Selection: the n_top operators of largest score (ties: smaller index) plus
 * the n_rand remaining operators of smallest d_rand key (ties: smaller index),
 * written ascending into d_idx[n_top + n_rand]. */
int swcs_select(swcs_ctx* ctx, const float* d_score, const uint32_t* d_rand, int64_t K,
                int64_t n_top, int64_t n_rand, int32_t* d_idx);

#ifdef __cplusplus
}
#endif

#endif /* SWCS_H */

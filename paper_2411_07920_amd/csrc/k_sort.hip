// Stable LSD radix sort of 64-bit keys (with optional 64-bit payloads),
// alive-entry compaction and the screener's top-k + random selection.
//
// One 8-bit digit per pass: (1) per-tile digit histograms, (2) one exclusive
// scan over (digit, tile) in digit-major order, (3) a stable scatter in which
// each 256-item row of a tile ranks its items by wave ballots on the digit
// bits and a prefix over the four waves.  Only ceil(key_bits / 8) passes run.
#include <type_traits>

#include "swcs_internal.h"

namespace swcs {

constexpr int kSortThreads = 256;
constexpr int kSortRows = 16;
constexpr int kSortTile = kSortThreads * kSortRows;

// Rows of 256 items per tile: 16 for large sorts, 1 for small ones (more
// tiles, shorter serial row loop per tile).
inline int sort_rows(u64 count) { return count < (1ULL << 20) ? 1 : kSortRows; }

// Tile handled by workgroup `block` of `nblocks`: workgroups are dispatched to
// the eight XCDs in turn, so XCD x (blocks x, x + 8, ...) is given a
// contiguous range of tiles.  Neighbouring tiles write neighbouring pieces of
// each digit's output run (scatter) and neighbouring counts of each digit
// (histogram), and these then meet in the same L2.
__device__ inline u64 xcd_tile(u64 block, u64 nblocks) {
  const u64 x = block & 7u, k = block >> 3;
  const u64 q = nblocks >> 3, r = nblocks & 7u;
  return x * q + (x < r ? x : r) + k;
}

template <int ROWS>
__global__ void __launch_bounds__(kSortThreads)
k_radix_hist(const u64* __restrict__ keys, u64 count, int shift, u64* __restrict__ counts,
             int nblocks) {
  __shared__ unsigned hist[256];
  hist[threadIdx.x] = 0;
  __syncthreads();
  const u64 b = xcd_tile(blockIdx.x, (u64)nblocks);
  const u64 base = b * (kSortThreads * ROWS);
  // all rows are loaded (indices clamped to the last key) before the first
  // LDS atomic, so the loads are in flight together
  u64 k[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; ++r) {
    const u64 i = base + (u64)r * kSortThreads + threadIdx.x;
    k[r] = keys[i < count ? i : count - 1];
  }
#pragma unroll
  for (int r = 0; r < ROWS; ++r)
    if (base + (u64)r * kSortThreads + threadIdx.x < count) atomicAdd(&hist[(k[r] >> shift) & 255u], 1u);
  __syncthreads();
  counts[(u64)threadIdx.x * nblocks + b] = hist[threadIdx.x];
}

// Exclusive scans.  Tiles of kScanChunk elements are loaded coalesced into
// LDS (kScanItems independent loads per thread), each thread scans
// kScanItems consecutive elements, and a block scan joins the threads.
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr u64 kScanChunk = (u64)kScanThreads * kScanItems;
constexpr u64 kScanSingleBlock = 1ULL << 16;

__device__ inline u64 block_exclusive_1024(u64 v, u64* part, u64* total) {
  part[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const u64 w = (threadIdx.x >= (unsigned)off) ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += w;
    __syncthreads();
  }
  const u64 incl = part[threadIdx.x];
  *total = part[kScanThreads - 1];
  return incl - v;
}

// Scans the tile data[base, base + kScanChunk) in place starting from
// `carry`; returns the tile total.  Every thread of the block calls it.
__device__ inline u64 scan_tile(u64* __restrict__ data, u64 len, u64 base, u64 carry, u64* stage,
                                u64* part) {
  // loads first (indices clamped, zeroed after), so the kScanItems loads of
  // a thread are in flight together
  u64 ld[kScanItems];
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const u64 i = base + (u64)j * kScanThreads + threadIdx.x;
    ld[j] = data[i < len ? i : len - 1];
  }
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const u64 i = base + (u64)j * kScanThreads + threadIdx.x;
    stage[(u64)j * kScanThreads + threadIdx.x] = (i < len) ? ld[j] : 0;
  }
  __syncthreads();
  u64 v[kScanItems], t = 0;
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = stage[(u64)threadIdx.x * kScanItems + j];
    t += v[j];
  }
  u64 total;
  u64 run = carry + block_exclusive_1024(t, part, &total);
  for (int j = 0; j < kScanItems; ++j) {
    stage[(u64)threadIdx.x * kScanItems + j] = run;
    run += v[j];
  }
  __syncthreads();
  for (int j = 0; j < kScanItems; ++j) {
    const u64 i = base + (u64)j * kScanThreads + threadIdx.x;
    if (i < len) data[i] = stage[(u64)j * kScanThreads + threadIdx.x];
  }
  __syncthreads();
  return total;
}

// In-place exclusive scan of data[len] with one block (short arrays, and the
// chunk sums of the multi-block scan below).
__global__ void __launch_bounds__(kScanThreads) k_scan_exclusive(u64* __restrict__ data, u64 len) {
  __shared__ u64 stage[kScanChunk];
  __shared__ u64 part[kScanThreads];
  u64 carry = 0;
  for (u64 base = 0; base < len; base += kScanChunk) carry += scan_tile(data, len, base, carry, stage, part);
}

// Multi-block exclusive scan: chunk sums, a scan of the sums, then each
// block scans its chunk from its offset.
__global__ void __launch_bounds__(kScanThreads)
k_scan_chunk_sums(const u64* __restrict__ data, u64 len, u64* __restrict__ sums) {
  __shared__ u64 red[kScanThreads];
  const u64 base = (u64)blockIdx.x * kScanChunk;
  u64 ld[kScanItems];
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const u64 i = base + (u64)j * kScanThreads + threadIdx.x;
    ld[j] = data[i < len ? i : len - 1];  // clamped: the loads issue together
  }
  u64 s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j)
    if (base + (u64)j * kScanThreads + threadIdx.x < len) s += ld[j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kScanThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kScanThreads)
k_scan_chunk_apply(u64* __restrict__ data, u64 len, const u64* __restrict__ offs) {
  __shared__ u64 stage[kScanChunk];
  __shared__ u64 part[kScanThreads];
  (void)scan_tile(data, len, (u64)blockIdx.x * kScanChunk, offs[blockIdx.x], stage, part);
}

// Extra scratch (u64 elements) that scan_exclusive needs for len elements.
u64 scan_scratch_elems(u64 len) { return len <= kScanSingleBlock ? 0 : (len + kScanChunk - 1) / kScanChunk; }

// Exclusive scan of data[len] in place; sums has scan_scratch_elems(len) elements.
void scan_exclusive(u64* data, u64 len, u64* sums, hipStream_t stream) {
  if (len <= kScanSingleBlock) {
    hipLaunchKernelGGL(k_scan_exclusive, dim3(1), dim3(1024), 0, stream, data, len);
    return;
  }
  const u64 nb = (len + kScanChunk - 1) / kScanChunk;
  hipLaunchKernelGGL(k_scan_chunk_sums, dim3((unsigned)nb), dim3(kScanThreads), 0, stream, data, len, sums);
  hipLaunchKernelGGL(k_scan_exclusive, dim3(1), dim3(1024), 0, stream, sums, nb);
  hipLaunchKernelGGL(k_scan_chunk_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, stream, data, len,
                     (const u64*)sums);
}

// Stable scatter of one tile of THREADS * ROWS items (the histogram's tile).
// Rows of THREADS items are ranked two at a time by wave ballots on the digit
// bits and prefixes over the waves (and over the first row of the pair for
// the second); the tile is first reordered by digit in LDS and then written
// out, so consecutive lanes store consecutive positions of one digit's run.
// The tile's digit counts come from the scanned offsets (the next tile's
// offset, or the next digit's first offset for the last tile).  Threads below
// 256 own one digit each in the per-digit arrays.
// Value type of a key-only sort: no value loads, stores or LDS staging.
struct NoVal {};

template <int THREADS, int ROWS, class V>
__global__ void __launch_bounds__(THREADS)
k_radix_scatter(const u64* __restrict__ keys_in, const V* __restrict__ vals_in, u64 count,
                int shift, const u64* __restrict__ offsets, int nblocks, u64* __restrict__ keys_out,
                V* __restrict__ vals_out) {
  constexpr int kTile = THREADS * ROWS;
  constexpr int kWaves = THREADS / 64;
  static_assert(THREADS >= 256, "one thread per digit");
  __shared__ u64 base_off[256];
  __shared__ unsigned local_off[256];
  __shared__ unsigned running[256];
  __shared__ unsigned wave_cnt[2][kWaves][256];
  __shared__ unsigned wave_tot[4];
  constexpr bool kVals = !std::is_same<V, NoVal>::value;
  __shared__ u64 s_key[kTile];
  __shared__ V s_val[kVals ? kTile : 1];
  const int lane = __lane_id();
  const int wave = threadIdx.x >> 6;
  const int t = threadIdx.x;
  const u64 b = xcd_tile(blockIdx.x, (u64)nblocks);
  // digit counts of the tile and their exclusive scan (waves 0-3 hold the
  // 256 digits; a wavefront scan, then the wave totals)
  unsigned cnt = 0, incl = 0;
  if (t < 256) {
    const u64 o = offsets[(u64)t * nblocks + b];
    const u64 nxt = (b + 1 < (u64)nblocks) ? offsets[(u64)t * nblocks + b + 1]
                                           : (t < 255 ? offsets[(u64)(t + 1) * nblocks] : count);
    base_off[t] = o;
    running[t] = 0;
    cnt = (unsigned)(nxt - o);
    incl = cnt;
    for (int off = 1; off < 64; off <<= 1) {
      const unsigned v = __shfl_up(incl, off);
      if (lane >= off) incl += v;
    }
    if (lane == 63) wave_tot[wave] = incl;
  }
  __syncthreads();
  if (t < 256) {
    unsigned before = 0;
    for (int w = 0; w < wave; ++w) before += wave_tot[w];
    local_off[t] = before + incl - cnt;
  }
  const u64 tile0 = b * (u64)kTile;
  const unsigned tile_n = (unsigned)((count - tile0) < (u64)kTile ? (count - tile0) : (u64)kTile);
  // every row's loads are issued before the ranking starts
  u64 key[ROWS];
  V val[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; ++r) {
    const unsigned i = (unsigned)r * THREADS + t;
    key[r] = (i < tile_n) ? keys_in[tile0 + i] : 0;
    if constexpr (kVals) val[r] = (vals_in && i < tile_n) ? vals_in[tile0 + i] : V(0);
  }
  // wave_cnt entries hold either a count of row pair p tagged (p + 1) << 16
  // or an offset tagged 0xffff << 16, so a stale count is never taken for a
  // current one and the table needs no clearing between pairs.
  if (t < 256)
    for (int w = 0; w < kWaves; ++w) wave_cnt[0][w][t] = wave_cnt[1][w][t] = 0xffff0000u;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < ROWS; r += 2) {
    const unsigned tag = (unsigned)(r / 2 + 1) << 16;
    bool valid[2];
    unsigned digit[2], below[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int rr = (r + h < ROWS) ? r + h : r;  // an odd last row has no partner
      valid[h] = r + h < ROWS && (unsigned)(r + h) * THREADS + t < tile_n;
      digit[h] = valid[h] ? (unsigned)((key[rr] >> shift) & 255u) : 0u;
      u64 peers = __ballot(valid[h]);
      for (int bit = 0; bit < 8; ++bit) {
        const u64 m = __ballot(valid[h] && ((digit[h] >> bit) & 1u));
        peers &= ((digit[h] >> bit) & 1u) ? m : ~m;
      }
      below[h] = (unsigned)__popcll(peers & ((1ULL << lane) - 1ULL));
      if (valid[h] && below[h] == 0) wave_cnt[h][wave][digit[h]] = tag | (unsigned)__popcll(peers);
    }
    __syncthreads();
    // column t (digit t): counts in (row, wave) order become the exclusive
    // positions of each (row, wave) run in the reordered tile
    if (t < 256) {
      // every count of the column is read before the first offset is
      // written back, so the reads are in flight together
      unsigned v[2 * kWaves];
#pragma unroll
      for (int j = 0; j < 2 * kWaves; ++j) v[j] = wave_cnt[j / kWaves][j % kWaves][t];
      const unsigned start = local_off[t] + running[t];
      unsigned at = start;
#pragma unroll
      for (int j = 0; j < 2 * kWaves; ++j) {
        wave_cnt[j / kWaves][j % kWaves][t] = 0xffff0000u | at;
        at += ((v[j] & 0xffff0000u) == tag) ? (v[j] & 0xffffu) : 0u;
      }
      running[t] += at - start;
    }
    __syncthreads();
    unsigned pos[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) pos[h] = (wave_cnt[h][wave][digit[h]] & 0xffffu) + below[h];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (!valid[h]) continue;
      const int rr = (r + h < ROWS) ? r + h : r;
      s_key[pos[h]] = key[rr];
      if constexpr (kVals) s_val[pos[h]] = val[rr];
    }
    __syncthreads();  // positions are read before the next pair's counts land
  }
  __syncthreads();
  for (unsigned i = t; i < tile_n; i += THREADS) {
    const u64 k = s_key[i];
    const unsigned digit = (unsigned)((k >> shift) & 255u);
    const u64 dst = base_off[digit] + (i - local_off[digit]);
    keys_out[dst] = k;
    if constexpr (kVals)
      if (vals_in) vals_out[dst] = s_val[i];
  }
}

// Scratch (u64 elements) for sorting any count up to `count`: the tiling
// switches from one-row to 16-row tiles at 2^20 items, so just below the
// switch a sort needs more scratch than just above it.
static u64 radix_sort_scratch_exact(u64 count) {
  const u64 tile = (u64)kSortThreads * sort_rows(count);
  const u64 nblocks = (count + tile - 1) / tile;
  const u64 len = 256 * (nblocks < 1 ? 1 : nblocks);
  return len + scan_scratch_elems(len);
}

u64 radix_sort_scratch_elems(u64 count) {
  u64 r = radix_sort_scratch_exact(count);
  if (count >= (1ULL << 20)) r = std::max(r, radix_sort_scratch_exact((1ULL << 20) - 1));
  return r;
}

// Sorts (keys, vals) ascending by the low key_bits bits of the key; tmp_* are
// ping-pong buffers of the same size.  With out_keys / out_vals the result
// stays in whichever pair of buffers the last pass wrote and the pointers are
// returned there; otherwise it is copied back to keys / vals if needed.
template <class V>
hipError_t radix_sort_impl(u64* keys, V* vals, u64* tmp_keys, V* tmp_vals, u64 count, int key_bits,
                           u64* scratch, u64 scratch_elems, hipStream_t stream, u64** out_keys,
                           V** out_vals) {
  if (out_keys) *out_keys = keys;
  if (out_vals) *out_vals = vals;
  if (count <= 1) return hipSuccess;
  const int rows = sort_rows(count);
  const u64 tile = (u64)kSortThreads * rows;
  const int nblocks = (int)((count + tile - 1) / tile);
  const u64 len = (u64)256 * nblocks;
  if (len + scan_scratch_elems(len) > scratch_elems) return hipErrorInvalidValue;
  const int passes = (key_bits + 7) / 8;
  u64 *kin = keys, *kout = tmp_keys;
  V *vin = vals, *vout = tmp_vals;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    if (rows == 1)
      hipLaunchKernelGGL(k_radix_hist<1>, dim3(nblocks), dim3(kSortThreads), 0, stream, kin, count,
                         shift, scratch, nblocks);
    else
      hipLaunchKernelGGL(k_radix_hist<kSortRows>, dim3(nblocks), dim3(kSortThreads), 0, stream, kin,
                         count, shift, scratch, nblocks);
    scan_exclusive(scratch, len, scratch + len, stream);
    // the scatter tile equals the histogram tile (kSortThreads * rows items)
    if (rows == 1)
      hipLaunchKernelGGL((k_radix_scatter<kSortThreads, 1, V>), dim3(nblocks), dim3(kSortThreads), 0, stream,
                         kin, vin, count, shift, scratch, nblocks, kout, vout);
    else
      hipLaunchKernelGGL((k_radix_scatter<2 * kSortThreads, kSortRows / 2, V>), dim3(nblocks),
                         dim3(2 * kSortThreads), 0, stream, kin, vin, count, shift, scratch, nblocks, kout, vout);
    u64* t = kin; kin = kout; kout = t;
    V* tv = vin; vin = vout; vout = tv;
  }
  if (out_keys && out_vals) {
    *out_keys = kin;
    *out_vals = vin;
    return hipGetLastError();
  }
  if (kin != keys) {
    hipError_t e = hipMemcpyAsync(keys, kin, count * sizeof(u64), hipMemcpyDeviceToDevice, stream);
    if constexpr (!std::is_same<V, NoVal>::value)
      if (e == hipSuccess && vals)
        e = hipMemcpyAsync(vals, vin, count * sizeof(V), hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t radix_sort_pairs(u64* keys, u64* vals, u64* tmp_keys, u64* tmp_vals, u64 count,
                            int key_bits, u64* scratch, u64 scratch_elems, hipStream_t stream,
                            u64** out_keys, u64** out_vals) {
  return radix_sort_impl<u64>(keys, vals, tmp_keys, tmp_vals, count, key_bits, scratch, scratch_elems,
                              stream, out_keys, out_vals);
}

hipError_t radix_sort_keys(u64* keys, u64* tmp_keys, u64 count, int key_bits, u64* scratch,
                           u64 scratch_elems, hipStream_t stream, u64** out_keys) {
  NoVal* none = nullptr;
  NoVal* out_none = nullptr;
  return radix_sort_impl<NoVal>(keys, none, tmp_keys, none, count, key_bits, scratch, scratch_elems, stream,
                                out_keys, out_keys ? &out_none : nullptr);
}

hipError_t radix_sort_pairs32(u64* keys, unsigned* vals, u64* tmp_keys, unsigned* tmp_vals, u64 count,
                              int key_bits, u64* scratch, u64 scratch_elems, hipStream_t stream,
                              u64** out_keys, unsigned** out_vals) {
  return radix_sort_impl<unsigned>(keys, vals, tmp_keys, tmp_vals, count, key_bits, scratch,
                                   scratch_elems, stream, out_keys, out_vals);
}

// ---------------------------------------------------------------- compaction
// Per-tile counts of alive entries, scan, then an order-preserving scatter.
__global__ void __launch_bounds__(kSortThreads)
k_alive_count(const double* __restrict__ amps, u64 n, u64* __restrict__ counts) {
  __shared__ unsigned c;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  const u64 base = (u64)blockIdx.x * kSortTile;
  unsigned mine = 0;
  for (int r = 0; r < kSortRows; ++r) {
    const u64 i = base + (u64)r * kSortThreads + threadIdx.x;
    if (i < n && !is_dead(amps[i])) ++mine;
  }
  atomicAdd(&c, mine);
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = c;
}

__global__ void __launch_bounds__(kSortThreads)
k_alive_scatter(const u64* __restrict__ keys, const double* __restrict__ amps,
                const double* __restrict__ vals, u64 n, const u64* __restrict__ offsets,
                u64* __restrict__ out_keys,
                double* __restrict__ out_amps, u64* __restrict__ d_count, int nblocks) {
  __shared__ unsigned wave_cnt[4];
  __shared__ unsigned running;
  const int lane = __lane_id();
  const int wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) running = 0;
  const u64 base = (u64)blockIdx.x * kSortTile;
  const u64 off = offsets[blockIdx.x];
  for (int r = 0; r < kSortRows; ++r) {
    const u64 i = base + (u64)r * kSortThreads + threadIdx.x;
    const bool keep = i < n && !is_dead(amps[i]);
    const u64 m = __ballot(keep);
    if (lane == 0) wave_cnt[wave] = (unsigned)__popcll(m);
    __syncthreads();
    if (keep) {
      unsigned pos = running + (unsigned)__popcll(m & ((1ULL << lane) - 1ULL));
      for (int w = 0; w < wave; ++w) pos += wave_cnt[w];
      out_keys[off + pos] = keys[i];
      out_amps[off + pos] = vals[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) running += wave_cnt[0] + wave_cnt[1] + wave_cnt[2] + wave_cnt[3];
    __syncthreads();
  }
  if (blockIdx.x == nblocks - 1 && threadIdx.x == 0) *d_count = off + running;
}

u64 compact_scratch_elems(u64 n) {
  const u64 len = (n + kSortTile - 1) / kSortTile + 1;
  return len + scan_scratch_elems(len);
}

// Alive entries in storage order: keys and vals[i] (vals = amps by default).
hipError_t launch_compact_alive(const DeviceState& st, u64 n, const double* vals, u64* out_keys,
                                double* out_amps, u64* d_count, u64* scratch, u64 scratch_elems,
                                hipStream_t stream) {
  if (!vals) vals = st.amps;
  const int nblocks = (int)((n + kSortTile - 1) / kSortTile);
  if (n == 0) return launch_fill_u32(d_count, 0u, 2, stream);
  if ((u64)nblocks + scan_scratch_elems((u64)nblocks) > scratch_elems) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_alive_count, dim3(nblocks), dim3(kSortThreads), 0, stream, st.amps, n,
                     scratch);
  scan_exclusive(scratch, (u64)nblocks, scratch + nblocks, stream);
  hipLaunchKernelGGL(k_alive_scatter, dim3(nblocks), dim3(kSortThreads), 0, stream, st.keys,
                     st.amps, vals, n, scratch, out_keys, out_amps, d_count, nblocks);
  return hipGetLastError();
}

// ---------------------------------------------------------------- selection
// Order-preserving map of a float to uint32 (larger float -> larger code).
__device__ inline unsigned float_code(float f) {
  const unsigned b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Sort keys for the two selection passes; payloads are the operator indices.
// The LSD sort is stable and inputs are in index order, so ties keep the
// smaller index first.
__global__ void k_select_keys_top(const float* __restrict__ score, long long K, u64* __restrict__ keys,
                                  u64* __restrict__ idx) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < K) {
    keys[i] = (u64)(~float_code(score[i]));  // larger score first
    idx[i] = (u64)i;
  }
}

__global__ void k_select_mark(const u64* __restrict__ idx_sorted, long long take,
                              unsigned char* __restrict__ flags) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < take) flags[idx_sorted[i]] = 1;
}

__global__ void k_select_keys_rand(const uint32_t* __restrict__ rnd,
                                   const unsigned char* __restrict__ flags, long long K,
                                   u64* __restrict__ keys, u64* __restrict__ idx) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < K) {
    keys[i] = ((u64)flags[i] << 32) | (u64)rnd[i];  // already chosen ones last
    idx[i] = (u64)i;
  }
}

__global__ void k_select_clear(unsigned char* flags, long long K) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < K) flags[i] = 0;
}

// Whole selection in one workgroup (pools up to kSelectBlockMax operators).
// Each choice is a radix select of the kth largest 64-bit key, most
// significant 8 bits first: top key = (score order, complemented index), so
// ties go to the smaller index; random key = complement of (rand, index) for
// operators not already chosen and 0 for chosen ones, so the smallest
// (rand, index) pairs rank first.  Keys are distinct, so after eight passes
// the prefix is the kth largest key itself and "key >= it" selects exactly k.
constexpr long long kSelectBlockMax = 1 << 17;

__device__ inline u64 select_key_top(const float* score, long long k) {
  return ((u64)float_code(score[k]) << 32) | (u64)(0xffffffffu - (unsigned)k);
}

__device__ inline u64 select_key_rand(const uint32_t* rnd, long long k, bool chosen) {
  return chosen ? 0ULL : ~(((u64)rnd[k] << 32) | (u64)(unsigned)k);
}

constexpr int kSelBatch = 8;  // keys in flight per thread in the selection passes

constexpr unsigned kSelCand = 4096;  // candidate keys kept in LDS once few enough remain

struct SelectState {
  u64 prefix, mask;
  unsigned long long remaining;
  int all;        // fewer candidates than requested: every candidate is taken
  int compacted;  // the candidates are in the LDS list
  unsigned ncand;
  unsigned bin;   // count of the chosen digit's bin in the last pass
  unsigned hist[256];
};

// Adds 1 to hist[digit] for every lane with v set; lanes of a wavefront with
// the same digit combine their count into one atomic.  Called by every lane
// of the wavefront.
__device__ inline void hist_add(unsigned* hist, bool v, unsigned dg) {
  u64 peers = __ballot(v);
  if (peers == 0ULL) return;  // uniform over the wavefront
  for (int bit = 0; bit < 8; ++bit) {
    const u64 m = __ballot(v && ((dg >> bit) & 1u));
    peers &= ((dg >> bit) & 1u) ? m : ~m;
  }
  if (v && (peers & ((1ULL << __lane_id()) - 1ULL)) == 0ULL) atomicAdd(&hist[dg], (unsigned)__popcll(peers));
}

// Radix select over keys produced by key_of(k): the kth largest key (or 0
// when there are fewer than kth keys).  Eight 8-bit digit passes from the
// top; the keys are read through key_of until the chosen bin holds at most
// kSelCand keys, which are then copied to an LDS list that the remaining
// passes read instead.  Every thread of the block calls it.
template <class KeyOf>
__device__ u64 block_radix_select(long long K, unsigned long long kth, KeyOf key_of,
                                  SelectState& st, u64* cand) {
  __syncthreads();  // every thread has read the previous call's result
  if (threadIdx.x == 0) {
    st.prefix = 0;
    st.mask = 0;
    st.remaining = kth;
    st.all = 0;
    st.compacted = 0;
    st.ncand = 0;
  }
  __syncthreads();
  for (int d = 7; d >= 0; --d) {
    if (threadIdx.x < 256) st.hist[threadIdx.x] = 0;
    __syncthreads();
    if (!st.all) {
      const u64 prefix = st.prefix, mask = st.mask;
      if (st.compacted) {
        const unsigned nc = st.ncand;
        for (unsigned i = threadIdx.x; i < nc; i += blockDim.x) {
          const u64 key = cand[i];
          if ((key & mask) == prefix) atomicAdd(&st.hist[(unsigned)(key >> (8 * d)) & 255u], 1u);
        }
      } else {
        // kSelBatch keys per thread are loaded before any is counted
        for (long long k0 = threadIdx.x; k0 < K; k0 += (long long)kSelBatch * blockDim.x) {
          u64 key[kSelBatch];
#pragma unroll
          for (int j = 0; j < kSelBatch; ++j) {
            const long long k = k0 + (long long)j * blockDim.x;
            key[j] = key_of(k < K ? k : K - 1);  // clamped: no branch between the loads
          }
#pragma unroll
          for (int j = 0; j < kSelBatch; ++j) {
            const long long k = k0 + (long long)j * blockDim.x;
            hist_add(st.hist, k < K && (key[j] & mask) == prefix, (unsigned)(key[j] >> (8 * d)) & 255u);
          }
        }
      }
    }
    __syncthreads();
    if (threadIdx.x < 64 && !st.all) {
      // lane l holds bins 255-4l .. 252-4l (descending); wavefront prefix sums
      const int l = (int)threadIdx.x;
      unsigned b[4], sum = 0;
      for (int q = 0; q < 4; ++q) {
        b[q] = st.hist[255 - 4 * l - q];
        sum += b[q];
      }
      unsigned long long incl = sum;
      for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long v = __shfl_up(incl, off);
        if (l >= off) incl += v;
      }
      const unsigned long long need = st.remaining;
      const u64 hit = __ballot(incl >= need);
      if (hit == 0ULL) {
        if (l == 0) st.all = 1;
      } else if (l == __ffsll((long long)hit) - 1) {
        unsigned long long cum = incl - sum;
        for (int q = 0; q < 4; ++q) {
          if (cum + b[q] >= need) {
            const u64 digit = (u64)(255 - 4 * l - q);
            st.prefix |= digit << (8 * d);
            st.mask |= 255ULL << (8 * d);
            st.remaining = need - cum;
            st.bin = b[q];
            break;
          }
          cum += b[q];
        }
      }
    }
    __syncthreads();
    if (d > 0 && !st.all && !st.compacted && st.bin <= kSelCand) {
      // copy the keys of the chosen bin to the LDS list
      const u64 prefix = st.prefix, mask = st.mask;
      for (long long k0 = threadIdx.x; k0 < K; k0 += (long long)kSelBatch * blockDim.x) {
        u64 key[kSelBatch];
#pragma unroll
        for (int j = 0; j < kSelBatch; ++j) {
          const long long k = k0 + (long long)j * blockDim.x;
          key[j] = key_of(k < K ? k : K - 1);  // clamped: no branch between the loads
        }
#pragma unroll
        for (int j = 0; j < kSelBatch; ++j) {
          const long long k = k0 + (long long)j * blockDim.x;
          const bool v = k < K && (key[j] & mask) == prefix;
          const u64 m = __ballot(v);
          if (m == 0ULL) continue;  // uniform over the wavefront
          const int leader = __ffsll((long long)m) - 1;
          unsigned base = 0;
          if (__lane_id() == leader) base = atomicAdd(&st.ncand, (unsigned)__popcll(m));
          base = __shfl(base, leader);
          if (v) cand[base + (unsigned)__popcll(m & ((1ULL << __lane_id()) - 1ULL))] = key[j];
        }
      }
      __syncthreads();
      if (threadIdx.x == 0) st.compacted = 1;
      __syncthreads();
    }
  }
  return st.all ? 0ULL : st.prefix;
}

__global__ void __launch_bounds__(1024)
k_select_block(const float* __restrict__ score, const uint32_t* __restrict__ rnd, long long K,
               long long n_top, long long n_rand, int* __restrict__ idx) {
  __shared__ SelectState st;
  __shared__ unsigned long long part[1024];
  __shared__ u64 cand[kSelCand];
  const u64 t_top = (n_top > 0)
      ? block_radix_select(K, (unsigned long long)n_top, [&](long long k) { return select_key_top(score, k); }, st, cand)
      : ~0ULL;
  const bool top_none = (n_top == 0);
  auto chosen_top = [&](long long k) { return !top_none && select_key_top(score, k) >= t_top; };
  const u64 t_rand = (n_rand > 0)
      ? block_radix_select(K, (unsigned long long)n_rand,
                           [&](long long k) { return select_key_rand(rnd, k, chosen_top(k)); }, st, cand)
      : ~0ULL;
  auto chosen = [&](long long k) {
    if (chosen_top(k)) return true;
    return n_rand > 0 && select_key_rand(rnd, k, false) >= t_rand && t_rand != 0ULL;
  };
  // ascending output: contiguous index ranges per thread (at most 128
  // entries, K <= kSelectBlockMax), flags evaluated kSelBatch at a time into
  // two 64-bit masks, block scan of counts
  const long long per = (K + blockDim.x - 1) / blockDim.x;
  const long long lo = (long long)threadIdx.x * per;
  const long long hi = (lo + per < K) ? lo + per : K;
  u64 f0 = 0, f1 = 0;
  unsigned long long cnt = 0;
  for (long long j0 = 0; j0 < per; j0 += kSelBatch) {
    bool c[kSelBatch];
#pragma unroll
    for (int j = 0; j < kSelBatch; ++j) c[j] = (lo + j0 + j < hi) && chosen(lo + j0 + j);
#pragma unroll
    for (int j = 0; j < kSelBatch; ++j) {
      if (!c[j]) continue;
      const long long jj = j0 + j;
      if (jj < 64) f0 |= 1ULL << jj;
      else f1 |= 1ULL << (jj - 64);
      ++cnt;
    }
  }
  part[threadIdx.x] = cnt;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const unsigned long long v = (threadIdx.x >= (unsigned)off) ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  long long pos = (long long)(part[threadIdx.x] - cnt);
  while (f0) {
    idx[pos++] = (int)(lo + __ffsll((long long)f0) - 1);
    f0 &= f0 - 1;
  }
  while (f1) {
    idx[pos++] = (int)(lo + 64 + __ffsll((long long)f1) - 1);
    f1 &= f1 - 1;
  }
}

// Ascending list of flagged indices: per-tile counts, scan, ordered scatter.
__global__ void __launch_bounds__(kSortThreads)
k_flag_count(const unsigned char* __restrict__ flags, long long K, u64* __restrict__ counts) {
  __shared__ unsigned c;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  const u64 base = (u64)blockIdx.x * kSortTile;
  unsigned mine = 0;
  for (int r = 0; r < kSortRows; ++r) {
    const u64 i = base + (u64)r * kSortThreads + threadIdx.x;
    if (i < (u64)K && flags[i]) ++mine;
  }
  atomicAdd(&c, mine);
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = c;
}

__global__ void __launch_bounds__(kSortThreads)
k_flag_scatter(const unsigned char* __restrict__ flags, long long K, const u64* __restrict__ offsets,
               int* __restrict__ idx) {
  __shared__ unsigned wave_cnt[4];
  __shared__ unsigned running;
  const int lane = __lane_id();
  const int wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) running = 0;
  const u64 base = (u64)blockIdx.x * kSortTile;
  const u64 off = offsets[blockIdx.x];
  for (int r = 0; r < kSortRows; ++r) {
    const u64 i = base + (u64)r * kSortThreads + threadIdx.x;
    const bool f = i < (u64)K && flags[i];
    const u64 m = __ballot(f);
    if (lane == 0) wave_cnt[wave] = (unsigned)__popcll(m);
    __syncthreads();
    if (f) {
      unsigned pos = running + (unsigned)__popcll(m & ((1ULL << lane) - 1ULL));
      for (int w = 0; w < wave; ++w) pos += wave_cnt[w];
      idx[off + pos] = (int)i;
    }
    __syncthreads();
    if (threadIdx.x == 0) running += wave_cnt[0] + wave_cnt[1] + wave_cnt[2] + wave_cnt[3];
    __syncthreads();
  }
}

u64 select_scratch_elems(long long K) {
  // keys, idx, tmp keys, tmp idx, flags (bytes, rounded up), sort scratch
  return 4 * (u64)K + ((u64)K + 7) / 8 + radix_sort_scratch_elems((u64)K) + 8;
}

hipError_t launch_select(const float* score, const uint32_t* rnd, long long K, long long n_top,
                         long long n_rand, int* idx, u64* scratch, u64 scratch_elems,
                         hipStream_t stream) {
  if (K <= kSelectBlockMax) {
    hipLaunchKernelGGL(k_select_block, dim3(1), dim3(1024), 0, stream, score, rnd, K, n_top, n_rand,
                       idx);
    return hipGetLastError();
  }
  if (scratch_elems < select_scratch_elems(K)) return hipErrorInvalidValue;
  u64* keys = scratch;
  u64* ids = scratch + K;
  u64* tk = scratch + 2 * K;
  u64* ti = scratch + 3 * K;
  unsigned char* flags = (unsigned char*)(scratch + 4 * K);
  u64* hist = scratch + 4 * K + (K + 7) / 8;
  const u64 hist_elems = radix_sort_scratch_elems((u64)K);
  const unsigned g = (unsigned)((K + 255) / 256);
  hipLaunchKernelGGL(k_select_clear, dim3(g), dim3(256), 0, stream, flags, K);
  if (n_top > 0) {
    hipLaunchKernelGGL(k_select_keys_top, dim3(g), dim3(256), 0, stream, score, K, keys, ids);
    hipError_t e = radix_sort_pairs(keys, ids, tk, ti, (u64)K, 32, hist, hist_elems, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_select_mark, dim3((unsigned)((n_top + 255) / 256)), dim3(256), 0, stream,
                       ids, n_top, flags);
  }
  if (n_rand > 0) {
    hipLaunchKernelGGL(k_select_keys_rand, dim3(g), dim3(256), 0, stream, rnd, flags, K, keys, ids);
    hipError_t e = radix_sort_pairs(keys, ids, tk, ti, (u64)K, 33, hist, hist_elems, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_select_mark, dim3((unsigned)((n_rand + 255) / 256)), dim3(256), 0, stream,
                       ids, n_rand, flags);
  }
  const int nblocks = (int)((K + kSortTile - 1) / kSortTile);
  hipLaunchKernelGGL(k_flag_count, dim3(nblocks), dim3(kSortThreads), 0, stream, flags, K, hist);
  hipLaunchKernelGGL(k_scan_exclusive, dim3(1), dim3(1024), 0, stream, hist, (u64)nblocks);
  hipLaunchKernelGGL(k_flag_scatter, dim3(nblocks), dim3(kSortThreads), 0, stream, flags, K, hist,
                     idx);
  return hipGetLastError();
}

}  // namespace swcs

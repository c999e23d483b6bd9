// segmented.hip -- sort many independent segments (sort_segmented).
//
// The scatter and sorting phases of the paper's method (Section 3.2,
// Figure 1 steps 3-9) for many lists at once: every segment of the input is
// sorted on its own, stably, and nothing crosses a segment boundary.  The
// host never reads the segment offsets, so one call is the same four
// launches whatever the number and sizes of the segments: three small
// planning launches whose cost does not grow with the keys, then one
// persistent sort launch that does all the sorting:
//
//   1. plan (count, base, fill): segment lengths -> size classes (floor
//      log2) -> a work list of the non-empty segments, largest class first,
//      so the longest segments start first (longest-processing-time order);
//   2. sort (persistent workgroups): each workgroup takes the next segment
//      of the work list from an atomic counter.  Segments of fewer than 1,024
//      keys are taken eight at a time, one per wave, and each wave sorts its
//      segment alone in its slice of LDS.  A segment of at most one tile
//      (8,192 keys) is read once, sorted entirely in LDS by the workgroup
//      (every digit pass a stable reorder by two 4-bit splits, ms_tile.hpp)
//      and written once.  A longer segment is read once for the digit histograms of every
//      pass; then each non-constant digit pass streams the segment tile by
//      tile, reordering each tile in LDS and writing its digit runs at
//      running per-digit offsets kept in LDS.  One workgroup owns the
//      segment, so no cross-workgroup look-back is needed.
#include <algorithm>

#include "ms_device.hpp"
#include "ms_runtime.hpp"
#include "ms_tile.hpp"

namespace ms {
namespace {

template <int THREADS>
struct SegCfg {
  static constexpr int kThreads = THREADS;
  static constexpr int kKpt = 16;
  static constexpr int kTile = kThreads * kKpt;
};
constexpr int kSegThreads = 512;
constexpr int kPersistentBlocks = 1024;
constexpr int kClasses = 64;
constexpr int kTinyClass = 9;  // floor(log2 len) <= 9: fewer than 1,024 keys, one wave
constexpr int kTinyKeys = kWave * 16;

__device__ __forceinline__ uint64_t seg_len(const uint64_t* off, uint64_t s, uint64_t n, uint64_t* begin) {
  uint64_t b = off[s], e = off[s + 1];
  b = b < n ? b : n;
  e = e < n ? e : n;
  *begin = b;
  return e > b ? e - b : 0;
}

// 1. plan: work list of non-empty segments, largest size class first, in
//    three launches over all segments at once (plan blocks b = 0 .. G-1 take
//    segments b*1024 + t, stepping by G*1024, in 1a and 1c alike).
//    ctr[0] = next work item (reset to 0), ctr[1] = number of work items,
//    ctr[2] = first item of the wave-sized class (ctr[3] unused).
constexpr uint32_t kPlanMaxBlocks = 1024;

__device__ __forceinline__ int seg_class(const uint64_t* off, uint64_t s, uint64_t nseg, uint64_t n) {
  if (s >= nseg) return -1;
  uint64_t b;
  const uint64_t len = seg_len(off, s, n, &b);
  return len ? 63 - __builtin_clzll(len) : -1;  // floor(log2 len); -1: empty
}

// 1a. row b of `bc`: how many of plan block b's segments fall in each class.
__global__ __launch_bounds__(1024) void seg_count_kernel(const uint64_t* __restrict__ off, uint64_t nseg,
                                                         uint64_t n, uint32_t* bc) {
  __shared__ uint32_t s_count[kClasses];
  const int tid = threadIdx.x;
  if (tid < kClasses) s_count[tid] = 0;
  __syncthreads();
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * 1024;
  for (uint64_t s = static_cast<uint64_t>(blockIdx.x) * 1024 + tid; s < nseg; s += stride) {
    const int c = seg_class(off, s, nseg, n);
    if (c >= 0) atomicAdd(&s_count[c], 1u);
  }
  __syncthreads();
  if (tid < kClasses) bc[static_cast<size_t>(blockIdx.x) * kClasses + tid] = s_count[tid];
}

// 1b. (one block of kClasses threads) the first work-list slot of every
// (plan block, class): classes largest first, blocks in order within a class.
__global__ __launch_bounds__(kClasses) void seg_base_kernel(const uint32_t* __restrict__ bc, uint32_t nblocks,
                                                            uint32_t* boff, uint32_t* ctr) {
  __shared__ uint32_t s_total[kClasses];
  __shared__ uint32_t s_first[kClasses];
  const int c = threadIdx.x;
  uint32_t total = 0;
  for (uint32_t b = 0; b < nblocks; ++b) total += bc[static_cast<size_t>(b) * kClasses + c];
  s_total[c] = total;
  __syncthreads();
  if (c == 0) {
    uint32_t run = 0, tiny_begin = 0;
    for (int k = kClasses - 1; k >= 0; --k) {
      if (k == kTinyClass) tiny_begin = run;
      s_first[k] = run;
      run += s_total[k];
    }
    ctr[0] = 0;
    ctr[1] = run;
    ctr[2] = tiny_begin;
    ctr[3] = tiny_begin;
  }
  __syncthreads();
  uint32_t run = s_first[c];
  for (uint32_t b = 0; b < nblocks; ++b) {
    boff[static_cast<size_t>(b) * kClasses + c] = run;
    run += bc[static_cast<size_t>(b) * kClasses + c];
  }
}

// 1c. plan block b writes its segments from its slots on (any order within a
// block: segments are sorted independently).
__global__ __launch_bounds__(1024) void seg_fill_kernel(const uint64_t* __restrict__ off, uint64_t nseg,
                                                        uint64_t n, const uint32_t* __restrict__ boff,
                                                        uint32_t* worklist) {
  __shared__ uint32_t s_next[kClasses];
  const int tid = threadIdx.x;
  if (tid < kClasses) s_next[tid] = boff[static_cast<size_t>(blockIdx.x) * kClasses + tid];
  __syncthreads();
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * 1024;
  for (uint64_t s = static_cast<uint64_t>(blockIdx.x) * 1024 + tid; s < nseg; s += stride) {
    const int c = seg_class(off, s, nseg, n);
    if (c >= 0) worklist[atomicAdd(&s_next[c], 1u)] = static_cast<uint32_t>(s);
  }
}

// Blocked load of up to one tile: thread t gets positions t*16 .. t*16+15 of
// [base, base + valid); positions past `valid` get all-ones keys (they sort
// after every real key) and zero values.
template <typename K, bool VALS, int KPT>
__device__ __forceinline__ void load_blocked(const K* src, const uint32_t* srcv, uint64_t base, int valid, K in_flip,
                                             K (&keys)[KPT], uint32_t (&vals)[KPT]) {
  const int first = threadIdx.x * KPT;
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const int idx = first + j;
    keys[j] = idx < valid ? flip_key(src[base + idx], in_flip) : ~K(0);
    if constexpr (VALS) vals[j] = idx < valid ? srcv[base + idx] : 0u;
  }
}

// Bits in which the first `valid` keys of a blocked tile differ from k0
// (block-wide OR), as two 32-bit halves in `s_diff`.  Contains barriers.
template <typename K, int KPT>
__device__ __forceinline__ uint64_t tile_diff_bits(const K (&keys)[KPT], int valid, K k0, uint32_t* s_diff) {
  if (threadIdx.x < 2) s_diff[threadIdx.x] = 0;
  __syncthreads();
  K diff = 0;
#pragma unroll
  for (int j = 0; j < KPT; ++j)
    if (static_cast<int>(threadIdx.x) * KPT + j < valid) diff |= keys[j] ^ k0;
  if (static_cast<uint32_t>(diff)) atomicOr(&s_diff[0], static_cast<uint32_t>(diff));
  if constexpr (sizeof(K) == 8)
    if (static_cast<uint32_t>(diff >> 32)) atomicOr(&s_diff[1], static_cast<uint32_t>(diff >> 32));
  __syncthreads();
  const uint64_t d = (static_cast<uint64_t>(s_diff[1]) << 32) | s_diff[0];
  __syncthreads();
  return d;
}

// A segment of at most one key per lane sorted by one wave with a bitonic
// network (Batcher's sorting network for 64 inputs: log2(64) merge levels,
// 21 compare-exchange stages, each a lane exchange).  Every lane carries its
// key (encoded), its input position and its value; items are ordered by
// (key, position), so equal keys keep their input order and the result is
// the stable sort.  Lanes past the segment hold the largest key with
// positions past it: they end last.
template <typename K, bool VALS>
__device__ __forceinline__ void wave_bitonic_sort(K& key, uint32_t& pos, uint32_t& val) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (uint32_t k = 2; k <= static_cast<uint32_t>(kWave); k <<= 1) {
#pragma unroll
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      const K ok = __shfl_xor(key, static_cast<int>(j), kWave);
      const uint32_t op = __shfl_xor(pos, static_cast<int>(j), kWave);
      uint32_t ov = 0;
      if constexpr (VALS) ov = __shfl_xor(val, static_cast<int>(j), kWave);
      const bool ascending = (lane & k) == 0;  // this run of k lanes is sorted upwards
      const bool lower = (lane & j) == 0;      // this lane is the lower of its pair
      const bool other_less = ok < key || (ok == key && op < pos);
      // The lower lane keeps the smaller item of an ascending run, the larger
      // of a descending one; the upper lane the other.
      if (lower == ascending ? other_less : !other_less) {
        key = ok;
        pos = op;
        if constexpr (VALS) val = ov;
      }
    }
  }
}

// 2. sort: persistent workgroups over the work list.  32-bit keys without
// values fit two 512-thread workgroups per CU (4 waves per SIMD, at most 128
// VGPRs), which the long segments' streaming needs to hide its memory
// latency; the compiler is held to that (the launch bound's second argument
// is the minimum number of waves per SIMD).
template <typename K, bool VALS>
constexpr int seg_min_waves_per_simd() {
  return sizeof(K) == 4 && !VALS ? 4 : 1;
}

template <typename K, bool VALS, int THREADS>
__global__ __launch_bounds__(THREADS, (seg_min_waves_per_simd<K, VALS>())) void segmented_kernel(const K* kin, const uint32_t* vin, K* kout,
                                                             uint32_t* vout, K* alt_k, uint32_t* alt_v,
                                                             const uint64_t* __restrict__ off, uint64_t n_total,
                                                             K flip, const uint32_t* __restrict__ worklist,
                                                             uint32_t* ctr, int small_limit) {
  constexpr int kKpt = SegCfg<THREADS>::kKpt;
  constexpr int kTile = SegCfg<THREADS>::kTile;
  constexpr int P = sizeof(K);
  constexpr int kStageBytes = padded16(kTile) * static_cast<int>(sizeof(K));
  constexpr int kCountBytes = SplitScratch<THREADS>::kCountWords * 4;
  __shared__ __attribute__((aligned(16))) uint8_t s_raw[kStageBytes > kCountBytes ? kStageBytes : kCountBytes];
  K* s_stage = reinterpret_cast<K*>(s_raw);
  uint32_t* s_counts = reinterpret_cast<uint32_t*>(s_raw);
  __shared__ uint32_t s_vstage[VALS ? padded16(kTile) : 1];
  __shared__ uint32_t s_hist[P][kRadix];  // segment digit counts of every pass
  __shared__ uint32_t s_thist[kRadix];    // tile digit counts
  __shared__ uint32_t s_run[kRadix];      // segment position of the next key of each digit
  __shared__ uint32_t s_doff[kRadix];     // s_run - tile start, per digit (mod 2^32)
  __shared__ uint32_t s_scan[THREADS / kWave];
  __shared__ uint32_t s_cscan[kRadix / kWave];
  __shared__ uint32_t s_diff[2];
  __shared__ uint32_t s_item;

  __shared__ uint32_t s_mode;
  const int tid = threadIdx.x;
  const bool inplace = kin == kout;
  K keys[kKpt];
  uint32_t vals[kKpt];
  constexpr int kWaves = THREADS / kWave;

  while (true) {
    __syncthreads();
    if (tid == 0) {
      const uint32_t i = atomicAdd(&ctr[0], 1u);
      s_item = i;
      s_mode = i < ctr[2] ? 0 : 1;
    }
    __syncthreads();
    const uint32_t item = s_item;
    if (s_mode == 1) {
      // Only wave-sized segments are left: every wave of the grid takes every
      // (grid waves)-th of them on its own, with no atomics (one counter would
      // queue every wave on one address) and no block barrier from here on.
      const uint32_t nwaves = gridDim.x * kWaves;
      for (uint32_t mine = ctr[2] + blockIdx.x * kWaves + tid / kWave; mine < ctr[1]; mine += nwaves) {
        uint64_t begin;
        const uint64_t len = seg_len(off, worklist[mine], n_total, &begin);
        const int valid = static_cast<int>(len);  // 1 .. kTinyKeys - 1
        const uint32_t lane = lane_id();
        if (valid <= small_limit) {  // wave-uniform: one segment per wave
          const bool mine_real = static_cast<int>(lane) < valid;
          K key = mine_real ? flip_key(kin[begin + lane], flip) : ~K(0);
          uint32_t pos = lane;
          uint32_t val = 0;
          if constexpr (VALS) val = mine_real ? vin[begin + lane] : 0u;
          wave_bitonic_sort<K, VALS>(key, pos, val);
          if (mine_real) {
            kout[begin + lane] = flip_key(key, flip);
            if constexpr (VALS) vout[begin + lane] = val;
          }
          continue;
        }
        const int wave = tid / kWave;
        K* wk = s_stage + wave * padded16(kTinyKeys);
        uint32_t* wv = s_vstage + (VALS ? wave * padded16(kTinyKeys) : 0);
        uint32_t* wc = reinterpret_cast<uint32_t*>(wk);
#pragma unroll
        for (int j = 0; j < kKpt; ++j) {
          const int idx = static_cast<int>(lane) * kKpt + j;
          keys[j] = idx < valid ? flip_key(kin[begin + idx], flip) : ~K(0);
          if constexpr (VALS) vals[j] = idx < valid ? vin[begin + idx] : 0u;
        }
        // bits in which the wave's real keys differ (wave-wide OR)
        const K k0 = flip_key(kin[begin], flip);
        K d = 0;
#pragma unroll
        for (int j = 0; j < kKpt; ++j)
          if (static_cast<int>(lane) * kKpt + j < valid) d |= keys[j] ^ k0;
        uint64_t diff = static_cast<uint64_t>(d);
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) diff |= __shfl_xor(diff, o, kWave);
        for (int p = 0; p < P; ++p) {
          if (((diff >> (8 * p)) & (kRadix - 1)) == 0) continue;  // uniform across the wave
          wave_sort_digit<kKpt, VALS>(keys, vals, 8 * p, wk, wv, wc);
        }
#pragma unroll
        for (int j = 0; j < kKpt; ++j) {
          const int idx = static_cast<int>(lane) * kKpt + j;
          if (idx < valid) {
            kout[begin + idx] = flip_key(keys[j], flip);
            if constexpr (VALS) vout[begin + idx] = vals[j];
          }
        }
      }
      return;
    }
    if (item >= ctr[1]) return;
    uint64_t begin;
    const uint64_t len = seg_len(off, worklist[item], n_total, &begin);
    if (len == 0) continue;
    const K k0 = flip_key(kin[begin], flip);

    if (len <= static_cast<uint64_t>(kTile)) {
      // ---- short segment: every pass in LDS ----
      const int valid = static_cast<int>(len);
      load_blocked<K, VALS>(kin, vin, begin, valid, flip, keys, vals);
      const uint64_t diff = tile_diff_bits(keys, valid, k0, s_diff);
      for (int p = 0; p < P; ++p) {
        if (((diff >> (8 * p)) & (kRadix - 1)) == 0) continue;  // same for the whole block
        tile_sort_digit<THREADS, kKpt, VALS>(keys, vals, 8 * p, s_stage, s_vstage, s_counts, s_scan, true);
      }
#pragma unroll
      for (int j = 0; j < kKpt; ++j) {
        const int idx = tid * kKpt + j;
        if (idx < valid) {
          kout[begin + idx] = flip_key(keys[j], flip);
          if constexpr (VALS) vout[begin + idx] = vals[j];
        }
      }
      continue;
    }

    // ---- long segment: one read for all histograms, then tile-streamed passes ----
    for (int i = tid; i < P * kRadix; i += THREADS) (&s_hist[0][0])[i] = 0;
    if (tid < 2) s_diff[tid] = 0;
    __syncthreads();
    {
      K diff = 0;
      for (uint64_t i = tid; i < len; i += THREADS) {
        const K k = flip_key(kin[begin + i], flip);
        diff |= k ^ k0;
#pragma unroll
        for (int p = 0; p < P; ++p) atomicAdd(&s_hist[p][digit_of(k, 8 * p)], 1u);
      }
      if (static_cast<uint32_t>(diff)) atomicOr(&s_diff[0], static_cast<uint32_t>(diff));
      if constexpr (sizeof(K) == 8)
        if (static_cast<uint32_t>(diff >> 32)) atomicOr(&s_diff[1], static_cast<uint32_t>(diff >> 32));
    }
    __syncthreads();
    const uint64_t all_diff = (static_cast<uint64_t>(s_diff[1]) << 32) | s_diff[0];
    int m = 0;
    for (int p = 0; p < P; ++p) m += ((all_diff >> (8 * p)) & (kRadix - 1)) != 0;

    const K* src = kin;
    const uint32_t* srcv = vin;
    int e = 0;
    for (int p = 0; p < P; ++p) {
      const int shift = 8 * p;
      if (((all_diff >> shift) & (kRadix - 1)) == 0) continue;
      // The last executed pass lands in the output; in place, the first
      // executed pass must not write the array it reads.
      const bool to_out = inplace ? (e % 2 == 1) : ((m - 1 - e) % 2 == 0);
      K* dst = to_out ? kout : alt_k;
      uint32_t* dstv = to_out ? vout : alt_v;
      const K out_flip = (e == m - 1) ? flip : K(0);
      const K in_flip = (e == 0) ? flip : K(0);  // intermediate buffers hold encoded keys

      uint32_t total;
      const uint32_t base = block_exclusive_scan_radix<THREADS>(tid < kRadix ? s_hist[p][tid] : 0u, s_cscan, &total);
      if (tid < kRadix) s_run[tid] = base;

      // The next tile's keys are loaded into the registers the sorted tile
      // has left, so that they arrive while this tile is scattered; barriers
      // inside the loop guard LDS only and do not wait for those loads.
      auto tile_valid = [&](uint64_t t) {
        const uint64_t rem = len - t;
        return rem < static_cast<uint64_t>(kTile) ? static_cast<int>(rem) : kTile;
      };
      load_blocked<K, VALS>(src, srcv, begin, tile_valid(0), in_flip, keys, vals);
      for (uint64_t t0 = 0; t0 < len; t0 += kTile) {
        const int valid = tile_valid(t0);
        for (int d = tid; d < kRadix; d += THREADS) s_thist[d] = 0;
        lds_barrier();
#pragma unroll
        for (int j = 0; j < kKpt; ++j) {
          const uint32_t d = digit_of(keys[j], shift);
          const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
          if (__builtin_amdgcn_ballot_w64(d == d0) == ~0ull) {
            if (lane_id() == 0) atomicAdd(&s_thist[d0], static_cast<uint32_t>(kWave));
          } else {
            atomicAdd(&s_thist[d], 1u);
          }
        }
        lds_barrier();
        const uint32_t cnt = tid < kRadix ? s_thist[tid] : 0u;
        tile_sort_digit<THREADS, kKpt, VALS>(keys, vals, shift, s_stage, s_vstage, s_counts, s_scan, false);
        if (t0 + kTile < len) load_blocked<K, VALS>(src, srcv, begin + t0 + kTile, tile_valid(t0 + kTile), in_flip,
                                                    keys, vals);
        uint32_t tile_total;
        const uint32_t start = block_exclusive_scan_radix<THREADS>(cnt, s_cscan, &tile_total);
        if (tid < kRadix) s_doff[tid] = s_run[tid] - start;
        lds_barrier();
        // Destinations stay inside the segment whenever the offsets keep the
        // contract; the clamp keeps overlapping segments (rewritten by other
        // workgroups between passes) inside their own range.
        for (int i = tid; i < valid; i += THREADS) {
          const K k = s_stage[pad16(i)];
          uint64_t rel = static_cast<uint32_t>(s_doff[digit_of(k, shift)] + static_cast<uint32_t>(i));
          rel = rel < len ? rel : len - 1;
          dst[begin + rel] = k ^ out_flip;
          if constexpr (VALS) dstv[begin + rel] = s_vstage[pad16(i)];
        }
        lds_barrier();
        if (tid < kRadix) s_run[tid] += cnt;
      }
      // This workgroup reads what it just wrote in the next pass.
      __threadfence();
      __syncthreads();
      src = dst;
      srcv = dstv;
      ++e;
    }

    // No pass ran (all keys equal) or the result ended in the workspace.
    const K* csrc = nullptr;
    const uint32_t* csrcv = nullptr;
    if (m == 0 && !inplace) {
      csrc = kin;
      csrcv = vin;
    } else if (m > 0 && inplace && (m % 2 == 1)) {
      csrc = alt_k;
      csrcv = alt_v;
    }
    if (csrc) {
      for (uint64_t i = tid; i < len; i += THREADS) {
        kout[begin + i] = csrc[begin + i];
        if constexpr (VALS) vout[begin + i] = csrcv[begin + i];
      }
    }
  }
}

struct SegLayout {
  size_t ctr = 0, bc = 0, boff = 0, worklist = 0, alt_k = 0, alt_v = 0, total = 0;
  uint32_t plan_blocks = 0;
};

SegLayout seg_layout(ms_key_type kt, bool has_vals, uint64_t n, uint64_t nseg) {
  SegLayout L;
  const uint64_t pb = (nseg + 1023) / 1024;
  L.plan_blocks = static_cast<uint32_t>(pb < kPlanMaxBlocks ? (pb ? pb : 1) : kPlanMaxBlocks);
  size_t off = 0;
  L.ctr = off;
  off += kAlign;
  L.bc = off;
  off += align_up(static_cast<size_t>(L.plan_blocks) * kClasses * sizeof(uint32_t));
  L.boff = off;
  off += align_up(static_cast<size_t>(L.plan_blocks) * kClasses * sizeof(uint32_t));
  L.worklist = off;
  off += align_up(nseg * sizeof(uint32_t));
  L.alt_k = off;
  off += align_up(n * key_bytes(kt));
  if (has_vals) {
    L.alt_v = off;
    off += align_up(n * sizeof(uint32_t));
  }
  L.total = off;
  return L;
}

template <typename K, bool VALS>
ms_status run_segmented(const void* kin, const uint32_t* vin, void* kout, uint32_t* vout, const uint64_t* off,
                        uint64_t nseg, uint64_t n, K flip, char* ws, const SegLayout& L, hipStream_t s) {
  uint32_t* ctr = reinterpret_cast<uint32_t*>(ws + L.ctr);
  uint32_t* worklist = reinterpret_cast<uint32_t*>(ws + L.worklist);
  K* alt_k = reinterpret_cast<K*>(ws + L.alt_k);
  uint32_t* alt_v = VALS ? reinterpret_cast<uint32_t*>(ws + L.alt_v) : nullptr;
  uint32_t* bc = reinterpret_cast<uint32_t*>(ws + L.bc);
  uint32_t* boff = reinterpret_cast<uint32_t*>(ws + L.boff);
  MS_LAUNCH("seg_plan", seg_count_kernel, L.plan_blocks, 1024, s, off, nseg, n, bc);
  MS_LAUNCH("seg_plan", seg_base_kernel, 1, kClasses, s, static_cast<const uint32_t*>(bc), L.plan_blocks, boff, ctr);
  MS_LAUNCH("seg_plan", seg_fill_kernel, L.plan_blocks, 1024, s, off, nseg, n, static_cast<const uint32_t*>(boff),
            worklist);
  int64_t want = tune_get(MS_TUNE_SEG_BLOCKS);
  if (want <= 0) want = kPersistentBlocks;
  const uint32_t blocks = static_cast<uint32_t>(nseg < static_cast<uint64_t>(want) ? nseg : want);
  const int small_limit = static_cast<int>(tune_get(MS_TUNE_SMALL_SORT));  // 0 or kWave
  MS_LAUNCH("seg_sort", (segmented_kernel<K, VALS, kSegThreads>), blocks, kSegThreads, s,
            static_cast<const K*>(kin), vin, static_cast<K*>(kout), vout, alt_k, alt_v, off, n, flip,
            static_cast<const uint32_t*>(worklist), ctr, small_limit);
  return MS_OK;
}

}  // namespace

size_t segmented_workspace_bytes(ms_key_type kt, bool has_vals, uint64_t n, uint64_t nseg) {
  if (nseg == 1) return radix_workspace_bytes(kt, has_vals, n);
  const size_t persistent = seg_layout(kt, has_vals, n, nseg).total;
  // Either path may run (MS_TUNE_SEG_PASSES can change after sizing), so the
  // workspace covers the segment passes whenever a launch per phase could
  // take the call; segments averaging 1,024 - 8,192 keys are covered only
  // when the one-launch queue is selected at sizing time (their per-segment
  // counters cost up to 8 B per key).
  const int mode = static_cast<int>(tune_get(MS_TUNE_SEG_PASSES));
  if (segsweep_eligible(n, nseg, mode == 2 ? 2 : 1))
    return std::max(persistent, segsweep_workspace_bytes(kt, has_vals, n, nseg));
  return persistent;
}

ms_status segmented_sort(const void* keys_in, const uint32_t* vals_in, void* keys_out, uint32_t* vals_out,
                         const uint64_t* offsets, uint64_t nseg, uint64_t n, ms_key_type kt, void* ws,
                         size_t ws_bytes, hipStream_t s) {
  // One segment is the whole list (offsets are {0, n} by contract): the
  // whole-list sort.
  if (nseg == 1) return radix_sort(keys_in, vals_in, keys_out, vals_out, n, kt, ws, ws_bytes, s);
  // Long segments: whole-device digit passes over all of them (a launch per
  // phase from 8,192 keys on average, the one-launch work queue from 1,024;
  // the host knows only the counts, which decide), unless the caller asked
  // for the persistent kernel with one workgroup per segment.
  const int seg_passes = static_cast<int>(tune_get(MS_TUNE_SEG_PASSES));
  if (seg_passes && segsweep_eligible(n, nseg, seg_passes)) {
    // Segments averaging 1,024 - 8,192 keys go to the queue only with a
    // workspace sized for it; otherwise to the persistent kernel, which is
    // their path by default.
    const bool queue_only = !segsweep_eligible(n, nseg, 1);
    if (!queue_only || ws_bytes >= segsweep_workspace_bytes(kt, vals_in != nullptr, n, nseg))
      return segsweep_sort(keys_in, vals_in, keys_out, vals_out, offsets, nseg, n, kt, ws, ws_bytes, s);
  }
  const bool vals = vals_in != nullptr;
  const SegLayout L = seg_layout(kt, vals, n, nseg);
  if (ws_bytes < L.total || !ws)
    return fail(MS_EINVAL, "sort_segmented: workspace too small: %zu bytes given, %zu needed", ws_bytes, L.total);
  if (nseg > 0x7fffffffull) return fail(MS_ENOTSUP, "sort_segmented: at most 2^31-1 segments per call");
  char* w = static_cast<char*>(ws);
  switch (kt) {
    case MS_KEY_I32:
      return vals ? run_segmented<uint32_t, true>(keys_in, vals_in, keys_out, vals_out, offsets, nseg, n, 0x80000000u, w, L, s)
                  : run_segmented<uint32_t, false>(keys_in, vals_in, keys_out, vals_out, offsets, nseg, n, 0x80000000u, w, L, s);
    case MS_KEY_U32:
      return vals ? run_segmented<uint32_t, true>(keys_in, vals_in, keys_out, vals_out, offsets, nseg, n, 0u, w, L, s)
                  : run_segmented<uint32_t, false>(keys_in, vals_in, keys_out, vals_out, offsets, nseg, n, 0u, w, L, s);
    case MS_KEY_U64:
      return vals ? run_segmented<uint64_t, true>(keys_in, vals_in, keys_out, vals_out, offsets, nseg, n, 0ull, w, L, s)
                  : run_segmented<uint64_t, false>(keys_in, vals_in, keys_out, vals_out, offsets, nseg, n, 0ull, w, L, s);
  }
  return fail(MS_ENOTSUP, "sort_segmented: unknown key type %d", static_cast<int>(kt));
}

}  // namespace ms

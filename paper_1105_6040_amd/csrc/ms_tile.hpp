// ms_tile.hpp -- stable in-LDS reordering of a register-resident tile by
// 4-bit sub-digits, shared by the radix kernels.
//
// Layout: a tile of THREADS * KPT keys is held "blocked": thread t holds tile
// positions t*KPT .. t*KPT+KPT-1 in its registers, in order.  A split by the
// 4 bits at `shift` gives every key its position in the stable order of those
// bits:
//   1. each thread counts its own keys per bucket in one 64-bit register
//      (16 buckets x 4-bit fields), learning for every key how many of its
//      own earlier keys share the bucket -- no LDS traffic, no ballots;
//   2. the per-(bucket, thread) totals go to LDS in bucket-major order and a
//      raking block scan turns them into exclusive prefixes, so the prefix of
//      (bucket b, thread t) counts every key of a smaller bucket plus the
//      keys of bucket b held by threads before t;
//   3. position = prefix[b][t] + own earlier keys of bucket b.  Equal
//      buckets keep thread order, then register order: the split is stable.
// Two splits (low nibble, then high nibble) order a tile by an 8-bit digit.
#pragma once

#include "ms_device.hpp"

namespace ms {

constexpr int kSubBits = 4;
constexpr int kSubBuckets = 1 << kSubBits;

// LDS arrays indexed in runs of 16 get one pad word per 16 entries, so that
// both a wave reading 64 consecutive entries and a wave whose lanes each read
// their own run of 16 hit distinct banks.
__device__ __forceinline__ uint32_t pad16(uint32_t i) { return i + (i >> 4); }
constexpr int padded16(int n) { return n + n / 16; }

// LDS needed by tile_split for a block of THREADS threads (32-bit words).
template <int THREADS>
struct SplitScratch {
  static constexpr int kCountWords = padded16(kSubBuckets * THREADS);
};

// Block-wide exclusive scan of one uint32 per thread; `scratch` holds
// THREADS / 64 words.  Contains a barrier; the caller must pass another one
// before the next call (the scratch is read until then).
template <int THREADS>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* scratch) {
  constexpr int kWaves = THREADS / kWave;
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const uint32_t incl = wave_inclusive_scan(v);
  if ((tid % kWave) == kWave - 1) scratch[wave] = incl;
  lds_barrier();
  uint32_t base = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w)
    if (w < wave) base += scratch[w];
  // No barrier after the reads: the caller meets one before `scratch` is
  // written again.
  return base + incl - v;
}

// Positions of the stable split of a blocked tile by bits [shift, shift+4).
// pos[j] receives the new tile position of key j of this thread.  `counts`
// holds SplitScratch<THREADS>::kCountWords words; `scan` THREADS/64 words.
// Requires KPT <= 16.  Contains barriers; all threads call it.
template <int THREADS, int KPT, typename K>
__device__ __forceinline__ void tile_split_positions(const K (&keys)[KPT], int shift, uint32_t (&pos)[KPT],
                                                     uint32_t* counts, uint32_t* scan) {
  static_assert(KPT <= 16, "4-bit per-thread counters hold at most 15 earlier keys");
  static_assert(THREADS % 16 == 0, "bucket rows of whole pad16 groups");
  const int tid = threadIdx.x;
  // Entry (bucket b, thread t) lives at pad16(b * THREADS + t), which is
  // b * padded16(THREADS) + pad16(t) since THREADS is a multiple of 16: one
  // base per thread plus a constant (or one multiply-add) per bucket.
  constexpr int kRow = padded16(THREADS);
  uint32_t* const column = counts + pad16(tid);

  // 1.  The last key is not counted into c (a bucket holding all KPT keys
  // would overflow its 4-bit field); its count is added in LDS instead.
  uint64_t c = 0;
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const uint32_t sh = (static_cast<uint32_t>(keys[j] >> shift) & (kSubBuckets - 1)) * kSubBits;
    pos[j] = static_cast<uint32_t>(c >> sh) & (kSubBuckets - 1);
    if (j + 1 < KPT) c += 1ull << sh;
  }
  const uint32_t last = static_cast<uint32_t>(keys[KPT - 1] >> shift) & (kSubBuckets - 1);
#pragma unroll
  for (int b = 0; b < kSubBuckets; ++b) column[b * kRow] = static_cast<uint32_t>(c >> (b * kSubBits)) & (kSubBuckets - 1);
  atomicAdd(&column[last * kRow], 1u);  // after this thread's own store to the word (LDS keeps a wave's order)
  lds_barrier();
  uint32_t* row = counts + tid * (kSubBuckets + 1);
  uint32_t v[kSubBuckets];
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < kSubBuckets; ++i) {
    v[i] = row[i];
    sum += v[i];
  }
  uint32_t run = block_exclusive_scan<THREADS>(sum, scan);
#pragma unroll
  for (int i = 0; i < kSubBuckets; ++i) {
    row[i] = run;
    run += v[i];
  }
  lds_barrier();
  // The buckets are extracted again rather than kept from step 1: holding
  // them through the scan would cost KPT registers at the kernel's peak.
  const int shift_again = opaque_uniform(shift);
#pragma unroll
  for (int j = 0; j < KPT; ++j)
    pos[j] += column[(static_cast<uint32_t>(keys[j] >> shift_again) & (kSubBuckets - 1)) * kRow];
  lds_barrier();  // callers may reuse `counts` (it can alias the key stage)
}

// One stable split of a blocked tile by bits [shift, shift+4) through
// `stage_k` (and `stage_v` for values), both indexed through pad16
// (padded16(THREADS * KPT) entries); `counts` may alias stage_k.  On return
// entry pad16(i) of the stage holds the i-th key of the split tile and, if
// `reload` is set, the tile is back in registers in blocked layout.
// Contains barriers.
template <int THREADS, int KPT, bool VALS, typename K>
__device__ __forceinline__ void tile_split_stage(K (&keys)[KPT], uint32_t (&vals)[KPT], int shift, K* stage_k,
                                                 uint32_t* stage_v, uint32_t* counts, uint32_t* scan,
                                                 bool reload) {
  static_assert(KPT == 16, "the blocked reload assumes 16 keys per thread");
  const int tid = threadIdx.x;
  uint32_t pos[KPT];
  tile_split_positions<THREADS, KPT>(keys, shift, pos, counts, scan);
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    stage_k[pad16(pos[j])] = keys[j];
    if constexpr (VALS) stage_v[pad16(pos[j])] = vals[j];
  }
  lds_barrier();
  if (reload) {
    // KPT == 16: pad16(tid * 16 + j) = 17 * tid + j.
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      keys[j] = stage_k[pad16(tid * KPT + j)];
      if constexpr (VALS) vals[j] = stage_v[pad16(tid * KPT + j)];
    }
    lds_barrier();
  }
}

// Full stable reorder of a blocked tile by the 8-bit digit at `shift`: the
// split by the low nibble, then by the high nibble.  On return the tile is in
// digit order in the stage and, if `reload` is set, back in registers in
// blocked layout.  Contains barriers.
template <int THREADS, int KPT, bool VALS, typename K>
__device__ __forceinline__ void tile_sort_digit(K (&keys)[KPT], uint32_t (&vals)[KPT], int shift, K* stage_k,
                                                uint32_t* stage_v, uint32_t* counts, uint32_t* scan, bool reload) {
  tile_split_stage<THREADS, KPT, VALS>(keys, vals, shift, stage_k, stage_v, counts, scan, true);
  tile_split_stage<THREADS, KPT, VALS>(keys, vals, shift + kSubBits, stage_k, stage_v, counts, scan, reload);
}

// Blocked load of the tile starting at `base` (raw bits: the codec is applied
// by the caller once the loads have landed); past the end keys read as `pad`
// and values as 0.
template <typename K, bool VALS, typename C, int KPT>
__device__ __forceinline__ void load_tile_keys(gptr<const K> src, gptr<const uint32_t> src_v, C my_base, C n, K pad,
                                               K (&keys)[KPT], uint32_t (&vals)[KPT]) {
  const bool vec_ok = (reinterpret_cast<uintptr_t>(src + my_base) % 16 == 0) && my_base + KPT <= n;
  if (vec_ok) {
    constexpr int kPer = 16 / sizeof(K);
    gptr<const uint4> p4 = (gptr<const uint4>)(src + my_base);
#pragma unroll
    for (int q = 0; q < KPT / kPer; ++q) {
      const uint4 v = p4[q];
      if constexpr (sizeof(K) == 4) {
        keys[4 * q + 0] = v.x;
        keys[4 * q + 1] = v.y;
        keys[4 * q + 2] = v.z;
        keys[4 * q + 3] = v.w;
      } else {
        keys[2 * q + 0] = (static_cast<uint64_t>(v.y) << 32) | v.x;
        keys[2 * q + 1] = (static_cast<uint64_t>(v.w) << 32) | v.z;
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const C idx = my_base + j;
      keys[j] = idx < n ? src[idx] : pad;
    }
  }
  if constexpr (VALS) {
    const bool vvec = (reinterpret_cast<uintptr_t>(src_v + my_base) % 16 == 0) && my_base + KPT <= n;
    if (vvec) {
      gptr<const uint4> p4 = (gptr<const uint4>)(src_v + my_base);
#pragma unroll
      for (int q = 0; q < KPT / 4; ++q) {
        const uint4 v = p4[q];
        vals[4 * q + 0] = v.x;
        vals[4 * q + 1] = v.y;
        vals[4 * q + 2] = v.z;
        vals[4 * q + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < KPT; ++j) {
        const C idx = my_base + j;
        vals[j] = idx < n ? src_v[idx] : 0u;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The same reorder for one wave on its own (64 lanes x KPT keys): used to sort
// many short lists at once, one per wave.  Lanes exchange data through the
// wave's own LDS slice; the wave executes LDS instructions in order, so a
// wave-scope fence (which also keeps the compiler from reordering) replaces
// the block barrier.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// LDS words of one wave's split counters (aliasing its key stage is fine).
constexpr int kWaveCountWords = padded16(kSubBuckets * kWave);

template <int KPT, typename K>
__device__ __forceinline__ void wave_split_positions(const K (&keys)[KPT], int shift, uint32_t (&pos)[KPT],
                                                     uint32_t* counts) {
  static_assert(KPT <= 16, "4-bit per-thread counters hold at most 15 earlier keys");
  const uint32_t lane = lane_id();
  uint64_t c = 0;
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const uint32_t sh = (static_cast<uint32_t>(keys[j] >> shift) & (kSubBuckets - 1)) * kSubBits;
    pos[j] = static_cast<uint32_t>(c >> sh) & (kSubBuckets - 1);
    if (j + 1 < KPT) c += 1ull << sh;
  }
  const uint32_t last = static_cast<uint32_t>(keys[KPT - 1] >> shift) & (kSubBuckets - 1);
  constexpr uint32_t kRow = kWave * 17 / 16;  // padded row of 64 entries
  uint32_t* mine = counts + pad16(lane);
#pragma unroll
  for (int b = 0; b < kSubBuckets; ++b)
    mine[b * kRow] = (static_cast<uint32_t>(c >> (b * kSubBits)) & (kSubBuckets - 1)) + (last == b);
  wave_sync();
  uint32_t* row = counts + lane * (kSubBuckets + 1);  // = pad16(lane * 16)
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < kSubBuckets; ++i) sum += row[i];
  uint32_t run = wave_inclusive_scan(sum) - sum;
#pragma unroll
  for (int i = 0; i < kSubBuckets; ++i) {
    const uint32_t v = row[i];
    row[i] = run;
    run += v;
  }
  wave_sync();
#pragma unroll
  for (int j = 0; j < KPT; ++j) pos[j] += mine[(static_cast<uint32_t>(keys[j] >> shift) & (kSubBuckets - 1)) * kRow];
  wave_sync();
}

// Stable reorder of one wave's blocked tile (64 x KPT keys) by the 8-bit
// digit at `shift`; stage_k / stage_v are the wave's own padded16(64 * KPT)
// entry slices and `counts` may alias stage_k.  Keys return in registers in
// blocked layout.
template <int KPT, bool VALS, typename K>
__device__ __forceinline__ void wave_sort_digit(K (&keys)[KPT], uint32_t (&vals)[KPT], int shift, K* stage_k,
                                                uint32_t* stage_v, uint32_t* counts) {
  static_assert(KPT == 16, "the blocked reload assumes 16 keys per lane");
  const uint32_t lane = lane_id();
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    uint32_t pos[KPT];
    wave_split_positions<KPT>(keys, shift + half * kSubBits, pos, counts);
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      stage_k[pad16(pos[j])] = keys[j];
      if constexpr (VALS) stage_v[pad16(pos[j])] = vals[j];
    }
    wave_sync();
    const K* my_k = stage_k + 17 * lane;
    const uint32_t* my_v = stage_v + 17 * lane;
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      keys[j] = my_k[j];
      if constexpr (VALS) vals[j] = my_v[j];
    }
    wave_sync();
  }
}

}  // namespace ms

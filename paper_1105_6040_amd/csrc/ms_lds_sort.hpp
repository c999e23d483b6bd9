// ms_lds_sort.hpp -- one workgroup sorts one short list entirely in LDS.
//
// Used for whole lists of at most one tile and for the short segments of a
// segmented sort: the list is read once, every 8-bit digit pass (stable rank
// by wave ballots and LDS counters, then a reorder through LDS) runs on-chip,
// and the result is written once.  Passes whose digit is the same for every
// key of the list are skipped.
#pragma once

#include <type_traits>

#include "ms_device.hpp"

namespace ms {

template <typename K>
struct LdsCfg {
  static constexpr int kThreads = 512;
  static constexpr int kKpt = sizeof(K) == 4 ? 16 : 8;
  static constexpr int kTile = kThreads * kKpt;
};

// LDS of one in-LDS list sort: per-wave digit counters, the key and value
// stages, scan scratch and the changed-bits words.
template <typename K, bool VALS>
struct LdsSortSmem {
  static constexpr int kWaves = LdsCfg<K>::kThreads / kWave;
  uint32_t (*whist)[kRadix];  // kWaves rows
  K* keys;                    // LdsCfg<K>::kTile entries
  uint32_t* vals;             // LdsCfg<K>::kTile entries when VALS
  uint32_t* scan;             // kRadix / kWave entries
  uint32_t* diff;             // 2 entries
};

// One workgroup of LdsCfg<K>::kThreads threads sorts the list
// [begin, begin + len) of kin/vin (1 <= len <= LdsCfg<K>::kTile) into the
// same positions of kout/vout, every digit pass on-chip.  Contains barriers;
// every thread of the block calls it.
template <typename K, bool VALS>
__device__ __forceinline__ void lds_sort_list(const K* __restrict__ kin, const uint32_t* __restrict__ vin, K* kout,
                                              uint32_t* vout, uint64_t begin, int len, K flip,
                                              const LdsSortSmem<K, VALS>& sm) {
  constexpr int kThreads = LdsCfg<K>::kThreads;
  constexpr int kKpt = LdsCfg<K>::kKpt;
  constexpr int kWaves = kThreads / kWave;
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const uint32_t lane = lane_id();
  uint32_t (*s_whist)[kRadix] = sm.whist;
  K* s_keys = sm.keys;
  uint32_t* s_vals = sm.vals;
  uint32_t* s_diff = sm.diff;

  // Only as many rounds of 64 keys per wave as the list needs: wave w holds
  // list positions [w * 64 * R, (w + 1) * 64 * R), slot j < R of lane l
  // position w * 64 * R + 64 * j + l; positions from len on hold padding that
  // sorts after every key.
  const int rounds = (len + kThreads - 1) / kThreads;  // R, 1 .. kKpt
  const int first = wave * kWave * rounds + static_cast<int>(lane);
  K keys[kKpt];
  uint32_t vals[VALS ? kKpt : 1];
#pragma unroll
  for (int j = 0; j < kKpt; ++j) {
    const int idx = first + j * kWave;
    const bool real = j < rounds && idx < len;
    keys[j] = real ? flip_key(kin[begin + idx], flip) : ~K(0);
    if constexpr (VALS) vals[j] = real ? vin[begin + idx] : 0u;
  }

  // Which bits differ among the real keys?  Passes over constant digits are skipped.
  if (tid < 2) s_diff[tid] = 0;
  __syncthreads();
  const K k0 = flip_key(kin[begin], flip);
  K diff = 0;
#pragma unroll
  for (int j = 0; j < kKpt; ++j)
    if (j < rounds && first + j * kWave < len) diff |= keys[j] ^ k0;
  if (static_cast<uint32_t>(diff)) atomicOr(&s_diff[0], static_cast<uint32_t>(diff));
  if constexpr (sizeof(K) == 8)
    if (static_cast<uint32_t>(diff >> 32)) atomicOr(&s_diff[1], static_cast<uint32_t>(diff >> 32));
  __syncthreads();
  const uint64_t all_diff = (static_cast<uint64_t>(s_diff[1]) << 32) | s_diff[0];

  // Full lists run the rounds as compile-time loops; shorter ones stop at
  // their last round.
  auto digit_passes = [&](auto full) {
    constexpr bool kFull = decltype(full)::value;
    const int R = kFull ? kKpt : rounds;
    for (int p = 0; p < static_cast<int>(sizeof(K)); ++p) {
      const int shift = 8 * p;
      if (((all_diff >> shift) & (kRadix - 1)) == 0) continue;  // uniform across the block

      for (int i = tid; i < kWaves * kRadix; i += kThreads) (&s_whist[0][0])[i] = 0;
      __syncthreads();
      uint32_t rank[kKpt];
      uint32_t* wh = s_whist[wave];
      wave_rank(keys, shift, rank, wh, R);
      __syncthreads();
      uint32_t cnt;
      tile_digit_starts<kThreads>(s_whist, sm.scan, &cnt);
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kKpt; ++j) {
        if (j >= R) break;
        const uint32_t pos = wh[digit_of(keys[j], shift)] + rank[j];
        s_keys[pos] = keys[j];
        if constexpr (VALS) s_vals[pos] = vals[j];
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kKpt; ++j) {
        if (j >= R) break;
        keys[j] = s_keys[first + j * kWave];
        if constexpr (VALS) vals[j] = s_vals[first + j * kWave];
      }
      __syncthreads();
    }
  };
  if (rounds == kKpt)
    digit_passes(std::true_type{});
  else
    digit_passes(std::false_type{});

#pragma unroll
  for (int j = 0; j < kKpt; ++j) {
    const int idx = first + j * kWave;
    if (j < rounds && idx < len) {
      kout[begin + idx] = flip_key(keys[j], flip);
      if constexpr (VALS) vout[begin + idx] = vals[j];
    }
  }
}

// In-LDS sort of one short list per workgroup (every pass on-chip).
//   seg_off == nullptr: a single list [0, n_total).
//   otherwise:          segment seg = (seg_list ? seg_list[b] : b) of the
//                       offsets array, clamped to n_total; segments longer
//                       than one tile are left to other kernels.
// Internal linkage: every translation unit that launches it owns its instance.
namespace {
template <typename K, bool VALS>
__global__ __launch_bounds__(LdsCfg<K>::kThreads) void lds_sort_kernel(
    const K* __restrict__ kin, const uint32_t* __restrict__ vin, K* kout, uint32_t* vout,
    const uint64_t* __restrict__ seg_off, const uint32_t* __restrict__ seg_list, uint64_t n_total, K flip) {
  constexpr int kTile = LdsCfg<K>::kTile;
  constexpr int kWaves = LdsCfg<K>::kThreads / kWave;
  __shared__ uint32_t s_whist[kWaves][kRadix];
  __shared__ K s_keys[kTile];
  __shared__ uint32_t s_vals[VALS ? kTile : 1];
  __shared__ uint32_t s_scan[kRadix / kWave];
  __shared__ uint32_t s_diff[2];

  uint64_t begin = 0, end = n_total;
  if (seg_off) {
    const uint64_t s = seg_list ? seg_list[blockIdx.x] : blockIdx.x;
    begin = seg_off[s];
    end = seg_off[s + 1];
    begin = begin < n_total ? begin : n_total;
    end = end < n_total ? end : n_total;
    if (end < begin) end = begin;
  }
  const uint64_t len64 = end - begin;
  if (len64 == 0 || len64 > static_cast<uint64_t>(kTile)) return;
  const LdsSortSmem<K, VALS> sm = {s_whist, s_keys, s_vals, s_scan, s_diff};
  lds_sort_list<K, VALS>(kin, vin, kout, vout, begin, static_cast<int>(len64), flip, sm);
}

}  // namespace

}  // namespace ms

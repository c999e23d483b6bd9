// ms_device.hpp -- device-side building blocks shared by the gfx950 kernels.
//
// Everything here is wave64 (CDNA4) code: lane masks are 64 bits wide and
// cross-lane votes use the amdgcn ballot / mbcnt builtins directly.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ms {

constexpr int kWave = 64;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

// ---------------------------------------------------------------------------
// Key codec.  Radix passes work on unsigned bit patterns; a signed int32 key
// becomes order-preserving unsigned by flipping bit 31 (`flip` = 0x80000000),
// unsigned keys pass through (`flip` = 0).  The map is its own inverse.
template <typename K>
__device__ __forceinline__ K flip_key(K k, K flip) { return k ^ flip; }

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K k, int shift) {
  return static_cast<uint32_t>(k >> shift) & (kRadix - 1);
}

// ---------------------------------------------------------------------------
// Lane helpers.
__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Number of set bits of `m` in lanes strictly below the calling lane.
__device__ __forceinline__ uint32_t count_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

// Peer mask of an 8-bit digit: bit j is set iff lane j holds the same digit.
// One ballot per digit bit; every lane of the wave must be active.
__device__ __forceinline__ uint64_t match_digit(uint32_t d) {
  uint64_t m = ~0ull;
#pragma unroll
  for (int b = 0; b < kRadixBits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t vote = __builtin_amdgcn_ballot_w64(bit);
    m &= bit ? vote : ~vote;
  }
  return m;
}

// Inclusive prefix sum across the 64 lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const T u = __shfl_up(v, off, kWave);
    if (lane >= static_cast<uint32_t>(off)) v += u;
  }
  return v;
}

// Exclusive prefix sum over the first kRadix threads of a block of THREADS
// threads (THREADS >= kRadix).  Threads >= kRadix contribute 0 and receive 0.
// All threads of the block must call it (it contains barriers).  `scratch`
// holds kRadix / kWave entries.  *total receives the sum over all digits.
template <int THREADS, typename T>
__device__ __forceinline__ T block_exclusive_scan_radix(T v, T* scratch, T* total) {
  static_assert(THREADS >= kRadix, "block must cover the radix");
  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const T incl = wave_inclusive_scan(tid < kRadix ? v : T(0));
  if (tid < kRadix && (tid % kWave) == kWave - 1) scratch[wave] = incl;
  __syncthreads();
  T base = 0, sum = 0;
#pragma unroll
  for (int w = 0; w < kRadix / kWave; ++w) {
    const T s = scratch[w];
    if (w < wave) base += s;
    sum += s;
  }
  __syncthreads();
  *total = sum;
  return tid < kRadix ? base + incl - v : T(0);
}

// ---------------------------------------------------------------------------
// Decoupled look-back status words.  One word per (tile, digit) holds a 2-bit
// flag in its top bits and a count below: NOT_READY (0), AGGREGATE (the
// tile's own count) or INCLUSIVE (the count of this digit in all tiles up to
// and including this one).  32-bit words serve lists below 2^30 keys, 64-bit
// words any larger list.
template <typename S>
struct Status {
  static constexpr int kBits = 8 * sizeof(S);
  static constexpr S kAgg = S(1) << (kBits - 2);
  static constexpr S kInc = S(2) << (kBits - 2);
  static constexpr S kFlagMask = S(3) << (kBits - 2);
  static constexpr S kValMask = ~kFlagMask;
};

template <typename S>
__device__ __forceinline__ S status_load(const S* p) {
  return __hip_atomic_load(const_cast<S*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename S>
__device__ __forceinline__ void status_store(S* p, S v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Tile ranking shared by the radix kernels.
//
// A tile of THREADS * KPT keys is held in registers, wave w owning tile
// positions [w*64*KPT, (w+1)*64*KPT) and slot j of lane l holding position
// w*64*KPT + j*64 + l.  `wave_rank` gives every key its rank among the keys of
// the same digit in its wave, in position order (so equal digits keep their
// order: the pass is stable), and leaves the wave's digit counts in `wh`
// (kRadix counters of this wave, zeroed by the caller).
template <typename K, int KPT>
__device__ __forceinline__ void wave_rank(const K (&keys)[KPT], int shift, uint32_t (&rank)[KPT], uint32_t* wh) {
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    const uint32_t d = digit_of(keys[j], shift);
    const uint64_t peers = match_digit(d);
    const uint32_t old = wh[d];
    // Every lane's read lands before any lane's write (the wave executes in
    // lockstep; this marks the dependence for the compiler and for emulation).
    __builtin_amdgcn_wave_barrier();
    rank[j] = old + count_below(peers);
    wh[d] = old + static_cast<uint32_t>(__popcll(peers));  // every peer stores the same value
  }
}

// After wave_rank and a barrier: turns the per-wave digit counts in
// whist[WAVES][kRadix] into the tile position of each wave's first key of
// each digit, so that key (wave w, digit d, rank r) goes to whist[w][d] + r.
// Thread t < kRadix receives the tile's count of digit t in *count and the
// tile position of its first key of digit t as the return value.  Contains
// barriers; every thread of the block calls it.
template <int THREADS>
__device__ __forceinline__ uint32_t tile_digit_starts(uint32_t (*whist)[kRadix], uint32_t* scan_scratch,
                                                      uint32_t* count) {
  constexpr int kWaves = THREADS / kWave;
  const int tid = threadIdx.x;
  uint32_t cnt = 0;
  if (tid < kRadix) {
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = whist[w][tid];
      whist[w][tid] = cnt;
      cnt += c;
    }
  }
  uint32_t total;
  const uint32_t start = block_exclusive_scan_radix<THREADS>(cnt, scan_scratch, &total);
  if (tid < kRadix) {
#pragma unroll
    for (int w = 0; w < kWaves; ++w) whist[w][tid] += start;
  }
  *count = cnt;
  return start;
}

// Decoupled look-back over the status rows of earlier tiles for one digit:
// `st` points at this tile's word for the digit, rows are `stride` words
// apart.  Reads kWindow predecessors at once (independent loads in flight),
// adds AGGREGATE counts nearest-first until an INCLUSIVE count ends the walk,
// and waits on a predecessor that has published nothing yet.  Tile 0
// publishes INCLUSIVE directly, so the walk always ends.  Returns the
// exclusive prefix of the digit over all earlier tiles.
template <typename C, typename S, int kWindow = 8>
__device__ __forceinline__ C lookback(const S* st, uint32_t tile, size_t stride) {
  using St = Status<S>;
  C excl = 0;
  int64_t p = static_cast<int64_t>(tile) - 1;
  while (true) {
    S w[kWindow];
#pragma unroll
    for (int i = 0; i < kWindow; ++i)
      w[i] = (p - i >= 0) ? status_load(st - static_cast<size_t>(static_cast<int64_t>(tile) - (p - i)) * stride)
                          : St::kInc;
    int used = 0;
    bool done = false;
#pragma unroll
    for (int i = 0; i < kWindow; ++i) {
      if (done || used < i) break;
      const S flag = w[i] & St::kFlagMask;
      if (flag == 0) break;
      excl += static_cast<C>(w[i] & St::kValMask);
      used = i + 1;
      if (flag == St::kInc) done = true;
    }
    if (done) return excl;
    p -= used;
    if (used == 0) __builtin_amdgcn_s_sleep(1);
  }
}

}  // namespace ms

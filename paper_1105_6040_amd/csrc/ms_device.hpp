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
// Global-memory view of a pointer the compiler cannot place by itself (one
// read from device memory rather than passed as a kernel argument).  Accesses
// through a generic pointer become FLAT instructions, which also count
// against the LDS wait counter: every later LDS access of the wave would then
// wait for them to finish.  Address spaces exist in device code only; the
// host pass (which parses device functions too) sees a plain pointer.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
#else
template <typename T>
using gptr = T*;
#endif

template <typename T>
__device__ __forceinline__ gptr<T> as_global(T* p) {
  return (gptr<T>)(p);
}

// LDS view of a shared-memory pointer, for the builtins that need one.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using lptr = __attribute__((address_space(3))) T*;
#else
template <typename T>
using lptr = T*;
#endif

// Workgroup barrier that orders LDS accesses only: it waits for the wave's
// own LDS operations, then meets the other waves.  Unlike __syncthreads it
// does not wait for global memory operations in flight, among them loads
// that land in LDS (which a plain barrier must treat as LDS writes): code
// using it must not pass data through global memory between threads of the
// workgroup, and reads LDS filled by such loads only in the wave that issued
// them, after waiting for them.
__device__ __forceinline__ void lds_barrier() {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
#else
  __syncthreads();
#endif
}

// Returns a wave-uniform value unchanged, hiding from the compiler that it is
// the same value, so that expressions computed from it are evaluated again
// instead of being kept in registers from an earlier evaluation.
__device__ __forceinline__ int opaque_uniform(int x) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+s"(x));
#endif
  return x;
}

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

// DPP controls (GFX9 encoding) used by the wave scan.
constexpr int kDppRowShr = 0x110;     // + n: lane reads lane - n of its row of 16
constexpr int kDppRowBcast15 = 0x142;  // lane 15 of each row to the next row
constexpr int kDppRowBcast31 = 0x143;  // lane 31 to rows 2 and 3

template <int kCtrl, int kRowMask, bool kBoundZero>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return static_cast<uint32_t>(
      __builtin_amdgcn_update_dpp(0, static_cast<int>(v), kCtrl, kRowMask, 0xf, kBoundZero));
}

// Inclusive prefix sum across the 64 lanes of a wave.  32-bit values use
// DPP lane moves (no LDS traffic): scans of shift 1, 2, 4, 8 within each row
// of 16 lanes, then the total of row 0 is added to row 1 and of row 2 to
// row 3 (row_bcast:15), then the total of rows 0-1 to rows 2-3
// (row_bcast:31).  Lanes a move does not reach receive 0.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  if constexpr (sizeof(T) == 4) {
    uint32_t x = static_cast<uint32_t>(v);
    x += dpp_u32<kDppRowShr + 1, 0xf, true>(x);
    x += dpp_u32<kDppRowShr + 2, 0xf, true>(x);
    x += dpp_u32<kDppRowShr + 4, 0xf, true>(x);
    x += dpp_u32<kDppRowShr + 8, 0xf, true>(x);
    x += dpp_u32<kDppRowBcast15, 0xa, false>(x);
    x += dpp_u32<kDppRowBcast31, 0xc, false>(x);
    return static_cast<T>(x);
  } else {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const T u = __shfl_up(v, off, kWave);
      if (lane >= static_cast<uint32_t>(off)) v += u;
    }
    return v;
  }
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
  lds_barrier();
  T base = 0, sum = 0;
#pragma unroll
  for (int w = 0; w < kRadix / kWave; ++w) {
    const T s = scratch[w];
    if (w < wave) base += s;
    sum += s;
  }
  lds_barrier();
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
// A tile of THREADS * R keys (R <= KPT rounds) is held in registers, wave w
// owning tile positions [w*64*R, (w+1)*64*R) and slot j < R of lane l holding
// position w*64*R + j*64 + l.  `wave_rank` gives every key its rank among the
// keys of the same digit in its wave, in position order (so equal digits keep
// their order: the pass is stable), and leaves the wave's digit counts in `wh`
// (kRadix counters of this wave, zeroed by the caller).  Slots j >= R are not
// read.  R is uniform across the block.
template <typename K, int KPT>
__device__ __forceinline__ void wave_rank(const K (&keys)[KPT], int shift, uint32_t (&rank)[KPT], uint32_t* wh,
                                          int rounds = KPT) {
#pragma unroll
  for (int j = 0; j < KPT; ++j) {
    if (j >= rounds) break;
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
// apart.  Starting at predecessor tile p and walking towards tile 0, reads
// kWindow predecessors at once (independent loads in flight), adds AGGREGATE
// counts nearest-first until an INCLUSIVE count ends the walk, and waits on a
// predecessor that has published nothing yet.  Tile 0 publishes INCLUSIVE
// directly, so the walk always ends.  Returns the count of the digit in tiles
// 0..p.
template <typename C, typename S, int kWindow = 8>
__device__ __forceinline__ C lookback_from(const S* st, uint32_t tile, int64_t p, size_t stride) {
  using St = Status<S>;
  C excl = 0;
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

// The exclusive prefix of the digit over all tiles before `tile`.
template <typename C, typename S, int kWindow = 8>
__device__ __forceinline__ C lookback(const S* st, uint32_t tile, size_t stride) {
  return lookback_from<C, S, kWindow>(st, tile, static_cast<int64_t>(tile) - 1, stride);
}

// Look-back agent: a workgroup of a pass that takes no tile but walks the
// status rows in tile order, and as soon as a tile's AGGREGATE word of a digit
// is visible publishes that tile's INCLUSIVE count, so that a tile usually
// finds its predecessor INCLUSIVE when it needs it instead of walking back
// itself.  It only reads words the tiles publish unconditionally (AGGREGATE or
// INCLUSIVE) and tiles never wait for it, so it adds no dependence a tile
// could block on.  An INCLUSIVE word already published (tile 0, or a tile
// that walked back by itself) restarts the running count at its value.
//
// One agent serves kDigits digits starting at digit0 (several agents share
// the radix, so that no single workgroup has to move all the status words).
// Thread t follows digit digit0 + t % kDigits over the kW tiles of chunk
// t / kDigits of the current window: THREADS / kDigits * kW rows per memory
// round trip.  `val` and `used` hold THREADS entries, `prefix` and `next`
// kDigits.  Contains barriers; every thread of the block calls it.  Returns
// when every tile of its digits has been published.
constexpr uint32_t kLbIncBit = 1u << 16;

template <int THREADS, int kDigits, int kW, typename C, typename S>
__device__ __forceinline__ void lookback_agent(S* status, uint32_t num_tiles, int digit0, C* val, uint32_t* used,
                                               C* prefix, uint32_t* next) {
  using St = Status<S>;
  constexpr int kChunks = THREADS / kDigits;
  static_assert(THREADS % kDigits == 0 && kRadix % kDigits == 0, "whole chunks of digits");
  const int tid = threadIdx.x;
  const int d = tid % kDigits;
  const int c = tid / kDigits;
  S* const column = status + digit0 + d;
  if (tid < kDigits) {
    next[tid] = 0;
    prefix[tid] = 0;
  }
  __syncthreads();
  while (true) {
    const uint32_t start = next[d];
    if (!__syncthreads_or(tid < kDigits && start < num_tiles)) break;
    // Read the chunk and fold it: u = words ready (published) from its start,
    // running = its effect on the count (set by an INCLUSIVE word, else added).
    const uint32_t base = start + static_cast<uint32_t>(c) * kW;
    S w[kW];
#pragma unroll
    for (int i = 0; i < kW; ++i)
      w[i] = base + i < num_tiles ? status_load(column + static_cast<size_t>(base + i) * kRadix) : S(0);
    uint32_t u = 0;
    bool stop = false, has_inc = false;
    C run = 0;
#pragma unroll
    for (int i = 0; i < kW; ++i) {
      const S flag = w[i] & St::kFlagMask;
      const bool ready = !stop && flag != 0;
      stop = !ready;
      u += ready ? 1u : 0u;
      const C v = static_cast<C>(w[i] & St::kValMask);
      if (ready && flag == St::kInc) {
        has_inc = true;
        run = v;
      } else if (ready) {
        run += v;
      }
    }
    val[tid] = run;
    used[tid] = u | (has_inc ? kLbIncBit : 0u);
    __syncthreads();
    // Count entering this chunk: the chunks before it, while each was ready
    // to its end.  Publish INCLUSIVE for the chunk's ready AGGREGATE words.
    C pin = prefix[d];
    bool reach = true;
#pragma unroll
    for (int k = 0; k < kChunks - 1; ++k) {
      if (k < c && reach) {
        const uint32_t uk = used[k * kDigits + d];
        const C vk = val[k * kDigits + d];
        pin = (uk & kLbIncBit) ? vk : pin + vk;
        reach = (uk & ~kLbIncBit) == static_cast<uint32_t>(kW);
      }
    }
    if (reach) {
      C incl = pin;
#pragma unroll
      for (int i = 0; i < kW; ++i) {
        if (static_cast<uint32_t>(i) < u) {
          const S flag = w[i] & St::kFlagMask;
          const C v = static_cast<C>(w[i] & St::kValMask);
          incl = flag == St::kInc ? v : incl + v;
          if (flag == St::kAgg) status_store(column + static_cast<size_t>(base + i) * kRadix, St::kInc | static_cast<S>(incl));
        }
      }
    }
    if (tid < kDigits) {
      C p = prefix[d];
      uint32_t adv = 0;
      bool go = true;
#pragma unroll
      for (int k = 0; k < kChunks; ++k) {
        if (go) {
          const uint32_t uk = used[k * kDigits + d];
          const C vk = val[k * kDigits + d];
          p = (uk & kLbIncBit) ? vk : p + vk;
          adv += uk & ~kLbIncBit;
          go = (uk & ~kLbIncBit) == static_cast<uint32_t>(kW);
        }
      }
      next[d] = start + adv;
      prefix[d] = p;
      if (adv == 0) __builtin_amdgcn_s_sleep(2);
    }
    __syncthreads();
  }
}

}  // namespace ms

// radix.hip -- stable LSD radix sort of one list on gfx950 (sort_keys, sort_pairs).
//
// This is the "sort phase" of the paper's scatter / sort / merge method
// (Section 3.2, Figure 1 step 9) for a whole list, redesigned for one GPU:
// instead of a comparison sort per process, the list is sorted by 8-bit
// digits from least to most significant, each digit pass a stable counting
// scatter, so the order of equal keys is kept (the paper's bubble sort keeps
// it too; its merge sort does with a left-first merge).
//
// Launch sequence on the caller's stream (no host synchronisation):
//   1. clear     zero the counters, histograms and first look-back buffer
//   2. histogram one read of all keys -> one 256-bin histogram per digit
//                pass; the last workgroup turns them into digit bases, marks
//                passes whose digit is the same for every key as trivial, and
//                writes the ping-pong plan (which buffer each pass reads and
//                writes) to device memory
//   3. P passes  onesweep: each workgroup takes the next tile id from an
//                atomic counter, ranks its tile by digit (wave ballots + LDS
//                counters), publishes its digit counts, looks back across
//                earlier tiles for their running prefix (decoupled look-back),
//                reorders the tile in LDS and writes digit runs coalesced
//   4. copy      only when the plan needs it (in-place sort with an odd
//                number of executed passes, or no pass executed)
// Lists of at most one LDS tile skip all that: one workgroup sorts them in
// LDS with every pass done on-chip.
#include <algorithm>
#include <mutex>
#include <vector>

#include "ms_device.hpp"
#include "ms_lds_sort.hpp"
#include "ms_tile.hpp"
#include "ms_runtime.hpp"

namespace ms {
namespace {

constexpr int kMaxPasses = 8;

struct PassPlan {
  const void* src_k;
  void* dst_k;
  const uint32_t* src_v;
  uint32_t* dst_v;
  uint32_t active;  // 0: the digit is constant over the list; pass skipped
  uint32_t first;   // the first executed pass: apply the key codec on load
  uint32_t last;    // the final executed pass: undo the key codec on store
  uint32_t pad;
};

struct SortPlan {
  PassPlan pass[kMaxPasses];
  const void* copy_src_k;
  void* copy_dst_k;
  const uint32_t* copy_src_v;
  uint32_t* copy_dst_v;
  uint32_t copy;  // 1: copy the n results from copy_src to copy_dst at the end
  uint32_t num_active;
  uint32_t pad[2];
};

struct Buffers {
  const void* keys_in;
  void* keys_out;
  void* alt_k;
  const uint32_t* vals_in;
  uint32_t* vals_out;
  uint32_t* alt_v;
};

// Onesweep tile geometry: THREADS threads (256, 512 or 1024; a tunable), 16
// keys per thread held in registers.  Threads 0..255 own one digit each in
// the look-back and scans.
template <int THREADS>
struct PassCfg {
  static constexpr int kThreads = THREADS;
  static constexpr int kKpt = 16;
  static constexpr int kTile = kThreads * kKpt;
  // Look-back agents publish prefixes for tiles of 512 and 1,024 threads:
  // kAgents workgroups, each serving kRadix / kAgents digits with chunks of
  // kAgentW rows.  256-thread tiles arrive faster than agents of their size
  // can read the status rows, so those tiles walk back by themselves.
  static constexpr bool kAgent = THREADS >= 512;
  // Agents and rows per chunk, measured per pass on 2^28 int32 keys
  // (1,024 threads): 4 agents of 2, 4, 8 or 16 rows 1.16 (the agents fall
  // behind), 0.813, 0.827 and 0.853 ms; 2 agents of 4, 8 or 16 rows 1.02,
  // 0.808 and 0.834 ms; 1 agent of 16 rows 0.917 ms; 8 agents of 4 rows
  // 0.839 ms.  2^26 (u64, u32) pairs (512 threads), whole sort: 2 agents of
  // 8, 16 or 32 rows 4.39, 4.17 and 4.28 ms, none 4.31 ms.
  static constexpr int kAgents = kAgent ? 2 : 0;
  static constexpr int kAgentW = THREADS == 1024 ? 8 : 16;
};
constexpr int kMinPassTile = PassCfg<256>::kTile;  // workspace is sized for the smallest tile

template <typename C>
__device__ __forceinline__ void atomic_add_c(C* p, C v) {
  if constexpr (sizeof(C) == 4) {
    atomicAdd(reinterpret_cast<unsigned int*>(p), static_cast<unsigned int>(v));
  } else {
    atomicAdd(reinterpret_cast<unsigned long long*>(p), static_cast<unsigned long long>(v));
  }
}

// ---------------------------------------------------------------------------
// 1. clear: zero two byte ranges (each a multiple of 16 bytes).
__global__ __launch_bounds__(256) void clear_kernel(uint4* a, size_t a16, uint4* b, size_t b16) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  const uint4 z = make_uint4(0, 0, 0, 0);
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < a16 + b16; i += stride) {
    if (i < a16)
      a[i] = z;
    else
      b[i - a16] = z;
  }
}

// ---------------------------------------------------------------------------
// 2. histogram + plan.
template <typename K, typename C>
__global__ __launch_bounds__(256) void histogram_kernel(const K* __restrict__ keys, C n, K flip,
                                                        C* __restrict__ ghist, C* __restrict__ gbase,
                                                        uint32_t* done, SortPlan* plan, Buffers buf,
                                                        int has_vals) {
  constexpr int P = sizeof(K);        // 8-bit digits
  constexpr int kCopies = 64 / P;     // counter copies spread same-digit lanes: 64 KB of LDS
  constexpr int kVec = 16 / sizeof(K);
  __shared__ uint32_t h[P * kRadix * kCopies];
  __shared__ C s_scan[kRadix / kWave];
  __shared__ uint32_t s_active[P];
  __shared__ uint32_t s_last;
  const int tid = threadIdx.x;

  for (int i = tid; i < P * kRadix * kCopies; i += 256) h[i] = 0;
  __syncthreads();

  const uint32_t copy = lane_id() % kCopies;
  auto count = [&](K k) {
    k = flip_key(k, flip);
#pragma unroll
    for (int p = 0; p < P; ++p) atomicAdd(&h[(p * kRadix + digit_of(k, 8 * p)) * kCopies + copy], 1u);
  };
  auto count_vec = [&](const uint4& v) {
    if constexpr (sizeof(K) == 4) {
      count(v.x);
      count(v.y);
      count(v.z);
      count(v.w);
    } else {
      count((static_cast<uint64_t>(v.y) << 32) | v.x);
      count((static_cast<uint64_t>(v.w) << 32) | v.z);
    }
  };

  // Unaligned head and the tail go through scalar loads in block 0.
  const uint64_t mis = (reinterpret_cast<uintptr_t>(keys) / sizeof(K)) % kVec;
  C head = mis ? static_cast<C>(kVec - mis) : C(0);
  if (head > n) head = n;
  const C nvec = (n - head) / kVec;
  const uint4* vbase = reinterpret_cast<const uint4*>(keys + head);
  const C stride = static_cast<C>(gridDim.x) * 256;
  C i = static_cast<C>(blockIdx.x) * 256 + tid;
  // Four vectors per thread per step; the next step's loads are issued
  // before this step's counting, so the LDS atomics overlap the HBM latency.
  if (i + 3 * stride < nvec) {
    uint4 a0 = vbase[i], a1 = vbase[i + stride], a2 = vbase[i + 2 * stride], a3 = vbase[i + 3 * stride];
    for (;;) {
      const C nxt = i + 4 * stride;
      const bool more = nxt + 3 * stride < nvec;
      uint4 b0 = a0, b1 = a1, b2 = a2, b3 = a3;
      if (more) {
        b0 = vbase[nxt];
        b1 = vbase[nxt + stride];
        b2 = vbase[nxt + 2 * stride];
        b3 = vbase[nxt + 3 * stride];
      }
      count_vec(a0);
      count_vec(a1);
      count_vec(a2);
      count_vec(a3);
      i = nxt;
      if (!more) break;
      a0 = b0;
      a1 = b1;
      a2 = b2;
      a3 = b3;
    }
  }
  for (; i < nvec; i += stride) count_vec(vbase[i]);
  if (blockIdx.x == 0) {
    for (C j = tid; j < head; j += 256) count(keys[j]);
    for (C j = head + nvec * kVec + tid; j < n; j += 256) count(keys[j]);
  }
  __syncthreads();

  for (int b = tid; b < P * kRadix; b += 256) {
    uint32_t s = 0;
#pragma unroll
    for (int c = 0; c < kCopies; ++c) s += h[b * kCopies + c];
    if (s) atomic_add_c(&ghist[b], static_cast<C>(s));
  }

  // The last block to finish builds the plan.
  __threadfence();
  __syncthreads();
  if (tid == 0) s_last = atomicAdd(done, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!s_last) return;
  __threadfence();

  for (int p = 0; p < P; ++p) {
    const C c = __hip_atomic_load(&ghist[p * kRadix + tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    C total;
    const C ex = block_exclusive_scan_radix<256>(c, s_scan, &total);
    gbase[p * kRadix + tid] = ex;
    const int trivial = __syncthreads_or(c == n);
    if (tid == 0) s_active[p] = !trivial;
  }
  __syncthreads();
  if (tid != 0) return;

  uint32_t m = 0;
  for (int p = 0; p < P; ++p) m += s_active[p];
  const bool inplace = buf.keys_in == buf.keys_out;
  const void* cur_k = buf.keys_in;
  const uint32_t* cur_v = buf.vals_in;
  uint32_t e = 0;
  for (int p = 0; p < kMaxPasses; ++p) {
    PassPlan pp = {};
    if (p < P && s_active[p]) {
      // The last executed pass must land in keys_out; earlier ones alternate.
      // In place, the first pass cannot write keys_out (it is being read).
      const bool to_out = inplace ? (e % 2 == 1) : ((m - 1 - e) % 2 == 0);
      pp.src_k = cur_k;
      pp.dst_k = to_out ? buf.keys_out : buf.alt_k;
      pp.src_v = cur_v;
      pp.dst_v = has_vals ? (to_out ? buf.vals_out : buf.alt_v) : nullptr;
      pp.active = 1;
      pp.first = e == 0;
      pp.last = e == m - 1;
      cur_k = pp.dst_k;
      cur_v = pp.dst_v;
      ++e;
    }
    plan->pass[p] = pp;
  }
  plan->copy = 0;
  plan->copy_src_k = nullptr;
  plan->copy_dst_k = nullptr;
  plan->copy_src_v = nullptr;
  plan->copy_dst_v = nullptr;
  if (m == 0 && !inplace) {  // every digit constant: the output is the input
    plan->copy = 1;
    plan->copy_src_k = buf.keys_in;
    plan->copy_dst_k = buf.keys_out;
    plan->copy_src_v = buf.vals_in;
    plan->copy_dst_v = buf.vals_out;
  } else if (m > 0 && inplace && (m % 2 == 1)) {  // result ended in the workspace
    plan->copy = 1;
    plan->copy_src_k = buf.alt_k;
    plan->copy_dst_k = buf.keys_out;
    plan->copy_src_v = buf.alt_v;
    plan->copy_dst_v = buf.vals_out;
  }
  plan->num_active = m;
}

// ---------------------------------------------------------------------------
// 3. one onesweep digit pass.
//
// Per tile: blocked load (vector loads when aligned) -> tile digit histogram
// in LDS -> publish the tile's digit counts (AGGREGATE) at once, so later
// tiles can look past this one while it works -> stable reorder of the tile
// by the digit (two 4-bit splits, ms_tile.hpp) -> look back for the count of
// each digit in all earlier tiles -> publish INCLUSIVE -> write the sorted
// tile: entry i goes to base[d] + earlier[d] + (i - start[d]), so threads
// i, i+1, ... write consecutive addresses inside every digit run.
//
// Workgroups are persistent: each takes tiles in arrival order from a counter
// until none are left.  The next tile's number is fetched while the current
// tile is being sorted and its keys are loaded before the current tile is
// written out, so neither round trip stands between two tiles.

// s_waitcnt immediate (GFX9 field layout: vmcnt in bits 3:0 and 15:14,
// expcnt 6:4, lgkmcnt 11:8) that waits until at most `vm` of the wave's vector
// memory operations are outstanding and leaves the other counters alone.
// Vector memory operations retire in issue order on this architecture, so it
// waits for everything issued before the last `vm` operations.
constexpr int waitcnt_vmcnt(int vm) { return (vm & 0xF) | ((vm >> 4) << 14) | (0x7 << 4) | (0xF << 8); }

// Loads of a tile's keys straight into LDS, one 16-byte chunk per lane and
// instruction: lane l of the wave lands at lds_dst + 16 * l (lds_dst is
// the same for every lane).  Written in
// assembly so that the compiler, which cannot tell which later LDS accesses
// such a load may touch, adds no waits for it: the caller waits for it by
// hand (read_prefetched_keys) in the issuing wave, before any exit.
__device__ __forceinline__ void global_to_lds_x4(gptr<const void> src, uint32_t* lds_dst) {
#if defined(__HIP_DEVICE_COMPILE__)
  // The destination is the same for the whole wave: make it a scalar.
  const uint32_t lds_addr =
      __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lptr<uint32_t>)lds_dst)));
  // M0 carries the LDS address; the compiler's own value of M0 is kept.
  uint32_t saved;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %1\n\t"
      "global_load_lds_dwordx4 %2, off\n\t"
      "s_mov_b32 m0, %0"
      : "=&s"(saved)
      : "s"(lds_addr), "v"(src)
      : "memory");
#else
  __builtin_amdgcn_global_load_lds(src, lds_dst, 16, 0, 0);
#endif
}

// Reads back this lane's four 16-byte chunks of a prefetch made by its wave
// (chunk q at lane_src + 256 q words) after waiting until at most `kLater` of
// the wave's vector memory operations are outstanding; the caller guarantees
// that at least that many were issued after the prefetch.
template <int kLater>
__device__ __forceinline__ void read_prefetched_keys(const uint32_t* lane_src, uint32_t (&k)[16]) {
#if defined(__HIP_DEVICE_COMPILE__)
  const uint32_t lds_addr = static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lptr<const uint32_t>)lane_src));
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  u32x4 a, b, c, d;
  asm volatile(
      "s_waitcnt vmcnt(%4)\n\t"
      "ds_read_b128 %0, %5\n\t"
      "ds_read_b128 %1, %5 offset:1024\n\t"
      "ds_read_b128 %2, %5 offset:2048\n\t"
      "ds_read_b128 %3, %5 offset:3072\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(a), "=&v"(b), "=&v"(c), "=&v"(d)
      : "n"(kLater), "v"(lds_addr)
      : "memory");
  k[0] = a.x; k[1] = a.y; k[2] = a.z; k[3] = a.w;
  k[4] = b.x; k[5] = b.y; k[6] = b.z; k[7] = b.w;
  k[8] = c.x; k[9] = c.y; k[10] = c.z; k[11] = c.w;
  k[12] = d.x; k[13] = d.y; k[14] = d.z; k[15] = d.w;
#else
  for (int q = 0; q < 4; ++q)
    for (int e = 0; e < 4; ++e) k[4 * q + e] = lane_src[256 * q + e];
#endif
}

template <typename K, bool VALS, typename C, typename S, int THREADS>
__global__ __launch_bounds__(THREADS) void onesweep_kernel(
    const SortPlan* __restrict__ plan, int pass, C n, K flip, const C* __restrict__ gbase,
    uint32_t* tile_counter, S* status_cur, S* status_next) {
  constexpr int kThreads = PassCfg<THREADS>::kThreads;
  constexpr int kKpt = PassCfg<THREADS>::kKpt;
  constexpr int kTile = PassCfg<THREADS>::kTile;
  using St = Status<S>;

  // The split counters are dead before the first key lands in the stage, so
  // the two share LDS.
  constexpr int kStageBytes = padded16(kTile) * static_cast<int>(sizeof(K));
  constexpr int kCountBytes = SplitScratch<kThreads>::kCountWords * 4;
  __shared__ __attribute__((aligned(16))) uint8_t s_raw[kStageBytes > kCountBytes ? kStageBytes : kCountBytes];
  K* s_stage = reinterpret_cast<K*>(s_raw);
  uint32_t* s_counts = reinterpret_cast<uint32_t*>(s_raw);
  __shared__ uint32_t s_vstage[VALS ? padded16(kTile) : 1];
  __shared__ uint32_t s_hist[kRadix];
  __shared__ C s_doff[kRadix];  // output index of the digit's first tile key, minus its tile position
  __shared__ uint32_t s_scan[kThreads / kWave];
  __shared__ C s_cscan[kRadix / kWave];
  __shared__ uint32_t s_ticket;
  __shared__ uint32_t s_ticket2;
  // Keys of the tile after the current one, loaded straight into LDS: wave w
  // owns entries [w * 64 * KPT, (w + 1) * 64 * KPT), filled by its 4 x 16-byte
  // loads per lane (lane l's 16 bytes of load q at 16 * (q * 64 + l)).
  constexpr bool kLdsPrefetch = THREADS == 1024 && sizeof(K) == 4 && !VALS;
  __shared__ __attribute__((aligned(16))) uint32_t s_next[kLdsPrefetch ? kTile : 4];
  // Used by the look-back agent only.
  constexpr bool kAgent = PassCfg<THREADS>::kAgent;
  __shared__ C s_lb_val[kAgent ? kThreads : 1];
  __shared__ uint32_t s_lb_used[kAgent ? kThreads : 1];

  const int tid = threadIdx.x;
  const PassPlan& pp = plan->pass[pass];

  const uint32_t num_tiles = static_cast<uint32_t>((n + kTile - 1) / kTile);
  if (!pp.active) {
    // Skipped pass: still clear the next pass's look-back rows.
    if (status_next)
      for (uint32_t row = blockIdx.x; row < num_tiles; row += gridDim.x)
        for (int d = tid; d < kRadix; d += kThreads) status_next[static_cast<size_t>(row) * kRadix + d] = 0;
    return;
  }

  // With agents, the first kAgents tickets make their workgroups look-back
  // agents and ticket t >= kAgents is tile t - kAgents; without, ticket t is
  // tile t.
  constexpr int kAgents = PassCfg<THREADS>::kAgents;
  constexpr uint32_t kFirstTile = kAgents;
  if (tid == 0) s_ticket = atomicAdd(tile_counter, 1u);
  __syncthreads();
  if constexpr (kAgent) {
    if (s_ticket < kFirstTile) {
      constexpr int kDigits = kRadix / kAgents;
      lookback_agent<kThreads, kDigits, PassCfg<THREADS>::kAgentW, C, S>(
          status_cur, num_tiles, static_cast<int>(s_ticket) * kDigits, s_lb_val, s_lb_used, s_doff, s_hist);
      return;
    }
  }
  uint32_t tile = s_ticket - kFirstTile;
  if (tile >= num_tiles) return;

  const int shift = 8 * pass;
  const gptr<const K> src = as_global(static_cast<const K*>(pp.src_k));
  const gptr<const uint32_t> src_v = as_global(static_cast<const uint32_t*>(pp.src_v));
  const gptr<K> dst = as_global(static_cast<K*>(pp.dst_k));
  const gptr<uint32_t> dst_v = as_global(pp.dst_v);
  const K in_flip = pp.first ? flip : K(0);  // intermediate buffers hold encoded keys
  const K out_flip = pp.last ? flip : K(0);
  const K pad = ~K(0) ^ in_flip;             // decodes to all-ones: sorts after every real key
  const bool src_aligned = reinterpret_cast<uintptr_t>(src) % 16 == 0;

  // This wave's prefetch slots: kKpt / 4 chunks of 64 lanes x 16 bytes.
  uint32_t* const s_next_wave = s_next + (tid / kWave) * (kKpt / 4) * kWave * 4;

  // Tickets run one tile ahead where keys are prefetched into LDS: `ahead`
  // is the tile after the current one once known (kNone before).  Every
  // workgroup holds the same lead, so tiles still start in ticket order.
  constexpr uint32_t kNone = ~0u;
  uint32_t ahead = kNone;
  bool in_lds = false;  // the current tile's keys were prefetched into s_next

  K keys[kKpt];
  uint32_t vals[kKpt];  // unused (and optimised away) for key-only sorts

  while (true) {
    const C tile_base = static_cast<C>(tile) * kTile;
    if (status_next)
      for (int d = tid; d < kRadix; d += kThreads) status_next[static_cast<size_t>(tile) * kRadix + d] = 0;
    for (int d = tid; d < kRadix; d += kThreads) s_hist[d] = 0;
    if constexpr (kLdsPrefetch) {
      if (in_lds) {
        // This wave's own prefetch, issued one tile ago: every thread has
        // issued at least the previous (full) tile's kKpt stores since, so
        // letting that many stay in flight still waits for the prefetch.
        uint32_t raw[kKpt];
        read_prefetched_keys<kKpt>(s_next_wave + (tid % kWave) * 4, raw);
#pragma unroll
        for (int j = 0; j < kKpt; ++j) keys[j] = flip_key(static_cast<K>(raw[j]), in_flip);
      } else {
        load_tile_keys<K, VALS, C, kKpt>(src, src_v, tile_base + static_cast<C>(tid) * kKpt, n, pad, keys, vals);
        // Finish these loads here, not where the two ways meet.
#pragma unroll
        for (int j = 0; j < kKpt; ++j) keys[j] = flip_key(keys[j], in_flip);
        __builtin_amdgcn_s_waitcnt(waitcnt_vmcnt(0));
      }
    } else {
      load_tile_keys<K, VALS, C, kKpt>(src, src_v, tile_base + static_cast<C>(tid) * kKpt, n, pad, keys, vals);
#pragma unroll
      for (int j = 0; j < kKpt; ++j) keys[j] = flip_key(keys[j], in_flip);
    }
    lds_barrier();

    // Tile digit histogram.  When all keys of the wave share one digit (long
    // runs: sorted or skewed input) one lane adds them all, sparing the LDS
    // 64 colliding atomics per instruction; otherwise every key adds itself.
    {
      const uint32_t d0 = digit_of(keys[0], shift);
      bool same = true;
#pragma unroll
      for (int j = 1; j < kKpt; ++j) same = same && digit_of(keys[j], shift) == d0;
      const uint32_t w0 = __builtin_amdgcn_readfirstlane(d0);
      if (__builtin_amdgcn_ballot_w64(same && d0 == w0) == ~0ull) {
        if (lane_id() == 0) atomicAdd(&s_hist[w0], static_cast<uint32_t>(kWave * kKpt));
      } else {
#pragma unroll
        for (int j = 0; j < kKpt; ++j) atomicAdd(&s_hist[digit_of(keys[j], shift)], 1u);
      }
    }
    lds_barrier();

    // Publish this tile's digit counts before sorting it.
    S* st = status_cur + static_cast<size_t>(tile) * kRadix + tid;
    uint32_t cnt = 0;
    if (tid < kRadix) {
      cnt = s_hist[tid];
      status_store(st, (tile == 0 ? St::kInc : St::kAgg) | static_cast<S>(cnt));
    }

    // Prefetch the keys of the tile after this one into LDS while this tile
    // is sorted (no registers held; nothing latency-critical queues behind
    // the loads), and take the next ticket.
    bool next_in_lds = false;
    if constexpr (kLdsPrefetch) {
      if (ahead != kNone && ahead < num_tiles && src_aligned &&
          (static_cast<C>(ahead) + 1) * kTile <= n) {
        const gptr<const K> from = src + static_cast<C>(ahead) * kTile + static_cast<C>(tid) * kKpt;
#pragma unroll
        for (int q = 0; q < kKpt / 4; ++q) global_to_lds_x4(from + 4 * q, s_next_wave + q * kWave * 4);
        next_in_lds = true;
      }
    }
    // atomicInc with the maximum bound is a fetch-and-add of one that the
    // compiler leaves as a single atomic (its rewrite of a one-lane atomicAdd
    // waits for the result right away, undoing the overlap).
    uint32_t ticket = 0;
    if (tid == 0) ticket = atomicInc(tile_counter, ~0u);

    // Sort the tile by the digit's low nibble.
    tile_split_stage<kThreads, kKpt, VALS>(keys, vals, shift, s_stage, s_vstage, s_counts, s_scan, true);

    // A second ticket while the first tile runs, so that the lead is one tile
    // from then on.
    uint32_t ticket2 = 0;
    const bool first_lead = kLdsPrefetch && ahead == kNone;
    if (first_lead && tid == 0) ticket2 = atomicInc(tile_counter, ~0u);

    // Read the predecessor's word while the second split runs: by the time it
    // is used the agent has usually published the predecessor's INCLUSIVE count.
    S pred = 0;
    if (tid < kRadix && tile != 0) pred = status_load(st - kRadix);

    // ... and by the high nibble: the stage now holds the tile in digit order.
    tile_split_stage<kThreads, kKpt, VALS>(keys, vals, shift + kSubBits, s_stage, s_vstage, s_counts, s_scan, false);

    if (tid == 0) {
      s_ticket = ticket;
      s_ticket2 = ticket2;
    }
    C tile_total;
    const C start = block_exclusive_scan_radix<kThreads>(static_cast<C>(cnt), s_cscan, &tile_total);

    // Without LDS prefetch the tile's registers now take the next tile's
    // keys: the loads land during the look-back.
    uint32_t next;
    if constexpr (kLdsPrefetch) {
      if (ahead == kNone) {
        next = s_ticket - kFirstTile;
        ahead = s_ticket2 - kFirstTile;
      } else {
        next = ahead;
        ahead = s_ticket - kFirstTile;
      }
    } else {
      next = s_ticket - kFirstTile;
    }
    const bool more = next < num_tiles;
    if constexpr (!kLdsPrefetch) {
      if (more)
        load_tile_keys<K, VALS, C, kKpt>(src, src_v, static_cast<C>(next) * kTile + static_cast<C>(tid) * kKpt, n,
                                         pad, keys, vals);
    }

    if (tid < kRadix) {
      C excl = 0;
      if (tile != 0) {
        // Otherwise walk back (the agent may be behind, or there is none),
        // 4 predecessors per read: the walk usually ends within a few, and
        // wider windows read status rows it never needed (16 cost 2.3 % on
        // this pass and 10 % on 512-thread pairs passes).
        excl = (pred & St::kFlagMask) == St::kInc ? static_cast<C>(pred & St::kValMask)
                                                  : lookback<C, S, 4>(st, tile, kRadix);
        status_store(st, St::kInc | static_cast<S>(excl + cnt));
      }
      s_doff[tid] = gbase[tid] + excl - start;
    }
    lds_barrier();

    const C remaining = n - tile_base;
    const int valid = remaining < static_cast<C>(kTile) ? static_cast<int>(remaining) : kTile;
#pragma unroll 4
    for (int i = tid; i < valid; i += kThreads) {
      const K k = s_stage[pad16(i)];
      const C o = s_doff[digit_of(k, shift)] + static_cast<C>(i);
      dst[o] = k ^ out_flip;
      if constexpr (VALS) dst_v[o] = s_vstage[pad16(i)];
    }
    if (!more) break;
    tile = next;
    in_lds = next_in_lds;
    lds_barrier();  // the stage, s_doff and s_hist are reused by the next tile
  }
  // A prefetch is only issued for a tile this workgroup goes on to process,
  // so none is in flight here.
}

// ---------------------------------------------------------------------------
// 5. The digit passes of sort_segmented for long segments: the paper's parts
// sorted by the whole device at once instead of one workgroup each.
//
// Every segment is cut into tiles from its own start (its last tile is
// partial) and the tiles of all segments are numbered in segment order; a
// table holds one record per tile.  A tile takes its digit bases from its own
// segment's histograms, and the segment's first tile publishes INCLUSIVE at
// once, so that the look-back of every other tile ends inside its segment.  A
// segment of one tile needs neither histograms nor look-back: its sorted tile
// is stored in place.  All passes run (no trivial-pass skip): even P
// ping-pongs keys_in -> workspace -> keys_out -> ... -> keys_out.
// Tiles of 8,192 keys (512 threads) or, for 32-bit keys without values,
// 16,384 keys (1,024 threads; a tunable).  The tile size is an argument of
// the planning kernels and a template parameter of the pass.
constexpr int kSegSweepThreads = 512;
// The one-launch path's queue table, a cleared block of the workspace of
// kQWordsAll words: per queue, its ticket counter and its counts of finished
// items per phase, each on a cache line of its own (every workgroup of an XCD
// counts there); then the queues' record starts (kMaxQueues + 1 of them, the
// last one the record count) and owners (XCC_ID + 1, 0 = unclaimed).
constexpr int kMaxQueues = 8;
constexpr int kLineWords = 32;
constexpr int kQTickets = 0;
constexpr int kQDone = kMaxQueues * kLineWords;
constexpr int kQStarts = 2 * kMaxQueues * kLineWords;
constexpr int kQOwners = kQStarts + kMaxQueues + 1;
constexpr int kQWords = kQOwners + kMaxQueues;
constexpr size_t kQWordsAll = 1024;
static_assert(kQWords <= static_cast<int>(kQWordsAll), "queue table fits its block");
// A launch per phase is used when the segments average more keys than one
// workgroup sorts in LDS (8,192): shorter ones are sorted faster by one
// workgroup each.  The one-launch work queue sorts a one-tile segment whole
// in LDS in its first phase, and pays off from segments averaging more than
// 1,024 keys (below that a wave sorts each segment on its own).
constexpr uint64_t kSegSweepMinAverage = 8192;
constexpr uint64_t kSegQueueMinAverage = 1024;
using SegSweepCfg = PassCfg<kSegSweepThreads>;  // the smallest tile: bounds the tile count

// One tile of the segment passes.  `count` holds the tile's key count
// (1 .. tile size) and two flags.
struct SegTile {
  uint64_t begin;  // index of the tile's first key
  uint32_t count;
  uint32_t seg;
};
constexpr uint32_t kTileFirst = 1u << 31;  // the segment's first tile
constexpr uint32_t kTileOnly = 1u << 30;   // the segment's only tile
constexpr uint32_t kTileCountMask = kTileOnly - 1;

// The tile table is planned in chunks of kSegChunk segments, one block each.
constexpr int kSegPlanThreads = 256;
constexpr int kSegPlanPerThread = 8;
constexpr uint32_t kSegChunk = kSegPlanThreads * kSegPlanPerThread;

// Segment s as [*begin, *begin + length): offsets clamped to n, a decreasing
// pair read as empty, so that offsets that break the contract never lead
// outside [0, n).
__device__ __forceinline__ uint64_t segment_span(const uint64_t* off, uint64_t s, uint64_t n, uint64_t* begin) {
  uint64_t b = off[s], e = off[s + 1];
  b = b < n ? b : n;
  e = e < n ? e : n;
  *begin = b;
  return e > b ? e - b : 0;
}

__device__ __forceinline__ uint64_t segment_tiles(const uint64_t* off, uint64_t s, uint64_t n, uint32_t tile) {
  uint64_t b;
  return (segment_span(off, s, n, &b) + tile - 1) / tile;
}

// A segment of this many keys or more needs 64-bit look-back status words
// (a 30-bit count field holds less); the planner raises *wide for it.
constexpr uint64_t kWideSegment = 1ull << 30;

// Tile counts are summed in 64 bits: offsets that break the contract
// (overlapping segments) may ask for more tiles than 32 bits count, and a
// wrapped sum would leave stale records inside the table.
static_assert(kSegPlanThreads == kRadix, "the planner's block scans cover kRadix threads");

// Tiles of this block's segments, each thread summing kSegPlanPerThread
// consecutive segments; returns the thread's exclusive start inside the block
// and the block total in *total.
__device__ __forceinline__ uint64_t chunk_tiles(const uint64_t* off, uint32_t nseg, uint64_t n, uint32_t tile,
                                                uint32_t* wide, uint64_t* s_scan, uint64_t* total) {
  const uint32_t s0 = blockIdx.x * kSegChunk + threadIdx.x * kSegPlanPerThread;
  uint64_t mine = 0;
  bool long_seg = false;
#pragma unroll
  for (int i = 0; i < kSegPlanPerThread; ++i)
    if (s0 + i < nseg) {
      uint64_t b;
      const uint64_t len = segment_span(off, s0 + i, n, &b);
      mine += (len + tile - 1) / tile;
      long_seg = long_seg || len >= kWideSegment;
    }
  if (long_seg) atomicOr(wide, 1u);
  return block_exclusive_scan_radix<kSegPlanThreads>(mine, s_scan, total);
}

// Plan step 1: tiles per chunk of segments.
__global__ __launch_bounds__(kSegPlanThreads) void segsweep_count_kernel(const uint64_t* __restrict__ off,
                                                                        uint32_t nseg, uint64_t n, uint32_t tile,
                                                                        uint32_t* wide,
                                                                        uint64_t* __restrict__ chunk_start) {
  __shared__ uint64_t s_scan[kRadix / kWave];
  uint64_t total;
  chunk_tiles(off, nseg, n, tile, wide, s_scan, &total);
  if (threadIdx.x == 0) chunk_start[blockIdx.x] = total;
}

// The pass plan of the segment passes (one thread): all P passes run,
// ping-ponging so that the last one writes keys_out.
template <typename K, bool VALS>
__device__ void write_segsweep_plan(SortPlan* plan, const Buffers& buf) {
  constexpr int P = sizeof(K);
  for (int p = 0; p < kMaxPasses; ++p) {
    PassPlan pp = {};
    if (p < P) {
      const bool to_out = p % 2 == 1;
      pp.src_k = p == 0 ? buf.keys_in : (to_out ? buf.alt_k : buf.keys_out);
      pp.dst_k = to_out ? buf.keys_out : buf.alt_k;
      pp.src_v = p == 0 ? buf.vals_in : (to_out ? buf.alt_v : buf.vals_out);
      pp.dst_v = VALS ? (to_out ? buf.vals_out : buf.alt_v) : nullptr;
      pp.active = 1;
      pp.first = p == 0;
      pp.last = p == P - 1;
    }
    plan->pass[p] = pp;
  }
  plan->copy = 0;
  plan->copy_src_k = nullptr;
  plan->copy_dst_k = nullptr;
  plan->copy_src_v = nullptr;
  plan->copy_dst_v = nullptr;
  plan->num_active = P;
}

// The one-launch path splits the tile table (segment order) into kMaxQueues
// contiguous queues of about equal tile counts, at segment boundaries: queue
// q starts at the first segment whose first tile is at or after
// ceil(q * total / kMaxQueues); a queue no segment starts in is empty.
// Every start defaults to the tile count (queue 0's to 0) ...
__device__ __forceinline__ void queue_start_defaults(uint32_t* qtab, uint32_t total) {
  qtab[kQStarts] = 0;
  for (int q = 1; q <= kMaxQueues; ++q) qtab[kQStarts + q] = total;
}

// ... and the one segment that crosses each boundary writes that queue's
// start: the segment starting at tile g whose predecessor starts at tile
// prev (prev_known false for segment 0).
__device__ __forceinline__ void mark_queue_starts(uint32_t* qtab, uint32_t total, uint64_t g, uint64_t prev,
                                                  bool prev_known) {
  for (int q = 1; q < kMaxQueues; ++q) {
    const uint64_t b = (static_cast<uint64_t>(q) * total + kMaxQueues - 1) / kMaxQueues;
    if ((!prev_known || prev < b) && b <= g) qtab[kQStarts + q] = static_cast<uint32_t>(g < total ? g : total);
  }
}

// Plan step 2 (one block): chunk starts by an exclusive scan of their tile
// counts, the tile count, and the pass plan (and, given qtab, the queue
// starts' defaults).
template <typename K, bool VALS>
__global__ __launch_bounds__(kSegPlanThreads) void segsweep_plan_kernel(uint64_t* __restrict__ chunk_start,
                                                                       uint32_t chunks, uint32_t max_tiles,
                                                                       uint32_t* __restrict__ num_tiles,
                                                                       SortPlan* plan, Buffers buf,
                                                                       uint32_t* __restrict__ qtab) {
  __shared__ uint64_t s_scan[kRadix / kWave];
  const int tid = threadIdx.x;
  uint64_t carry = 0;  // the same in every thread
  for (uint32_t c0 = 0; c0 < chunks; c0 += kSegPlanThreads) {
    const uint32_t c = c0 + tid;
    const uint64_t v = c < chunks ? chunk_start[c] : 0u;
    uint64_t sum;
    const uint64_t ex = block_exclusive_scan_radix<kSegPlanThreads>(v, s_scan, &sum);
    if (c < chunks) chunk_start[c] = carry + ex;
    carry += sum;
  }
  if (tid != 0) return;
  // Offsets within the contract give at most max_tiles tiles (the size of
  // the record and status tables); overlapping ones may give more, which
  // are dropped.
  *num_tiles = static_cast<uint32_t>(carry < max_tiles ? carry : max_tiles);
  if (qtab) queue_start_defaults(qtab, *num_tiles);
  write_segsweep_plan<K, VALS>(plan, buf);
}

// Plan step 3: the records of this block's chunk of segments, whose first
// tile is number `base`; written by all threads of the block (a tile finds
// its segment by a binary search over the chunk's segment starts in LDS).
// Records from max_tiles on are not written: the local starts are held
// saturated at the room left below max_tiles.  Returns the chunk's tile
// count.  Given qtab, also marks the queue starts that fall in the chunk
// (num_tiles: the tile count from plan step 2, or nullptr when this block
// holds every segment and sets the defaults itself).
__device__ uint64_t fill_chunk(const uint64_t* __restrict__ off, uint32_t nseg, uint64_t n, uint32_t tile,
                               uint64_t base, uint32_t max_tiles, uint32_t* wide, SegTile* __restrict__ tiles,
                               uint32_t* qtab, const uint32_t* num_tiles) {
  __shared__ uint64_t s_scan[kRadix / kWave];
  __shared__ uint32_t s_start[kSegChunk + 1];  // tile start of each segment of the chunk, block-relative
  __shared__ uint64_t s_off[kSegChunk + 1];    // the chunk's offsets, clamped to n
  const uint32_t first_seg = blockIdx.x * kSegChunk;
  const uint32_t nloc = nseg - first_seg < kSegChunk ? nseg - first_seg : kSegChunk;
  const uint32_t room = static_cast<uint32_t>(base < max_tiles ? max_tiles - base : 0u);
  uint64_t total;
  const uint64_t start = chunk_tiles(off, nseg, n, tile, wide, s_scan, &total);
  uint32_t all = 0;  // the capped tile count, for the queue starts
  if (qtab) {
    if (num_tiles) {
      all = *num_tiles;
    } else {
      all = static_cast<uint32_t>(total < max_tiles ? total : max_tiles);
      if (threadIdx.x == 0) queue_start_defaults(qtab, all);
      __syncthreads();
    }
  }
  {
    const uint32_t l0 = threadIdx.x * kSegPlanPerThread;
    uint64_t run = start;
#pragma unroll
    for (int i = 0; i < kSegPlanPerThread; ++i)
      if (l0 + i < nloc) {
        s_start[l0 + i] = static_cast<uint32_t>(run < room ? run : room);
        const uint32_t sg = first_seg + l0 + i;
        const uint64_t len = segment_tiles(off, sg, n, tile);
        if (qtab) {
          const uint64_t g = base + run;
          const uint64_t prev = sg == 0 ? 0 : g - segment_tiles(off, sg - 1, n, tile);
          mark_queue_starts(qtab, all, g, prev, sg != 0);
        }
        run += len;
      }
    if (threadIdx.x == 0) s_start[nloc] = static_cast<uint32_t>(total < room ? total : room);
    for (uint32_t i = threadIdx.x; i <= nloc; i += kSegPlanThreads) {
      const uint64_t v = off[first_seg + i];
      s_off[i] = v < n ? v : n;
    }
  }
  __syncthreads();
  const uint32_t end = s_start[nloc];
  for (uint32_t t = threadIdx.x; t < end; t += kSegPlanThreads) {
    // The last local segment whose start is <= t: a non-empty one, since
    // t < its successor's start.
    uint32_t lo = 0, hi = nloc;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) / 2;
      if (s_start[mid] <= t)
        lo = mid;
      else
        hi = mid;
    }
    const uint32_t s = first_seg + lo;
    const uint32_t j = t - s_start[lo];
    const uint64_t sb = s_off[lo], se = s_off[lo + 1] > sb ? s_off[lo + 1] : sb;  // as segment_span
    const uint64_t b = sb + static_cast<uint64_t>(j) * tile;
    const uint64_t e = se;
    const uint32_t cnt = static_cast<uint32_t>(e - b < static_cast<uint64_t>(tile) ? e - b : tile);
    const bool only = s_start[lo + 1] - s_start[lo] == 1;
    SegTile r;
    r.begin = b;
    r.count = cnt | (j == 0 ? kTileFirst : 0u) | (only ? kTileOnly : 0u);
    r.seg = s;
    tiles[base + t] = r;
  }
  return total;
}

__global__ __launch_bounds__(kSegPlanThreads) void segsweep_fill_kernel(const uint64_t* __restrict__ off,
                                                                       uint32_t nseg, uint64_t n, uint32_t tile,
                                                                       const uint64_t* __restrict__ chunk_start,
                                                                       uint32_t max_tiles, uint32_t* wide,
                                                                       SegTile* __restrict__ tiles,
                                                                       uint32_t* __restrict__ qtab,
                                                                       const uint32_t* __restrict__ num_tiles) {
  fill_chunk(off, nseg, n, tile, chunk_start[blockIdx.x], max_tiles, wide, tiles, qtab, num_tiles);
}

// The whole plan in one launch when the segments form one chunk (at most
// kSegChunk): records, tile count and pass plan.
template <typename K, bool VALS>
__global__ __launch_bounds__(kSegPlanThreads) void segsweep_plan1_kernel(const uint64_t* __restrict__ off,
                                                                        uint32_t nseg, uint64_t n, uint32_t tile,
                                                                        uint32_t max_tiles, uint32_t* wide,
                                                                        uint32_t* __restrict__ num_tiles,
                                                                        SegTile* __restrict__ tiles, SortPlan* plan,
                                                                        Buffers buf, uint32_t* __restrict__ qtab) {
  const uint64_t total = fill_chunk(off, nseg, n, tile, 0u, max_tiles, wide, tiles, qtab, nullptr);
  if (threadIdx.x != 0) return;
  *num_tiles = static_cast<uint32_t>(total < max_tiles ? total : max_tiles);
  write_segsweep_plan<K, VALS>(plan, buf);
}

// Digit histograms of every segment of more than one tile (all P digit
// positions): each block counts a contiguous range of tiles in LDS and adds
// its counts to the segment's row whenever the segment changes.
template <typename K, typename C>
__global__ __launch_bounds__(256) void segsweep_hist_kernel(const K* __restrict__ keys, K flip,
                                                            const SegTile* __restrict__ tiles,
                                                            const uint32_t* __restrict__ num_tiles,
                                                            C* __restrict__ seg_hist) {
  constexpr int P = sizeof(K);
  constexpr int kCopies = 64 / P;
  constexpr int kInFlight = 16;  // loads per thread issued before their counts
  __shared__ uint32_t h[P * kRadix * kCopies];
  const int tid = threadIdx.x;
  for (int i = tid; i < P * kRadix * kCopies; i += 256) h[i] = 0;
  __syncthreads();
  const uint32_t total = *num_tiles;
  const uint32_t t0 = static_cast<uint32_t>(static_cast<uint64_t>(total) * blockIdx.x / gridDim.x);
  const uint32_t t1 = static_cast<uint32_t>(static_cast<uint64_t>(total) * (blockIdx.x + 1) / gridDim.x);
  const uint32_t copy = lane_id() % kCopies;
  auto flush = [&](uint32_t s) {
    __syncthreads();
    for (int b = tid; b < P * kRadix; b += 256) {
      uint32_t sum = 0;
#pragma unroll
      for (int c = 0; c < kCopies; ++c) {
        sum += h[b * kCopies + c];
        h[b * kCopies + c] = 0;
      }
      if (sum) atomic_add_c(&seg_hist[static_cast<size_t>(s) * P * kRadix + b], static_cast<C>(sum));
    }
    __syncthreads();
  };
  uint32_t cur = ~0u;
  for (uint32_t t = t0; t < t1; ++t) {
    const SegTile r = tiles[t];
    if (r.count & kTileOnly) continue;  // uniform over the block
    if (r.seg != cur && cur != ~0u) flush(cur);
    cur = r.seg;
    const uint32_t cnt = r.count & kTileCountMask;
    const K* src = keys + r.begin;
    for (uint32_t i0 = 0; i0 < cnt; i0 += 256 * kInFlight) {
      K v[kInFlight];
#pragma unroll
      for (int q = 0; q < kInFlight; ++q) {
        const uint32_t i = i0 + q * 256 + tid;
        v[q] = i < cnt ? src[i] : K(0);
      }
#pragma unroll
      for (int q = 0; q < kInFlight; ++q) {
        if (i0 + q * 256 + tid < cnt) {
          const K k = flip_key(v[q], flip);
#pragma unroll
          for (int p = 0; p < P; ++p) atomicAdd(&h[(p * kRadix + digit_of(k, 8 * p)) * kCopies + copy], 1u);
        }
      }
    }
  }
  if (cur != ~0u) flush(cur);
}

// Digit bases: row (s, p) of seg_base = off[s] + exclusive scan of the
// segment's digit-p counts.  One block per row; one-tile segments have no
// histogram and need no bases.
template <typename C>
__global__ __launch_bounds__(256) void segsweep_base_kernel(const uint64_t* __restrict__ off, uint64_t n, int P,
                                                            uint32_t tile, const C* __restrict__ seg_hist,
                                                            C* __restrict__ seg_base) {
  __shared__ C s_scan[kRadix / kWave];
  const uint32_t row = blockIdx.x;
  const uint64_t s = row / P;
  uint64_t b;
  if (segment_span(off, s, n, &b) <= tile) return;
  const C c = seg_hist[static_cast<size_t>(row) * kRadix + threadIdx.x];
  C total;
  const C ex = block_exclusive_scan_radix<256>(c, s_scan, &total);
  seg_base[static_cast<size_t>(row) * kRadix + threadIdx.x] = static_cast<C>(b) + ex;
}

// One digit pass over the tiles of every segment (persistent workgroups,
// tiles by ticket as in onesweep_kernel, without agents or LDS prefetch).
template <typename K, bool VALS, typename C, typename S, int THREADS>
__global__ __launch_bounds__(THREADS) void segsweep_pass_kernel(
    const SortPlan* __restrict__ plan, int pass, const SegTile* __restrict__ tiles,
    const uint32_t* __restrict__ num_tiles_p, C n, K flip, const C* __restrict__ seg_base, uint32_t* tile_counter,
    S* status_cur, S* status_next, const uint32_t* __restrict__ gate, uint32_t want) {
  // Lists of 2^30 keys and more launch the pass with both status widths; the
  // planner's flag (a segment of 2^30 keys or more) lets exactly one run.
  if (gate != nullptr && *gate != want) return;
  constexpr int kThreads = THREADS;
  constexpr int kKpt = PassCfg<THREADS>::kKpt;
  constexpr int kTile = PassCfg<THREADS>::kTile;
  constexpr int P = sizeof(K);
  using St = Status<S>;

  constexpr int kStageBytes = padded16(kTile) * static_cast<int>(sizeof(K));
  constexpr int kCountBytes = SplitScratch<kThreads>::kCountWords * 4;
  __shared__ __attribute__((aligned(16))) uint8_t s_raw[kStageBytes > kCountBytes ? kStageBytes : kCountBytes];
  K* s_stage = reinterpret_cast<K*>(s_raw);
  uint32_t* s_counts = reinterpret_cast<uint32_t*>(s_raw);
  __shared__ uint32_t s_vstage[VALS ? padded16(kTile) : 1];
  __shared__ uint32_t s_hist[kRadix];
  __shared__ C s_doff[kRadix];
  __shared__ uint32_t s_scan[kThreads / kWave];
  __shared__ C s_cscan[kRadix / kWave];
  __shared__ uint32_t s_ticket;

  const int tid = threadIdx.x;
  if (tid == 0) s_ticket = atomicAdd(tile_counter, 1u);
  __syncthreads();
  const uint32_t num_tiles = *num_tiles_p;
  uint32_t tile = s_ticket;
  if (tile >= num_tiles) return;

  const PassPlan& pp = plan->pass[pass];
  const int shift = 8 * pass;
  const gptr<const K> src = as_global(static_cast<const K*>(pp.src_k));
  const gptr<const uint32_t> src_v = as_global(static_cast<const uint32_t*>(pp.src_v));
  const gptr<K> dst = as_global(static_cast<K*>(pp.dst_k));
  const gptr<uint32_t> dst_v = as_global(pp.dst_v);
  const K in_flip = pp.first ? flip : K(0);
  const K out_flip = pp.last ? flip : K(0);
  const K pad = ~K(0) ^ in_flip;  // decodes to all-ones: sorts after every real key of the tile

  // The tile's record: first key, key count and flags, segment.
  SegTile r = tiles[tile];
  C tile_base = static_cast<C>(r.begin);
  C tile_end = tile_base + static_cast<C>(r.count & kTileCountMask);

  K keys[kKpt];
  uint32_t vals[kKpt];
  load_tile_keys<K, VALS, C, kKpt>(src, src_v, tile_base + static_cast<C>(tid) * kKpt, tile_end, pad, keys, vals);

  while (true) {
    const bool first = (r.count & kTileFirst) != 0;
    const bool only = (r.count & kTileOnly) != 0;
#pragma unroll
    for (int q = 0; q < kKpt; ++q) keys[q] = flip_key(keys[q], in_flip);
    if (status_next)
      for (int d = tid; d < kRadix; d += kThreads) status_next[static_cast<size_t>(tile) * kRadix + d] = 0;
    for (int d = tid; d < kRadix; d += kThreads) s_hist[d] = 0;
    lds_barrier();

    {
      const uint32_t d0 = digit_of(keys[0], shift);
      bool same = true;
#pragma unroll
      for (int q = 1; q < kKpt; ++q) same = same && digit_of(keys[q], shift) == d0;
      const uint32_t w0 = __builtin_amdgcn_readfirstlane(d0);
      if (__builtin_amdgcn_ballot_w64(same && d0 == w0) == ~0ull) {
        if (lane_id() == 0) atomicAdd(&s_hist[w0], static_cast<uint32_t>(kWave * kKpt));
      } else {
#pragma unroll
        for (int q = 0; q < kKpt; ++q) atomicAdd(&s_hist[digit_of(keys[q], shift)], 1u);
      }
    }
    lds_barrier();

    // A segment's first tile has no predecessor in its segment; a segment's
    // only tile has no successor either, and publishes nothing.
    S* st = status_cur + static_cast<size_t>(tile) * kRadix + tid;
    uint32_t cnt = 0;
    if (tid < kRadix) {
      cnt = s_hist[tid];
      if (!only) status_store(st, (first ? St::kInc : St::kAgg) | static_cast<S>(cnt));
    }
    uint32_t ticket = 0;
    if (tid == 0) ticket = atomicInc(tile_counter, ~0u);

    tile_split_stage<kThreads, kKpt, VALS>(keys, vals, shift, s_stage, s_vstage, s_counts, s_scan, true);
    S pred = 0;
    if (tid < kRadix && !first) pred = status_load(st - kRadix);
    tile_split_stage<kThreads, kKpt, VALS>(keys, vals, shift + kSubBits, s_stage, s_vstage, s_counts, s_scan, false);

    if (tid == 0) s_ticket = ticket;
    C tile_total;
    const C start = block_exclusive_scan_radix<kThreads>(static_cast<C>(cnt), s_cscan, &tile_total);

    // The next tile's keys load into the registers during the look-back.
    const uint32_t next = s_ticket;
    const bool more = next < num_tiles;
    const uint32_t cur_seg = r.seg;
    const C cur_base = tile_base, cur_end = tile_end;
    if (more) {
      r = tiles[next];
      tile_base = static_cast<C>(r.begin);
      tile_end = tile_base + static_cast<C>(r.count & kTileCountMask);
      load_tile_keys<K, VALS, C, kKpt>(src, src_v, tile_base + static_cast<C>(tid) * kKpt, tile_end, pad, keys, vals);
    }

    if (tid < kRadix) {
      if (only) {
        s_doff[tid] = cur_base;  // the segment's digit-d keys start at cur_base + start[d]: the tile in place
      } else {
        C excl = 0;
        if (!first) {
          excl = (pred & St::kFlagMask) == St::kInc ? static_cast<C>(pred & St::kValMask)
                                                    : lookback<C, S, 4>(st, tile, kRadix);
          status_store(st, St::kInc | static_cast<S>(excl + cnt));
        }
        s_doff[tid] = seg_base[(static_cast<size_t>(cur_seg) * P + pass) * kRadix + tid] + excl - start;
      }
    }
    lds_barrier();

    const C remaining = cur_end - cur_base;
    const int valid = remaining < static_cast<C>(kTile) ? static_cast<int>(remaining) : kTile;
    // Destinations lie inside the tile's segment whenever the offsets keep
    // the contract; the clamp (a branch here costs ~10 % of the pass) keeps
    // overlapping segments, whose keys other tiles rewrite between passes,
    // inside the array.
#pragma unroll 4
    for (int i = tid; i < valid; i += kThreads) {
      const K k = s_stage[pad16(i)];
      C o = s_doff[digit_of(k, shift)] + static_cast<C>(i);
      o = o < n ? o : n - 1;
      dst[o] = k ^ out_flip;
      if constexpr (VALS) dst_v[o] = s_vstage[pad16(i)];
    }
    if (!more) break;
    tile = next;
    lds_barrier();  // the stage, s_doff and s_hist are reused by the next tile
  }
}

// ---------------------------------------------------------------------------
// 6. The same segment passes as ONE persistent launch: a work queue of
// (phase, tile) items over the tile table above.  Phase 0 of a segment of
// several tiles counts its keys for the P digit histograms; phase 1 + p is
// digit pass p over its tiles (decoupled look-back inside the segment, bases
// from the segment's histogram).  A segment of one tile is sorted whole in
// LDS in phase 0 and has nothing to do in the later phases.
//
// XCD-aware: the chip's L2 is one cache per XCD, and one XCD's L2 is not
// kept coherent with another's inside a kernel.  Keys written in one phase
// are read by other workgroups in the next, so every segment is given to one
// XCD: the table is cut into kMaxQueues queues of consecutive segments with
// about equal tile counts, and each queue is served by one XCD -- queue x by
// the XCD whose XCC_ID is x, claimed for it by the first of its workgroups.
// A workgroup whose queue has no tickets left claims an unclaimed queue that
// still has some (so that every queue is served on a device with fewer
// XCDs), and exits when there is none.
//
// Tickets of a queue run phase-major (every tile's phase 0, then every tile's
// phase 1, ...), and an item of phase f > 0 waits until every item of phase
// f - 1 of its queue has counted itself done (a count per phase and queue).
// An item only waits for items with earlier tickets of its own queue -- that
// count and, inside a pass, the look-back -- so no wait can deadlock, even
// with a workgroup holding its next ticket while it runs the current item
// (tickets run one item ahead).  A finishing item waits for its own stores
// before it counts itself done; a workgroup that sees a phase complete
// invalidates its CU's L1 and its XCD's non-coherent L2 lines before reading
// the keys of the next phase (once per phase and workgroup).  Look-back
// status words and the per-segment histograms are read and written with
// device-coherent atomics, as in the other passes.
//
// Look-back rows: two buffers, pass p in buffer p % 2; phase 0 clears a
// tile's row in both, and pass p (p >= 1) clears the tile's row of buffer
// (p + 1) % 2 for pass p + 1, once pass p - 1 -- the last reader of that
// row -- is complete.

__device__ __forceinline__ uint32_t xcc_id() {
#if defined(__HIP_DEVICE_COMPILE__)
  uint32_t v;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
  return v & 0xF;
#else
  return blockIdx.x % kMaxQueues;  // the dispatch order the register reports on the GPU
#endif
}

// Invalidates this CU's vector L1 and the non-coherent lines of its XCD's L2
// (the acquire side of device scope), so that the following loads read what
// other CUs have written.  Measured: the L1 invalidation alone still let
// stale keys through to the next phase now and then.
__device__ __forceinline__ void invalidate_caches() {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("buffer_inv sc1" ::: "memory");
#endif
}

// The claim of a ticket by thread 0: from queue q while it has tickets left
// (t_first: a ticket of q already taken, or ~0u to take one here), else from
// this XCD's own queue (number XCC_ID, claimed for the XCD by whichever of its
// workgroups comes first), else from another queue this XCD owns with tickets
// left, else from a queue claimed now for this XCD.  Returns the queue (-1:
// none is left) and the ticket in *t.  With as many queues as XCDs every XCD
// serves its own; the other claims keep every queue served on a device with
// fewer XCDs (or other XCC_IDs).
template <int P>
__device__ int claim_ticket(uint32_t* qtab, uint32_t nq, uint32_t me, int q, uint32_t t_first, uint32_t* t) {
  uint32_t* const owner = qtab + kQOwners;
  auto total = [&](uint32_t k) { return (P + 1) * (qtab[kQStarts + k + 1] - qtab[kQStarts + k]); };
  auto left = [&](uint32_t k) {
    return __hip_atomic_load(&qtab[kQTickets + k * kLineWords], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
           total(k);
  };
  auto owner_of = [&](uint32_t k) { return __hip_atomic_load(&owner[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); };
  bool have = t_first != ~0u;
  while (true) {
    if (q >= 0) {
      const uint32_t tot = total(q);
      const uint32_t v = have ? t_first : atomicAdd(&qtab[kQTickets + q * kLineWords], 1u);
      have = false;
      if (v < tot) {
        *t = v;
        return q;
      }
      q = -1;
    }
    const uint32_t x = me - 1;
    if (x < nq) {
      uint32_t v = owner_of(x);
      if (v == 0) {
        v = atomicCAS(&owner[x], 0u, me);
        if (v == 0) v = me;
      }
      if (v == me && left(x)) {
        q = static_cast<int>(x);
        continue;
      }
    }
    for (uint32_t k = 0; k < nq && q < 0; ++k)
      if (owner_of(k) == me && left(k)) q = static_cast<int>(k);
    if (q >= 0) continue;
    // No queue of this XCD has tickets left: claim the first unclaimed one.
    // A lost race means another workgroup -- perhaps of this XCD -- just
    // claimed it: look at the owned queues again before claiming another.
    // Owners only ever change from 0, so this ends after at most nq lost
    // races.
    bool unclaimed = false;
    for (uint32_t k = 0; k < nq; ++k) {
      if (owner_of(k) != 0 || !left(k)) continue;
      unclaimed = true;
      if (atomicCAS(&owner[k], 0u, me) == 0u) q = static_cast<int>(k);
      break;
    }
    if (!unclaimed) return -1;
  }
}

template <typename K, bool VALS, typename C, typename S>
__device__ __forceinline__ void segqueue_body(const SortPlan* __restrict__ plan, const SegTile* __restrict__ tiles,
                                              uint32_t* __restrict__ qtab, const uint64_t* __restrict__ off,
                                              uint64_t n, K flip, C* __restrict__ seg_hist, S* status0, S* status1,
                                              const uint32_t* __restrict__ gate, uint32_t want) {
  // Lists of 2^30 keys and more launch the queue with both status widths;
  // the planner's flag (a segment of 2^30 keys or more) lets exactly one run.
  if (gate != nullptr && *gate != want) return;
  constexpr uint32_t nq = kMaxQueues;
  constexpr int kThreads = kSegSweepThreads;
  constexpr int kKpt = PassCfg<kThreads>::kKpt;
  constexpr int kTile = PassCfg<kThreads>::kTile;
  constexpr int P = sizeof(K);
  using St = Status<S>;

  constexpr int kStageBytes = padded16(kTile) * static_cast<int>(sizeof(K));
  constexpr int kCountBytes = SplitScratch<kThreads>::kCountWords * 4;
  constexpr int kRawBytes = std::max(std::max(kStageBytes, kCountBytes), P * kRadix * 4);
  __shared__ __attribute__((aligned(16))) uint8_t s_raw[kRawBytes];
  K* s_stage = reinterpret_cast<K*>(s_raw);
  uint32_t* s_counts = reinterpret_cast<uint32_t*>(s_raw);
  uint32_t* s_h = reinterpret_cast<uint32_t*>(s_raw);  // phase 0: P x kRadix counters
  __shared__ uint32_t s_vstage[VALS ? padded16(kTile) : 1];
  __shared__ uint32_t s_hist[kRadix];
  __shared__ C s_doff[kRadix];
  __shared__ uint32_t s_scan[kThreads / kWave];
  __shared__ C s_cscan[kRadix / kWave];
  __shared__ C s_cscan2[kRadix / kWave];
  __shared__ int s_q;
  __shared__ uint32_t s_ticket;

  const int tid = threadIdx.x;
  const uint32_t me = xcc_id() + 1;

  // The first ticket.
  if (tid == 0) {
    uint32_t t = 0;
    s_q = claim_ticket<P>(qtab, nq, me, -1, ~0u, &t);
    s_ticket = t;
  }
  __syncthreads();
  // The current item's queue and ticket, uniform: kept in scalar registers.
  int q = __builtin_amdgcn_readfirstlane(s_q);
  uint32_t ticket = __builtin_amdgcn_readfirstlane(s_ticket);
  int known = -1;              // phases of queue q known to be complete: 0 .. known
  bool loaded = false;         // the current item's keys are already in `keys`
  K keys[kKpt];
  uint32_t vals[kKpt];

  while (q >= 0) {
    const uint32_t T = qtab[kQStarts + q + 1] - qtab[kQStarts + q];
    const uint32_t phase = ticket / T;
    const uint32_t i = qtab[kQStarts + q] + ticket % T;
    uint32_t* const qdone = qtab + kQDone + q * kLineWords;
    const SegTile r = tiles[i];
    const uint32_t cnt = r.count & kTileCountMask;
    const uint64_t tbeg = r.begin;
    const uint64_t tend = tbeg + cnt;
    const bool only = (r.count & kTileOnly) != 0;
    const bool first = (r.count & kTileFirst) != 0;
    const uint32_t seg = r.seg;
    C* const h = seg_hist + static_cast<size_t>(seg) * P * kRadix;

    // The next ticket of this queue, taken now and resolved later: tickets
    // run one item ahead.
    uint32_t raw_next = 0;
    if (tid == 0) raw_next = atomicAdd(&qtab[kQTickets + q * kLineWords], 1u);

    if (only || phase == 0) {
      if (only && phase == 0) {
        // The whole segment in one tile: every digit pass in LDS, in place.
        const K* src = static_cast<const K*>(plan->pass[0].src_k);
        const uint32_t* srcv = plan->pass[0].src_v;
        K* dst = static_cast<K*>(plan->pass[P - 1].dst_k);
        uint32_t* dstv = plan->pass[P - 1].dst_v;
        load_tile_keys<K, VALS, uint64_t, kKpt>(as_global(src), as_global(srcv),
                                                tbeg + static_cast<uint64_t>(tid) * kKpt, tend, ~K(0) ^ flip, keys,
                                                vals);
#pragma unroll
        for (int k = 0; k < kKpt; ++k) keys[k] = flip_key(keys[k], flip);
        for (int p = 0; p < P; ++p)
          tile_sort_digit<kThreads, kKpt, VALS>(keys, vals, 8 * p, s_stage, s_vstage, s_counts, s_scan,
                                                p + 1 < P);
        for (int e = tid; e < static_cast<int>(cnt); e += kThreads) {
          dst[tbeg + e] = s_stage[pad16(e)] ^ flip;
          if constexpr (VALS) dstv[tbeg + e] = s_vstage[pad16(e)];
        }
      } else if (!only) {
        // Phase 0: the tile's counts of every digit added to its segment's
        // histograms; its look-back rows cleared in both buffers.  Keys are
        // read striped (lane-consecutive, whatever the segment's alignment)
        // and counted into kCopies copies of the counters, lane l using copy
        // l % kCopies, so that lanes meeting on a bin rarely share a word.
        constexpr int kCopies = 32 / P;
        static_assert(P * kRadix * kCopies * 4 <= kRawBytes, "counter copies fit the stage");
        for (int e = tid; e < kRadix; e += kThreads) {
          status_store(&status0[static_cast<size_t>(i) * kRadix + e], S(0));
          status_store(&status1[static_cast<size_t>(i) * kRadix + e], S(0));
        }
        for (int e = tid; e < P * kRadix * kCopies; e += kThreads) s_h[e] = 0;
        __syncthreads();
        const gptr<const K> hsrc = as_global(static_cast<const K*>(plan->pass[0].src_k)) + tbeg;
#pragma unroll
        for (int k = 0; k < kKpt; ++k) {
          const uint32_t e = static_cast<uint32_t>(k * kThreads + tid);
          keys[k] = e < cnt ? hsrc[e] : K(0);
        }
        const uint32_t copy = lane_id() % kCopies;
#pragma unroll
        for (int k = 0; k < kKpt; ++k) {
          if (static_cast<uint32_t>(k * kThreads + tid) < cnt) {
            const K key = flip_key(keys[k], flip);
#pragma unroll
            for (int p = 0; p < P; ++p) atomicAdd(&s_h[(p * kRadix + digit_of(key, 8 * p)) * kCopies + copy], 1u);
          }
        }
        __syncthreads();
        for (int e = tid; e < P * kRadix; e += kThreads) {
          uint32_t sum = 0;
#pragma unroll
          for (int c = 0; c < kCopies; ++c) sum += s_h[e * kCopies + c];
          if (sum) atomic_add_c(&h[e], static_cast<C>(sum));
        }
      }
      // Every wave's stores and atomics complete before the item counts
      // itself done (a one-tile segment's later phases have nothing to do).
      __builtin_amdgcn_s_waitcnt(waitcnt_vmcnt(0));
      __syncthreads();
      if (tid == 0) {
        __hip_atomic_fetch_add(&qdone[phase], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t t = 0;
        const int nq2 = claim_ticket<P>(qtab, nq, me, q, raw_next, &t);
        s_q = nq2;
        s_ticket = t;
      }
      __syncthreads();
      const int q2 = __builtin_amdgcn_readfirstlane(s_q);
      if (q2 != q) known = -1;
      q = q2;
      ticket = __builtin_amdgcn_readfirstlane(s_ticket);
      loaded = false;
      __syncthreads();  // s_q and s_ticket are written again by the next item
      continue;
    }

    // Digit pass p of a tile of a segment of several tiles, once phase p - 1
    // (and so every earlier phase) of the whole queue is complete.
    const int p = static_cast<int>(phase) - 1;
    if (known < static_cast<int>(phase) - 1) {
      if (tid == 0) {
        // Back off while waiting: every poll is a device-coherent read of the
        // line that finishing items count themselves done on.
        int nap = 1;
        while (__hip_atomic_load(&qdone[phase - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < T) {
          for (int k = 0; k < nap; ++k) __builtin_amdgcn_s_sleep(8);
          nap = nap < 16 ? 2 * nap : 16;
        }
      }
      __syncthreads();
      invalidate_caches();  // the previous phase's keys, written by other CUs
      known = static_cast<int>(phase) - 1;
    }
    uint64_t sb;
    (void)segment_span(off, seg, n, &sb);
    const C hc = tid < kRadix
                     ? __hip_atomic_load(&h[p * kRadix + tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                     : C(0);

    S* const cur = (p & 1) ? status1 : status0;
    if (p >= 1) {
      // The row's last reader, pass p - 1 of this queue, is complete.
      S* const later = (p & 1) ? status0 : status1;
      for (int e = tid; e < kRadix; e += kThreads) status_store(&later[static_cast<size_t>(i) * kRadix + e], S(0));
    }
    const PassPlan& pp = plan->pass[p];
    const int shift = 8 * p;
    const gptr<const K> src = as_global(static_cast<const K*>(pp.src_k));
    const gptr<const uint32_t> src_v = as_global(static_cast<const uint32_t*>(pp.src_v));
    const gptr<K> dst = as_global(static_cast<K*>(pp.dst_k));
    const gptr<uint32_t> dst_v = as_global(pp.dst_v);
    const K in_flip = pp.first ? flip : K(0);
    const K out_flip = pp.last ? flip : K(0);
    const K pad = ~K(0) ^ in_flip;

    if (!loaded)
      load_tile_keys<K, VALS, C, kKpt>(src, src_v, static_cast<C>(tbeg) + static_cast<C>(tid) * kKpt,
                                       static_cast<C>(tend), pad, keys, vals);
#pragma unroll
    for (int k = 0; k < kKpt; ++k) keys[k] = flip_key(keys[k], in_flip);
    for (int e = tid; e < kRadix; e += kThreads) s_hist[e] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kKpt; ++k)
      if (static_cast<uint32_t>(tid * kKpt + k) < cnt) atomicAdd(&s_hist[digit_of(keys[k], shift)], 1u);
    __syncthreads();
    S* const st = cur + static_cast<size_t>(i) * kRadix + tid;
    uint32_t tcnt = 0;
    if (tid < kRadix) {
      tcnt = s_hist[tid];
      status_store(st, (first ? St::kInc : St::kAgg) | static_cast<S>(tcnt));
    }
    tile_split_stage<kThreads, kKpt, VALS>(keys, vals, shift, s_stage, s_vstage, s_counts, s_scan, true);
    // The next item, known by now unless this queue ran out of tickets.
    if (tid == 0) {
      uint32_t t = 0;
      s_q = claim_ticket<P>(qtab, nq, me, q, raw_next, &t);
      s_ticket = t;
    }
    S pred = 0;
    if (tid < kRadix && !first) pred = status_load(st - kRadix);
    tile_split_stage<kThreads, kKpt, VALS>(keys, vals, shift + kSubBits, s_stage, s_vstage, s_counts, s_scan, false);
    C tile_total, seg_total;
    const C start = block_exclusive_scan_radix<kThreads>(static_cast<C>(tcnt), s_cscan, &tile_total);
    const C base = block_exclusive_scan_radix<kThreads>(hc, s_cscan2, &seg_total);

    // The next item's keys load into the registers during the look-back and
    // the scatter when it is a tile of this same pass (of a segment of
    // several tiles): its dependency is then already met.
    const int nq2 = __builtin_amdgcn_readfirstlane(s_q);
    const uint32_t nticket = __builtin_amdgcn_readfirstlane(s_ticket);
    bool next_loaded = false;
    if (nq2 == q && nticket / T == phase) {
      const SegTile nr = tiles[qtab[kQStarts + q] + nticket % T];
      if ((nr.count & kTileOnly) == 0) {
        const C nb = static_cast<C>(nr.begin);
        load_tile_keys<K, VALS, C, kKpt>(src, src_v, nb + static_cast<C>(tid) * kKpt,
                                         nb + static_cast<C>(nr.count & kTileCountMask), pad, keys, vals);
        next_loaded = true;
      }
    }

    if (tid < kRadix) {
      C excl = 0;
      if (!first) {
        excl = (pred & St::kFlagMask) == St::kInc ? static_cast<C>(pred & St::kValMask)
                                                  : lookback<C, S, 4>(st, i, kRadix);
        status_store(st, St::kInc | static_cast<S>(excl + tcnt));
      }
      s_doff[tid] = static_cast<C>(sb) + base + excl - start;
    }
    __syncthreads();
#pragma unroll 4
    for (int e = tid; e < static_cast<int>(cnt); e += kThreads) {
      const K k = s_stage[pad16(e)];
      C o = s_doff[digit_of(k, shift)] + static_cast<C>(e);
      o = o < static_cast<C>(n) ? o : static_cast<C>(n) - 1;
      dst[o] = k ^ out_flip;
      if constexpr (VALS) dst_v[o] = s_vstage[pad16(e)];
    }
    // Every wave's stores complete before the tile counts itself done.
    __builtin_amdgcn_s_waitcnt(waitcnt_vmcnt(0));
    __syncthreads();
    if (tid == 0) __hip_atomic_fetch_add(&qdone[phase], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (nq2 != q) known = -1;
    q = nq2;
    ticket = nticket;
    loaded = next_loaded;
  }
}

template <typename K, bool VALS, typename C, typename S>
__global__ __launch_bounds__(kSegSweepThreads) void segqueue_kernel(
    const SortPlan* __restrict__ plan, const SegTile* __restrict__ tiles, uint32_t* __restrict__ qtab,
    const uint64_t* __restrict__ off, uint64_t n, K flip, C* __restrict__ seg_hist, S* status0, S* status1,
    const uint32_t* __restrict__ gate, uint32_t want) {
  segqueue_body<K, VALS, C, S>(plan, tiles, qtab, off, n, flip, seg_hist, status0, status1, gate, want);
}

// The same for 32-bit keys without values, held to 128 registers so that two
// workgroups share a CU (a few registers spill; with values or 64-bit keys
// the spills would cost more than the second workgroup gains).
template <typename K, bool VALS, typename C, typename S>
__global__ __launch_bounds__(kSegSweepThreads) __attribute__((amdgpu_waves_per_eu(4))) void segqueue_kernel_x2(
    const SortPlan* __restrict__ plan, const SegTile* __restrict__ tiles, uint32_t* __restrict__ qtab,
    const uint64_t* __restrict__ off, uint64_t n, K flip, C* __restrict__ seg_hist, S* status0, S* status1,
    const uint32_t* __restrict__ gate, uint32_t want) {
  segqueue_body<K, VALS, C, S>(plan, tiles, qtab, off, n, flip, seg_hist, status0, status1, gate, want);
}

// ---------------------------------------------------------------------------
// 4. copy n results when the plan asks for it.
template <typename K, bool VALS>
__global__ __launch_bounds__(256) void plan_copy_kernel(const SortPlan* __restrict__ plan, uint64_t n) {
  if (!plan->copy) return;
  const gptr<const K> sk = as_global(static_cast<const K*>(plan->copy_src_k));
  const gptr<K> dk = as_global(static_cast<K*>(plan->copy_dst_k));
  const gptr<const uint32_t> sv = as_global(plan->copy_src_v);
  const gptr<uint32_t> dv = as_global(plan->copy_dst_v);
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    dk[i] = sk[i];
    if constexpr (VALS) dv[i] = sv[i];
  }
}

// ---------------------------------------------------------------------------
// Host side.
struct Layout {
  size_t plan = 0, ctrs = 0, ghist = 0, gbase = 0, status0 = 0, status1 = 0, alt_k = 0, alt_v = 0, total = 0;
  size_t status_bytes = 0;
  uint32_t num_tiles = 0;
  bool big = false;
  bool small = false;
};

Layout make_layout(ms_key_type kt, bool has_vals, uint64_t n) {
  Layout L;
  const int kb = key_bytes(kt);
  const int lds_tile = kb == 4 ? LdsCfg<uint32_t>::kTile : LdsCfg<uint64_t>::kTile;
  if (n <= static_cast<uint64_t>(lds_tile)) {
    L.small = true;
    return L;  // no workspace
  }
  const int P = kb;
  L.big = n >= (1ull << 30);
  const size_t cb = L.big ? 8 : 4;  // counter and status word bytes
  L.num_tiles = static_cast<uint32_t>((n + kMinPassTile - 1) / kMinPassTile);
  size_t off = 0;
  L.plan = off;
  off += align_up(sizeof(SortPlan));
  L.ctrs = off;
  off += align_up((1 + kMaxPasses) * sizeof(uint32_t));
  L.ghist = off;
  off += align_up(P * kRadix * cb);
  L.gbase = off;
  off += align_up(P * kRadix * cb);
  L.status_bytes = align_up(static_cast<size_t>(L.num_tiles) * kRadix * cb);
  L.status0 = off;
  off += L.status_bytes;
  L.status1 = off;
  off += L.status_bytes;
  L.alt_k = off;
  off += align_up(n * kb);
  if (has_vals) {
    L.alt_v = off;
    off += align_up(n * sizeof(uint32_t));
  }
  L.total = off;
  return L;
}

template <typename K, bool VALS>
ms_status run_small(const void* kin, const uint32_t* vin, void* kout, uint32_t* vout, uint64_t n, K flip,
                    hipStream_t s) {
  MS_LAUNCH("lds_sort", (lds_sort_kernel<K, VALS>), 1, LdsCfg<K>::kThreads, s, static_cast<const K*>(kin), vin,
            static_cast<K*>(kout), vout, static_cast<const uint64_t*>(nullptr),
            static_cast<const uint32_t*>(nullptr), n, flip);
  return MS_OK;
}

// Workgroups of `kernel` the current device holds at once (`fallback` when
// the runtime cannot say), remembered per kernel and device.
uint64_t resident_blocks(const void* kernel, int threads, uint64_t fallback) {
  struct Entry {
    const void* kernel;
    int device;
    uint64_t blocks;
  };
  static std::mutex mu;
  static std::vector<Entry> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fallback;
  {
    std::lock_guard<std::mutex> lock(mu);
    for (const Entry& e : cache)
      if (e.kernel == kernel && e.device == dev) return e.blocks;
  }
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu <= 0 ||
      cus <= 0) {
    (void)hipGetLastError();
    return fallback;
  }
  const uint64_t blocks = static_cast<uint64_t>(per_cu) * static_cast<uint64_t>(cus);
  std::lock_guard<std::mutex> lock(mu);
  cache.push_back({kernel, dev, blocks});
  return blocks;
}

// Compute units of the current device (`fallback` when the runtime cannot say).
uint64_t device_cus(uint64_t fallback) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
    (void)hipGetLastError();
    return fallback;
  }
  return static_cast<uint64_t>(cus);
}

template <typename K, bool VALS, typename C, typename S, int THREADS>
ms_status launch_pass_t(uint64_t n, SortPlan* plan, int p, K flip, const C* gbase, uint32_t* ctr, S* cur, S* next,
                        hipStream_t s) {
  const uint64_t tiles = (n + PassCfg<THREADS>::kTile - 1) / PassCfg<THREADS>::kTile;
  // Persistent workgroups: as many as fit on the device at once (never more
  // than tiles), plus the look-back agents.
  const uint64_t blocks =
      std::min<uint64_t>(tiles, resident_blocks(reinterpret_cast<const void*>(&onesweep_kernel<K, VALS, C, S, THREADS>),
                                                THREADS, tiles)) +
      PassCfg<THREADS>::kAgents;
  MS_LAUNCH("onesweep_pass", (onesweep_kernel<K, VALS, C, S, THREADS>), static_cast<uint32_t>(blocks), THREADS, s,
            static_cast<const SortPlan*>(plan), p, static_cast<C>(n), flip, gbase, ctr, cur, next);
  return MS_OK;
}

// LDS bytes of one onesweep workgroup (the larger of stage and counters, plus
// the value stage); configurations above the 160 KB of a CU fall back.
template <typename K, bool VALS, int THREADS>
constexpr int pass_lds_bytes() {
  constexpr int stage = padded16(PassCfg<THREADS>::kTile) * static_cast<int>(sizeof(K));
  constexpr int counts = SplitScratch<THREADS>::kCountWords * 4;
  constexpr bool prefetch = THREADS == 1024 && sizeof(K) == 4 && !VALS;
  return (stage > counts ? stage : counts) + (VALS ? padded16(PassCfg<THREADS>::kTile) * 4 : 0) +
         (prefetch ? PassCfg<THREADS>::kTile * 4 : 0) + (PassCfg<THREADS>::kAgent ? THREADS * 8 : 0) + 4096;
}

// 1,024-thread tiles are used for 32-bit keys without values, counted in
// 32-bit words (lists below 2^30 keys), only: the other forms need more than
// the 128 VGPRs a 1,024-thread workgroup may hold and would run with register
// spills, so they take 512-thread tiles.
template <typename K, bool VALS, typename S>
constexpr bool pass_1024_ok() {
  return sizeof(K) == 4 && !VALS && sizeof(S) == 4 && pass_lds_bytes<K, VALS, 1024>() <= 160 * 1024;
}

template <typename K, bool VALS, typename C, typename S>
ms_status launch_pass(int threads, uint64_t n, SortPlan* plan, int p, K flip, const C* gbase, uint32_t* ctr, S* cur,
                      S* next, hipStream_t s) {
  switch (threads) {
    case 1024:
      if constexpr (pass_1024_ok<K, VALS, S>())
        return launch_pass_t<K, VALS, C, S, 1024>(n, plan, p, flip, gbase, ctr, cur, next, s);
      else
        return launch_pass_t<K, VALS, C, S, 512>(n, plan, p, flip, gbase, ctr, cur, next, s);
    case 512:
      return launch_pass_t<K, VALS, C, S, 512>(n, plan, p, flip, gbase, ctr, cur, next, s);
    default:
      return launch_pass_t<K, VALS, C, S, 256>(n, plan, p, flip, gbase, ctr, cur, next, s);
  }
}

template <typename K, bool VALS, typename C, typename S>
ms_status run_onesweep(const void* kin, const uint32_t* vin, void* kout, uint32_t* vout, uint64_t n, K flip,
                       char* ws, const Layout& L, hipStream_t s) {
  constexpr int P = sizeof(K);
  SortPlan* plan = reinterpret_cast<SortPlan*>(ws + L.plan);
  uint32_t* ctrs = reinterpret_cast<uint32_t*>(ws + L.ctrs);
  C* ghist = reinterpret_cast<C*>(ws + L.ghist);
  C* gbase = reinterpret_cast<C*>(ws + L.gbase);
  S* status[2] = {reinterpret_cast<S*>(ws + L.status0), reinterpret_cast<S*>(ws + L.status1)};

  const size_t a16 = (L.gbase - L.ctrs) / 16;  // counters + histograms
  const size_t b16 = L.status_bytes / 16;
  MS_LAUNCH("clear", clear_kernel, 1024, 256, s, reinterpret_cast<uint4*>(ws + L.ctrs), a16,
            reinterpret_cast<uint4*>(ws + L.status0), b16);

  Buffers buf = {kin, kout, ws + L.alt_k, vin, vout, VALS ? reinterpret_cast<uint32_t*>(ws + L.alt_v) : nullptr};
  const uint64_t per_block = 256ull * 16;
  uint64_t hblocks = (n + per_block - 1) / per_block;
  // One workgroup per CU by default: the read is bound by the LDS atomics,
  // and a second workgroup per CU only adds its clearing and flushing.
  const int64_t tuned = tune_get(MS_TUNE_HIST_BLOCKS);
  const uint64_t hmax = tuned > 0 ? static_cast<uint64_t>(tuned) : device_cus(256);
  if (hblocks > hmax) hblocks = hmax;
  MS_LAUNCH("histogram", (histogram_kernel<K, C>), static_cast<uint32_t>(hblocks), 256, s,
            static_cast<const K*>(kin), static_cast<C>(n), flip, ghist, gbase, ctrs, plan, buf, VALS ? 1 : 0);

  const int threads = static_cast<int>(tune_get(MS_TUNE_PASS_THREADS));
  for (int p = 0; p < P; ++p) {
    S* next = p + 1 < P ? status[(p + 1) & 1] : nullptr;
    ms_status st = launch_pass<K, VALS, C, S>(threads, n, plan, p, flip, gbase + p * kRadix, ctrs + 1 + p,
                                              status[p & 1], next, s);
    if (st != MS_OK) return st;
  }
  MS_LAUNCH("plan_copy", (plan_copy_kernel<K, VALS>), 1024, 256, s, static_cast<const SortPlan*>(plan), n);
  return MS_OK;
}

template <typename K, bool VALS>
ms_status dispatch(const void* kin, const uint32_t* vin, void* kout, uint32_t* vout, uint64_t n, K flip,
                   void* ws, const Layout& L, hipStream_t s) {
  if (L.small) return run_small<K, VALS>(kin, vin, kout, vout, n, flip, s);
  char* w = static_cast<char*>(ws);
  if (L.big) return run_onesweep<K, VALS, uint64_t, uint64_t>(kin, vin, kout, vout, n, flip, w, L, s);
  return run_onesweep<K, VALS, uint32_t, uint32_t>(kin, vin, kout, vout, n, flip, w, L, s);
}

// ---------------------------------------------------------------------------
// Segmented digit passes (long segments).
struct SegSweepLayout {
  size_t plan = 0, ctrs = 0, hist = 0, qtab = 0, base = 0, chunks = 0, records = 0, status0 = 0, status1 = 0,
         alt_k = 0, alt_v = 0, total = 0;
  size_t ctrs_hist_bytes = 0, status_bytes = 0;
  uint64_t tiles = 0;  // bound on the tile count: every segment adds at most one partial tile
  uint32_t num_chunks = 0;
  bool big = false;
};

SegSweepLayout segsweep_layout(ms_key_type kt, bool has_vals, uint64_t n, uint64_t nseg) {
  SegSweepLayout L;
  const int kb = key_bytes(kt);
  const int P = kb;
  L.big = n >= (1ull << 30);
  const size_t cb = L.big ? 8 : 4;
  L.tiles = (n + SegSweepCfg::kTile - 1) / SegSweepCfg::kTile + nseg;
  L.num_chunks = static_cast<uint32_t>((nseg + kSegChunk - 1) / kSegChunk);
  size_t off = 0;
  L.plan = off;
  off += align_up(sizeof(SortPlan));
  // Counters and histograms are cleared together: ctrs[0] receives the tile
  // count, ctrs[1 + p] is pass p's tile ticket, ctrs[1 + kMaxPasses] the
  // planner's flag for a segment of 2^30 keys or more.
  L.ctrs = off;
  off += align_up((2 + kMaxPasses) * sizeof(uint32_t));
  L.hist = off;
  off += align_up(nseg * P * kRadix * cb);
  L.qtab = off;  // one-launch path: queue table
  off += align_up(kQWordsAll * sizeof(uint32_t));
  L.ctrs_hist_bytes = off - L.ctrs;
  L.base = off;
  off += align_up(nseg * P * kRadix * cb);
  L.chunks = off;  // chunk tile starts
  off += align_up(static_cast<size_t>(L.num_chunks) * sizeof(uint64_t));
  L.records = off;
  off += align_up(static_cast<size_t>(L.tiles) * sizeof(SegTile));
  L.status_bytes = align_up(static_cast<size_t>(L.tiles) * kRadix * cb);
  L.status0 = off;
  off += L.status_bytes;
  L.status1 = off;
  off += L.status_bytes;
  L.alt_k = off;
  off += align_up(n * kb);
  if (has_vals) {
    L.alt_v = off;
    off += align_up(n * sizeof(uint32_t));
  }
  L.total = off;
  return L;
}

// One digit pass of the segment passes; gate/want as in the kernel.
template <typename K, bool VALS, typename C, typename S, int THREADS>
ms_status launch_segsweep_pass(const SortPlan* plan, int p, const SegTile* records, const uint32_t* num_tiles,
                               uint64_t n, K flip, const C* base, uint32_t* counter, char* status_cur,
                               char* status_next, const uint32_t* gate, uint32_t want, uint64_t max_tiles,
                               hipStream_t s) {
  const uint64_t blocks = std::min<uint64_t>(
      max_tiles, resident_blocks(reinterpret_cast<const void*>(&segsweep_pass_kernel<K, VALS, C, S, THREADS>),
                                 THREADS, 256));
  MS_LAUNCH("segsweep_pass", (segsweep_pass_kernel<K, VALS, C, S, THREADS>), static_cast<uint32_t>(blocks), THREADS,
            s, plan, p, records, num_tiles, static_cast<C>(n), flip, base, counter,
            reinterpret_cast<S*>(status_cur), reinterpret_cast<S*>(status_next), gate, want);
  return MS_OK;
}

// The tile table of the segment passes (1 or 3 launches): records in
// segment order, the tile count in ctrs[0], the pass plan and, given qtab,
// the one-launch path's queue starts.
template <typename K, bool VALS>
ms_status plan_segment_tiles(const uint64_t* off, uint32_t nseg, uint64_t n, uint32_t tile, char* ws,
                             const SegSweepLayout& L, const Buffers& buf, uint32_t* qtab, hipStream_t s) {
  SortPlan* plan = reinterpret_cast<SortPlan*>(ws + L.plan);
  uint32_t* ctrs = reinterpret_cast<uint32_t*>(ws + L.ctrs);
  uint64_t* chunk_start = reinterpret_cast<uint64_t*>(ws + L.chunks);
  SegTile* records = reinterpret_cast<SegTile*>(ws + L.records);
  uint32_t* wide = ctrs + 1 + kMaxPasses;
  const uint32_t max_tiles = static_cast<uint32_t>(L.tiles);
  if (L.num_chunks == 1) {
    MS_LAUNCH("segsweep_plan", (segsweep_plan1_kernel<K, VALS>), 1, kSegPlanThreads, s, off, nseg, n, tile,
              max_tiles, wide, ctrs, records, plan, buf, qtab);
  } else {
    MS_LAUNCH("segsweep_plan", segsweep_count_kernel, L.num_chunks, kSegPlanThreads, s, off, nseg, n, tile, wide,
              chunk_start);
    MS_LAUNCH("segsweep_plan", (segsweep_plan_kernel<K, VALS>), 1, kSegPlanThreads, s, chunk_start, L.num_chunks,
              max_tiles, ctrs, plan, buf, qtab);
    MS_LAUNCH("segsweep_plan", segsweep_fill_kernel, L.num_chunks, kSegPlanThreads, s, off, nseg, n, tile,
              static_cast<const uint64_t*>(chunk_start), max_tiles, wide, records, qtab,
              static_cast<const uint32_t*>(ctrs));
  }
  return MS_OK;
}

template <typename K, bool VALS, typename C, int THREADS>
ms_status run_segsweep(const void* kin, const uint32_t* vin, void* kout, uint32_t* vout, const uint64_t* off,
                       uint32_t nseg, uint64_t n, K flip, char* ws, const SegSweepLayout& L, hipStream_t s) {
  constexpr int P = sizeof(K);
  constexpr uint32_t kTile = PassCfg<THREADS>::kTile;
  SortPlan* plan = reinterpret_cast<SortPlan*>(ws + L.plan);
  uint32_t* ctrs = reinterpret_cast<uint32_t*>(ws + L.ctrs);
  C* hist = reinterpret_cast<C*>(ws + L.hist);
  C* base = reinterpret_cast<C*>(ws + L.base);
  SegTile* records = reinterpret_cast<SegTile*>(ws + L.records);
  char* status[2] = {ws + L.status0, ws + L.status1};
  const uint32_t* num_tiles = ctrs;
  uint32_t* wide = ctrs + 1 + kMaxPasses;

  MS_LAUNCH("clear", clear_kernel, 1024, 256, s, reinterpret_cast<uint4*>(ws + L.ctrs), L.ctrs_hist_bytes / 16,
            reinterpret_cast<uint4*>(ws + L.status0), L.status_bytes / 16);
  Buffers buf = {kin, kout, ws + L.alt_k, vin, vout, VALS ? reinterpret_cast<uint32_t*>(ws + L.alt_v) : nullptr};
  {
    const ms_status st = plan_segment_tiles<K, VALS>(off, nseg, n, kTile, ws, L, buf, nullptr, s);
    if (st != MS_OK) return st;
  }
  const uint64_t hblocks = std::min<uint64_t>(L.tiles, 2 * device_cus(256));
  MS_LAUNCH("segsweep_hist", (segsweep_hist_kernel<K, C>), static_cast<uint32_t>(hblocks), 256, s,
            static_cast<const K*>(kin), flip, static_cast<const SegTile*>(records), num_tiles, hist);
  MS_LAUNCH("segsweep_base", segsweep_base_kernel<C>, nseg * P, 256, s, off, n, P, kTile,
            static_cast<const C*>(hist), base);
  // Segment-local counts fit 30-bit status fields unless a segment has 2^30
  // keys or more; below 2^30 keys in all no segment can, and only the 32-bit
  // form is launched.
  for (int p = 0; p < P; ++p) {
    char* next = p + 1 < P ? status[(p + 1) & 1] : nullptr;
    const SortPlan* cplan = plan;
    const SegTile* crec = records;
    const C* cbase = base;
    ms_status st = launch_segsweep_pass<K, VALS, C, uint32_t, THREADS>(
        cplan, p, crec, num_tiles, n, flip, cbase, ctrs + 1 + p, status[p & 1], next, L.big ? wide : nullptr, 0u,
        L.tiles, s);
    if (st != MS_OK) return st;
    if (L.big) {
      st = launch_segsweep_pass<K, VALS, C, uint64_t, THREADS>(cplan, p, crec, num_tiles, n, flip, cbase,
                                                               ctrs + 1 + p, status[p & 1], next, wide, 1u, L.tiles, s);
      if (st != MS_OK) return st;
    }
  }
  return MS_OK;
}

// One launch of the work queue with status words of type S; gate/want as in
// segqueue_body (nullptr: always runs).
template <typename K, bool VALS, typename C, typename S>
ms_status launch_segqueue(const uint64_t* off, uint64_t n, K flip, char* ws, const SegSweepLayout& L,
                          const uint32_t* gate, uint32_t want, hipStream_t s) {
  const SortPlan* plan = reinterpret_cast<const SortPlan*>(ws + L.plan);
  const SegTile* records = reinterpret_cast<const SegTile*>(ws + L.records);
  uint32_t* qtab = reinterpret_cast<uint32_t*>(ws + L.qtab);
  C* hist = reinterpret_cast<C*>(ws + L.hist);
  S* status0 = reinterpret_cast<S*>(ws + L.status0);
  S* status1 = reinterpret_cast<S*>(ws + L.status1);
  // The grid is what the device holds at once: workgroups loop over tickets.
  if constexpr (sizeof(K) == 4 && !VALS) {
    const uint64_t blocks = resident_blocks(reinterpret_cast<const void*>(&segqueue_kernel_x2<K, VALS, C, S>),
                                            kSegSweepThreads, 256);
    MS_LAUNCH("segqueue", (segqueue_kernel_x2<K, VALS, C, S>), static_cast<uint32_t>(blocks), kSegSweepThreads, s,
              plan, records, qtab, off, n, flip, hist, status0, status1, gate, want);
  } else {
    const uint64_t blocks = resident_blocks(reinterpret_cast<const void*>(&segqueue_kernel<K, VALS, C, S>),
                                            kSegSweepThreads, 256);
    MS_LAUNCH("segqueue", (segqueue_kernel<K, VALS, C, S>), static_cast<uint32_t>(blocks), kSegSweepThreads, s,
              plan, records, qtab, off, n, flip, hist, status0, status1, gate, want);
  }
  return MS_OK;
}

// The segment passes as one persistent launch (segqueue_kernel), after the
// clearing and planning launches.  Segment-local counts fit 30-bit status
// fields unless a segment has 2^30 keys or more; below 2^30 keys in all no
// segment can, and only the 32-bit form is launched; otherwise the queue is
// launched in both widths, the unselected one returning at entry.
template <typename K, bool VALS, typename C>
ms_status run_segqueue(const void* kin, const uint32_t* vin, void* kout, uint32_t* vout, const uint64_t* off,
                       uint32_t nseg, uint64_t n, K flip, char* ws, const SegSweepLayout& L, hipStream_t s) {
  constexpr uint32_t kTile = SegSweepCfg::kTile;
  uint32_t* qtab = reinterpret_cast<uint32_t*>(ws + L.qtab);
  // Counters, histograms and the queue table only: a tile clears its own
  // look-back rows before they are used.
  MS_LAUNCH("clear", clear_kernel, 1024, 256, s, reinterpret_cast<uint4*>(ws + L.ctrs), L.ctrs_hist_bytes / 16,
            static_cast<uint4*>(nullptr), size_t(0));
  Buffers buf = {kin, kout, ws + L.alt_k, vin, vout, VALS ? reinterpret_cast<uint32_t*>(ws + L.alt_v) : nullptr};
  ms_status st = plan_segment_tiles<K, VALS>(off, nseg, n, kTile, ws, L, buf, qtab, s);
  if (st != MS_OK) return st;
  if constexpr (sizeof(C) == 8) {
    if (L.big) {
      const uint32_t* wide = reinterpret_cast<const uint32_t*>(ws + L.ctrs) + 1 + kMaxPasses;
      st = launch_segqueue<K, VALS, C, uint32_t>(off, n, flip, ws, L, wide, 0u, s);
      if (st != MS_OK) return st;
      return launch_segqueue<K, VALS, C, uint64_t>(off, n, flip, ws, L, wide, 1u, s);
    }
  }
  return launch_segqueue<K, VALS, C, uint32_t>(off, n, flip, ws, L, nullptr, 0u, s);
}

template <typename K, bool VALS>
ms_status segsweep_dispatch(const void* kin, const uint32_t* vin, void* kout, uint32_t* vout, const uint64_t* off,
                            uint32_t nseg, uint64_t n, K flip, char* ws, const SegSweepLayout& L, hipStream_t s) {
  // MS_TUNE_SEG_PASSES = 2: all phases in one persistent launch.
  if (tune_get(MS_TUNE_SEG_PASSES) == 2) {
    if (L.big) return run_segqueue<K, VALS, uint64_t>(kin, vin, kout, vout, off, nseg, n, flip, ws, L, s);
    return run_segqueue<K, VALS, uint32_t>(kin, vin, kout, vout, off, nseg, n, flip, ws, L, s);
  }
  // 16,384-key tiles only where 1,024 threads fit their registers without
  // spilling: 32-bit keys without values.
  if constexpr (sizeof(K) == 4 && !VALS) {
    if (tune_get(MS_TUNE_SEG_PASS_THREADS) == 1024) {
      if (L.big) return run_segsweep<K, VALS, uint64_t, 1024>(kin, vin, kout, vout, off, nseg, n, flip, ws, L, s);
      return run_segsweep<K, VALS, uint32_t, 1024>(kin, vin, kout, vout, off, nseg, n, flip, ws, L, s);
    }
  }
  if (L.big) return run_segsweep<K, VALS, uint64_t, 512>(kin, vin, kout, vout, off, nseg, n, flip, ws, L, s);
  return run_segsweep<K, VALS, uint32_t, 512>(kin, vin, kout, vout, off, nseg, n, flip, ws, L, s);
}

}  // namespace

size_t radix_workspace_bytes(ms_key_type kt, bool has_vals, uint64_t n) {
  return make_layout(kt, has_vals, n).total;
}

ms_status radix_sort(const void* keys_in, const uint32_t* vals_in, void* keys_out, uint32_t* vals_out,
                     uint64_t n, ms_key_type kt, void* ws, size_t ws_bytes, hipStream_t s) {
  if (n == 0) return MS_OK;
  const Layout L = make_layout(kt, vals_in != nullptr, n);
  if (ws_bytes < L.total || (L.total && !ws))
    return fail(MS_EINVAL, "workspace too small: %zu bytes given, %zu needed", ws_bytes, L.total);
  const bool vals = vals_in != nullptr;
  switch (kt) {
    case MS_KEY_I32:
      return vals ? dispatch<uint32_t, true>(keys_in, vals_in, keys_out, vals_out, n, 0x80000000u, ws, L, s)
                  : dispatch<uint32_t, false>(keys_in, vals_in, keys_out, vals_out, n, 0x80000000u, ws, L, s);
    case MS_KEY_U32:
      return vals ? dispatch<uint32_t, true>(keys_in, vals_in, keys_out, vals_out, n, 0u, ws, L, s)
                  : dispatch<uint32_t, false>(keys_in, vals_in, keys_out, vals_out, n, 0u, ws, L, s);
    case MS_KEY_U64:
      return vals ? dispatch<uint64_t, true>(keys_in, vals_in, keys_out, vals_out, n, 0ull, ws, L, s)
                  : dispatch<uint64_t, false>(keys_in, vals_in, keys_out, vals_out, n, 0ull, ws, L, s);
  }
  return fail(MS_ENOTSUP, "unknown key type %d", static_cast<int>(kt));
}

bool segsweep_eligible(uint64_t n, uint64_t nseg, int mode) {
  // Tile numbers and segment ids are 32-bit; the base kernel runs one block
  // per (segment, digit position) in one grid dimension.
  if (nseg < 1 || nseg * kMaxPasses >= (1ull << 31)) return false;
  const uint64_t tiles = (n + SegSweepCfg::kTile - 1) / SegSweepCfg::kTile + nseg;
  // The average bounds the per-segment histograms and bases to 8 KiB per
  // `min_average` keys.
  const uint64_t min_average = mode == 1 ? kSegSweepMinAverage : kSegQueueMinAverage;
  return n > min_average * nseg && tiles < (1ull << 32);
}

size_t segsweep_workspace_bytes(ms_key_type kt, bool has_vals, uint64_t n, uint64_t nseg) {
  return segsweep_layout(kt, has_vals, n, nseg).total;
}

ms_status segsweep_sort(const void* keys_in, const uint32_t* vals_in, void* keys_out, uint32_t* vals_out,
                        const uint64_t* offsets, uint64_t nseg, uint64_t n, ms_key_type kt, void* ws,
                        size_t ws_bytes, hipStream_t s) {
  if (!segsweep_eligible(n, nseg, static_cast<int>(tune_get(MS_TUNE_SEG_PASSES))))
    return fail(MS_EINVAL, "sort_segmented: internal: segment passes not eligible");
  const bool vals = vals_in != nullptr;
  const SegSweepLayout L = segsweep_layout(kt, vals, n, nseg);
  if (ws_bytes < L.total || !ws)
    return fail(MS_EINVAL, "sort_segmented: workspace too small: %zu bytes given, %zu needed", ws_bytes, L.total);
  char* w = static_cast<char*>(ws);
  const uint32_t ns = static_cast<uint32_t>(nseg);
  switch (kt) {
    case MS_KEY_I32:
      return vals ? segsweep_dispatch<uint32_t, true>(keys_in, vals_in, keys_out, vals_out, offsets, ns, n, 0x80000000u, w, L, s)
                  : segsweep_dispatch<uint32_t, false>(keys_in, vals_in, keys_out, vals_out, offsets, ns, n, 0x80000000u, w, L, s);
    case MS_KEY_U32:
      return vals ? segsweep_dispatch<uint32_t, true>(keys_in, vals_in, keys_out, vals_out, offsets, ns, n, 0u, w, L, s)
                  : segsweep_dispatch<uint32_t, false>(keys_in, vals_in, keys_out, vals_out, offsets, ns, n, 0u, w, L, s);
    case MS_KEY_U64:
      return vals ? segsweep_dispatch<uint64_t, true>(keys_in, vals_in, keys_out, vals_out, offsets, ns, n, 0ull, w, L, s)
                  : segsweep_dispatch<uint64_t, false>(keys_in, vals_in, keys_out, vals_out, offsets, ns, n, 0ull, w, L, s);
  }
  return fail(MS_ENOTSUP, "sort_segmented: unknown key type %d", static_cast<int>(kt));
}

}  // namespace ms

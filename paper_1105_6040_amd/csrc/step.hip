// step.hip -- continuous batching of sort requests: one step per launch.
//
// A serving loop sorts many independent requests (each the whole method of
// Section 3.2 on its own list) by advancing every active request one phase
// per step.  A request of at most one LDS tile is sorted completely in its
// single phase.  A longer request has P + 1 phases (P = key bytes, 8-bit
// digits): phase 0 reads its keys once for the P digit histograms, phase
// 1 + p is digit pass p (a stable counting scatter by decoupled look-back
// over the request's own tiles, as in the whole-list sort).  One step is one
// launch over all the requests it names, whatever their phases, so requests
// that arrive while others are on the GPU join at the next step and a
// finished one leaves at once: the batch changes at every pass boundary.
//
// Work items are tiles: request j contributes tiles(j) consecutive tickets
// (1 for a one-tile request; ceil(n / 8192) for a histogram or digit pass).
// Persistent workgroups take tickets in order from a counter, so a tile
// only ever waits on tiles with earlier tickets of its own request (the
// look-back, and the histogram's "counters cleared" flag raised by the
// request's tile 0), which are already running: no wait can deadlock.
//
// Per-request state lives in the request's `work` area (owned by the
// caller, kept between its steps): P digit histograms, P rows of look-back
// status words per tile, and the ping-pong buffers.  Phase 0 clears the
// status rows and (its tile 0) the histograms, so the area needs no
// initialisation.  Passes ping-pong in -> alt -> out -> alt -> out ..., P
// being even, so the last pass lands in keys_out.
#include <algorithm>
#include <mutex>
#include <vector>

#include "ms_device.hpp"
#include "ms_lds_sort.hpp"
#include "ms_runtime.hpp"
#include "ms_tile.hpp"

namespace ms {
namespace {

constexpr int kStepThreads = 512;
constexpr int kStepKpt = 16;
constexpr int kStepTile = kStepThreads * kStepKpt;  // keys per histogram / pass tile
constexpr uint32_t kMaxStepRequests = MS_STEP_MAX_REQUESTS;
constexpr uint64_t kMaxStepKeys = (1ull << 30) - 1;  // 30-bit counts in the status words

static_assert(sizeof(ms_step_request) == 56, "descriptor layout");
static_assert(LdsCfg<uint32_t>::kThreads == kStepThreads && LdsCfg<uint64_t>::kThreads == kStepThreads,
              "one workgroup shape for every phase");

// Step control block (the caller's step workspace): the ticket counter,
// then one "histograms cleared" flag per request of the step.  Cleared by a
// small kernel before every step.
constexpr int kCtlTicket = 0;
constexpr int kCtlReady = 64;
constexpr size_t kCtlWords = kCtlReady + kMaxStepRequests;

template <typename K>
__host__ __device__ constexpr uint64_t step_small_max() {
  return static_cast<uint64_t>(LdsCfg<K>::kTile);
}

__host__ __device__ inline uint64_t step_tiles_of(uint64_t n) { return (n + kStepTile - 1) / kStepTile; }

// Byte offsets inside a request's work area.
struct StepWork {
  size_t hist = 0, status = 0, alt_k = 0, alt_v = 0, total = 0;
};

__host__ __device__ inline size_t step_align(size_t x) { return (x + 255) / 256 * 256; }

__host__ __device__ inline StepWork step_work(int key_bytes, bool has_vals, uint64_t n) {
  StepWork w;
  const uint64_t small = key_bytes == 4 ? step_small_max<uint32_t>() : step_small_max<uint64_t>();
  if (n <= small) return w;  // sorted in LDS in one phase: no state
  const int P = key_bytes;
  const uint64_t tiles = step_tiles_of(n);
  size_t o = 0;
  w.hist = o;
  o += step_align(static_cast<size_t>(P) * kRadix * 4);
  w.status = o;
  o += step_align(static_cast<size_t>(P) * tiles * kRadix * 4);
  w.alt_k = o;
  o += step_align(n * key_bytes);
  if (has_vals) {
    w.alt_v = o;
    o += step_align(n * 4);
  }
  w.total = o;
  return w;
}

// Tickets request r takes in this step (0 for an empty request, a phase out
// of range, or a list beyond the supported length).
template <typename K>
__device__ __forceinline__ uint32_t step_request_tiles(const ms_step_request& r) {
  constexpr int P = sizeof(K);
  if (r.n == 0 || r.n > kMaxStepKeys) return 0;
  if (r.n <= step_small_max<K>()) return r.phase == 0 ? 1u : 0u;
  return r.phase <= static_cast<uint32_t>(P) ? static_cast<uint32_t>(step_tiles_of(r.n)) : 0u;
}

__global__ __launch_bounds__(256) void step_clear_kernel(uint32_t* ctl) {
  for (size_t i = threadIdx.x; i < kCtlWords; i += 256) ctl[i] = 0;
}

// LDS of the step kernel: the phases share one raw buffer.
template <typename K, bool VALS>
struct StepLds {
  static constexpr int kStage = padded16(kStepTile) * static_cast<int>(sizeof(K));
  static constexpr int kCounts = SplitScratch<kStepThreads>::kCountWords * 4;
  static constexpr int kPassBytes = (kStage > kCounts ? kStage : kCounts) + (VALS ? padded16(kStepTile) * 4 : 0);
  static constexpr int kLdsSortBytes = LdsSortSmem<K, VALS>::kWaves * kRadix * 4 +
                                       LdsCfg<K>::kTile * static_cast<int>(sizeof(K)) +
                                       (VALS ? LdsCfg<K>::kTile * 4 : 0);
  static constexpr int kHistBytes = static_cast<int>(sizeof(K)) * kRadix * 4;
  static constexpr int kBytes = std::max(kPassBytes, std::max(kLdsSortBytes, kHistBytes));
};

template <typename K, bool VALS>
__global__ __launch_bounds__(kStepThreads) void step_kernel(const ms_step_request* __restrict__ reqs, uint32_t num_reqs,
                                                            K flip, uint32_t* ctl) {
  constexpr int P = sizeof(K);
  constexpr int kKpt = kStepKpt;
  using St = Status<uint32_t>;
  using L = StepLds<K, VALS>;

  __shared__ __attribute__((aligned(16))) uint8_t s_raw[L::kBytes];
  __shared__ uint32_t s_prefix[kMaxStepRequests + 1];
  __shared__ uint32_t s_scan[kStepThreads / kWave];
  __shared__ uint32_t s_cscan[kRadix / kWave];
  __shared__ uint32_t s_cscan2[kRadix / kWave];
  __shared__ uint32_t s_hist[kRadix];
  __shared__ uint32_t s_doff[kRadix];
  __shared__ uint32_t s_small[kRadix / kWave + 2];
  __shared__ uint32_t s_ticket;

  const int tid = threadIdx.x;

  // Tile prefix over the step's requests (two per thread).
  static_assert(kMaxStepRequests == 2 * kStepThreads, "two requests per thread");
  const uint32_t j0 = 2 * tid, j1 = 2 * tid + 1;
  const uint32_t t0 = j0 < num_reqs ? step_request_tiles<K>(reqs[j0]) : 0u;
  const uint32_t t1 = j1 < num_reqs ? step_request_tiles<K>(reqs[j1]) : 0u;
  const uint32_t ex = block_exclusive_scan<kStepThreads>(t0 + t1, s_scan);
  if (tid == 0) s_prefix[0] = 0;
  if (j0 < num_reqs) s_prefix[j0 + 1] = ex + t0;
  if (j1 < num_reqs) s_prefix[j1 + 1] = ex + t0 + t1;
  __syncthreads();
  const uint32_t total = s_prefix[num_reqs];

  while (true) {
    if (tid == 0) s_ticket = atomicAdd(&ctl[kCtlTicket], 1u);
    __syncthreads();
    const uint32_t ticket = s_ticket;
    if (ticket >= total) break;
    // The request of this ticket: the last j with s_prefix[j] <= ticket.
    uint32_t lo = 0, hi = num_reqs - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) / 2;
      if (s_prefix[mid] <= ticket) lo = mid; else hi = mid - 1;
    }
    const uint32_t j = lo;
    const uint32_t tile = ticket - s_prefix[j];
    const ms_step_request r = reqs[j];
    const uint64_t n = r.n;

    if (n <= step_small_max<K>()) {
      // ---- a one-tile request: its whole sort in LDS.
      const LdsSortSmem<K, VALS> sm = {
          reinterpret_cast<uint32_t(*)[kRadix]>(s_raw),
          reinterpret_cast<K*>(s_raw + LdsSortSmem<K, VALS>::kWaves * kRadix * 4),
          reinterpret_cast<uint32_t*>(s_raw + LdsSortSmem<K, VALS>::kWaves * kRadix * 4 +
                                      LdsCfg<K>::kTile * sizeof(K)),
          s_small, s_small + kRadix / kWave};
      lds_sort_list<K, VALS>(static_cast<const K*>(r.keys_in), r.vals_in, static_cast<K*>(r.keys_out), r.vals_out,
                             0, static_cast<int>(n), flip, sm);
    } else {
      const StepWork w = step_work(P, VALS, n);
      char* const work = static_cast<char*>(r.work);
      uint32_t* const ghist = reinterpret_cast<uint32_t*>(work + w.hist);
      uint32_t* const status = reinterpret_cast<uint32_t*>(work + w.status);
      const uint32_t tiles = static_cast<uint32_t>(step_tiles_of(n));
      const uint64_t tile_base = static_cast<uint64_t>(tile) * kStepTile;
      const uint64_t tile_end = std::min<uint64_t>(n, tile_base + kStepTile);

      if (r.phase == 0) {
        // ---- histogram phase: this tile's keys counted for every digit.
        uint32_t* const h = reinterpret_cast<uint32_t*>(s_raw);
        for (int i = tid; i < P * kRadix; i += kStepThreads) h[i] = 0;
        // This tile's look-back rows of every pass start NOT_READY.
        for (int i = tid; i < P * kRadix; i += kStepThreads)
          status[(static_cast<size_t>(i / kRadix) * tiles + tile) * kRadix + i % kRadix] = 0;
        __syncthreads();
        K keys[kKpt];
        uint32_t unused[kKpt];
        load_tile_keys<K, false, uint64_t, kKpt>(as_global(static_cast<const K*>(r.keys_in)), nullptr,
                                                 tile_base + static_cast<uint64_t>(tid) * kKpt, tile_end, K(0), keys,
                                                 unused);
#pragma unroll
        for (int q = 0; q < kKpt; ++q) {
          if (tile_base + static_cast<uint64_t>(tid) * kKpt + q < tile_end) {
            const K k = flip_key(keys[q], flip);
#pragma unroll
            for (int p = 0; p < P; ++p) atomicAdd(&h[p * kRadix + digit_of(k, 8 * p)], 1u);
          }
        }
        // Tile 0 clears the request's histograms and raises its flag; the
        // other tiles add theirs once the flag is up.
        if (tile == 0) {
          for (int i = tid; i < P * kRadix; i += kStepThreads) ghist[i] = 0;
          __threadfence();
          __syncthreads();
          if (tid == 0) __hip_atomic_store(&ctl[kCtlReady + j], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
          if (tid == 0)
            while (__hip_atomic_load(&ctl[kCtlReady + j], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0)
              __builtin_amdgcn_s_sleep(2);
          __syncthreads();
        }
        for (int i = tid; i < P * kRadix; i += kStepThreads)
          if (h[i]) atomicAdd(&ghist[i], h[i]);
      } else {
        // ---- digit pass p = phase - 1 over this tile.
        const int p = static_cast<int>(r.phase) - 1;
        const int shift = 8 * p;
        K* const alt_k = reinterpret_cast<K*>(work + w.alt_k);
        uint32_t* const alt_v = VALS ? reinterpret_cast<uint32_t*>(work + w.alt_v) : nullptr;
        K* const out_k = static_cast<K*>(r.keys_out);
        const K* const src_k = p == 0 ? static_cast<const K*>(r.keys_in) : ((p & 1) ? alt_k : out_k);
        K* const dst_k = (p & 1) ? out_k : alt_k;
        const uint32_t* const src_v = p == 0 ? r.vals_in : ((p & 1) ? alt_v : r.vals_out);
        uint32_t* const dst_v = (p & 1) ? r.vals_out : alt_v;
        const K in_flip = p == 0 ? flip : K(0);
        const K out_flip = p == P - 1 ? flip : K(0);
        const K pad = ~K(0) ^ in_flip;  // decodes to all-ones: after every real key

        K* const s_stage = reinterpret_cast<K*>(s_raw);
        uint32_t* const s_counts = reinterpret_cast<uint32_t*>(s_raw);
        uint32_t* const s_vstage = reinterpret_cast<uint32_t*>(s_raw + (L::kStage > L::kCounts ? L::kStage : L::kCounts));

        K keys[kKpt];
        uint32_t vals[kKpt];
        load_tile_keys<K, VALS, uint64_t, kKpt>(as_global(src_k), as_global(src_v),
                                                tile_base + static_cast<uint64_t>(tid) * kKpt, tile_end, pad, keys,
                                                vals);
#pragma unroll
        for (int q = 0; q < kKpt; ++q) keys[q] = flip_key(keys[q], in_flip);
        for (int d = tid; d < kRadix; d += kStepThreads) s_hist[d] = 0;
        __syncthreads();
        const int valid = static_cast<int>(tile_end - tile_base);
#pragma unroll
        for (int q = 0; q < kKpt; ++q)
          if (tid * kKpt + q < valid) atomicAdd(&s_hist[digit_of(keys[q], shift)], 1u);
        __syncthreads();

        uint32_t* const st = status + (static_cast<size_t>(p) * tiles + tile) * kRadix + tid;
        uint32_t cnt = 0;
        if (tid < kRadix) {
          cnt = s_hist[tid];
          if (tiles > 1) status_store(st, (tile == 0 ? St::kInc : St::kAgg) | cnt);
        }
        tile_split_stage<kStepThreads, kKpt, VALS>(keys, vals, shift, s_stage, s_vstage, s_counts, s_scan, true);
        uint32_t pred = 0;
        if (tid < kRadix && tile != 0) pred = status_load(st - kRadix);
        tile_split_stage<kStepThreads, kKpt, VALS>(keys, vals, shift + kSubBits, s_stage, s_vstage, s_counts, s_scan,
                                                   false);
        uint32_t tile_total, list_total;
        const uint32_t start = block_exclusive_scan_radix<kStepThreads>(cnt, s_cscan, &tile_total);
        const uint32_t hcount = tid < kRadix ? ghist[p * kRadix + tid] : 0u;
        const uint32_t base = block_exclusive_scan_radix<kStepThreads>(hcount, s_cscan2, &list_total);
        if (tid < kRadix) {
          uint32_t excl = 0;
          if (tile != 0) {
            excl = (pred & St::kFlagMask) == St::kInc ? (pred & St::kValMask) : lookback<uint32_t, uint32_t, 16>(st, tile, kRadix);
            status_store(st, St::kInc | (excl + cnt));
          }
          s_doff[tid] = base + excl - start;
        }
        __syncthreads();
        // Destinations stay inside the request even if its phases were run
        // out of order (then the order is unspecified, never an overrun).
        for (int i = tid; i < valid; i += kStepThreads) {
          const K k = s_stage[pad16(i)];
          uint64_t o = static_cast<uint64_t>(s_doff[digit_of(k, shift)]) + static_cast<uint64_t>(i);
          o = o < n ? o : n - 1;
          dst_k[o] = k ^ out_flip;
          if constexpr (VALS) dst_v[o] = s_vstage[pad16(i)];
        }
      }
    }
    __syncthreads();  // LDS and s_ticket are reused by the next ticket
  }
}

template <typename K, bool VALS>
ms_status run_step(const ms_step_request* reqs, uint32_t num_reqs, K flip, uint32_t* ctl, hipStream_t s) {
  // Persistent workgroups: as many as the device holds at once.
  static std::mutex mu;
  static std::vector<std::pair<int, uint32_t>> cache;  // (device, blocks)
  int dev = 0;
  uint32_t blocks = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    std::lock_guard<std::mutex> lock(mu);
    for (auto& e : cache)
      if (e.first == dev) blocks = e.second;
    if (!blocks) {
      int per_cu = 0, cus = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&step_kernel<K, VALS>),
                                                       kStepThreads, 0) == hipSuccess &&
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && per_cu > 0 &&
          cus > 0) {
        blocks = static_cast<uint32_t>(per_cu * cus);
        cache.push_back({dev, blocks});
      }
    }
  }
  (void)hipGetLastError();
  if (!blocks) blocks = 256;
  MS_LAUNCH("step_clear", step_clear_kernel, 1, 256, s, ctl);
  MS_LAUNCH("step", (step_kernel<K, VALS>), blocks, kStepThreads, s, reqs, num_reqs, flip, ctl);
  return MS_OK;
}

}  // namespace

size_t step_control_bytes() { return step_align(kCtlWords * 4); }

ms_status step_request_plan(ms_key_type kt, bool has_vals, uint64_t n, uint32_t* phases, size_t* work_bytes) {
  const int kb = key_bytes(kt);
  if (n > kMaxStepKeys)
    return fail(MS_ENOTSUP, "sort_step: a request holds at most %llu keys (got %llu)",
                static_cast<unsigned long long>(kMaxStepKeys), static_cast<unsigned long long>(n));
  const uint64_t small = kb == 4 ? step_small_max<uint32_t>() : step_small_max<uint64_t>();
  *phases = n == 0 ? 0u : (n <= small ? 1u : static_cast<uint32_t>(kb + 1));
  *work_bytes = step_work(kb, has_vals, n).total;
  return MS_OK;
}

ms_status sort_step_run(const ms_step_request* reqs, uint32_t num_reqs, ms_key_type kt, bool has_vals, void* ws,
                        hipStream_t s) {
  uint32_t* ctl = static_cast<uint32_t*>(ws);
  switch (kt) {
    case MS_KEY_I32:
      return has_vals ? run_step<uint32_t, true>(reqs, num_reqs, 0x80000000u, ctl, s)
                      : run_step<uint32_t, false>(reqs, num_reqs, 0x80000000u, ctl, s);
    case MS_KEY_U32:
      return has_vals ? run_step<uint32_t, true>(reqs, num_reqs, 0u, ctl, s)
                      : run_step<uint32_t, false>(reqs, num_reqs, 0u, ctl, s);
    case MS_KEY_U64:
      return has_vals ? run_step<uint64_t, true>(reqs, num_reqs, 0ull, ctl, s)
                      : run_step<uint64_t, false>(reqs, num_reqs, 0ull, ctl, s);
  }
  return fail(MS_ENOTSUP, "sort_step: unknown key type %d", static_cast<int>(kt));
}

}  // namespace ms

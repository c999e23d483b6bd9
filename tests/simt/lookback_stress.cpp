// lookback_stress.cpp -- the decoupled look-back of ms_device.hpp under real
// concurrency in the CPU emulator: every block publishes a per-digit count
// (AGGREGATE) after a random delay, looks back, publishes INCLUSIVE after
// another delay, and records its exclusive prefix.  The prefixes must equal
// the serial exclusive scan of the counts.  Two forms: the plain walk, and
// the form of the onesweep pass: one extra workgroup runs the look-back agent
// (publishing INCLUSIVE in tile order from the AGGREGATE words) while every
// tile reads its predecessor's word once and walks back only if that word is
// not INCLUSIVE yet.
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "hip/hip_runtime.h"
#include "ms_device.hpp"

static uint32_t mix(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  return x ^ (x >> 16);
}

template <int kWindow>
__global__ void stress_kernel(uint32_t* status, uint32_t* counter, const uint32_t* counts, uint32_t* excl_out,
                              uint64_t* agg_seen) {
  using St = ms::Status<uint32_t>;
  __shared__ uint32_t s_tile;
  const int tid = threadIdx.x;
  if (tid == 0) s_tile = atomicAdd(counter, 1u);
  __syncthreads();
  const uint32_t tile = s_tile;
  for (uint32_t k = mix(tile * 977 + tid) % 7; k > 0; --k) ms::status_load(status);  // jitter
  uint32_t* st = status + tile * 64 + tid;
  const uint32_t cnt = counts[tile * 64 + tid];
  ms::status_store(st, (tile == 0 ? St::kInc : St::kAgg) | cnt);
  for (uint32_t k = mix(tile * 131 + tid * 7) % 11; k > 0; --k) ms::status_load(status);  // jitter
  uint32_t excl = 0;
  if (tile != 0) {
    // count predecessors still AGGREGATE when first seen (coverage of the walk)
    if (ms::status_load(st - 64) >> 30 == 1) atomicAdd(reinterpret_cast<unsigned long long*>(agg_seen), 1ull);
    excl = ms::lookback<uint32_t, uint32_t, kWindow>(st, tile, 64);
    for (uint32_t k = mix(tile * 71 + tid * 3) % 13; k > 0; --k) ms::status_load(status);  // jitter
    ms::status_store(st, St::kInc | (excl + cnt));
  }
  excl_out[tile * 64 + tid] = excl;
}

template <int THREADS, int kAgents, int kW>
__global__ void agent_kernel(uint32_t* status, uint32_t* counter, const uint32_t* counts, uint32_t* excl_out,
                             uint32_t tiles, uint64_t* hits, uint64_t* walks) {
  using St = ms::Status<uint32_t>;
  constexpr int R = ms::kRadix;
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_val[THREADS];
  __shared__ uint32_t s_used[THREADS];
  __shared__ uint32_t s_prefix[R];
  __shared__ uint32_t s_next[R];
  const int tid = threadIdx.x;
  if (tid == 0) s_tile = atomicAdd(counter, 1u);
  __syncthreads();
  if (s_tile < kAgents) {
    constexpr int kDigits = R / kAgents;
    ms::lookback_agent<THREADS, kDigits, kW, uint32_t, uint32_t>(status, tiles, static_cast<int>(s_tile) * kDigits,
                                                                 s_val, s_used, s_prefix, s_next);
    return;
  }
  const uint32_t tile = s_tile - kAgents;
  if (tid >= R) return;
  uint32_t* st = status + tile * R + tid;
  const uint32_t cnt = counts[tile * R + tid];
  for (uint32_t k = mix(tile * 977 + tid) % 7; k > 0; --k) ms::status_load(status);  // jitter
  ms::status_store(st, (tile == 0 ? St::kInc : St::kAgg) | cnt);
  for (uint32_t k = mix(tile * 131 + tid * 7) % 23; k > 0; --k) ms::status_load(status);  // jitter
  const uint32_t pred = tile != 0 ? ms::status_load(st - R) : 0u;
  for (uint32_t k = mix(tile * 37 + tid * 5) % 11; k > 0; --k) ms::status_load(status);  // jitter
  uint32_t excl = 0;
  if (tile != 0) {
    if ((pred & St::kFlagMask) == St::kInc) {
      excl = pred & St::kValMask;
      atomicAdd(reinterpret_cast<unsigned long long*>(hits), 1ull);
    } else {
      excl = ms::lookback<uint32_t, uint32_t, 4>(st, tile, R);  // the passes' window
      atomicAdd(reinterpret_cast<unsigned long long*>(walks), 1ull);
    }
    ms::status_store(st, St::kInc | (excl + cnt));
  }
  excl_out[tile * R + tid] = excl;
}

template <int THREADS, int kAgents, int kW>
static int run_agent(int tiles) {
  constexpr int R = ms::kRadix;
  std::vector<uint32_t> status(tiles * R, 0), counts(tiles * R), excl(tiles * R, 0xffffffffu);
  uint32_t counter = 0;
  uint64_t hits = 0, walks = 0;
  for (int i = 0; i < tiles * R; ++i) counts[i] = mix(i + 999) % 1000;
  hipLaunchKernelGGL((agent_kernel<THREADS, kAgents, kW>), dim3(tiles + kAgents), dim3(THREADS), 0, nullptr,
                     status.data(), &counter, counts.data(), excl.data(), static_cast<uint32_t>(tiles), &hits, &walks);
  int bad = 0;
  for (int d = 0; d < R; ++d) {
    uint32_t run = 0, incl = 0;
    for (int t = 0; t < tiles; ++t) {
      if (excl[t * R + d] != run) ++bad;
      run += counts[t * R + d];
      incl = run;
      // every word ends INCLUSIVE with the true inclusive count
      if (status[t * R + d] != (ms::Status<uint32_t>::kInc | incl)) ++bad;
    }
  }
  // Both ways of finding the prefix must have been taken for the run to count.
  const bool covered = hits > 0 && walks > 0;
  printf("%s lookback agents=%d threads=%d window=%d tiles=%d wrong=%d predecessor-inclusive=%llu walked=%llu\n",
         bad || !covered ? "FAIL" : "ok  ", kAgents, THREADS, kW, tiles, bad, static_cast<unsigned long long>(hits),
         static_cast<unsigned long long>(walks));
  return bad || !covered ? 1 : 0;
}

template <int kWindow>
static int run(int tiles) {
  std::vector<uint32_t> status(tiles * 64, 0), counts(tiles * 64), excl(tiles * 64, 0xffffffffu);
  uint32_t counter = 0;
  uint64_t agg_seen = 0;
  for (int i = 0; i < tiles * 64; ++i) counts[i] = mix(i + 12345) % 1000;
  hipLaunchKernelGGL((stress_kernel<kWindow>), dim3(tiles), dim3(64), 0, nullptr, status.data(), &counter,
                     counts.data(), excl.data(), &agg_seen);
  int bad = 0;
  for (int d = 0; d < 64; ++d) {
    uint32_t run = 0;
    for (int t = 0; t < tiles; ++t) {
      if (excl[t * 64 + d] != run) ++bad;
      run += counts[t * 64 + d];
    }
  }
  printf("%s lookback window=%d tiles=%d wrong=%d aggregate-predecessors-seen=%llu\n", bad ? "FAIL" : "ok  ",
         kWindow, tiles, bad, static_cast<unsigned long long>(agg_seen));
  return bad ? 1 : 0;
}

int main() {
  int fails = 0;
  fails += run<1>(300);
  fails += run<4>(400);
  fails += run<8>(500);
  fails += run<16>(700);
  fails += run_agent<256, 1, 16>(150);
  fails += run_agent<512, 2, 16>(150);
  fails += run_agent<1024, 2, 8>(150);  // the 1,024-thread pass's agents
  return fails ? 1 : 0;
}

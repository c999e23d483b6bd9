// segmented.hip -- sort many independent segments (sort_segmented).
//
// The scatter and sorting phases of the paper's method (Section 3.2,
// Figure 1 steps 3-9) for many lists at once: every segment of the input is
// sorted on its own, stably, and nothing crosses a segment boundary.  The
// host never reads the segment offsets; each workgroup reads the ones it
// needs, so one call costs the same few launches whatever the segment count.
//
//   short segments (at most one LDS tile): one workgroup each, every digit
//       pass in LDS (one read and one write of HBM per key);
//   longer segments: a persistent grid of workgroups takes segments from an
//       atomic counter; the workgroup reads its segment once for the digit
//       histograms of every pass, then runs each non-constant digit pass
//       tile by tile, keeping running digit offsets in LDS (one workgroup
//       owns the segment, so no cross-workgroup look-back is needed).
#include "ms_device.hpp"
#include "ms_lds_sort.hpp"
#include "ms_runtime.hpp"

namespace ms {
namespace {

template <typename K>
struct SegCfg {
  static constexpr int kThreads = 256;
  static constexpr int kKpt = sizeof(K) == 4 ? 16 : 8;
  static constexpr int kTile = kThreads * kKpt;
};

constexpr int kPersistentBlocks = 2048;

__global__ void zero_words_kernel(uint32_t* p, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0;
}

template <typename K, bool VALS>
__global__ __launch_bounds__(SegCfg<K>::kThreads) void segment_radix_kernel(
    const K* kin, const uint32_t* vin, K* kout, uint32_t* vout, K* alt_k, uint32_t* alt_v,
    const uint64_t* __restrict__ off, uint64_t nseg, uint64_t n_total, K flip, uint32_t* next_seg,
    uint64_t short_cap) {
  constexpr int kThreads = SegCfg<K>::kThreads;
  constexpr int kKpt = SegCfg<K>::kKpt;
  constexpr int kTile = SegCfg<K>::kTile;
  constexpr int kWaves = kThreads / kWave;
  constexpr int P = sizeof(K);

  __shared__ uint32_t s_hist[P][kRadix];       // segment digit counts per pass
  __shared__ uint32_t s_whist[kWaves][kRadix];
  __shared__ uint32_t s_run[kRadix];           // segment position of the next key of each digit
  __shared__ uint32_t s_doff[kRadix];          // s_run - tile start, per digit (mod 2^32)
  __shared__ K s_keys[kTile];
  __shared__ uint32_t s_vals[VALS ? kTile : 1];
  __shared__ uint32_t s_scan[kRadix / kWave];
  __shared__ uint32_t s_diff[2];
  __shared__ uint32_t s_seg;

  const int tid = threadIdx.x;
  const int wave = tid / kWave;
  const uint32_t lane = lane_id();
  const int first = wave * kWave * kKpt + static_cast<int>(lane);
  const bool inplace = kin == kout;

  while (true) {
    __syncthreads();
    if (tid == 0) s_seg = atomicAdd(next_seg, 1u);
    __syncthreads();
    const uint64_t seg = s_seg;
    if (seg >= nseg) return;
    uint64_t begin = off[seg], end = off[seg + 1];
    begin = begin < n_total ? begin : n_total;
    end = end < n_total ? end : n_total;
    if (end <= begin) continue;
    const uint64_t len = end - begin;
    if (len <= short_cap) continue;  // sorted by the in-LDS kernel

    // One read: digit histograms of every pass and the bits that vary.
    for (int i = tid; i < P * kRadix; i += kThreads) (&s_hist[0][0])[i] = 0;
    if (tid < 2) s_diff[tid] = 0;
    __syncthreads();
    const K k0 = flip_key(kin[begin], flip);
    K diff = 0;
    for (uint64_t i = tid; i < len; i += kThreads) {
      const K k = flip_key(kin[begin + i], flip);
      diff |= k ^ k0;
#pragma unroll
      for (int p = 0; p < P; ++p) atomicAdd(&s_hist[p][digit_of(k, 8 * p)], 1u);
    }
    if (static_cast<uint32_t>(diff)) atomicOr(&s_diff[0], static_cast<uint32_t>(diff));
    if constexpr (sizeof(K) == 8)
      if (static_cast<uint32_t>(diff >> 32)) atomicOr(&s_diff[1], static_cast<uint32_t>(diff >> 32));
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
      const uint32_t base = block_exclusive_scan_radix<kThreads>(tid < kRadix ? s_hist[p][tid] : 0u, s_scan, &total);
      if (tid < kRadix) s_run[tid] = base;

      for (uint64_t t0 = 0; t0 < len; t0 += kTile) {
        const uint64_t rem = len - t0;
        const int valid = rem < static_cast<uint64_t>(kTile) ? static_cast<int>(rem) : kTile;
        K keys[kKpt];
        uint32_t vals[VALS ? kKpt : 1];
#pragma unroll
        for (int j = 0; j < kKpt; ++j) {
          const int idx = first + j * kWave;
          keys[j] = idx < valid ? flip_key(src[begin + t0 + idx], in_flip) : ~K(0);
          if constexpr (VALS) vals[j] = idx < valid ? srcv[begin + t0 + idx] : 0u;
        }
        for (int i = tid; i < kWaves * kRadix; i += kThreads) (&s_whist[0][0])[i] = 0;
        __syncthreads();
        uint32_t rank[kKpt];
        wave_rank(keys, shift, rank, s_whist[wave]);
        __syncthreads();
        uint32_t cnt;
        const uint32_t start = tile_digit_starts<kThreads>(s_whist, s_scan, &cnt);
        if (tid < kRadix) s_doff[tid] = s_run[tid] - start;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kKpt; ++j) {
          const uint32_t pos = s_whist[wave][digit_of(keys[j], shift)] + rank[j];
          s_keys[pos] = keys[j];
          if constexpr (VALS) s_vals[pos] = vals[j];
        }
        __syncthreads();
        for (int i = tid; i < valid; i += kThreads) {
          const K k = s_keys[i];
          const uint64_t o = begin + static_cast<uint32_t>(s_doff[digit_of(k, shift)] + static_cast<uint32_t>(i));
          dst[o] = k ^ out_flip;
          if constexpr (VALS) dstv[o] = s_vals[i];
        }
        __syncthreads();
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
      for (uint64_t i = tid; i < len; i += kThreads) {
        kout[begin + i] = csrc[begin + i];
        if constexpr (VALS) vout[begin + i] = csrcv[begin + i];
      }
    }
  }
}

struct SegLayout {
  size_t ctr = 0, alt_k = 0, alt_v = 0, total = 0;
};

SegLayout seg_layout(ms_key_type kt, bool has_vals, uint64_t n) {
  SegLayout L;
  size_t off = 0;
  L.ctr = off;
  off += kAlign;
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
  K* alt_k = reinterpret_cast<K*>(ws + L.alt_k);
  uint32_t* alt_v = VALS ? reinterpret_cast<uint32_t*>(ws + L.alt_v) : nullptr;
  MS_LAUNCH("seg_clear", zero_words_kernel, 1, 64, s, ctr, 1);
  MS_LAUNCH("seg_lds_sort", (lds_sort_kernel<K, VALS>), static_cast<uint32_t>(nseg), LdsCfg<K>::kThreads, s,
            static_cast<const K*>(kin), vin, static_cast<K*>(kout), vout, off,
            static_cast<const uint32_t*>(nullptr), n, flip);
  const uint32_t blocks = static_cast<uint32_t>(nseg < kPersistentBlocks ? nseg : kPersistentBlocks);
  MS_LAUNCH("seg_radix", (segment_radix_kernel<K, VALS>), blocks, SegCfg<K>::kThreads, s,
            static_cast<const K*>(kin), vin, static_cast<K*>(kout), vout, alt_k, alt_v, off, nseg, n, flip, ctr,
            static_cast<uint64_t>(LdsCfg<K>::kTile));
  return MS_OK;
}

}  // namespace

size_t segmented_workspace_bytes(ms_key_type kt, bool has_vals, uint64_t n, uint64_t nseg) {
  (void)nseg;
  return seg_layout(kt, has_vals, n).total;
}

ms_status segmented_sort(const void* keys_in, const uint32_t* vals_in, void* keys_out, uint32_t* vals_out,
                         const uint64_t* offsets, uint64_t nseg, uint64_t n, ms_key_type kt, void* ws,
                         size_t ws_bytes, hipStream_t s) {
  const bool vals = vals_in != nullptr;
  const SegLayout L = seg_layout(kt, vals, n);
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

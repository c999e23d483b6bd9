// merge.hip -- the merge phase: stable merge of adjacent sorted runs (merge_runs).
//
// The paper's merge phase combines the sorted parts into one ordered list,
// either by neighbour exchanges (Figure 1 merge loop) or by the master
// merging every part (Section 3.2.2).  With the left run's item first on
// equal keys, every schedule gives the same list: the stable sort of the
// concatenation.  Here the runs are merged in ceil(log2 R) rounds of pairwise
// merges, each round one launch over all output positions: round r merges
// groups of 2^r input runs pairwise, (group 2j, group 2j+1), and copies an
// unpaired last group.
//
// A workgroup produces one tile of kTile consecutive outputs.  When the tile
// lies inside one pair (the usual case once runs are longer than a tile), one
// wave finds the merge-path co-rank of each end of the tile (how many of the
// pair's first d outputs come from the left run) by a 64-way search, the
// tile's slices of both runs are loaded into LDS with coalesced reads, every
// thread co-ranks its kItems outputs inside LDS and merges them, and the tile
// is written back with coalesced stores.  Otherwise every thread finds the
// pair and co-rank of its first output itself and merges from global memory,
// crossing into the next pair if its outputs span a pair boundary.
#include "ms_device.hpp"
#include "ms_tile.hpp"
#include "ms_runtime.hpp"

namespace ms {
namespace {

// Tiles of 256 threads x kItems outputs: BIG tiles (16 32-bit or 8 64-bit
// keys per thread) for long lists, half that below kBigTileMin keys, where
// more, shorter tiles keep more of the device busy.
template <typename K, bool BIG>
struct MergeCfg {
  static constexpr int kThreads = 256;
  static constexpr int kItems = (sizeof(K) == 4 ? 16 : 8) / (BIG ? 1 : 2);
  static constexpr int kTile = kThreads * kItems;
};
constexpr uint64_t kBigTileMin = 1ull << 22;

__device__ __forceinline__ uint64_t clamp_off(const uint64_t* off, uint64_t idx, uint64_t n) {
  const uint64_t v = off[idx];
  return v < n ? v : n;
}

// Boundary of group g of `width` runs: run_offsets[min(g*width, nruns)],
// clamped to n and made non-decreasing against the previous boundary.
__device__ __forceinline__ uint64_t group_begin(const uint64_t* off, uint64_t nruns, uint64_t width, uint64_t g,
                                                uint64_t n) {
  const uint64_t idx = g * width < nruns ? g * width : nruns;
  return clamp_off(off, idx, n);
}

// Merge-path co-rank of diagonal d of the pair (A = src[a0, a0 + la),
// B = src[a1, a1 + lb)): the number i of A items among the first d outputs,
// i.e. the count of m in [max(0, d - lb), min(d, la)) with A[m] <= B[d-1-m]
// (true below i, false from i on).  One wave probes 64 evenly spaced m per
// round, so the range shrinks 64-fold per memory round trip.  All lanes of
// the wave call it and get the result.
template <typename K>
__device__ __forceinline__ uint64_t corank_wave(const K* __restrict__ src, uint64_t a0, uint64_t a1, uint64_t la,
                                                uint64_t lb, uint64_t d, K flip) {
  uint64_t lo = d > lb ? d - lb : 0, hi = d < la ? d : la;  // the answer lies in [lo, hi]
  const uint64_t lane = lane_id();
  while (hi > lo) {
    const uint64_t step = (hi - lo + kWave - 1) / kWave;
    const uint64_t m = lo + lane * step;
    bool le = false;
    if (m < hi) le = flip_key(src[a0 + m], flip) <= flip_key(src[a1 + (d - 1 - m)], flip);
    const uint32_t t = static_cast<uint32_t>(__popcll(__builtin_amdgcn_ballot_w64(le)));  // probes 0..t-1 hold
    if (step == 1) return lo + t;  // every candidate probed
    if (t == 0) return lo;
    const uint64_t first_false = lo + t * step;
    lo = lo + (t - 1) * step + 1;
    if (first_false < hi) hi = first_false;
  }
  return lo;
}

template <typename K, bool VALS, bool BIG>
__global__ __launch_bounds__(256) void merge_round_kernel(
    const K* __restrict__ src, const uint32_t* __restrict__ srcv, K* __restrict__ dst, uint32_t* __restrict__ dstv,
    const uint64_t* __restrict__ off, uint64_t nruns, uint64_t n, uint64_t width, K flip) {
  constexpr int kThreads = MergeCfg<K, BIG>::kThreads;
  static_assert(kThreads == 256, "the launch bound");
  constexpr int kItems = MergeCfg<K, BIG>::kItems;
  constexpr int kTile = MergeCfg<K, BIG>::kTile;
  // Indexed through pad16 on the tile path (one pad word per 16 entries):
  // each thread's outputs and its slices of the runs lie ~8-16 entries from
  // its neighbours', which would otherwise put a wave's accesses in a few banks.
  __shared__ K s_out[padded16(kTile)];
  __shared__ uint32_t s_outv[VALS ? padded16(kTile) : 1];

  __shared__ uint64_t s_pair[3];  // a0, a1, b1 of the pair holding the whole tile; a0 = ~0: none
  __shared__ uint64_t s_rank[2];

  const int tid = threadIdx.x;
  const uint64_t tile_begin = static_cast<uint64_t>(blockIdx.x) * kTile;
  const uint64_t tile_end = tile_begin + kTile < n ? tile_begin + kTile : n;
  const uint64_t ngroups = (nruns + width - 1) / width;
  const uint64_t npairs = (ngroups + 1) / 2;

  if (tid == 0) {
    uint64_t lo = 0, hi = npairs;  // last pair whose start is <= tile_begin
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) / 2;
      if (group_begin(off, nruns, width, 2 * mid, n) <= tile_begin)
        lo = mid;
      else
        hi = mid;
    }
    uint64_t a0 = group_begin(off, nruns, width, 2 * lo, n);
    uint64_t a1 = group_begin(off, nruns, width, 2 * lo + 1, n);
    uint64_t b1 = (lo + 1 == npairs) ? n : group_begin(off, nruns, width, 2 * lo + 2, n);
    if (a1 < a0) a1 = a0;
    if (b1 < a1) b1 = a1;
    const bool inside = a0 <= tile_begin && tile_end <= b1;
    s_pair[0] = inside ? a0 : ~0ull;
    s_pair[1] = a1;
    s_pair[2] = b1;
  }
  __syncthreads();
  if (s_pair[0] != ~0ull) {
    const uint64_t a0 = s_pair[0], a1 = s_pair[1], b1 = s_pair[2];
    const uint64_t la = a1 - a0, lb = b1 - a1;
    const uint64_t d0 = tile_begin - a0, d1 = tile_end - a0;
    const int wave = tid / kWave;
    if (wave < 2) {
      const uint64_t r = corank_wave<K>(src, a0, a1, la, lb, wave == 0 ? d0 : d1, flip);
      if (lane_id() == 0) s_rank[wave] = r;
    }
    __syncthreads();
    const uint64_t i0 = s_rank[0], i1 = s_rank[1];
    const int na = static_cast<int>(i1 - i0);               // A items of the tile
    const int total = static_cast<int>(tile_end - tile_begin);
    const int nb = total - na;
    const uint64_t b0 = a1 + (d0 - i0);                     // first B item of the tile
#pragma unroll
    for (int q = 0; q < kItems; ++q) {  // all loads in flight at once
      const int e = q * kThreads + tid;
      if (e < total) {
        const uint64_t from = e < na ? a0 + i0 + e : b0 + (e - na);
        s_out[pad16(e)] = src[from];
        if constexpr (VALS) s_outv[pad16(e)] = srcv[from];
      }
    }
    __syncthreads();
    // This thread's outputs: tile positions [dd, dd + kItems) of A' = s_out[0, na)
    // and B' = s_out[na, total).
    const int dd = tid * kItems;
    K ok[kItems];
    uint32_t ov[kItems];
    int cnt = 0;
    if (dd < total) {
      int lo = dd > nb ? dd - nb : 0, hi = dd < na ? dd : na;
      while (lo < hi) {
        const int mid = (lo + hi) / 2;
        if (flip_key(s_out[pad16(mid)], flip) <= flip_key(s_out[pad16(na + dd - 1 - mid)], flip))
          lo = mid + 1;
        else
          hi = mid;
      }
      int i = lo, k = dd - lo;
      cnt = total - dd < kItems ? total - dd : kItems;
      // The heads of both runs stay in registers: one LDS read per output
      // (an index past its run reads a neighbour that is never taken).
      K ha = s_out[pad16(i < kTile ? i : kTile - 1)];
      K hb = s_out[pad16(na + k < kTile ? na + k : kTile - 1)];
#pragma unroll
      for (int q = 0; q < kItems; ++q) {
        if (q < cnt) {
          const bool take_a = k >= nb || (i < na && flip_key(ha, flip) <= flip_key(hb, flip));
          ok[q] = take_a ? ha : hb;
          if constexpr (VALS) ov[q] = s_outv[pad16(take_a ? i : na + k)];
          i += take_a;
          k += !take_a;
          const int nxt = take_a ? i : na + k;
          const K h = s_out[pad16(nxt < kTile ? nxt : kTile - 1)];
          ha = take_a ? h : ha;
          hb = take_a ? hb : h;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
      if (q < cnt) {
        s_out[pad16(dd + q)] = ok[q];
        if constexpr (VALS) s_outv[pad16(dd + q)] = ov[q];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
      const int e = q * kThreads + tid;
      if (e < total) {
        dst[tile_begin + e] = s_out[pad16(e)];
        if constexpr (VALS) dstv[tile_begin + e] = s_outv[pad16(e)];
      }
    }
    return;
  }

  uint64_t p = tile_begin + static_cast<uint64_t>(tid) * kItems;
  int produced = 0;
  while (produced < kItems && p < n) {
    // Last pair whose start is <= p (pair starts are non-decreasing).
    uint64_t lo = 0, hi = npairs;  // answer in [lo, hi)
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) / 2;
      if (group_begin(off, nruns, width, 2 * mid, n) <= p)
        lo = mid;
      else
        hi = mid;
    }
    const uint64_t j = lo;
    uint64_t a0 = group_begin(off, nruns, width, 2 * j, n);
    uint64_t a1 = group_begin(off, nruns, width, 2 * j + 1, n);
    uint64_t b1 = (j + 1 == npairs) ? n : group_begin(off, nruns, width, 2 * j + 2, n);
    if (a1 < a0) a1 = a0;
    if (b1 < a1) b1 = a1;
    if (p < a0 || p >= b1) {  // offsets that break the contract: emit nothing more
      break;
    }
    const uint64_t la = a1 - a0, lb = b1 - a1;
    const uint64_t d = p - a0;
    // co-rank: i = number of left-run items among the first d outputs
    uint64_t ilo = d > lb ? d - lb : 0, ihi = d < la ? d : la;
    while (ilo < ihi) {
      const uint64_t mid = (ilo + ihi) / 2;
      if (flip_key(src[a0 + mid], flip) <= flip_key(src[a1 + (d - 1 - mid)], flip))
        ilo = mid + 1;
      else
        ihi = mid;
    }
    uint64_t i = ilo, k = d - ilo;
    while (produced < kItems && p < b1) {
      bool take_a;
      if (i >= la)
        take_a = false;
      else if (k >= lb)
        take_a = true;
      else
        take_a = flip_key(src[a0 + i], flip) <= flip_key(src[a1 + k], flip);
      const uint64_t from = take_a ? a0 + i : a1 + k;
      s_out[tid * kItems + produced] = src[from];
      if constexpr (VALS) s_outv[tid * kItems + produced] = srcv[from];
      if (take_a)
        ++i;
      else
        ++k;
      ++produced;
      ++p;
    }
  }
  __syncthreads();
  for (int t = tid; t < kTile; t += kThreads) {
    const uint64_t q = tile_begin + t;
    if (q < n) {
      dst[q] = s_out[t];
      if constexpr (VALS) dstv[q] = s_outv[t];
    }
  }
}

template <typename K, bool VALS>
__global__ __launch_bounds__(256) void copy_kernel(const K* __restrict__ src, const uint32_t* __restrict__ srcv,
                                                   K* __restrict__ dst, uint32_t* __restrict__ dstv, uint64_t n) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    dst[i] = src[i];
    if constexpr (VALS) dstv[i] = srcv[i];
  }
}

struct MergeLayout {
  size_t alt_k = 0, alt_v = 0, total = 0;
  int rounds = 0;
};

int ceil_log2(uint64_t x) {
  int r = 0;
  while ((1ull << r) < x) ++r;
  return r;
}

MergeLayout merge_layout(ms_key_type kt, bool has_vals, uint64_t n, uint64_t nruns) {
  MergeLayout L;
  L.rounds = nruns > 1 ? ceil_log2(nruns) : 0;
  if (L.rounds < 2) return L;  // one round reads the input and writes the output directly
  size_t off = 0;
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
ms_status run_merge(const void* kin, const uint32_t* vin, void* kout, uint32_t* vout, const uint64_t* off,
                    uint64_t nruns, uint64_t n, K flip, char* ws, const MergeLayout& L, hipStream_t s) {
  if (L.rounds == 0) {
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    MS_LAUNCH("merge_copy", (copy_kernel<K, VALS>), static_cast<uint32_t>(blocks), 256, s,
              static_cast<const K*>(kin), vin, static_cast<K*>(kout), vout, n);
    return MS_OK;
  }
  K* alt_k = L.rounds >= 2 ? reinterpret_cast<K*>(ws + L.alt_k) : nullptr;
  uint32_t* alt_v = (VALS && L.rounds >= 2) ? reinterpret_cast<uint32_t*>(ws + L.alt_v) : nullptr;
  const K* src = static_cast<const K*>(kin);
  const uint32_t* srcv = vin;
  const bool big = n >= kBigTileMin;
  const uint64_t tile = big ? MergeCfg<K, true>::kTile : MergeCfg<K, false>::kTile;
  const uint64_t blocks = (n + tile - 1) / tile;
  if (blocks > 0x7fffffffull) return fail(MS_ENOTSUP, "merge_runs: list too long");
  for (int r = 0; r < L.rounds; ++r) {
    const bool to_out = ((L.rounds - 1 - r) % 2) == 0;
    K* dst = to_out ? static_cast<K*>(kout) : alt_k;
    uint32_t* dstv = to_out ? vout : alt_v;
    if (big)
      MS_LAUNCH("merge_round", (merge_round_kernel<K, VALS, true>), static_cast<uint32_t>(blocks), 256, s, src, srcv,
                dst, dstv, off, nruns, n, 1ull << r, flip);
    else
      MS_LAUNCH("merge_round", (merge_round_kernel<K, VALS, false>), static_cast<uint32_t>(blocks), 256, s, src,
                srcv, dst, dstv, off, nruns, n, 1ull << r, flip);
    src = dst;
    srcv = dstv;
  }
  return MS_OK;
}

// ---------------------------------------------------------------------------
// Figure 1's merge loop as odd/even transposition merge-split over p equal
// parts: p phases, each one merge_round_kernel launch of width 1 over the
// phase's pairs (an odd phase works on the view that starts one part in, and
// part 0 is copied).  Merging a pair into the same positions and keeping the
// first s outputs in the lower part is the count-preserving split.

// The scatter phase of Figure 1: the p + 1 boundaries of p contiguous parts,
// part i = [floor(i*n/p), floor((i+1)*n/p)), so that part sizes differ by at
// most one when p does not divide n.  i*n is formed in 128 bits: it exceeds
// 64 bits for lists and part counts both beyond 2^32.
__global__ __launch_bounds__(256) void part_offsets_kernel(uint64_t* off, uint64_t n, uint64_t p) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * 256;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * 256 + threadIdx.x; i <= p; i += stride)
    off[i] = static_cast<uint64_t>((static_cast<unsigned __int128>(i) * n) / p);
}

// Grid of the partition launch: one thread per boundary, at most 65,536
// workgroups striding over the rest.
uint32_t part_offsets_blocks(uint64_t p) {
  const uint64_t b = (p + 256) / 256;
  return static_cast<uint32_t>(b < 65536 ? b : 65536);
}

struct SplitLayout {
  size_t off = 0, alt_k = 0, alt_v = 0, total = 0;
};

SplitLayout split_layout(ms_key_type kt, bool has_vals, uint64_t n, uint64_t p) {
  SplitLayout L;
  if (p < 2 || n == 0) return L;  // one part: a copy
  size_t o = 0;
  L.off = o;
  o += align_up((p + 1) * sizeof(uint64_t));
  L.alt_k = o;
  o += align_up(n * key_bytes(kt));
  if (has_vals) {
    L.alt_v = o;
    o += align_up(n * sizeof(uint32_t));
  }
  L.total = o;
  return L;
}

template <typename K, bool VALS>
ms_status run_merge_split(const void* kin, const uint32_t* vin, void* kout, uint32_t* vout, uint64_t n, uint64_t p,
                          K flip, char* ws, const SplitLayout& L, hipStream_t s) {
  uint64_t cblocks = (n + 255) / 256;
  if (cblocks > 4096) cblocks = 4096;
  if (p < 2) {
    MS_LAUNCH("merge_copy", (copy_kernel<K, VALS>), static_cast<uint32_t>(cblocks), 256, s,
              static_cast<const K*>(kin), vin, static_cast<K*>(kout), vout, n);
    return MS_OK;
  }
  uint64_t* off = reinterpret_cast<uint64_t*>(ws + L.off);
  K* alt_k = reinterpret_cast<K*>(ws + L.alt_k);
  uint32_t* alt_v = VALS ? reinterpret_cast<uint32_t*>(ws + L.alt_v) : nullptr;
  MS_LAUNCH("part_offsets", part_offsets_kernel, part_offsets_blocks(p), 256, s, off, n, p);
  const uint64_t sz = n / p;
  const bool big = n >= kBigTileMin;
  const uint64_t tile = big ? MergeCfg<K, true>::kTile : MergeCfg<K, false>::kTile;
  const K* src = static_cast<const K*>(kin);
  const uint32_t* srcv = vin;
  for (uint64_t k = 0; k < p; ++k) {
    const bool to_out = ((p - 1 - k) % 2) == 0;
    K* dst = to_out ? static_cast<K*>(kout) : alt_k;
    uint32_t* dstv = to_out ? vout : alt_v;
    // Even phase: parts (0,1), (2,3), ... of the whole list.  Odd phase: part
    // 0 copied, then parts (1,2), (3,4), ... as pairs of the view one part in.
    const uint64_t skip = (k % 2 == 1) ? sz : 0;
    if (skip)
      MS_LAUNCH("merge_copy", (copy_kernel<K, VALS>), static_cast<uint32_t>(cblocks), 256, s, src, srcv, dst, dstv,
                sz);
    const uint64_t m = n - skip;
    const uint64_t blocks = (m + tile - 1) / tile;
    const K* vs = src + skip;
    K* vd = dst + skip;
    const uint32_t* vsv = VALS ? srcv + skip : nullptr;
    uint32_t* vdv = VALS ? dstv + skip : nullptr;
    if (big)
      MS_LAUNCH("merge_split_phase", (merge_round_kernel<K, VALS, true>), static_cast<uint32_t>(blocks), 256, s, vs,
                vsv, vd, vdv, static_cast<const uint64_t*>(off), p - (skip ? 1 : 0), m, 1ull, flip);
    else
      MS_LAUNCH("merge_split_phase", (merge_round_kernel<K, VALS, false>), static_cast<uint32_t>(blocks), 256, s,
                vs, vsv, vd, vdv, static_cast<const uint64_t*>(off), p - (skip ? 1 : 0), m, 1ull, flip);
    src = dst;
    srcv = dstv;
  }
  return MS_OK;
}

}  // namespace

ms_status partition_offsets(uint64_t n, uint64_t p, uint64_t* off, hipStream_t s) {
  MS_LAUNCH("part_offsets", part_offsets_kernel, part_offsets_blocks(p), 256, s, off, n, p);
  return MS_OK;
}

size_t merge_split_workspace_bytes(ms_key_type kt, bool has_vals, uint64_t n, uint64_t nparts) {
  return split_layout(kt, has_vals, n, nparts).total;
}

ms_status merge_split_parts(const void* keys_in, const uint32_t* vals_in, void* keys_out, uint32_t* vals_out,
                            uint64_t n, uint64_t nparts, ms_key_type kt, void* ws, size_t ws_bytes, hipStream_t s) {
  const bool vals = vals_in != nullptr;
  const SplitLayout L = split_layout(kt, vals, n, nparts);
  if (ws_bytes < L.total || (L.total && !ws))
    return fail(MS_EINVAL, "merge_split: workspace too small: %zu bytes given, %zu needed", ws_bytes, L.total);
  if ((n + MergeCfg<uint64_t, false>::kTile - 1) / MergeCfg<uint64_t, false>::kTile > 0x7fffffffull)
    return fail(MS_ENOTSUP, "merge_split: list too long");
  char* w = static_cast<char*>(ws);
  switch (kt) {
    case MS_KEY_I32:
      return vals ? run_merge_split<uint32_t, true>(keys_in, vals_in, keys_out, vals_out, n, nparts, 0x80000000u, w, L, s)
                  : run_merge_split<uint32_t, false>(keys_in, vals_in, keys_out, vals_out, n, nparts, 0x80000000u, w, L, s);
    case MS_KEY_U32:
      return vals ? run_merge_split<uint32_t, true>(keys_in, vals_in, keys_out, vals_out, n, nparts, 0u, w, L, s)
                  : run_merge_split<uint32_t, false>(keys_in, vals_in, keys_out, vals_out, n, nparts, 0u, w, L, s);
    case MS_KEY_U64:
      return vals ? run_merge_split<uint64_t, true>(keys_in, vals_in, keys_out, vals_out, n, nparts, 0ull, w, L, s)
                  : run_merge_split<uint64_t, false>(keys_in, vals_in, keys_out, vals_out, n, nparts, 0ull, w, L, s);
  }
  return fail(MS_ENOTSUP, "merge_split: unknown key type %d", static_cast<int>(kt));
}

size_t merge_workspace_bytes(ms_key_type kt, bool has_vals, uint64_t n, uint64_t nruns) {
  return merge_layout(kt, has_vals, n, nruns).total;
}

ms_status merge_sorted_runs(const void* keys_in, const uint32_t* vals_in, void* keys_out, uint32_t* vals_out,
                            const uint64_t* offsets, uint64_t nruns, uint64_t n, ms_key_type kt, void* ws,
                            size_t ws_bytes, hipStream_t s) {
  const bool vals = vals_in != nullptr;
  const MergeLayout L = merge_layout(kt, vals, n, nruns);
  if (ws_bytes < L.total || (L.total && !ws))
    return fail(MS_EINVAL, "merge_runs: workspace too small: %zu bytes given, %zu needed", ws_bytes, L.total);
  char* w = static_cast<char*>(ws);
  switch (kt) {
    case MS_KEY_I32:
      return vals ? run_merge<uint32_t, true>(keys_in, vals_in, keys_out, vals_out, offsets, nruns, n, 0x80000000u, w, L, s)
                  : run_merge<uint32_t, false>(keys_in, vals_in, keys_out, vals_out, offsets, nruns, n, 0x80000000u, w, L, s);
    case MS_KEY_U32:
      return vals ? run_merge<uint32_t, true>(keys_in, vals_in, keys_out, vals_out, offsets, nruns, n, 0u, w, L, s)
                  : run_merge<uint32_t, false>(keys_in, vals_in, keys_out, vals_out, offsets, nruns, n, 0u, w, L, s);
    case MS_KEY_U64:
      return vals ? run_merge<uint64_t, true>(keys_in, vals_in, keys_out, vals_out, offsets, nruns, n, 0ull, w, L, s)
                  : run_merge<uint64_t, false>(keys_in, vals_in, keys_out, vals_out, offsets, nruns, n, 0ull, w, L, s);
  }
  return fail(MS_ENOTSUP, "merge_runs: unknown key type %d", static_cast<int>(kt));
}

}  // namespace ms

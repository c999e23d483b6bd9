// probe.hip -- achievable HBM bandwidth, measured with kernels written here.
//
// Three streaming kernels with the sort passes' access width (16-byte
// vector loads and stores, fully coalesced): a read (every byte of `src`
// read once, folded into one word per workgroup so nothing is optimised
// away), a write (every byte of `dst` written once) and a copy (read `src`,
// write `dst`), each with ordinary or non-temporal (streaming) accesses.
// Their rates are the practical ceiling the sort's roofline fraction is read
// against, and under rocprofv3 their byte counters calibrate the counters of
// the sort kernels.  Not part of the sort path.
#include "ms_runtime.hpp"

namespace ms {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeUnroll = 8;
constexpr int kWaveSize = 64;
constexpr uint32_t kProbeBlocks = 2048;  // 8 workgroups per compute unit

template <bool NT>
__device__ __forceinline__ uint4 ld16(const uint4* p) {
  if constexpr (NT) {
    uint4 v;
    v.x = __builtin_nontemporal_load(&p->x);
    v.y = __builtin_nontemporal_load(&p->y);
    v.z = __builtin_nontemporal_load(&p->z);
    v.w = __builtin_nontemporal_load(&p->w);
    return v;
  } else {
    return *p;
  }
}

template <bool NT>
__device__ __forceinline__ void st16(uint4* p, uint4 v) {
  if constexpr (NT) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
    __builtin_nontemporal_store(v.z, &p->z);
    __builtin_nontemporal_store(v.w, &p->w);
  } else {
    *p = v;
  }
}

// kind: 0 read, 1 write, 2 copy.  n16 = number of 16-byte words.  Each
// workgroup streams one contiguous chunk (DRAM pages stay open), 256 threads
// x kProbeUnroll independent 16-byte accesses in flight per step.
template <int KIND, bool NT>
__global__ __launch_bounds__(kProbeThreads) void probe_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                              size_t n16, uint32_t* __restrict__ sink) {
  constexpr size_t kStep = static_cast<size_t>(kProbeThreads) * kProbeUnroll;
  const size_t per_block = (n16 + gridDim.x - 1) / gridDim.x;
  const size_t chunk = (per_block + kStep - 1) / kStep * kStep;
  const size_t begin = static_cast<size_t>(blockIdx.x) * chunk;
  const size_t end = begin + chunk < n16 ? begin + chunk : n16;
  uint32_t acc = 0;
  const uint4 pattern = make_uint4(0x9e3779b9u, 0x7f4a7c15u, 0x85ebca6bu, 0xc2b2ae35u);
  size_t i = begin + threadIdx.x;
  for (; i + (kProbeUnroll - 1) * kProbeThreads < end; i += kStep) {
    uint4 v[kProbeUnroll];
    if constexpr (KIND != 1) {
#pragma unroll
      for (int u = 0; u < kProbeUnroll; ++u) v[u] = ld16<NT>(src + i + u * kProbeThreads);
    }
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) {
      if constexpr (KIND == 0) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
      if constexpr (KIND == 1) st16<NT>(dst + i + u * kProbeThreads, pattern);
      if constexpr (KIND == 2) st16<NT>(dst + i + u * kProbeThreads, v[u]);
    }
  }
  for (; i < end; i += kProbeThreads) {
    if constexpr (KIND == 0) {
      const uint4 v = ld16<NT>(src + i);
      acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if constexpr (KIND == 1) st16<NT>(dst + i, pattern);
    if constexpr (KIND == 2) st16<NT>(dst + i, ld16<NT>(src + i));
  }
  if constexpr (KIND == 0) {
    // One word per workgroup, so the loads cannot be dropped.
#pragma unroll
    for (int o = kWaveSize / 2; o > 0; o /= 2) acc ^= __shfl_xor(acc, o, kWaveSize);
    if ((threadIdx.x % kWaveSize) == 0) atomicXor(&sink[blockIdx.x], acc);
  }
}

template <int KIND, bool NT>
ms_status launch_probe(const void* src, void* dst, size_t n16, uint32_t blocks, uint32_t* sink, hipStream_t s) {
  MS_LAUNCH(KIND == 0 ? (NT ? "probe_read_nt" : "probe_read")
                      : KIND == 1 ? (NT ? "probe_write_nt" : "probe_write") : (NT ? "probe_copy_nt" : "probe_copy"),
            (probe_kernel<KIND, NT>), blocks, kProbeThreads, s, static_cast<const uint4*>(src),
            static_cast<uint4*>(dst), n16, sink);
  return MS_OK;
}

}  // namespace

size_t probe_sink_bytes() { return kProbeBlocks * sizeof(uint32_t); }

ms_status hbm_probe(int kind, const void* src, void* dst, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  uint32_t* sink = static_cast<uint32_t*>(dst);
  switch (kind) {
    case 0: return launch_probe<0, false>(src, nullptr, n16, kProbeBlocks, sink, s);
    case 1: return launch_probe<1, false>(nullptr, dst, n16, kProbeBlocks, nullptr, s);
    case 2: return launch_probe<2, false>(src, dst, n16, kProbeBlocks, nullptr, s);
    case 3: return launch_probe<0, true>(src, nullptr, n16, kProbeBlocks, sink, s);
    case 4: return launch_probe<1, true>(nullptr, dst, n16, kProbeBlocks, nullptr, s);
    case 5: return launch_probe<2, true>(src, dst, n16, kProbeBlocks, nullptr, s);
  }
  return fail(MS_EINVAL, "ms_hbm_probe: unknown kind %d", kind);
}

}  // namespace ms

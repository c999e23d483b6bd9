// Host-side stand-in for <hip/hip_runtime.h> used ONLY by the CPU SIMT
// emulator tests (tests/simt).  It lets the library's kernel sources compile
// with a host C++ compiler: every GPU thread of a block runs as a cooperative
// fiber, __syncthreads() is a block barrier, wave64 collectives (ballot,
// readfirstlane, shfl, wave_barrier) rendezvous the 64 lanes of a wave.
// Several blocks of a grid run at once, each on its own OS thread (so blocks
// really do wait on each other, as in a decoupled look-back); a block's
// __shared__ arrays are thread-local to its OS thread.  Built with
// AddressSanitizer, out-of-bounds accesses to device buffers or LDS arrays
// are reported on the CPU.  Not a model of the GPU memory ordering.
#pragma once

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <stddef.h>
#include <string.h>

#include <functional>

// ---------------------------------------------------------------------------
// Qualifiers.
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
// Each running block owns an OS thread, so thread-local statics are its LDS.
#define __shared__ static thread_local
#define __align__(n) alignas(n)
// A __device__ variable is an ordinary host object here; its "symbol
// address" is its address.
#define HIP_SYMBOL(x) (reinterpret_cast<const void*>(&(x)))
// Non-temporal accesses are ordinary accesses here.
template <typename T>
inline T __builtin_nontemporal_load(const T* p) { return *p; }
template <typename T>
inline void __builtin_nontemporal_store(T v, T* p) { *p = v; }

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

struct uint4 {
  unsigned x, y, z, w;
};
inline uint4 make_uint4(unsigned a, unsigned b, unsigned c, unsigned d) { return uint4{a, b, c, d}; }
typedef uint4 HIP_vector_type_uint4;

// ---------------------------------------------------------------------------
// Runtime API subset.
typedef void* hipStream_t;
typedef void* hipEvent_t;
typedef enum hipError_t { hipSuccess = 0, hipErrorUnknown = 999 } hipError_t;
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "simt"; }
inline hipError_t hipEventCreate(hipEvent_t* e) {
  *e = nullptr;
  return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.f;
  return hipSuccess;
}
inline hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
// The emulated device: one device of kSimtCUs compute units holding one
// workgroup each, so persistent kernels loop over many tiles per workgroup.
constexpr int kSimtCUs = 2;
typedef enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount = 1 } hipDeviceAttribute_t;
inline hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  *p = const_cast<void*>(symbol);
  return hipSuccess;
}
inline hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
inline hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
  *v = a == hipDeviceAttributeMultiprocessorCount ? kSimtCUs : 0;
  return hipSuccess;
}
// SIMT_BLOCKS_PER_CU (default 1) sets the blocks a CU holds, so that a
// persistent kernel's grid can be made large enough for its look-back agents.
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void*, int, size_t) {
  const char* e = getenv("SIMT_BLOCKS_PER_CU");
  *n = e && atoi(e) > 0 ? atoi(e) : 1;
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Emulator core (tests/simt/simt.cpp).
namespace simt {
struct Idx {
  unsigned x, y, z;
};
const Idx& thread_idx();
const Idx& block_idx();
const Idx& block_dim();
const Idx& grid_dim();
void barrier();
int barrier_or(int p);
uint64_t ballot(bool p);
uint64_t shfl_u64(uint64_t v, int src_lane);  // value of `src_lane` (caller computes it)
void wave_sync();
uint32_t lane();
void yield();
void launch(dim3 grid, dim3 block, const std::function<void()>& body);
}  // namespace simt

#define threadIdx (::simt::thread_idx())
#define blockIdx (::simt::block_idx())
#define blockDim (::simt::block_dim())
#define gridDim (::simt::grid_dim())

inline void __syncthreads() { simt::barrier(); }
inline int __syncthreads_or(int p) { return simt::barrier_or(p); }
inline void __threadfence() {}
inline void __threadfence_block() {}

inline uint64_t __builtin_amdgcn_ballot_w64(bool p) { return simt::ballot(p); }
inline uint32_t __builtin_amdgcn_mbcnt_lo(uint32_t m, uint32_t acc) {
  const uint32_t l = simt::lane();
  const uint32_t mask = l >= 32 ? 0xffffffffu : ((1u << l) - 1u);
  return acc + static_cast<uint32_t>(__builtin_popcount(m & mask));
}
inline uint32_t __builtin_amdgcn_mbcnt_hi(uint32_t m, uint32_t acc) {
  const uint32_t l = simt::lane();
  const uint32_t mask = l < 32 ? 0u : ((1u << (l - 32)) - 1u);
  return acc + static_cast<uint32_t>(__builtin_popcount(m & mask));
}
inline uint32_t __builtin_amdgcn_readfirstlane(uint32_t v) { return static_cast<uint32_t>(simt::shfl_u64(v, 0)); }
inline void __builtin_amdgcn_s_sleep(int) { simt::yield(); }
inline void __builtin_amdgcn_wave_barrier() { simt::wave_sync(); }
// Global-to-LDS load: lane l copies `size` bytes from its `src` to
// dst + offset + l * size (dst is the same for every lane of the wave).  The
// emulator copies at once, so waits for it are no-ops.
inline void __builtin_amdgcn_global_load_lds(const void* src, void* dst, unsigned size, int offset, int) {
  memcpy(static_cast<char*>(dst) + offset + simt::lane() * size, src, size);
}
inline void __builtin_amdgcn_s_waitcnt(int) {}
// DPP move (GFX9 rules) for the controls the kernels use: row_shr:1..15
// (0x111..0x11f, within rows of 16 lanes) and row_bcast:15 / row_bcast:31
// (0x142 / 0x143).  Lanes of rows disabled by row_mask keep `old`; lanes
// whose source lies outside the row read 0 with bound_ctrl, else keep `old`.
inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
  const int l = static_cast<int>(simt::lane());
  const int row = l / 16, r = l % 16;
  int from = -1;
  if (ctrl >= 0x111 && ctrl <= 0x11f) {
    const int n = ctrl - 0x110;
    from = r >= n ? l - n : -1;
  } else if (ctrl == 0x142) {
    from = row >= 1 ? row * 16 - 1 : -1;
  } else if (ctrl == 0x143) {
    from = row >= 2 ? 31 : -1;
  } else {
    fprintf(stderr, "simt: unsupported dpp control 0x%x\n", ctrl);
    abort();
  }
  if (bank_mask != 0xf) {
    fprintf(stderr, "simt: unsupported dpp bank mask 0x%x\n", bank_mask);
    abort();
  }
  const uint64_t got = simt::shfl_u64(static_cast<uint32_t>(src), from >= 0 ? from : l);
  if (!((row_mask >> row) & 1)) return old;
  if (from < 0) return bound_ctrl ? 0 : old;
  return static_cast<int>(static_cast<uint32_t>(got));
}
inline void __builtin_amdgcn_fence(int, const char*) {}
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline int __popc(unsigned x) { return __builtin_popcount(x); }

template <typename T>
inline T __shfl_up(T v, unsigned delta, int width = 64) {
  (void)width;
  const uint32_t l = simt::lane();
  const int src = l >= delta ? static_cast<int>(l - delta) : static_cast<int>(l);
  uint64_t bits = 0;
  memcpy(&bits, &v, sizeof(T));
  const uint64_t got = simt::shfl_u64(bits, src);
  T out;
  memcpy(&out, &got, sizeof(T));
  return out;
}

template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64) {
  (void)width;
  const int src = static_cast<int>(simt::lane()) ^ mask;
  uint64_t bits = 0;
  memcpy(&bits, &v, sizeof(T));
  const uint64_t got = simt::shfl_u64(bits, src);
  T out;
  memcpy(&out, &got, sizeof(T));
  return out;
}

template <typename T>
inline T __shfl(T v, int src_lane, int width = 64) {
  if (width != 64) {
    fprintf(stderr, "simt: only full-wave __shfl is emulated\n");
    abort();
  }
  uint64_t bits = 0;
  memcpy(&bits, &v, sizeof(T));
  const uint64_t got = simt::shfl_u64(bits, src_lane & 63);
  T out;
  memcpy(&out, &got, sizeof(T));
  return out;
}

// Atomics: blocks run on parallel OS threads, so real atomics.
template <typename T>
inline T atomicAdd(T* p, T v) {
  return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}
// atomicInc: old = *p; *p = old >= bound ? 0 : old + 1; returns old.
inline unsigned atomicInc(unsigned* p, unsigned bound) {
  unsigned old = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (!__atomic_compare_exchange_n(p, &old, old >= bound ? 0u : old + 1u, false, __ATOMIC_SEQ_CST,
                                      __ATOMIC_SEQ_CST)) {
  }
  return old;
}
template <typename T>
inline T atomicOr(T* p, T v) {
  return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST);
}
template <typename T>
inline T atomicXor(T* p, T v) {
  return __atomic_fetch_xor(p, v, __ATOMIC_SEQ_CST);
}
template <typename T>
inline T atomicCAS(T* p, T expected, T desired) {
  __atomic_compare_exchange_n(p, &expected, desired, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST);
  return expected;  // the old value
}

#define __HIP_MEMORY_SCOPE_AGENT 0
#define __HIP_MEMORY_SCOPE_WORKGROUP 0
template <typename T>
inline T __hip_atomic_load(T* p, int, int) {
  simt::yield();  // let other fibers run between polls
  return __atomic_load_n(p, __ATOMIC_SEQ_CST);
}
template <typename T>
inline void __hip_atomic_store(T* p, T v, int, int) {
  __atomic_store_n(p, v, __ATOMIC_SEQ_CST);
}
template <typename T>
inline T __hip_atomic_fetch_add(T* p, T v, int, int) {
  return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}

#define hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, ...) \
  ::simt::launch(GRID, BLOCK, [&]() { KERNEL(__VA_ARGS__); })

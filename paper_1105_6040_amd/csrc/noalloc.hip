// noalloc.hip -- sort_keys for callers that cannot allocate device memory.
//
// The same sort as sort_keys (the same kernels and launches), with its
// workspace taken from a fixed array in the library's device memory instead
// of a caller's buffer, so a call needs neither hipMalloc nor a workspace
// argument: usable under HIP graph capture, in serving loops that must not
// allocate, and from harnesses that forbid allocation.
//
// The array is a file-scope __device__ variable.  In host code its name is
// only a host-side stand-in, not a device address, so the library looks up
// its real address once per device with hipGetSymbolAddress (with that
// device current) and passes that pointer to the kernels.  Every GPU holds
// its own copy of the array until the process ends.
#include <mutex>

#include "ms_runtime.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's copy of `scratch`, looked up on first
// use with the device current.  nullptr (and *err set) on failure.
void* scratch_on_current_device(int* dev_out, ms_status* err) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *err = ms::fail(MS_EDEVICE, "sort_keys_noalloc: hipGetDevice failed: %s", hipGetErrorString(e));
    return nullptr;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    *err = ms::fail(MS_ENOTSUP, "sort_keys_noalloc: device %d beyond the %d devices supported", dev, kMaxDevices);
    return nullptr;
  }
  *dev_out = dev;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *err = ms::fail(MS_EDEVICE, "sort_keys_noalloc: hipGetSymbolAddress of the scratch array failed on device %d: %s",
                      dev, hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

ms_status sort_keys_noalloc(const void* keys_in, void* keys_out, uint64_t n, ms_key_type kt, void* stream) {
  if (kt != MS_KEY_I32 && kt != MS_KEY_U32 && kt != MS_KEY_U64)
    return ms::fail(MS_ENOTSUP, "sort_keys_noalloc: unknown key type %d", static_cast<int>(kt));
  if (n == 0) return MS_OK;
  if (!keys_in || !keys_out)
    return ms::fail(MS_EINVAL, "sort_keys_noalloc: NULL key pointer with n = %llu", static_cast<unsigned long long>(n));
  const size_t need = ms::radix_workspace_bytes(kt, false, n);
  if (need > kScratchBytes)
    return ms::fail(MS_EINVAL,
                    "sort_keys_noalloc: n = %llu keys need %zu bytes of scratch, beyond the %zu-byte static scratch "
                    "array; use sort_keys with a workspace",
                    static_cast<unsigned long long>(n), need, kScratchBytes);
  ms_status err = MS_OK;
  int dev = 0;
  void* ws = need ? scratch_on_current_device(&dev, &err) : nullptr;
  if (need && !ws) return err;
  return ms::radix_sort(keys_in, nullptr, keys_out, nullptr, n, kt, ws, kScratchBytes, static_cast<hipStream_t>(stream));
}

}  // extern "C"

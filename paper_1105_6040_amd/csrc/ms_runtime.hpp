// ms_runtime.hpp -- host-side internals: error reporting, launch checking,
// optional per-kernel event timing, and the internal entry points each
// kernel family exports to the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "mi355sort.h"

namespace ms {

// Record a message for ms_last_error() and return `st`.
ms_status fail(ms_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

// Event timing around every launch while enabled (see ms_timing_enable).
void timing_begin(const char* name, hipStream_t s);
void timing_end(const char* name, hipStream_t s);

// After a launch: MS_OK, or MS_EDEVICE with the HIP error text recorded.
ms_status check_launch(const char* name);

// Launch a kernel with the timing hooks and a launch-error check.
#define MS_LAUNCH(NAME, KERNEL, GRID, BLOCK, STREAM, ...)                             \
  do {                                                                              \
    ::ms::timing_begin(NAME, STREAM);                                               \
    hipLaunchKernelGGL(KERNEL, dim3(GRID), dim3(BLOCK), 0, STREAM, __VA_ARGS__);     \
    ::ms::timing_end(NAME, STREAM);                                                 \
    const ms_status _st = ::ms::check_launch(NAME);                                 \
    if (_st != MS_OK) return _st;                                                   \
  } while (0)

// Tunable launch parameters (ms_tune_set / ms_tune_get).
int64_t tune_get(ms_tune_param p);

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

inline int key_bytes(ms_key_type kt) { return kt == MS_KEY_U64 ? 8 : 4; }

// ---- radix sort of one list (sort_keys / sort_pairs) -----------------------
size_t radix_workspace_bytes(ms_key_type kt, bool has_vals, uint64_t n);
ms_status radix_sort(const void* keys_in, const uint32_t* vals_in, void* keys_out, uint32_t* vals_out,
                     uint64_t n, ms_key_type kt, void* ws, size_t ws_bytes, hipStream_t s);

// ---- segmented sort ---------------------------------------------------------
size_t segmented_workspace_bytes(ms_key_type kt, bool has_vals, uint64_t n, uint64_t nseg);
ms_status segmented_sort(const void* keys_in, const uint32_t* vals_in, void* keys_out,
                         uint32_t* vals_out, const uint64_t* offsets, uint64_t nseg, uint64_t n,
                         ms_key_type kt, void* ws, size_t ws_bytes, hipStream_t s);

// Whole-device digit passes over many segments (radix.hip), in one of two
// forms (MS_TUNE_SEG_PASSES = mode): a launch per phase (mode 1) for
// segments averaging more than 8,192 keys, or the one-launch work queue
// (mode 2) for segments averaging more than 1,024.  sort_segmented takes
// this path when the host-known counts allow it for the mode; with
// mode == 0 the threshold of the lowest form is returned (workspace sizing
// covers every form).
bool segsweep_eligible(uint64_t n, uint64_t nseg, int mode);
size_t segsweep_workspace_bytes(ms_key_type kt, bool has_vals, uint64_t n, uint64_t nseg);
ms_status segsweep_sort(const void* keys_in, const uint32_t* vals_in, void* keys_out, uint32_t* vals_out,
                        const uint64_t* offsets, uint64_t nseg, uint64_t n, ms_key_type kt, void* ws,
                        size_t ws_bytes, hipStream_t s);

// ---- continuous batching (step.hip) and the bandwidth probe (probe.hip) -----
size_t step_control_bytes();
ms_status step_request_plan(ms_key_type kt, bool has_vals, uint64_t n, uint32_t* phases, size_t* work_bytes);
ms_status sort_step_run(const ms_step_request* reqs, uint32_t num_reqs, ms_key_type kt, bool has_vals, void* ws,
                        hipStream_t s);
size_t probe_sink_bytes();
ms_status hbm_probe(int kind, const void* src, void* dst, size_t bytes, hipStream_t s);

// ---- scatter phase: part boundaries ------------------------------------------
ms_status partition_offsets(uint64_t n, uint64_t p, uint64_t* off, hipStream_t s);

// ---- merge of sorted runs ---------------------------------------------------
size_t merge_workspace_bytes(ms_key_type kt, bool has_vals, uint64_t n, uint64_t nruns);
size_t merge_split_workspace_bytes(ms_key_type kt, bool has_vals, uint64_t n, uint64_t nparts);
ms_status merge_split_parts(const void* keys_in, const uint32_t* vals_in, void* keys_out, uint32_t* vals_out,
                            uint64_t n, uint64_t nparts, ms_key_type kt, void* ws, size_t ws_bytes, hipStream_t s);
ms_status merge_sorted_runs(const void* keys_in, const uint32_t* vals_in, void* keys_out,
                            uint32_t* vals_out, const uint64_t* offsets, uint64_t nruns, uint64_t n,
                            ms_key_type kt, void* ws, size_t ws_bytes, hipStream_t s);

}  // namespace ms

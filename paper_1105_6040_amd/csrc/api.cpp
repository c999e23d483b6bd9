// api.cpp -- the C ABI (include/mi355sort.h): argument checks, workspace
// sizing, dispatch to the kernel families, error text and kernel timing.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ms_runtime.hpp"

namespace ms {

namespace {
thread_local char t_error[512] = "";

struct PendingTiming {
  std::string name;
  hipEvent_t start;
  hipEvent_t stop;
};

struct TimingState {
  bool enabled = false;
  std::vector<PendingTiming> pending;
  hipEvent_t open_start = nullptr;
  std::map<std::string, std::pair<uint64_t, double>> totals;  // name -> (launches, ms)
};
TimingState g_timing;
std::mutex g_timing_mu;

bool valid_kt(ms_key_type kt) { return kt == MS_KEY_I32 || kt == MS_KEY_U32 || kt == MS_KEY_U64; }

std::atomic<int64_t> g_tune[MS_TUNE_COUNT] = {{1024}, {0}, {0}, {64}, {512}, {1}};
}  // namespace

int64_t tune_get(ms_tune_param p) { return (p >= 0 && p < MS_TUNE_COUNT) ? g_tune[p].load() : 0; }

ms_status fail(ms_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(t_error, sizeof(t_error), fmt, ap);
  va_end(ap);
  return st;
}

ms_status check_launch(const char* name) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MS_EDEVICE, "launch of %s failed: %s", name, hipGetErrorString(e));
  return MS_OK;
}

void timing_begin(const char* name, hipStream_t s) {
  (void)name;
  std::lock_guard<std::mutex> lk(g_timing_mu);
  if (!g_timing.enabled) return;
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  (void)hipEventRecord(e, s);
  g_timing.open_start = e;
}

void timing_end(const char* name, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_timing_mu);
  if (!g_timing.enabled || !g_timing.open_start) return;
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  (void)hipEventRecord(e, s);
  g_timing.pending.push_back({name, g_timing.open_start, e});
  g_timing.open_start = nullptr;
}

}  // namespace ms

using ms::fail;

extern "C" {

const char* ms_last_error(void) { return ms::t_error; }

ms_status ms_workspace_size(ms_op op, ms_key_type kt, int has_values, uint64_t n_total, uint64_t num_segments,
                            size_t* bytes) {
  if (!bytes) return fail(MS_EINVAL, "ms_workspace_size: bytes is NULL");
  if (!ms::valid_kt(kt)) return fail(MS_ENOTSUP, "unknown key type %d", static_cast<int>(kt));
  switch (op) {
    case MS_OP_SORT_KEYS:
      *bytes = ms::radix_workspace_bytes(kt, false, n_total);
      return MS_OK;
    case MS_OP_SORT_PAIRS:
      *bytes = ms::radix_workspace_bytes(kt, true, n_total);
      return MS_OK;
    case MS_OP_SORT_SEGMENTED:
      *bytes = ms::segmented_workspace_bytes(kt, has_values != 0, n_total, num_segments);
      return MS_OK;
    case MS_OP_MERGE_RUNS:
      *bytes = ms::merge_workspace_bytes(kt, has_values != 0, n_total, num_segments);
      return MS_OK;
    case MS_OP_MERGE_SPLIT:
      *bytes = ms::merge_split_workspace_bytes(kt, has_values != 0, n_total, num_segments);
      return MS_OK;
    case MS_OP_SORT_STEP:
      *bytes = ms::step_control_bytes();
      return MS_OK;
  }
  return fail(MS_ENOTSUP, "unknown op %d", static_cast<int>(op));
}

ms_status sort_keys(const void* keys_in, void* keys_out, uint64_t n, ms_key_type kt, void* ws, size_t ws_bytes,
                    void* stream) {
  if (!ms::valid_kt(kt)) return fail(MS_ENOTSUP, "sort_keys: unknown key type %d", static_cast<int>(kt));
  if (n == 0) return MS_OK;
  if (!keys_in || !keys_out) return fail(MS_EINVAL, "sort_keys: NULL key pointer with n = %llu",
                                         static_cast<unsigned long long>(n));
  return ms::radix_sort(keys_in, nullptr, keys_out, nullptr, n, kt, ws, ws_bytes,
                        static_cast<hipStream_t>(stream));
}

ms_status sort_pairs(const void* keys_in, const uint32_t* vals_in, void* keys_out, uint32_t* vals_out, uint64_t n,
                     ms_key_type kt, void* ws, size_t ws_bytes, void* stream) {
  if (!ms::valid_kt(kt)) return fail(MS_ENOTSUP, "sort_pairs: unknown key type %d", static_cast<int>(kt));
  if (n == 0) return MS_OK;
  if (!keys_in || !keys_out || !vals_in || !vals_out)
    return fail(MS_EINVAL, "sort_pairs: NULL pointer with n = %llu", static_cast<unsigned long long>(n));
  if ((keys_in == keys_out) != (static_cast<const void*>(vals_in) == static_cast<const void*>(vals_out)))
    return fail(MS_EINVAL, "sort_pairs: keys and values must both be in place or both out of place");
  return ms::radix_sort(keys_in, vals_in, keys_out, vals_out, n, kt, ws, ws_bytes,
                        static_cast<hipStream_t>(stream));
}

ms_status part_offsets(uint64_t n, uint64_t num_parts, uint64_t* offsets_out, void* stream) {
  if (num_parts == 0) return fail(MS_EINVAL, "part_offsets: num_parts must be at least 1");
  if (num_parts == UINT64_MAX)
    return fail(MS_EINVAL, "part_offsets: num_parts + 1 boundaries do not fit in 64 bits");
  if (!offsets_out) return fail(MS_EINVAL, "part_offsets: NULL offsets_out");
  return ms::partition_offsets(n, num_parts, offsets_out, static_cast<hipStream_t>(stream));
}

ms_status ms_step_plan(ms_key_type kt, int has_values, uint64_t n, uint32_t* phases, size_t* work_bytes) {
  if (!phases || !work_bytes) return fail(MS_EINVAL, "ms_step_plan: NULL output pointer");
  if (!ms::valid_kt(kt)) return fail(MS_ENOTSUP, "ms_step_plan: unknown key type %d", static_cast<int>(kt));
  return ms::step_request_plan(kt, has_values != 0, n, phases, work_bytes);
}

ms_status sort_step(const ms_step_request* reqs, uint64_t num_reqs, ms_key_type kt, int has_values, void* ws,
                    size_t ws_bytes, void* stream) {
  if (!ms::valid_kt(kt)) return fail(MS_ENOTSUP, "sort_step: unknown key type %d", static_cast<int>(kt));
  if (num_reqs > MS_STEP_MAX_REQUESTS)
    return fail(MS_EINVAL, "sort_step: %llu requests in one step, at most %d", static_cast<unsigned long long>(num_reqs),
                MS_STEP_MAX_REQUESTS);
  if (num_reqs == 0) return MS_OK;
  if (!reqs) return fail(MS_EINVAL, "sort_step: NULL request table with %llu requests",
                         static_cast<unsigned long long>(num_reqs));
  if (!ws || ws_bytes < ms::step_control_bytes())
    return fail(MS_EINVAL, "sort_step: workspace too small: %zu bytes given, %zu needed", ws_bytes,
                ms::step_control_bytes());
  return ms::sort_step_run(reqs, static_cast<uint32_t>(num_reqs), kt, has_values != 0, ws,
                           static_cast<hipStream_t>(stream));
}

ms_status ms_hbm_probe(int kind, const void* src, void* dst, size_t bytes, void* stream) {
  if (kind < 0 || kind > 5) return fail(MS_EINVAL, "ms_hbm_probe: unknown kind %d", kind);
  if (bytes % 16) return fail(MS_EINVAL, "ms_hbm_probe: %zu bytes is not a multiple of 16", bytes);
  const bool reads = kind != 1 && kind != 4;
  if ((reads && !src) || !dst) return fail(MS_EINVAL, "ms_hbm_probe: NULL pointer");
  return ms::hbm_probe(kind, src, dst, bytes, static_cast<hipStream_t>(stream));
}

static ms_status check_ranged(const char* what, const void* keys_in, const uint32_t* vals_in, const void* keys_out,
                              const uint32_t* vals_out, const uint64_t* offsets, uint64_t count,
                              uint64_t n_total, ms_key_type kt) {
  if (!ms::valid_kt(kt)) return fail(MS_ENOTSUP, "%s: unknown key type %d", what, static_cast<int>(kt));
  if ((vals_in == nullptr) != (vals_out == nullptr))
    return fail(MS_EINVAL, "%s: give both vals_in and vals_out, or neither", what);
  if (n_total > 0 && (!keys_in || !keys_out))
    return fail(MS_EINVAL, "%s: NULL key pointer with n_total = %llu", what,
                static_cast<unsigned long long>(n_total));
  if (count > 0 && !offsets) return fail(MS_EINVAL, "%s: NULL offsets with %llu entries", what,
                                         static_cast<unsigned long long>(count));
  return MS_OK;
}

ms_status sort_segmented(const void* keys_in, const uint32_t* vals_in, void* keys_out, uint32_t* vals_out,
                         const uint64_t* seg_offsets, uint64_t num_segments, uint64_t n_total, ms_key_type kt,
                         void* ws, size_t ws_bytes, void* stream) {
  ms_status st = check_ranged("sort_segmented", keys_in, vals_in, keys_out, vals_out, seg_offsets, num_segments,
                              n_total, kt);
  if (st != MS_OK) return st;
  if (num_segments == 0) {
    if (n_total) return fail(MS_EINVAL, "sort_segmented: no segments but n_total = %llu",
                             static_cast<unsigned long long>(n_total));
    return MS_OK;
  }
  if (vals_in && ((keys_in == keys_out) != (static_cast<const void*>(vals_in) == static_cast<const void*>(vals_out))))
    return fail(MS_EINVAL, "sort_segmented: keys and values must both be in place or both out of place");
  if (n_total == 0) return MS_OK;
  return ms::segmented_sort(keys_in, vals_in, keys_out, vals_out, seg_offsets, num_segments, n_total, kt, ws,
                            ws_bytes, static_cast<hipStream_t>(stream));
}

ms_status merge_runs(const void* keys_in, const uint32_t* vals_in, void* keys_out, uint32_t* vals_out,
                     const uint64_t* run_offsets, uint64_t num_runs, uint64_t n_total, ms_key_type kt, void* ws,
                     size_t ws_bytes, void* stream) {
  ms_status st =
      check_ranged("merge_runs", keys_in, vals_in, keys_out, vals_out, run_offsets, num_runs, n_total, kt);
  if (st != MS_OK) return st;
  if (num_runs == 0) return fail(MS_EINVAL, "merge_runs: num_runs must be at least 1");
  if (n_total == 0) return MS_OK;
  if (keys_in == keys_out || (vals_in && static_cast<const void*>(vals_in) == static_cast<const void*>(vals_out)))
    return fail(MS_EINVAL, "merge_runs: output must not alias the input");
  return ms::merge_sorted_runs(keys_in, vals_in, keys_out, vals_out, run_offsets, num_runs, n_total, kt, ws,
                               ws_bytes, static_cast<hipStream_t>(stream));
}

ms_status merge_split(const void* keys_in, const uint32_t* vals_in, void* keys_out, uint32_t* vals_out,
                      uint64_t n_total, uint64_t num_parts, ms_key_type kt, void* ws, size_t ws_bytes,
                      void* stream) {
  if (!ms::valid_kt(kt)) return fail(MS_ENOTSUP, "merge_split: unknown key type %d", static_cast<int>(kt));
  if ((vals_in == nullptr) != (vals_out == nullptr))
    return fail(MS_EINVAL, "merge_split: give both vals_in and vals_out, or neither");
  if (num_parts == 0) return fail(MS_EINVAL, "merge_split: num_parts must be at least 1");
  if (n_total % num_parts != 0)
    return fail(MS_EINVAL, "merge_split: %llu parts do not divide %llu keys into equal parts",
                static_cast<unsigned long long>(num_parts), static_cast<unsigned long long>(n_total));
  if (n_total == 0) return MS_OK;
  if (!keys_in || !keys_out)
    return fail(MS_EINVAL, "merge_split: NULL key pointer with n_total = %llu",
                static_cast<unsigned long long>(n_total));
  if (keys_in == keys_out || (vals_in && static_cast<const void*>(vals_in) == static_cast<const void*>(vals_out)))
    return fail(MS_EINVAL, "merge_split: output must not alias the input");
  return ms::merge_split_parts(keys_in, vals_in, keys_out, vals_out, n_total, num_parts, kt, ws, ws_bytes,
                               static_cast<hipStream_t>(stream));
}

ms_status ms_tune_set(ms_tune_param p, int64_t value) {
  switch (p) {
    case MS_TUNE_PASS_THREADS:
      if (value != 256 && value != 512 && value != 1024)
        return fail(MS_EINVAL, "MS_TUNE_PASS_THREADS must be 256, 512 or 1024 (got %lld)",
                    static_cast<long long>(value));
      ms::g_tune[p] = value;
      return MS_OK;
    case MS_TUNE_SEG_BLOCKS:
    case MS_TUNE_HIST_BLOCKS:
      if (value < 0 || value > 65536)
        return fail(MS_EINVAL, "tuning parameter %d must be in [0, 65536] (got %lld)", static_cast<int>(p),
                    static_cast<long long>(value));
      ms::g_tune[p] = value;
      return MS_OK;
    case MS_TUNE_SMALL_SORT:
      if (value != 0 && value != 64)
        return fail(MS_EINVAL, "MS_TUNE_SMALL_SORT must be 0 or 64 (got %lld)", static_cast<long long>(value));
      ms::g_tune[p] = value;
      return MS_OK;
    case MS_TUNE_SEG_PASSES:
      if (value < 0 || value > 2)
        return fail(MS_EINVAL, "MS_TUNE_SEG_PASSES must be 0, 1 or 2 (got %lld)", static_cast<long long>(value));
      ms::g_tune[p] = value;
      return MS_OK;
    case MS_TUNE_SEG_PASS_THREADS:
      if (value != 512 && value != 1024)
        return fail(MS_EINVAL, "MS_TUNE_SEG_PASS_THREADS must be 512 or 1024 (got %lld)",
                    static_cast<long long>(value));
      ms::g_tune[p] = value;
      return MS_OK;
    default:
      return fail(MS_EINVAL, "unknown tuning parameter %d", static_cast<int>(p));
  }
}

int64_t ms_tune_get(ms_tune_param p) { return ms::tune_get(p); }

ms_status ms_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(ms::g_timing_mu);
  ms::g_timing.enabled = on != 0;
  return MS_OK;
}

ms_status ms_timing_reset(void) {
  std::lock_guard<std::mutex> lk(ms::g_timing_mu);
  for (auto& p : ms::g_timing.pending) {
    (void)hipEventSynchronize(p.stop);
    (void)hipEventDestroy(p.start);
    (void)hipEventDestroy(p.stop);
  }
  ms::g_timing.pending.clear();
  ms::g_timing.totals.clear();
  return MS_OK;
}

int ms_timing_read(char* names_out, uint64_t* count_out, double* ms_out, int max_entries) {
  std::lock_guard<std::mutex> lk(ms::g_timing_mu);
  for (auto& p : ms::g_timing.pending) {
    float ms_elapsed = 0.f;
    if (hipEventSynchronize(p.stop) == hipSuccess && hipEventElapsedTime(&ms_elapsed, p.start, p.stop) == hipSuccess) {
      auto& t = ms::g_timing.totals[p.name];
      t.first += 1;
      t.second += ms_elapsed;
    }
    (void)hipEventDestroy(p.start);
    (void)hipEventDestroy(p.stop);
  }
  ms::g_timing.pending.clear();
  int i = 0;
  for (const auto& kv : ms::g_timing.totals) {
    if (i < max_entries) {
      if (names_out) {
        snprintf(names_out + 64 * i, 64, "%s", kv.first.c_str());
      }
      if (count_out) count_out[i] = kv.second.first;
      if (ms_out) ms_out[i] = kv.second.second;
    }
    ++i;
  }
  return i;
}

}  // extern "C"

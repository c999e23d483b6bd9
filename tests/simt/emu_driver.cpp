// emu_driver.cpp -- runs the library's C ABI on the CPU SIMT emulator (host
// buffers stand in for device memory) and compares every result with the
// CPU oracle.  Prints one line per case; exit status 1 on any mismatch.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

#include "mi355sort.h"

extern "C" {
int oracle_sort(int kt, const void* kin, const uint32_t* vin, void* kout, uint32_t* vout, uint64_t n);
int oracle_sort_segmented(int kt, const void* kin, const uint32_t* vin, void* kout, uint32_t* vout,
                          const uint64_t* off, uint64_t nseg);
int oracle_merge_runs(int kt, const void* kin, const uint32_t* vin, void* kout, uint32_t* vout,
                      const uint64_t* off, uint64_t nruns);
int oracle_merge_split(int kt, const void* kin, const uint32_t* vin, void* kout, uint32_t* vout, uint64_t n,
                       uint64_t p);
}

static uint64_t g_state = 0x9e3779b97f4a7c15ull;
static uint64_t rnd() {  // splitmix64: input generation only
  uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

static int failures = 0;

static void fill(std::vector<uint64_t>& bits, int kt, size_t n, const std::string& dist) {
  bits.resize(n);
  for (size_t i = 0; i < n; ++i) {
    uint64_t r = rnd();
    if (dist == "small") r %= 1024;
    else if (dist == "equal") r = 12345;
    else if (dist == "few") r = (r % 4) * 0x9e3779b97f4a7c15ull;
    else if (dist == "sorted") r = i * 7919;
    else if (dist == "low12") r &= 0xfff;
    if (kt != MS_KEY_U64) r &= 0xffffffffull;
    bits[i] = r;
  }
}

template <typename K>
static std::vector<K> narrow(const std::vector<uint64_t>& b) {
  std::vector<K> out(b.size());
  for (size_t i = 0; i < b.size(); ++i) out[i] = static_cast<K>(b[i]);
  return out;
}

template <typename K>
static void run_sort(int kt, size_t n, const std::string& dist, bool pairs, bool inplace, int threads) {
  std::vector<uint64_t> bits;
  fill(bits, kt, n, dist);
  std::vector<K> kin = narrow<K>(bits), kout(n), kexp(n);
  std::vector<uint32_t> vin(n), vout(n), vexp(n);
  for (size_t i = 0; i < n; ++i) vin[i] = static_cast<uint32_t>(i);
  ms_tune_set(MS_TUNE_PASS_THREADS, threads);
  size_t wsb = 0;
  ms_workspace_size(pairs ? MS_OP_SORT_PAIRS : MS_OP_SORT_KEYS, (ms_key_type)kt, pairs, n, 0, &wsb);
  std::vector<char> ws(wsb + 1);
  oracle_sort(kt, kin.data(), pairs ? vin.data() : nullptr, kexp.data(), pairs ? vexp.data() : nullptr, n);
  K* ko = inplace ? kin.data() : kout.data();
  uint32_t* vo = inplace ? vin.data() : vout.data();
  ms_status st = pairs ? sort_pairs(kin.data(), vin.data(), ko, vo, n, (ms_key_type)kt, ws.data(), wsb, nullptr)
                       : sort_keys(kin.data(), ko, n, (ms_key_type)kt, ws.data(), wsb, nullptr);
  bool ok = st == MS_OK && memcmp(ko, kexp.data(), n * sizeof(K)) == 0 &&
            (!pairs || memcmp(vo, vexp.data(), n * 4) == 0);
  printf("%s %s kt=%d n=%zu dist=%s pairs=%d inplace=%d threads=%d\n", ok ? "ok  " : "FAIL",
         pairs ? "sort_pairs" : "sort_keys", kt, n, dist.c_str(), pairs, inplace, threads);
  fflush(stdout);
  if (!ok) ++failures;
}

template <typename K>
static void run_segmented(int kt, const std::vector<uint64_t>& lengths, bool pairs, const char* dist = "few") {
  std::vector<uint64_t> off(lengths.size() + 1, 0);
  for (size_t s = 0; s < lengths.size(); ++s) off[s + 1] = off[s] + lengths[s];
  const size_t n = off.back();
  std::vector<uint64_t> bits;
  fill(bits, kt, n, dist);
  std::vector<K> kin = narrow<K>(bits), kout(n), kexp(n);
  std::vector<uint32_t> vin(n), vout(n), vexp(n);
  for (size_t i = 0; i < n; ++i) vin[i] = static_cast<uint32_t>(i);
  size_t wsb = 0;
  ms_workspace_size(MS_OP_SORT_SEGMENTED, (ms_key_type)kt, pairs, n, lengths.size(), &wsb);
  std::vector<char> ws(wsb + 1);
  oracle_sort_segmented(kt, kin.data(), pairs ? vin.data() : nullptr, kexp.data(), pairs ? vexp.data() : nullptr,
                        off.data(), lengths.size());
  ms_status st = sort_segmented(kin.data(), pairs ? vin.data() : nullptr, kout.data(), pairs ? vout.data() : nullptr,
                                off.data(), lengths.size(), n, (ms_key_type)kt, ws.data(), wsb, nullptr);
  bool ok = st == MS_OK && memcmp(kout.data(), kexp.data(), n * sizeof(K)) == 0 &&
            (!pairs || memcmp(vout.data(), vexp.data(), n * 4) == 0);
  printf("%s sort_segmented kt=%d nseg=%zu n=%zu pairs=%d dist=%s\n", ok ? "ok  " : "FAIL", kt, lengths.size(), n, pairs,
         dist);
  if (!ok && st == MS_OK) {
    size_t bad = 0;
    while (bad < n && kout[bad] == kexp[bad] && (!pairs || vout[bad] == vexp[bad])) ++bad;
    size_t seg = 0;
    while (seg + 1 < off.size() && off[seg + 1] <= bad) ++seg;
    size_t nbad = 0;
    for (size_t i = 0; i < n; ++i) nbad += kout[i] != kexp[i];
    printf("     first difference at %zu (segment %zu, offset %zu): got %llu expected %llu; %zu keys differ\n", bad,
           seg, bad - off[seg], (unsigned long long)kout[bad], (unsigned long long)kexp[bad], nbad);
    if (getenv("DBGQ"))
      for (size_t sg = 0; sg + 1 < off.size(); ++sg) {
        size_t c = 0;
        for (size_t i = off[sg]; i < off[sg + 1]; ++i) c += kout[i] != kexp[i];
        printf("     segment %zu [%llu, %llu): %zu differ\n", sg, (unsigned long long)off[sg],
               (unsigned long long)off[sg + 1], c);
      }
  }
  fflush(stdout);
  if (!ok) ++failures;
}

// Offsets that break the contract (decreasing pairs, overlapping segments,
// entries beyond n): the order is unspecified, but the call must succeed and
// every access stay inside the buffers (buffers and workspace are sized
// exactly, so AddressSanitizer sees any access past them).
template <typename K>
static void run_malformed(int kt, const std::vector<uint64_t>& off, size_t n, bool pairs, int seg_passes) {
  std::vector<uint64_t> bits;
  fill(bits, kt, n, "uniform");
  std::vector<K> kin = narrow<K>(bits), kout(n);
  std::vector<uint32_t> vin(n), vout(n);
  for (size_t i = 0; i < n; ++i) vin[i] = static_cast<uint32_t>(i);
  const uint64_t nseg = off.size() - 1;
  size_t wsb = 0;
  ms_workspace_size(MS_OP_SORT_SEGMENTED, (ms_key_type)kt, pairs, n, nseg, &wsb);
  std::vector<char> ws(wsb);
  ms_tune_set(MS_TUNE_SEG_PASSES, seg_passes);
  ms_status st = sort_segmented(kin.data(), pairs ? vin.data() : nullptr, kout.data(), pairs ? vout.data() : nullptr,
                                off.data(), nseg, n, (ms_key_type)kt, ws.data(), wsb, nullptr);
  ms_tune_set(MS_TUNE_SEG_PASSES, 1);
  const bool ok = st == MS_OK;
  printf("%s sort_segmented malformed offsets kt=%d nseg=%llu n=%zu pairs=%d seg_passes=%d\n", ok ? "ok  " : "FAIL",
         kt, static_cast<unsigned long long>(nseg), n, pairs, seg_passes);
  fflush(stdout);
  if (!ok) ++failures;
}

template <typename K>
static void run_merge_split(int kt, size_t n, uint64_t p, bool pairs, const char* dist) {
  std::vector<uint64_t> bits;
  fill(bits, kt, n, dist);
  std::vector<K> raw = narrow<K>(bits), kin(n), kout(n), kexp(n);
  std::vector<uint32_t> vraw(n), vin(n), vout(n), vexp(n);
  for (size_t i = 0; i < n; ++i) vraw[i] = static_cast<uint32_t>(i);
  std::vector<uint64_t> off(p + 1);
  for (uint64_t i = 0; i <= p; ++i) off[i] = i * (n / p);
  oracle_sort_segmented(kt, raw.data(), vraw.data(), kin.data(), vin.data(), off.data(), p);  // sorted parts
  oracle_merge_split(kt, raw.data(), pairs ? vraw.data() : nullptr, kexp.data(), pairs ? vexp.data() : nullptr, n, p);
  size_t wsb = 0;
  ms_workspace_size(MS_OP_MERGE_SPLIT, (ms_key_type)kt, pairs, n, p, &wsb);
  std::vector<char> ws(wsb + 1);
  ms_status st = merge_split(kin.data(), pairs ? vin.data() : nullptr, kout.data(), pairs ? vout.data() : nullptr, n, p,
                             (ms_key_type)kt, ws.data(), wsb, nullptr);
  bool ok = st == MS_OK && memcmp(kout.data(), kexp.data(), n * sizeof(K)) == 0 &&
            (!pairs || memcmp(vout.data(), vexp.data(), n * 4) == 0);
  printf("%s merge_split kt=%d n=%zu p=%llu pairs=%d dist=%s\n", ok ? "ok  " : "FAIL", kt, n,
         static_cast<unsigned long long>(p), pairs, dist);
  fflush(stdout);
  if (!ok) ++failures;
}

template <typename K>
static void run_merge(int kt, const std::vector<uint64_t>& lengths) {
  std::vector<uint64_t> off(lengths.size() + 1, 0);
  for (size_t s = 0; s < lengths.size(); ++s) off[s + 1] = off[s] + lengths[s];
  const size_t n = off.back();
  std::vector<uint64_t> bits;
  fill(bits, kt, n, "small");
  std::vector<K> raw = narrow<K>(bits), kin(n), kout(n), kexp(n);
  std::vector<uint32_t> vraw(n), vin(n), vout(n), vexp(n);
  for (size_t i = 0; i < n; ++i) vraw[i] = static_cast<uint32_t>(i);
  oracle_sort_segmented(kt, raw.data(), vraw.data(), kin.data(), vin.data(), off.data(), lengths.size());
  size_t wsb = 0;
  ms_workspace_size(MS_OP_MERGE_RUNS, (ms_key_type)kt, 1, n, lengths.size(), &wsb);
  std::vector<char> ws(wsb + 1);
  oracle_merge_runs(kt, kin.data(), vin.data(), kexp.data(), vexp.data(), off.data(), lengths.size());
  ms_status st = merge_runs(kin.data(), vin.data(), kout.data(), vout.data(), off.data(), lengths.size(), n,
                            (ms_key_type)kt, ws.data(), wsb, nullptr);
  bool ok = st == MS_OK && memcmp(kout.data(), kexp.data(), n * sizeof(K)) == 0 &&
            memcmp(vout.data(), vexp.data(), n * 4) == 0;
  printf("%s merge_runs kt=%d nruns=%zu n=%zu\n", ok ? "ok  " : "FAIL", kt, lengths.size(), n);
  fflush(stdout);
  if (!ok) ++failures;
}

// Continuous batching: requests of the given lengths join the step loop at
// the given steps (arrival step per request) and every step advances each
// active request by one phase (sort_step); each result against the oracle.
template <typename K>
static void run_steps(int kt, const std::vector<uint64_t>& lengths, const std::vector<int>& arrive, bool pairs,
                      const char* dist) {
  const size_t m = lengths.size();
  std::vector<std::vector<K>> kin(m), kout(m), kexp(m);
  std::vector<std::vector<uint32_t>> vin(m), vout(m), vexp(m);
  std::vector<std::vector<char>> work(m);
  std::vector<uint32_t> phases(m), phase(m, 0);
  for (size_t i = 0; i < m; ++i) {
    std::vector<uint64_t> bits;
    fill(bits, kt, lengths[i], dist);
    kin[i] = narrow<K>(bits);
    kout[i].assign(lengths[i], K(0));
    kexp[i].assign(lengths[i], K(0));
    vin[i].resize(lengths[i]);
    for (size_t j = 0; j < lengths[i]; ++j) vin[i][j] = static_cast<uint32_t>(j * 3 + i);
    vout[i].assign(lengths[i], 0);
    vexp[i].assign(lengths[i], 0);
    oracle_sort(kt, kin[i].data(), pairs ? vin[i].data() : nullptr, kexp[i].data(), pairs ? vexp[i].data() : nullptr,
                lengths[i]);
    size_t wb = 0;
    if (ms_step_plan((ms_key_type)kt, pairs, lengths[i], &phases[i], &wb) != MS_OK) {
      printf("FAIL ms_step_plan: %s\n", ms_last_error());
      ++failures;
      return;
    }
    work[i].assign(wb + 1, char(0x5a));  // garbage: the histogram phase must clear what it uses
  }
  size_t wsb = 0;
  ms_workspace_size(MS_OP_SORT_STEP, (ms_key_type)kt, pairs, 0, MS_STEP_MAX_REQUESTS, &wsb);
  std::vector<char> ws(wsb, char(0x33));
  bool ok = true;
  int steps = 0;
  for (int step = 0; step < 1000; ++step) {
    std::vector<ms_step_request> table;
    for (size_t i = 0; i < m; ++i) {
      if (arrive[i] > step || phase[i] >= phases[i]) continue;
      ms_step_request r = {};
      r.keys_in = kin[i].data();
      r.vals_in = pairs ? vin[i].data() : nullptr;
      r.keys_out = kout[i].data();
      r.vals_out = pairs ? vout[i].data() : nullptr;
      r.work = work[i].data();
      r.n = lengths[i];
      r.phase = phase[i]++;
      table.push_back(r);
    }
    bool pending = false;
    for (size_t i = 0; i < m; ++i) pending |= phase[i] < phases[i];
    if (table.empty() && !pending) break;
    if (table.empty()) continue;
    ++steps;
    ms_status st = sort_step(table.data(), table.size(), (ms_key_type)kt, pairs, ws.data(), ws.size(), nullptr);
    if (st != MS_OK) {
      printf("FAIL sort_step: %s\n", ms_last_error());
      ok = false;
      break;
    }
  }
  for (size_t i = 0; i < m && ok; ++i) {
    const bool good = lengths[i] == 0 ||
                      (memcmp(kout[i].data(), kexp[i].data(), lengths[i] * sizeof(K)) == 0 &&
                       (!pairs || memcmp(vout[i].data(), vexp[i].data(), lengths[i] * 4) == 0));
    if (!good) {
      printf("     request %zu (n=%llu) differs from the oracle\n", i, (unsigned long long)lengths[i]);
      ok = false;
    }
  }
  printf("%s sort_step kt=%d requests=%zu steps=%d pairs=%d dist=%s\n", ok ? "ok  " : "FAIL", kt, m, steps, pairs,
         dist);
  fflush(stdout);
  if (!ok) ++failures;
}

int main(int argc, char** argv) {
  const std::string what = argc > 1 ? argv[1] : "all";
  if (what == "quick") {  // a few cases per kernel family, for the CPU test suite
    run_sort<uint32_t>(MS_KEY_I32, 20001, "uniform", false, false, 256);
    run_sort<uint32_t>(MS_KEY_I32, 12000, "sorted", false, true, 512);
    run_sort<uint64_t>(MS_KEY_U64, 9000, "few", true, false, 256);
    run_sort<uint32_t>(MS_KEY_I32, 300, "uniform", true, false, 256);
    // 1,024-thread tiles: look-back agent, persistent workgroups over several tiles each
    run_sort<uint32_t>(MS_KEY_I32, 120000, "uniform", false, false, 1024);
    run_sort<uint32_t>(MS_KEY_U32, 70001, "small", false, true, 1024);
    run_segmented<uint32_t>(MS_KEY_I32, {0, 5, 9000, 1, 300, 1000, 64, 2, 900, 17, 18, 19, 20}, true);
    // segments of at most 64 keys: bitonic network (default) and radix passes
    run_segmented<uint64_t>(MS_KEY_U64, {64, 63, 1, 2, 3, 33, 65, 0, 16, 48}, true, "few");
    ms_tune_set(MS_TUNE_SMALL_SORT, 0);
    run_segmented<uint32_t>(MS_KEY_U32, {64, 63, 1, 2, 3, 33, 65, 0, 16, 48}, true, "few");
    ms_tune_set(MS_TUNE_SMALL_SORT, 64);
    // A few long segments: whole-device digit passes (empty, one-key and
    // partial-tile segments among them)
    run_segmented<uint32_t>(MS_KEY_I32, {40000, 0, 20000, 1, 50000}, false, "uniform");
    run_segmented<uint64_t>(MS_KEY_U64, {70000, 30001}, true, "few");
    // one-tile segments (stored in place, no histogram) among multi-tile ones
    run_segmented<uint32_t>(MS_KEY_I32, {8192, 1, 0, 30000, 5, 8193, 100, 16385, 7, 40000}, true, "uniform");
    // 16,384-key tiles (32-bit keys without values)
    ms_tune_set(MS_TUNE_SEG_PASS_THREADS, 1024);
    run_segmented<uint32_t>(MS_KEY_I32, {8192, 1, 0, 30000, 5, 16384, 100, 16385, 7, 40000}, false, "uniform");
    ms_tune_set(MS_TUNE_SEG_PASS_THREADS, 512);
    run_merge<uint32_t>(MS_KEY_U32, {3000, 0, 2500, 1});
    run_merge<uint32_t>(MS_KEY_I32, {20000, 30000, 5, 70000});
    run_merge_split<uint32_t>(MS_KEY_I32, 5 * 4001, 5, true, "few");
    // overlapping segments whose tiles exceed the tile table: both paths
    run_malformed<uint32_t>(MS_KEY_I32, {0, 30000, 10000, 50000, 20000, 60000}, 60000, true, 1);
    run_malformed<uint32_t>(MS_KEY_U32, {0, 15000, 5000, 12000, 3000, 20000}, 20000, false, 1);
    // the segment passes as one persistent launch (work queue of phases)
    ms_tune_set(MS_TUNE_SEG_PASSES, 2);
    run_segmented<uint32_t>(MS_KEY_I32, {8192, 1, 0, 30000, 5, 8193, 100, 16385, 7, 40000}, true, "uniform");
    run_segmented<uint64_t>(MS_KEY_U64, {3, 8192, 20000, 4097, 0, 1, 16384, 9000, 2, 30000}, false, "few");
    ms_tune_set(MS_TUNE_SEG_PASSES, 1);
    // continuous batching: one-tile and multi-tile requests joining at different steps
    run_steps<uint32_t>(MS_KEY_U32, {20000, 5, 8192, 8193, 1, 30001, 700, 16384}, {0, 0, 1, 1, 2, 2, 5, 7}, true,
                        "uniform");
    run_steps<uint32_t>(MS_KEY_I32, {9000, 3, 25000}, {0, 3, 4}, false, "few");
  }
  if (what == "segqueue") {
    ms_tune_set(MS_TUNE_SEG_PASSES, 2);
    run_segmented<uint32_t>(MS_KEY_I32, {40000, 0, 20000, 1, 50000}, false, "uniform");
    run_segmented<uint32_t>(MS_KEY_U32, {16384, 16383, 16385, 8191, 8193}, true, "small");
    run_segmented<uint64_t>(MS_KEY_U64, {70000, 30001}, true, "few");
    run_segmented<uint32_t>(MS_KEY_I32, {100000}, true, "sorted");
    run_segmented<uint32_t>(MS_KEY_I32, {8192, 1, 0, 30000, 5, 8193, 100, 16385, 7, 40000}, true, "uniform");
    run_segmented<uint64_t>(MS_KEY_U64, {3, 8192, 20000, 8191, 0, 1, 16384, 9000, 2, 30000}, false, "few");
    run_segmented<uint32_t>(MS_KEY_I32, {9000, 16383, 12000, 10000, 15000, 9500, 16000, 11000}, true, "uniform");
    run_segmented<uint32_t>(MS_KEY_U32, {18599, 3000, 1200, 40000}, true, "low12");
    // segments averaging 1,024 - 8,192 keys: mostly one-tile segments sorted whole in phase 0
    run_segmented<uint32_t>(MS_KEY_I32, {3000, 1, 0, 2500, 8192, 700, 8193, 4000, 1500, 2048}, false, "uniform");
    run_segmented<uint64_t>(MS_KEY_U64, {2000, 3000, 0, 9000, 1200}, true, "few");
    run_malformed<uint32_t>(MS_KEY_I32, {0, 30000, 10000, 50000, 20000, 60000}, 60000, true, 2);
    run_malformed<uint32_t>(MS_KEY_U32, {0, 15000, 5000, 12000, 3000, 20000}, 20000, false, 2);
    ms_tune_set(MS_TUNE_SEG_PASSES, 1);
  }
  if (what == "step") {
    run_steps<uint32_t>(MS_KEY_U32, {20000, 5, 8192, 8193, 1, 30001, 700, 16384}, {0, 0, 1, 1, 2, 2, 5, 7}, true,
                        "uniform");
    run_steps<uint32_t>(MS_KEY_I32, {9000, 3, 25000, 0, 40000}, {0, 3, 4, 4, 9}, false, "few");
    run_steps<uint32_t>(MS_KEY_U32, {18599, 12000, 9000}, {0, 0, 0}, true, "low12");
    run_steps<uint64_t>(MS_KEY_U64, {4096, 4097, 8192, 20001, 3}, {0, 1, 2, 3, 3}, true, "uniform");
    run_steps<uint64_t>(MS_KEY_U64, {9000, 17000}, {0, 2}, false, "small");
  }
  if (what == "manyseg") {  // hundreds of short segments (with lowered thresholds: several planning chunks)
    std::vector<uint64_t> lens;
    for (int i = 0; i < 700; ++i) lens.push_back(rnd() % 300);
    lens[5] = 0;
    lens[699] = 0;
    run_segmented<uint32_t>(MS_KEY_I32, lens, true, "uniform");
    lens.resize(300);
    run_segmented<uint64_t>(MS_KEY_U64, lens, false, "few");
    run_malformed<uint32_t>(MS_KEY_U32, {0, 9000, 0, 9000, 0, 9000, 0, 9000, 3000, 9000}, 9000, false, 1);
  }
  if (what == "malformed") {
    for (int sp : {1, 0}) {
      run_malformed<uint32_t>(MS_KEY_I32, {0, 30000, 10000, 50000, 20000, 60000}, 60000, true, sp);
      run_malformed<uint32_t>(MS_KEY_I32, {0, 30000, 10000, 50000, 20000, 60000}, 60000, false, sp);
      run_malformed<uint64_t>(MS_KEY_U64, {0, 70000, 20000, 60000}, 60000, true, sp);
      run_malformed<uint32_t>(MS_KEY_U32, {0, 15000, 5000, 12000, 3000, 20000}, 20000, false, sp);
      run_malformed<uint32_t>(MS_KEY_U32, {0, 40000, 40000, 100, 100, 50000}, 50000, true, sp);
    }
  }
  if (what == "all" || what == "sort") {
    for (int threads : {256, 512, 1024}) {
      run_sort<uint32_t>(MS_KEY_I32, 40000, "uniform", false, false, threads);
      run_sort<uint32_t>(MS_KEY_U32, 20001, "small", false, false, threads);
      run_sort<uint32_t>(MS_KEY_I32, 20001, "sorted", false, false, threads);
    }
    run_sort<uint32_t>(MS_KEY_I32, 9000, "equal", false, false, 256);
    run_sort<uint32_t>(MS_KEY_I32, 9000, "uniform", false, true, 256);
    run_sort<uint32_t>(MS_KEY_U32, 12345, "few", true, false, 256);
    run_sort<uint32_t>(MS_KEY_U32, 12345, "uniform", true, true, 512);
    run_sort<uint64_t>(MS_KEY_U64, 10000, "uniform", false, false, 256);
    run_sort<uint64_t>(MS_KEY_U64, 10000, "few", true, false, 512);
    run_sort<uint32_t>(MS_KEY_I32, 100, "uniform", false, false, 256);
  }
  if (what == "quick" || what == "lds") {
    // one-workgroup in-LDS sorts: only the rounds of 64 keys per wave the
    // list needs (one round, a partial last round, every round)
    for (size_t n : {1, 2, 65, 511, 513, 1000, 4097, 8191})
      run_sort<uint32_t>(n % 2 ? MS_KEY_I32 : MS_KEY_U32, n, n % 3 ? "uniform" : "few", n % 4 == 1, false, 512);
    run_sort<uint64_t>(MS_KEY_U64, 2049, "few", true, false, 512);
    run_sort<uint64_t>(MS_KEY_U64, 4096, "uniform", false, true, 512);
  }
  if (what == "low12") {
    run_segmented<uint32_t>(MS_KEY_U32, {18599, 3000, 1200, 40000}, true, "low12");
    run_sort<uint32_t>(MS_KEY_U32, 18599, "low12", true, false, 1024);
  }
  if (what == "segsweep") {
    run_segmented<uint32_t>(MS_KEY_I32, {40000, 0, 20000, 1, 50000}, false, "uniform");
    run_segmented<uint32_t>(MS_KEY_U32, {16384, 16383, 16385, 8191, 8193}, true, "small");
    run_segmented<uint64_t>(MS_KEY_U64, {70000, 30001}, true, "few");
    run_segmented<uint32_t>(MS_KEY_I32, {100000}, true, "sorted");
    run_segmented<uint32_t>(MS_KEY_I32, {8192, 1, 0, 30000, 5, 8193, 100, 16385, 7, 40000}, true, "uniform");
    run_segmented<uint64_t>(MS_KEY_U64, {3, 8192, 20000, 8191, 0, 1, 16384, 9000, 2, 30000}, false, "few");
    run_segmented<uint32_t>(MS_KEY_I32, {9000, 16383, 12000, 10000, 15000, 9500, 16000, 11000}, true, "uniform");
    ms_tune_set(MS_TUNE_SEG_PASS_THREADS, 1024);
    run_segmented<uint32_t>(MS_KEY_U32, {16384, 16383, 16385, 8191, 8193, 40000}, false, "small");
    run_segmented<uint32_t>(MS_KEY_I32, {8192, 1, 0, 30000, 5, 16384, 100, 16385, 7, 40000}, false, "uniform");
    run_segmented<uint32_t>(MS_KEY_I32, {20000, 30000}, true, "uniform");  // pairs: 8,192-key tiles
    ms_tune_set(MS_TUNE_SEG_PASS_THREADS, 512);
  }
  if (what == "all" || what == "segmented" || what == "seg") {
    run_segmented<uint32_t>(MS_KEY_I32, {0, 5, 9000, 1, 0, 8192, 8193, 300}, false);
    run_segmented<uint32_t>(MS_KEY_I32, {20000, 17, 16, 4000, 0, 1}, true);
    run_segmented<uint32_t>(MS_KEY_I32, {5, 1023, 1024, 700, 64, 65, 1, 2, 1000, 900, 3, 800}, true);
    run_segmented<uint64_t>(MS_KEY_U64, {5, 1023, 1024, 700, 9000, 65, 1, 2, 1000, 900, 3, 800}, false);
    run_segmented<uint32_t>(MS_KEY_U32, {7000, 10000, 3}, true);
    run_segmented<uint64_t>(MS_KEY_U64, {5000, 4096, 4097, 0}, true);
  }
  if (what == "mergebig") {  // lists of 2^22 keys and more: the larger merge tiles (slow on the emulator)
    run_merge<uint32_t>(MS_KEY_I32, {1u << 21, (1u << 21) + 3, 77, 0, 5});
    run_merge_split<uint32_t>(MS_KEY_U32, 4 * ((1u << 20) + 1), 4, false, "few");
  }
  if (what == "all" || what == "merge") {
    run_merge<uint32_t>(MS_KEY_I32, {3000, 0, 2500, 4000, 1});
    run_merge<uint64_t>(MS_KEY_U64, {1000, 2000});
    // runs of several tiles: most tiles lie inside one pair
    run_merge<uint32_t>(MS_KEY_U32, {20000, 30000, 5, 70000});
    run_merge<uint64_t>(MS_KEY_U64, {9000, 9001, 4095});
    for (uint64_t p : {1, 2, 3, 4, 7})
      run_merge_split<uint32_t>(MS_KEY_U32, p * 3001, p, p % 2 == 1, "small");
    run_merge_split<uint64_t>(MS_KEY_U64, 4 * 5000, 4, true, "few");
  }
  printf("%d failure(s)\n", failures);
  return failures ? 1 : 0;
}

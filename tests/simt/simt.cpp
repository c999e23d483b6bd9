// simt.cpp -- cooperative-fiber SIMT emulator behind tests/simt/include/hip.
//
// Each thread of a block is a ucontext fiber.  The scheduler runs fibers
// round-robin until each blocks on a block barrier, a wave collective, a
// yield or its end; a barrier releases when every live thread of the block is
// waiting on it, a wave collective when every live lane of the wave is.
// kWorkers OS threads each run one block at a time, taking blockIdx values in
// order, so up to kWorkers blocks are in flight together.  A block whose
// threads can make no progress (a collective some lanes never reach, or a
// spin on data no running block will write) aborts with a message.
#include <sched.h>
#include <setjmp.h>
#include <stdio.h>
#include <stdlib.h>
#include <ucontext.h>

#include <atomic>
#include <thread>
#include <vector>

#include "hip/hip_runtime.h"

#if defined(__SANITIZE_ADDRESS__)
#define SIMT_ASAN 1
#elif defined(__has_feature)
#if __has_feature(address_sanitizer)
#define SIMT_ASAN 1
#endif
#endif
#ifdef SIMT_ASAN
#include <sanitizer/common_interface_defs.h>
#endif

namespace simt {
namespace {

enum State { kRunnable, kBarrier, kWave, kYield, kDone };
enum WaveOp { kNone, kBallot, kShfl, kSync };

constexpr size_t kStack = 512 * 1024;

struct Fiber {
  ucontext_t ctx;      // used once, to start the fiber on its own stack
  jmp_buf jb;          // every later switch: _setjmp/_longjmp (no signal-mask syscalls)
  bool started = false;
  Idx tid;
  uint32_t lane = 0, wave = 0;
  State st = kRunnable;
  char* stack = nullptr;
  int bval = 0;           // barrier_or input / result
  WaveOp op = kNone;
  uint64_t wval = 0;      // collective input / result
  int wsrc = 0;           // shfl source lane
};

struct Grid {
  std::vector<Fiber> f;
  ucontext_t sched;
  jmp_buf sched_jb;
  Idx bidx{0, 0, 0}, bdim{1, 1, 1}, gdim{1, 1, 1};
  const std::function<void()>* body = nullptr;
  int cur = -1;
#ifdef SIMT_ASAN
  void* fake_stack = nullptr;
  const void* sched_stack_bottom = nullptr;
  size_t sched_stack_size = 0;
#endif
};
thread_local Grid g;
int g_workers = 4;

void to_sched() {
  Fiber& me = g.f[g.cur];
#ifdef SIMT_ASAN
  void* fs = nullptr;
  __sanitizer_start_switch_fiber(&fs, g.sched_stack_bottom, g.sched_stack_size);
#endif
  if (!_setjmp(me.jb)) _longjmp(g.sched_jb, 1);
#ifdef SIMT_ASAN
  __sanitizer_finish_switch_fiber(fs, nullptr, nullptr);
#endif
}

void entry() {
#ifdef SIMT_ASAN
  __sanitizer_finish_switch_fiber(nullptr, &g.sched_stack_bottom, &g.sched_stack_size);
#endif
  (*g.body)();
  g.f[g.cur].st = kDone;
#ifdef SIMT_ASAN
  __sanitizer_start_switch_fiber(nullptr, g.sched_stack_bottom, g.sched_stack_size);
#endif
  _longjmp(g.sched_jb, 1);
}

void run_fiber(int i) {
  g.cur = i;
  Fiber& fb = g.f[i];
  fb.st = kRunnable;
#ifdef SIMT_ASAN
  void* fs = nullptr;
  __sanitizer_start_switch_fiber(&fs, fb.stack, kStack);
#endif
  if (!_setjmp(g.sched_jb)) {
    if (!fb.started) {
      fb.started = true;
      swapcontext(&g.sched, &fb.ctx);  // first entry; later returns come through sched_jb
    } else {
      _longjmp(fb.jb, 1);
    }
  }
#ifdef SIMT_ASAN
  __sanitizer_finish_switch_fiber(fs, &g.sched_stack_bottom, &g.sched_stack_size);
#endif
  g.cur = -1;
}

[[noreturn]] void die(const char* what) {
  fprintf(stderr, "simt: %s (block %u)\n", what, g.bidx.x);
  abort();
}

// Sweeps of a block whose every live thread only spins before the run is
// declared a livelock (SIMT_LIVELOCK_SWEEPS; blocks that wait on slow
// neighbours under AddressSanitizer may need more than the default).
long livelock_sweeps() {
  static const long v = [] {
    const char* e = getenv("SIMT_LIVELOCK_SWEEPS");
    const long x = e ? atol(e) : 0;
    return x > 0 ? x : 20000000L;
  }();
  return v;
}

void run_block() {
  const int n = static_cast<int>(g.f.size());
  const int nwaves = (n + 63) / 64;
  long idle_sweeps = 0;
  while (true) {
    bool progress = false, any_live = false, any_yield = false;
    for (int i = 0; i < n; ++i) {
      Fiber& fb = g.f[i];
      if (fb.st == kRunnable || fb.st == kYield) {
        const bool was_yield = fb.st == kYield;
        run_fiber(i);
        if (!(was_yield && g.f[i].st == kYield)) progress = true;
        if (g.f[i].st == kYield) any_yield = true;
      }
    }
    // wave collectives
    for (int w = 0; w < nwaves; ++w) {
      int live = 0, waiting = 0;
      WaveOp op = kNone;
      for (int i = w * 64; i < n && i < (w + 1) * 64; ++i) {
        if (g.f[i].st == kDone) continue;
        ++live;
        if (g.f[i].st == kWave) {
          if (op != kNone && g.f[i].op != op) die("lanes of one wave wait in different collectives");
          op = g.f[i].op;
          ++waiting;
        }
      }
      if (live == 0 || waiting != live) continue;
      uint64_t vals[64] = {0};
      bool alive[64] = {false};
      for (int i = w * 64; i < n && i < (w + 1) * 64; ++i)
        if (g.f[i].st == kWave) {
          vals[i - w * 64] = g.f[i].wval;
          alive[i - w * 64] = true;
        }
      uint64_t mask = 0;
      if (op == kBallot)
        for (int l = 0; l < 64; ++l)
          if (alive[l] && vals[l]) mask |= 1ull << l;
      for (int i = w * 64; i < n && i < (w + 1) * 64; ++i) {
        Fiber& fb = g.f[i];
        if (fb.st != kWave) continue;
        if (op == kBallot) {
          fb.wval = mask;
        } else if (op == kSync) {
          fb.wval = 0;
        } else {
          if (fb.wsrc < 0 || fb.wsrc >= 64) die("shfl source lane out of range");
          fb.wval = alive[fb.wsrc] ? vals[fb.wsrc] : 0;
        }
        fb.st = kRunnable;
        fb.op = kNone;
      }
      progress = true;
    }
    // block barrier
    int live = 0, at_bar = 0, orv = 0;
    for (auto& fb : g.f) {
      if (fb.st == kDone) continue;
      ++live;
      if (fb.st == kBarrier) {
        ++at_bar;
        orv |= fb.bval;
      }
    }
    if (live == 0) break;
    any_live = true;
    if (at_bar == live) {
      for (auto& fb : g.f)
        if (fb.st == kBarrier) {
          fb.bval = orv != 0;
          fb.st = kRunnable;
        }
      progress = true;
    }
    if (progress) {
      idle_sweeps = 0;
    } else if (any_live) {
      if (!any_yield) die("deadlock: threads wait on a barrier or collective others never reach");
      if (++idle_sweeps > livelock_sweeps()) die("livelock: threads spin on data no running block will write");
      if (idle_sweeps % 64 == 0) sched_yield();
    }
  }
}

}  // namespace

const Idx& thread_idx() { return g.f[g.cur].tid; }
const Idx& block_idx() { return g.bidx; }
const Idx& block_dim() { return g.bdim; }
const Idx& grid_dim() { return g.gdim; }
uint32_t lane() { return g.f[g.cur].lane; }

void barrier() {
  g.f[g.cur].st = kBarrier;
  g.f[g.cur].bval = 0;
  to_sched();
}

int barrier_or(int p) {
  g.f[g.cur].st = kBarrier;
  g.f[g.cur].bval = p != 0;
  to_sched();
  return g.f[g.cur].bval;
}

uint64_t ballot(bool p) {
  Fiber& me = g.f[g.cur];
  me.st = kWave;
  me.op = kBallot;
  me.wval = p ? 1 : 0;
  to_sched();
  return g.f[g.cur].wval;
}

uint64_t shfl_u64(uint64_t v, int src_lane) {
  Fiber& me = g.f[g.cur];
  me.st = kWave;
  me.op = kShfl;
  me.wval = v;
  me.wsrc = src_lane;
  to_sched();
  return g.f[g.cur].wval;
}

void wave_sync() {
  Fiber& me = g.f[g.cur];
  me.st = kWave;
  me.op = kSync;
  me.wval = 0;
  to_sched();
}

void yield() {
  if (g.cur < 0) return;
  g.f[g.cur].st = kYield;
  to_sched();
}

void launch(dim3 grid, dim3 block, const std::function<void()>& body) {
  if (grid.y != 1 || grid.z != 1 || block.y != 1 || block.z != 1) die("only 1-D launches are emulated");
  if (grid.x == 0) return;
  const char* env = getenv("SIMT_WORKERS");
  if (env) g_workers = atoi(env) > 0 ? atoi(env) : 1;
  std::atomic<unsigned> next{0};
  auto worker = [&]() {
    const unsigned nthreads = block.x;
    g.body = &body;
    g.bdim = Idx{block.x, 1, 1};
    g.gdim = Idx{grid.x, 1, 1};
    g.f.assign(nthreads, Fiber());
    for (unsigned t = 0; t < nthreads; ++t) g.f[t].stack = static_cast<char*>(malloc(kStack));
    while (true) {
      const unsigned b = next.fetch_add(1);
      if (b >= grid.x) break;
      g.bidx = Idx{b, 0, 0};
      for (unsigned t = 0; t < nthreads; ++t) {
        Fiber& fb = g.f[t];
        fb.tid = Idx{t, 0, 0};
        fb.lane = t % 64;
        fb.wave = t / 64;
        fb.st = kRunnable;
        fb.op = kNone;
        fb.started = false;
        getcontext(&fb.ctx);
        fb.ctx.uc_stack.ss_sp = fb.stack;
        fb.ctx.uc_stack.ss_size = kStack;
        fb.ctx.uc_link = &g.sched;
        makecontext(&fb.ctx, entry, 0);
      }
      run_block();
    }
    for (auto& fb : g.f) free(fb.stack);
    g.f.clear();
  };
  const int nw = static_cast<int>(grid.x) < g_workers ? static_cast<int>(grid.x) : g_workers;
  std::vector<std::thread> pool;
  for (int w = 0; w < nw; ++w) pool.emplace_back(worker);
  for (auto& t : pool) t.join();
}

}  // namespace simt

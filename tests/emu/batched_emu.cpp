// batched_emu.cpp -- CPU emulation of the batched inversion kernel, for tests.
//
// Runs the workgroup building blocks of paper_2208_01239_amd/csrc/batched_dev.hpp
// unchanged, with every GPU thread as a cooperative fiber.  The scheduler runs
// all fibers until each one blocks (workgroup barrier, wave-level exchange) or
// finishes, then releases what can be released, and checks on the way:
//   - a workgroup barrier is released only when every thread of the workgroup
//     waits at the same call site, having passed the same number of barriers;
//   - a wave exchange (lane shuffle, first-lane read, matrix-core product)
//     needs all 64 lanes of the wave;
//   - nothing is left waiting forever (deadlock), and the total number of
//     barriers stays under a limit (a loop that never advances).
// Any violation stops the run and is reported with the fiber, block and count.
//
// The matrix-core products are emulated from their operand layouts: lane l
// supplies A(l % 16, l / 16) and B(l / 16, l % 16) and holds four entries of
// column l % 16 of the 16 x 16 result (rows (l / 16) + 4 v in FP64,
// 4 (l / 16) + v in FP32).
#include <setjmp.h>
#include <ucontext.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <vector>

namespace frob {
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
}  // namespace frob

namespace emu {

enum State { RUN = 0, WGBAR = 1, WAVEBAR = 2, DONE = 3 };
enum Err { OK = 0, ERR_DIVERGENT_BARRIER = 1, ERR_DEADLOCK = 2, ERR_WATCHDOG = 3, ERR_EXITED_AT_BARRIER = 4,
           ERR_WAVE_DIVERGENCE = 5 };

struct Fiber {
  ucontext_t uc;
  jmp_buf jb;
  std::vector<char> stack;
  State st = RUN;
  bool started = false;
  int block = 0, tid = 0;
  long long bars = 0;       // workgroup barriers passed
  const void* site = nullptr;
};

struct Machine {
  std::vector<Fiber> f;
  int nt = 0, nblocks = 0;
  int cur = -1;
  jmp_buf sched;
  ucontext_t sched_uc;
  std::function<void(int block)> body;
  std::vector<uint64_t> xch;         // per-fiber exchange word
  std::vector<double> xa, xb;        // matrix-core operands
  long long total_bars = 0, limit = 0;
  int err = OK;
  char msg[256] = {0};
};

static Machine* M = nullptr;

static void fail(int code, const char* fmt, int a, int b, long long c) {
  if (M->err == OK) {
    M->err = code;
    std::snprintf(M->msg, sizeof(M->msg), fmt, a, b, c);
  }
}

// leave the current fiber for the scheduler
static void yield_to_sched() {
  Fiber& me = M->f[M->cur];
  if (!_setjmp(me.jb)) _longjmp(M->sched, 1);
}

static void fiber_entry() {
  Fiber& me = M->f[M->cur];
  M->body(me.block);
  M->f[M->cur].st = DONE;
  _longjmp(M->sched, 1);
}

// Run `body` on nblocks workgroups of nt threads.  Returns an Err code.
static int run(int nblocks, int nt, size_t stack_bytes, long long limit, std::function<void(int)> body,
               long long* bars_per_block) {
  Machine m;
  M = &m;
  m.nt = nt;
  m.nblocks = nblocks;
  m.limit = limit;
  m.body = std::move(body);
  const int total = nblocks * nt;
  m.f.resize(total);
  m.xch.assign(total, 0);
  m.xa.assign(total, 0.0);
  m.xb.assign(total, 0.0);
  for (int i = 0; i < total; ++i) {
    Fiber& fb = m.f[i];
    fb.block = i / nt;
    fb.tid = i % nt;
    fb.stack.resize(stack_bytes);
    getcontext(&fb.uc);
    fb.uc.uc_stack.ss_sp = fb.stack.data();
    fb.uc.uc_stack.ss_size = stack_bytes;
    fb.uc.uc_link = nullptr;
    makecontext(&fb.uc, (void (*)())fiber_entry, 0);
  }
  for (;;) {
    // run every runnable fiber until it blocks or finishes
    for (int i = 0; i < total && m.err == OK; ++i) {
      if (m.f[i].st != RUN) continue;
      m.cur = i;
      if (!_setjmp(m.sched)) {
        if (!m.f[i].started) {
          m.f[i].started = true;
          swapcontext(&m.sched_uc, &m.f[i].uc);
        } else {
          _longjmp(m.f[i].jb, 1);
        }
      }
    }
    if (m.err != OK) break;
    bool released = false, all_done = true;
    // wave exchanges: all 64 lanes present
    for (int w = 0; w < total / 64; ++w) {
      int waiting = 0, done = 0;
      for (int l = 0; l < 64; ++l) {
        const State s = m.f[w * 64 + l].st;
        waiting += s == WAVEBAR;
        done += s == DONE;
      }
      if (waiting == 64) {
        for (int l = 0; l < 64; ++l) m.f[w * 64 + l].st = RUN;
        released = true;
      } else if (waiting > 0) {
        fail(ERR_WAVE_DIVERGENCE, "wave %d: %d lanes at a lane exchange, the others elsewhere (%lld done)", w,
             waiting, (long long)done);
      }
    }
    if (m.err != OK) break;
    if (released) continue;
    // workgroup barriers
    for (int b = 0; b < nblocks && m.err == OK; ++b) {
      int at = 0, done = 0;
      const Fiber* first = nullptr;
      for (int t = 0; t < nt; ++t) {
        const Fiber& fb = m.f[b * nt + t];
        if (fb.st == WGBAR) {
          ++at;
          if (!first) first = &fb;
          else if (fb.site != first->site || fb.bars != first->bars)
            fail(ERR_DIVERGENT_BARRIER, "block %d thread %d waits at a different barrier (count %lld)", b, t,
                 fb.bars);
        }
        done += fb.st == DONE;
      }
      if (done < nt) all_done = false;
      if (at == nt) {
        for (int t = 0; t < nt; ++t) m.f[b * nt + t].st = RUN;
        released = true;
      } else if (at > 0 && at + done == nt) {
        fail(ERR_EXITED_AT_BARRIER, "block %d: %d threads wait at a barrier that %d exited threads never reach", b,
             at, (long long)done);
      }
    }
    if (m.err != OK) break;
    if (all_done) break;
    if (!released) {
      fail(ERR_DEADLOCK, "deadlock: no barrier can be released (%d blocks, %d threads)", nblocks, nt, 0);
      break;
    }
  }
  if (bars_per_block)
    for (int b = 0; b < nblocks; ++b) bars_per_block[b] = m.f[b * nt].bars;
  const int e = m.err;
  if (e != OK) std::fprintf(stderr, "emu: %s\n", m.msg);
  M = nullptr;
  return e;
}

static void wave_sync() {
  M->f[M->cur].st = WAVEBAR;
  yield_to_sched();
}

}  // namespace emu

// ------------------------------------------------- primitives of batched_dev.hpp
namespace frob {
namespace bat {
#define BB_FN __attribute__((noinline))
#define BB_IN inline
#define BB_GLOBAL
inline int bb_tid() { return emu::M->f[emu::M->cur].tid; }
__attribute__((noinline)) void bb_sync() {
  emu::Fiber& me = emu::M->f[emu::M->cur];
  me.site = __builtin_return_address(0);
  me.bars += 1;
  if (++emu::M->total_bars > emu::M->limit)
    emu::fail(emu::ERR_WATCHDOG, "watchdog: more than %d barriers (block %d, count %lld)", (int)emu::M->limit,
              me.block, me.bars);
  me.st = emu::WGBAR;
  emu::yield_to_sched();
}
template <class V>
inline V bb_shfl_xor(V v, int mask) {
  static_assert(sizeof(V) <= 8, "exchange word");
  const int g = emu::M->cur;
  uint64_t w = 0;
  std::memcpy(&w, &v, sizeof(V));
  emu::M->xch[g] = w;
  emu::wave_sync();
  const int src = (g & ~63) | ((g & 63) ^ mask);
  V r;
  std::memcpy(&r, &emu::M->xch[src], sizeof(V));
  emu::wave_sync();
  return r;
}
inline int bb_first(int v) {
  const int g = emu::M->cur;
  emu::M->xch[g] = (uint64_t)(uint32_t)v;
  emu::wave_sync();
  const int r = (int)(uint32_t)emu::M->xch[g & ~63];
  emu::wave_sync();
  return r;
}
template <class S, class V>
inline V mfma_emu(S a, S b, V c, bool f64) {
  const int g = emu::M->cur, base = g & ~63, l = g & 63;
  emu::M->xa[g] = a;
  emu::M->xb[g] = b;
  emu::wave_sync();
  V d;
  const int j = l & 15;
  for (int v = 0; v < 4; ++v) {
    const int r = f64 ? (l >> 4) + 4 * v : 4 * (l >> 4) + v;
    S acc = c[v];
    for (int k = 0; k < 4; ++k) acc += (S)emu::M->xa[base + 16 * k + r] * (S)emu::M->xb[base + 16 * k + j];
    d[v] = acc;
  }
  emu::wave_sync();
  return d;
}
inline d4 bb_mfma(double a, double b, d4 c) { return mfma_emu<double, d4>(a, b, c, true); }
inline f4 bb_mfma(float a, float b, f4 c) { return mfma_emu<float, f4>(a, b, c, false); }
inline int bb_atomic_add(int* p, int v) {
  const int old = *p;
  *p = old + v;
  return old;
}
}  // namespace bat
}  // namespace frob

#include "../../paper_2208_01239_amd/csrc/batched_dev.hpp"

using namespace frob::bat;

namespace {

template <typename T>
int run_batch(int count, int nmax, const int* n, const int* kind, void* const* A, void* const* B, void* const* Xr,
              void* const* Xi, int* info, int grid, const int* nb_table, long long limit, long long* bars) {
  std::vector<int> order(count), counter(1, 12345);
  // queue order and reset by the order kernel's body (one workgroup of 1024)
  std::vector<int> hist(BNMAX + 2);
  int e = emu::run(1, 1024, 32 << 10, limit,
                   [&](int) { batched_order_body(1024, count, n, order.data(), counter.data(), hist.data()); },
                   nullptr);
  if (e) return e;
  const long long slot = 3 * (long long)nmax * nmax + ((long long)nmax * (long long)sizeof(int) + sizeof(T) - 1) /
                                                        (long long)sizeof(T) + 64;
  std::vector<T> ws((size_t)slot * grid);
  BatchArgs g;
  g.count = count; g.n = n; g.kind = kind;
  g.A = A; g.B = B; g.Xr = Xr; g.Xi = Xi; g.info = info;
  g.nmax = nmax; g.order = order.data(); g.counter = counter.data();
  g.ws = ws.data(); g.slot_elems = slot;
  for (int k = 0; k < 2; ++k)
    for (int c = 0; c < 4; ++c) g.nb_table[k][c] = nb_table[4 * k + c];
  std::vector<Smem<T>> sm(grid);
  return emu::run(grid, BT, 256 << 10, limit, [&](int b) { batched_worker<T>(g, sm[b], b); }, bars);
}

}  // namespace

extern "C" {

// The persistent kernel on `grid` emulated workgroups (storage 0: FP64
// matrices, 1: FP32).  bars (may be null) receives the barrier count of each
// workgroup's thread 0.  Returns 0, or the emu::Err code of the violation.
int emu_batched_run(int storage, int count, int nmax, const int* n, const int* kind, void* const* A, void* const* B,
                    void* const* Xr, void* const* Xi, int* info, int grid, const int* nb_table, long long limit,
                    long long* bars) {
  if (storage == 1) return run_batch<float>(count, nmax, n, kind, A, B, Xr, Xi, info, grid, nb_table, limit, bars);
  return run_batch<double>(count, nmax, n, kind, A, B, Xr, Xi, info, grid, nb_table, limit, bars);
}

// The in-workgroup Cholesky alone with a given block width (FP64, one
// workgroup), for the behaviour of block widths outside the table's range.
// *ret receives the returned pivot status when the run completes.
int emu_potrf(int n, double* a, int nb, long long limit, int* ret) {
  Smem<double>* sm = new Smem<double>();
  int r = -1;
  const int e = emu::run(1, BT, 256 << 10, limit, [&](int) { const int v = wg_potrf<double>(*sm, n, a, n, nb);
                                                                if (bb_tid() == 0) r = v; }, nullptr);
  delete sm;
  if (ret) *ret = r;
  return e;
}

}  // extern "C"

extern "C" {

// Self-test of the checker on small bodies with known defects:
//   mode 0: uniform barriers (no error expected)
//   mode 1: thread 0 takes one extra barrier at another call site
//   mode 2: half of a wave reaches a lane exchange, the other half does not
//   mode 3: one wave leaves before the last barrier
int emu_selftest(int mode) {
  return emu::run(1, BT, 64 << 10, 10000, [mode](int) {
    const int t = bb_tid();
    bb_sync();
    if (mode == 1 && t == 0) bb_sync();
    if (mode == 2 && (t & 63) < 32) (void)bb_shfl_xor(t, 1);
    if (mode == 3 && t >= 192) return;
    bb_sync();
  }, nullptr);
}

}  // extern "C"

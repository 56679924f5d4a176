// Host emulation runtime for the CPU kernel test (see shim/hip/hip_runtime.h).
//
// Every workgroup runs as blockDim.x cooperative fibers (ucontext) on one OS
// thread.  A fiber runs until it reaches a synchronisation point:
//   * __syncthreads: released when every unfinished fiber of the workgroup
//     waits there;
//   * a wave-wide exchange (__shfl_xor, DPP, permlane swaps, readfirstlane):
//     each lane publishes its value, then the 64 fibers of the wave are
//     released together, read their partner's value, and meet once more so
//     that the exchange buffer can be reused.
// A state where no fiber can run before all have finished (a barrier some
// participant never reaches, a wave exchange inside divergent code) aborts
// with a message.  A fiber is entered once through makecontext/swapcontext;
// later switches use _setjmp/_longjmp, which do not save the signal mask (a
// system call per switch otherwise).  The fibers' stack switches are
// announced to AddressSanitizer.
#include <setjmp.h>
#include <ucontext.h>

#include <cstdarg>
#include <vector>

#include "hip/hip_runtime.h"

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#define EMU_ASAN 1
#endif
#endif
#ifdef EMU_ASAN
extern "C" {
void __sanitizer_start_switch_fiber(void** fake_stack_save, const void* bottom,
                                    size_t size);
void __sanitizer_finish_switch_fiber(void* fake_stack_save,
                                     const void** bottom_old, size_t* size_old);
}
#endif

EmuIdx threadIdx, blockIdx, blockDim, gridDim;

namespace {

constexpr size_t kStack = 64 * 1024;
enum State { kRun = 0, kBlockBar = 1, kWaveBar = 2, kDone = 3 };

struct Fiber {
  ucontext_t ctx;
  jmp_buf jb;
  int started;
  State st;
  char* stack;
};

ucontext_t g_sched;
jmp_buf g_sched_jb;
std::vector<Fiber> g_f;
const std::function<void()>* g_body = nullptr;
int g_cur = -1;
int g_nthreads = 0;
const void* g_sched_stack = nullptr;
size_t g_sched_size = 0;

// exchange buffers, one slot per thread of the workgroup
uint32_t g_x0[1024], g_x1[1024];
double g_xd[1024];

[[noreturn]] void fail(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::fprintf(stderr, "emu: ");
  std::vfprintf(stderr, fmt, ap);
  std::fprintf(stderr, "\n");
  va_end(ap);
  std::abort();
}

void to_scheduler() {
  Fiber& f = g_f[g_cur];
#ifdef EMU_ASAN
  void* fake = nullptr;
  __sanitizer_start_switch_fiber(&fake, g_sched_stack, g_sched_size);
#endif
  if (!_setjmp(f.jb)) _longjmp(g_sched_jb, 1);
#ifdef EMU_ASAN
  __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#endif
}

// A fiber is a worker that runs the kernel body once per workgroup: after
// each body it reports done and waits for the next workgroup, so the
// context is created once per fiber, not once per workgroup.
void entry() {
#ifdef EMU_ASAN
  __sanitizer_finish_switch_fiber(nullptr, &g_sched_stack, &g_sched_size);
#endif
  for (;;) {
    (*g_body)();
    g_f[g_cur].st = kDone;
    to_scheduler();
  }
}

void set_tid(int t) {
  threadIdx.x = (unsigned)t;
  threadIdx.y = threadIdx.z = 0;
}

void resume(int t) {
  g_cur = t;
  set_tid(t);
  Fiber& f = g_f[t];
  f.st = kRun;
#ifdef EMU_ASAN
  void* fake = nullptr;
  __sanitizer_start_switch_fiber(&fake, f.stack, kStack);
#endif
  if (!_setjmp(g_sched_jb)) {
    if (!f.started) {
      f.started = 1;
      swapcontext(&g_sched, &f.ctx);
    } else {
      _longjmp(f.jb, 1);
    }
  }
#ifdef EMU_ASAN
  __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#endif
  g_cur = -1;
}

void wait_state(State s) {
  g_f[g_cur].st = s;
  const int t = g_cur;
  to_scheduler();
  set_tid(t);
  g_cur = t;
}

// Runs one workgroup to completion.
void run_group() {
  const int n = g_nthreads;
  for (int t = 0; t < n; ++t) g_f[t].st = kRun;
  std::vector<char> runnable(n, 1);
  for (;;) {
    bool ran = false;
    for (int t = 0; t < n; ++t)
      if (runnable[t]) {
        runnable[t] = 0;
        resume(t);
        ran = true;
      }
    if (ran) continue;
    // everyone is waiting or done: release what can be released
    int done = 0, block = 0;
    for (int t = 0; t < n; ++t) {
      done += g_f[t].st == kDone;
      block += g_f[t].st == kBlockBar;
    }
    if (done == n) return;
    bool released = false;
    for (int w = 0; w * 64 < n; ++w) {
      int waiting = 0;
      for (int l = 0; l < 64 && w * 64 + l < n; ++l)
        waiting += g_f[w * 64 + l].st == kWaveBar;
      if (waiting == 0) continue;
      if (waiting != 64)
        fail("wave %d: %d of 64 lanes reached a wave exchange (block %u)", w,
             waiting, blockIdx.x);
      for (int l = 0; l < 64; ++l) runnable[w * 64 + l] = 1;
      released = true;
    }
    if (released) continue;
    if (block > 0 && block + done == n) {
      for (int t = 0; t < n; ++t)
        if (g_f[t].st == kBlockBar) runnable[t] = 1;
      continue;
    }
    fail("deadlock in block %u: %d done, %d at __syncthreads", blockIdx.x,
         done, block);
  }
}

int lane() { return (int)threadIdx.x & 63; }
int wave_base() { return (int)threadIdx.x & ~63; }

}  // namespace

void emu_launch(dim3 grid, dim3 block, const std::function<void()>& body) {
  if (block.y != 1 || block.z != 1 || block.x % 64 != 0 || block.x > 1024)
    fail("unsupported block shape %u x %u x %u", block.x, block.y, block.z);
  if (grid.y != 1 || grid.z != 1) fail("unsupported grid shape");
  if (g_cur >= 0) fail("kernel launch from device code");
  if (g_f.empty()) {
    g_f.resize(1024);
    for (size_t t = 0; t < g_f.size(); ++t) {
      Fiber& f = g_f[t];
      f.stack = (char*)std::malloc(kStack);
      getcontext(&f.ctx);
      f.ctx.uc_stack.ss_sp = f.stack;
      f.ctx.uc_stack.ss_size = kStack;
      f.ctx.uc_link = nullptr;
      makecontext(&f.ctx, entry, 0);
      f.started = 0;
      f.st = kDone;
    }
  }
  g_nthreads = (int)block.x;
  g_body = &body;
  blockDim.x = block.x;
  blockDim.y = blockDim.z = 1;
  gridDim.x = grid.x;
  gridDim.y = gridDim.z = 1;
  for (unsigned b = 0; b < grid.x; ++b) {
    blockIdx.x = b;
    blockIdx.y = blockIdx.z = 0;
    run_group();
  }
  g_body = nullptr;
}

void __syncthreads() {
  if (g_cur < 0) fail("__syncthreads outside a kernel");
  wait_state(kBlockBar);
}

static void wave_sync() {
  if (g_cur < 0) fail("wave exchange outside a kernel");
  wait_state(kWaveBar);
}

double __shfl_xor(double v, int mask, int width) {
  if (width != 64) fail("shuffle width %d", width);
  const int t = (int)threadIdx.x;
  g_xd[t] = v;
  wave_sync();
  const double r = g_xd[wave_base() + ((lane() ^ mask) & 63)];
  wave_sync();
  return r;
}

float __shfl_xor(float v, int mask, int width) {
  return (float)__shfl_xor((double)v, mask, width);
}

int __shfl_xor(int v, int mask, int width) {
  return (int)__shfl_xor((double)v, mask, width);
}

int emu_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask,
                   bool bound_ctrl) {
  (void)old;
  if (row_mask != 0xF || bank_mask != 0xF || !bound_ctrl)
    fail("unsupported DPP masks");
  const int t = (int)threadIdx.x, l = lane();
  g_x0[t] = (uint32_t)src;
  wave_sync();
  const int row = l & ~15, in = l & 15;
  int from;
  if (ctrl == 0x128) {  // row_ror:8
    from = row + ((in + 8) & 15);
  } else if (ctrl == 0x141) {  // row_half_mirror
    from = (l & ~7) + (7 - (l & 7));
  } else if (ctrl < 0x100) {  // quad_perm
    from = (l & ~3) + ((ctrl >> (2 * (l & 3))) & 3);
  } else {
    fail("unsupported DPP control 0x%x", ctrl);
  }
  const uint32_t r = g_x0[wave_base() + from];
  wave_sync();
  return (int)r;
}

// v_permlane32_swap: lanes 32..63 of the first operand trade places with
// lanes 0..31 of the second.
EmuPair emu_permlane32_swap(unsigned a, unsigned b, bool fi, bool bc) {
  (void)fi;
  (void)bc;
  const int t = (int)threadIdx.x, l = lane(), wb = wave_base();
  g_x0[t] = a;
  g_x1[t] = b;
  wave_sync();
  EmuPair r;
  if (l < 32) {
    r.v[0] = g_x0[wb + l];
    r.v[1] = g_x0[wb + l + 32];
  } else {
    r.v[0] = g_x1[wb + l - 32];
    r.v[1] = g_x1[wb + l];
  }
  wave_sync();
  return r;
}

// v_permlane16_swap: within each half of the wave, lanes 16..31 of the first
// operand trade places with lanes 0..15 of the second.
EmuPair emu_permlane16_swap(unsigned a, unsigned b, bool fi, bool bc) {
  (void)fi;
  (void)bc;
  const int t = (int)threadIdx.x, l = lane(), wb = wave_base();
  g_x0[t] = a;
  g_x1[t] = b;
  wave_sync();
  EmuPair r;
  if ((l & 16) == 0) {
    r.v[0] = g_x0[wb + l];
    r.v[1] = g_x0[wb + l + 16];
  } else {
    r.v[0] = g_x1[wb + l - 16];
    r.v[1] = g_x1[wb + l];
  }
  wave_sync();
  return r;
}

int emu_readfirstlane(int v) {
  const int t = (int)threadIdx.x;
  g_x0[t] = (uint32_t)v;
  wave_sync();
  const int r = (int)g_x0[wave_base()];
  wave_sync();
  return r;
}

// ------------------------------------------------------------ runtime --

hipError_t hipMalloc(void** p, size_t bytes) {
  *p = std::malloc(bytes ? bytes : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* p, int v, size_t bytes, hipStream_t) {
  std::memset(p, v, bytes);
  return hipSuccess;
}
hipError_t hipMemcpy(void* d, const void* s, size_t bytes, hipMemcpyKind) {
  std::memmove(d, s, bytes);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t bytes,
                          hipMemcpyKind k, hipStream_t) {
  return hipMemcpy(d, s, bytes, k);
}
hipError_t hipMemcpy2D(void* d, size_t dp, const void* s, size_t sp, size_t w,
                       size_t h, hipMemcpyKind) {
  for (size_t r = 0; r < h; ++r)
    std::memmove((char*)d + r * dp, (const char*)s + r * sp, w);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "emulated HIP error"; }
struct EmuEvent {
  int unused;
};
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new EmuEvent();
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.f;
  return hipSuccess;
}
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) {
  return hipErrorNotSupported;
}
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t*) {
  return hipErrorNotSupported;
}
hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, void*, char*,
                               size_t) {
  return hipErrorNotSupported;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }

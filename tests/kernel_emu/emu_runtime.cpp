// Fiber runtime of the host build of the library's kernels (hip/hip_runtime.h).
//
// Every lane of a workgroup is a fiber with its own stack; a fiber gives way
// only at __syncthreads and at wave-level operations, so a run is one valid,
// sequentially consistent schedule of the kernel.  What it checks:
//   * a barrier that some live lane never reaches (deadlock: reported with
//     the waiting lanes), lanes released by one barrier that arrived from
//     different source lines (counted);
//   * a wave-level operation reached by part of a wave only, or by lanes at
//     different source lines, a lane read that did not take part, an MFMA
//     without all 64 lanes;
//   * with -fsanitize=address (every device buffer is its own host
//     allocation): overflows of device buffers, of per-lane private arrays
//     and of the shared-memory objects; with -fsanitize=array-bounds also
//     indexes past one member array of the shared-memory struct into the next;
//   * with emu_race.cpp: races between waves and between workgroups.
// Freshly allocated device buffers can be filled with 0xFF bytes (NaN as
// doubles), so that a read of memory nobody wrote shows in the results.
#include "hip/hip_runtime.h"

#include <pthread.h>
#include <stdio.h>
#include <stdlib.h>
#include <sys/mman.h>
#include <time.h>

#include <vector>

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#define EMU_ASAN 1
#include <sanitizer/asan_interface.h>
#include <sanitizer/common_interface_defs.h>
#endif
#endif

#if !defined(__x86_64__) || !defined(__linux__)
#error "the fiber switch below is written for x86-64 Linux (System V calling convention)"
#endif

// Saves the callee-saved registers and the stack pointer of the running
// fiber in *save_sp and resumes the fiber whose stack pointer is new_sp.
extern "C" void emu_swap(void** save_sp, void* new_sp);
asm(R"(
.text
.globl emu_swap
.type emu_swap,@function
emu_swap:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
.size emu_swap, .-emu_swap
)");

#ifdef EMU_LDS_SECTION
extern "C" char __start_emu_lds[] __attribute__((weak));
extern "C" char __stop_emu_lds[] __attribute__((weak));
#endif

#ifdef EMU_RACE
extern "C" void emu_race_launch_end();
extern "C" void emu_race_register(void* p, size_t n);
extern "C" void emu_race_unregister(void* p);
extern "C" void emu_race_lds_setup();
#endif

namespace emu {

Lane* g_cur = nullptr;
dim3 g_block, g_bdim, g_gdim;
uint64_t g_epoch = 1;     // barrier intervals, unique over all workgroups
uint64_t g_launch = 0;
uint32_t g_group = 0;

namespace {

enum State { READY = 0, WAIT_BAR = 1, WAIT_WAVE = 2, DONE = 3 };

constexpr size_t kStack = 4u << 20;

struct Fiber {
  void* sp = nullptr;
  char* stack = nullptr;   // usable region [stack, stack + kStack)
  int state = DONE;
  unsigned wait_gen = 0;
  void* fake = nullptr;
  Lane lane;
};

enum Op { OP_NONE, OP_SHFL, OP_SHFL_XOR, OP_READLANE, OP_DPP, OP_MFMA };
const char* op_name(int k) {
  static const char* n[] = {"none", "shfl", "shfl_xor", "readlane", "dpp", "mfma"};
  return n[k];
}

struct Wave {
  int count = 0, nlive = 0, kind = OP_NONE;
  unsigned gen = 0;
  const char* file = nullptr;
  int line = 0;
  uint64_t arrived = 0, alive = 0;
  double in_d[64], in_b[64], out_d[64];
  int in_i[64], in_j[64], out_i[64];
  v4 in_c[64], out_c[64];
};

struct Group {
  int n = 0, nlive = 0;
  int bar_count = 0;
  unsigned bar_gen = 0;
  const char* bar_file = nullptr;
  int bar_line = 0;
  std::vector<Fiber> f;
  std::vector<Wave> w;
  int cur = -1;
  void* main_sp = nullptr;
  void* main_fake = nullptr;
  const void* main_bottom = nullptr;
  size_t main_size = 0;
  const std::function<void()>* body = nullptr;
};

Group G;
uint64_t n_launch = 0, n_groups = 0, n_bar = 0, n_wave = 0, n_mfma = 0;
uint64_t n_bar_mismatch = 0;
uint64_t clock_ticks = 0;
// per launch: workgroups, MFMA instructions (per wave), barriers
std::vector<uint64_t> launch_log;

[[noreturn]] void fail(const char* fmt, const char* file, int line, const char* extra = "") {
  fprintf(stderr, "EMU ERROR: ");
  fprintf(stderr, fmt, extra);
  fprintf(stderr, " at %s:%d (block %u, lane %u)\n", file ? file : "?", line, g_block.x,
          g_cur ? g_cur->tid.x : 0u);
  fflush(stderr);
  abort();
}

void start_switch(Fiber* from, const void* to_bottom, size_t to_size, bool dying) {
#ifdef EMU_ASAN
  __sanitizer_start_switch_fiber(dying ? nullptr : (from ? &from->fake : &G.main_fake), to_bottom,
                                 to_size);
#else
  (void)from; (void)to_bottom; (void)to_size; (void)dying;
#endif
}
void finish_switch(void* fake) {
#ifdef EMU_ASAN
  __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#else
  (void)fake;
#endif
}

// switch from fiber `from` (or main: -1) to fiber `to` (or main: -1)
void switch_to(int from, int to, bool dying) {
  Fiber* ff = from >= 0 ? &G.f[from] : nullptr;
  void** save = ff ? &ff->sp : &G.main_sp;
  void* dest;
  if (to >= 0) {
    Fiber& t = G.f[to];
    start_switch(ff, t.stack, kStack, dying);
    g_cur = &t.lane;
    G.cur = to;
    dest = t.sp;
  } else {
    start_switch(ff, G.main_bottom, G.main_size, dying);
    g_cur = nullptr;
    G.cur = -1;
    dest = G.main_sp;
  }
  emu_swap(save, dest);
  // resumed
  finish_switch(ff ? ff->fake : G.main_fake);
}

void dump_and_fail(const char* why) {
  fprintf(stderr, "EMU ERROR: %s in block %u; live lanes %d of %d\n", why, g_block.x, G.nlive, G.n);
  if (G.bar_count)
    fprintf(stderr, "  barrier: %d lanes waiting (first from %s:%d)\n", G.bar_count, G.bar_file,
            G.bar_line);
  for (size_t w = 0; w < G.w.size(); ++w) {
    const Wave& W = G.w[w];
    if (W.count)
      fprintf(stderr, "  wave %zu: %d of %d live lanes at %s (%s:%d)\n", w, W.count, W.nlive,
              op_name(W.kind), W.file, W.line);
  }
  fflush(stderr);
  abort();
}

// continue with the next ready fiber after the current one
void run_next(bool dying) {
  const int n = G.n, c = G.cur;
  for (int k = 1; k <= n; ++k) {
    const int j = (c + k) % n;
    if (G.f[j].state == READY) {
      if (j == c) return;
      switch_to(c, j, dying);
      return;
    }
  }
  if (G.nlive == 0) {
    switch_to(c, -1, dying);
    return;
  }
  dump_and_fail("deadlock (no lane can run)");
}

void release_barrier() {
  G.bar_gen++;
  g_epoch++;
  G.bar_count = 0;
  for (auto& f : G.f)
    if (f.state == WAIT_BAR) f.state = READY;
}

void complete_wave(int w);

void fiber_exit() {
  Fiber& me = G.f[G.cur];
  me.state = DONE;
  G.nlive--;
  const int w = me.lane.tid.x >> 6, l = me.lane.tid.x & 63;
  Wave& W = G.w[w];
  W.nlive--;
  W.alive &= ~(1ull << l);
  if (G.bar_count > 0 && G.bar_count == G.nlive) release_barrier();
  if (W.count > 0 && W.count == W.nlive) complete_wave(w);
  run_next(true);
  fprintf(stderr, "EMU internal: finished fiber resumed\n");
  abort();
}

void fiber_entry() {
#ifdef EMU_ASAN
  const void* ob;
  size_t os;
  __sanitizer_finish_switch_fiber(nullptr, &ob, &os);
  if (!G.main_bottom) {
    G.main_bottom = ob;
    G.main_size = os;
  }
#endif
  (*G.body)();
  fiber_exit();
}

void init_fiber(Fiber& f, unsigned tid) {
  if (!f.stack) {
    char* base = (char*)mmap(nullptr, kStack + 4096, PROT_READ | PROT_WRITE,
                             MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
    if (base == MAP_FAILED) {
      perror("mmap");
      abort();
    }
    mprotect(base, 4096, PROT_NONE);   // guard page below the stack
    f.stack = base + 4096;
  }
#ifdef EMU_ASAN
  __asan_unpoison_memory_region(f.stack, kStack);
#endif
  uintptr_t top = ((uintptr_t)(f.stack + kStack)) & ~(uintptr_t)15;
  void** sp = (void**)top;
  *--sp = nullptr;                      // alignment slot: rsp % 16 == 8 at entry
  *--sp = (void*)&fiber_entry;          // return address of emu_swap
  for (int r = 0; r < 6; ++r) *--sp = nullptr;   // rbp rbx r12 r13 r14 r15
  f.sp = sp;
  f.state = READY;
  f.wait_gen = 0;
  f.fake = nullptr;
  f.lane.tid = dim3(tid, 0, 0);
}

Wave& wave_enter(int kind, const char* file, int line, int& w, int& l) {
  w = g_cur->tid.x >> 6;
  l = g_cur->tid.x & 63;
  Wave& W = G.w[w];
  if (W.count == 0) {
    W.kind = kind;
    W.file = file;
    W.line = line;
    W.arrived = 0;
  } else if (W.kind != kind || W.line != line || strcmp(W.file, file) != 0) {
    fprintf(stderr, "EMU ERROR: wave %d: lanes at %s (%s:%d) and %s (%s:%d)\n", w,
            op_name(W.kind), W.file, W.line, op_name(kind), file, line);
    fail("divergent wave operation", file, line);
  }
  return W;
}

void wave_wait(Wave& W, int w, int l) {
  W.arrived |= 1ull << l;
  W.count++;
  n_wave++;
  if (W.count == W.nlive) {
    complete_wave(w);
  } else {
    Fiber& me = G.f[G.cur];
    me.state = WAIT_WAVE;
    me.wait_gen = W.gen;
    run_next(false);
  }
}

int dpp_src(int ctrl, int l) {
  const int row = l & ~15, r = l & 15;
  if (ctrl >= 0 && ctrl <= 0xFF) {
    const int q = r & 3;
    return row + (r & ~3) + ((ctrl >> (2 * q)) & 3);
  }
  if (ctrl == 0x140) return row + (15 - r);                 // row_mirror
  if (ctrl == 0x141) return row + (r & 8) + (7 - (r & 7));  // row_half_mirror
  return -1;
}

void complete_wave(int w) {
  Wave& W = G.w[w];
  const uint64_t arr = W.arrived;
  auto need = [&](int src, const char* what) {
    if (src < 0 || src > 63 || !((arr >> src) & 1)) {
      fprintf(stderr, "EMU ERROR: wave %d %s reads lane %d, which did not take part\n", w, what,
              src);
      fail("read of an inactive lane", W.file, W.line);
    }
  };
  switch (W.kind) {
    case OP_SHFL:
      for (int l = 0; l < 64; ++l)
        if ((arr >> l) & 1) {
          const int s = ((W.in_i[l] % 64) + 64) % 64;
          need(s, "shfl");
          W.out_d[l] = W.in_d[s];
        }
      break;
    case OP_SHFL_XOR:
      for (int l = 0; l < 64; ++l)
        if ((arr >> l) & 1) {
          const int s = l ^ W.in_i[l];
          need(s, "shfl_xor");
          W.out_d[l] = W.in_d[s];
        }
      break;
    case OP_READLANE: {
      int sel = -1;
      for (int l = 0; l < 64; ++l)
        if ((arr >> l) & 1) {
          if (sel < 0) sel = W.in_j[l];
          else if (W.in_j[l] != sel) fail("readlane with a lane index that is not uniform", W.file, W.line);
        }
      need(sel, "readlane");
      for (int l = 0; l < 64; ++l) W.out_i[l] = W.in_i[sel];
      break;
    }
    case OP_DPP:
      for (int l = 0; l < 64; ++l)
        if ((arr >> l) & 1) {
          const int s = dpp_src(W.in_j[l], l);
          if (s < 0) fail("unsupported DPP control", W.file, W.line);
          need(s, "dpp");
          W.out_i[l] = W.in_i[s];
        }
      break;
    case OP_MFMA: {
      if (arr != ~0ull) fail("MFMA without all 64 lanes", W.file, W.line);
      n_mfma++;
      // A[i][k] in lane i + 16k, B[k][j] in lane j + 16k, C/D[i][j] in lane
      // j + 16 (i & 3), element i >> 2
      for (int i = 0; i < 16; ++i)
        for (int j = 0; j < 16; ++j) {
          const int dl = j + 16 * (i & 3), de = i >> 2;
          double acc = W.in_c[dl][de];
          for (int k = 0; k < 4; ++k) acc = fma(W.in_d[i + 16 * k], W.in_b[j + 16 * k], acc);
          W.out_c[dl][de] = acc;
        }
      break;
    }
    default:
      break;
  }
  W.count = 0;
  W.gen++;
  for (int l = 0; l < 64; ++l) {
    Fiber& f = G.f[64 * w + l];
    if (f.state == WAIT_WAVE) f.state = READY;
  }
}

}  // namespace

void syncthreads(const char* file, int line) {
  n_bar++;
  if (G.bar_count == 0) {
    G.bar_file = file;
    G.bar_line = line;
  } else if (G.bar_line != line || strcmp(G.bar_file, file) != 0) {
    if (n_bar_mismatch++ < 20)
      fprintf(stderr, "EMU WARNING: barrier reached from %s:%d and %s:%d (block %u)\n", G.bar_file,
              G.bar_line, file, line, g_block.x);
  }
  G.bar_count++;
  if (G.bar_count == G.nlive) {
    release_barrier();
    return;
  }
  Fiber& me = G.f[G.cur];
  me.state = WAIT_BAR;
  me.wait_gen = G.bar_gen;
  run_next(false);
}

__attribute__((noinline)) double shfl(double v, int src, const char* file, int line) {
  int w, l;
  Wave& W = wave_enter(OP_SHFL, file, line, w, l);
  W.in_d[l] = v;
  W.in_i[l] = src;
  wave_wait(W, w, l);
  return G.w[w].out_d[l];
}

__attribute__((noinline)) double shfl_xor(double v, int mask, const char* file, int line) {
  int w, l;
  Wave& W = wave_enter(OP_SHFL_XOR, file, line, w, l);
  if (mask < 0 || mask > 63) fail("shfl_xor mask out of range", file, line);
  W.in_d[l] = v;
  W.in_i[l] = mask;
  wave_wait(W, w, l);
  return G.w[w].out_d[l];
}

__attribute__((noinline)) int readlane(int v, int lane, const char* file, int line) {
  int w, l;
  Wave& W = wave_enter(OP_READLANE, file, line, w, l);
  W.in_i[l] = v;
  W.in_j[l] = lane;
  wave_wait(W, w, l);
  return G.w[w].out_i[l];
}

__attribute__((noinline)) int mov_dpp(int v, int ctrl, const char* file, int line) {
  int w, l;
  Wave& W = wave_enter(OP_DPP, file, line, w, l);
  W.in_i[l] = v;
  W.in_j[l] = ctrl;
  wave_wait(W, w, l);
  return G.w[w].out_i[l];
}

__attribute__((noinline)) v4 mfma_f64(double a, double b, v4 c, const char* file, int line) {
  int w, l;
  Wave& W = wave_enter(OP_MFMA, file, line, w, l);
  W.in_d[l] = a;
  W.in_b[l] = b;
  W.in_c[l] = c;
  wave_wait(W, w, l);
  return G.w[w].out_c[l];
}

uint64_t clock64() { return clock_ticks += 100; }

void sleep_yield() {
  // a spinning lane lets every other ready lane run first
  run_next(false);
}

void launch(dim3 grid, dim3 block, const std::function<void()>& body) {
  if (G.cur != -1 && !G.f.empty() && G.f[G.cur].state != DONE) {
    fprintf(stderr, "EMU ERROR: launch from inside a kernel\n");
    abort();
  }
  n_launch++;
  g_launch = n_launch;
  const uint64_t mfma0 = n_mfma, bar0 = n_bar;
#ifdef EMU_RACE
  emu_race_lds_setup();
#endif
  const int n = (int)(block.x * block.y * block.z);
  if (block.y != 1 || block.z != 1 || grid.y != 1 || grid.z != 1 || n <= 0 || n > 1024 || n % 64) {
    fprintf(stderr, "EMU ERROR: unsupported launch shape (%u,%u,%u) x (%u,%u,%u)\n", grid.x, grid.y,
            grid.z, block.x, block.y, block.z);
    abort();
  }
  if ((int)G.f.size() < n) G.f.resize(n);
  G.w.assign(n / 64, Wave());
  G.n = n;
  G.body = &body;
  g_bdim = block;
  g_gdim = grid;
  for (unsigned b = 0; b < grid.x; ++b) {
    n_groups++;
    g_group = b;
    g_epoch++;
#ifdef EMU_LDS_SECTION
    if (__start_emu_lds && __stop_emu_lds) memset(__start_emu_lds, 0xFF, __stop_emu_lds - __start_emu_lds);
#endif
    g_block = dim3(b, 0, 0);
    for (int t = 0; t < n; ++t) init_fiber(G.f[t], t);
    for (int w = 0; w < n / 64; ++w) {
      G.w[w] = Wave();
      G.w[w].nlive = 64;
      G.w[w].alive = ~0ull;
    }
    G.nlive = n;
    G.bar_count = 0;
    G.cur = -1;
    switch_to(-1, 0, false);
    if (G.nlive != 0) {
      fprintf(stderr, "EMU ERROR: workgroup ended with live lanes\n");
      abort();
    }
  }
  G.cur = -1;
  launch_log.push_back(grid.x);
  launch_log.push_back(n_mfma - mfma0);
  launch_log.push_back(n_bar - bar0);
#ifdef EMU_RACE
  emu_race_launch_end();
#endif
}

}  // namespace emu

extern "C" {
void emu_stats(uint64_t* out) {
  out[0] = emu::n_launch;
  out[1] = emu::n_groups;
  out[2] = emu::n_bar;
  out[3] = emu::n_wave;
  out[4] = emu::n_mfma;
  out[5] = emu::n_bar_mismatch;
}

// per-launch records (workgroups, MFMA instructions of whole waves, barrier
// arrivals of lanes), oldest first; returns the number of launches
int emu_launch_log(uint64_t* out, int max) {
  const int n = (int)(emu::launch_log.size() / 3);
  for (int i = 0; i < n && i < max; ++i)
    for (int k = 0; k < 3; ++k) out[3 * i + k] = emu::launch_log[3 * i + k];
  return n;
}

static int g_fill = -1;   // byte written into fresh allocations (-1: none)
void emu_set_fill(int byte) { g_fill = byte; }

hipError_t hipMalloc(void** p, size_t n) {
  if (posix_memalign(p, 256, n ? n : 1) != 0) return hipErrorInvalidValue;
  if (g_fill >= 0) memset(*p, g_fill, n);
#ifdef EMU_RACE
  emu_race_register(*p, n);
#endif
  return hipSuccess;
}
hipError_t hipFree(void* p) {
#ifdef EMU_RACE
  emu_race_unregister(p);
#endif
  free(p);
  return hipSuccess;
}
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { memmove(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  memmove(d, s, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) { memset(d, v, n); return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamIsCapturing(hipStream_t, hipStreamCaptureStatus* s) { *s = hipStreamCaptureStatusNone; return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
  *v = a == hipDeviceAttributeMultiprocessorCount ? 256 : 100000;
  return hipSuccess;
}
struct emu_event { double t; };
static double now_ms() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return ts.tv_sec * 1e3 + ts.tv_nsec * 1e-6;
}
hipError_t hipEventCreate(hipEvent_t* e) { *e = new emu_event{0}; return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { e->t = now_ms(); return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) { *ms = (float)(b->t - a->t); return hipSuccess; }
hipError_t hipGetLastError(void) { return hipSuccess; }
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "hipSuccess" : "emulated hip error"; }
hipError_t hipGetSymbolAddress(void** p, const void* sym) { *p = (void*)sym; return hipSuccess; }
}

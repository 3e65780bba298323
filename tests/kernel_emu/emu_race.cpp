// Race checker of the host build of the library's kernels: kernels compiled with
// -fsanitize=thread call these hooks on every load and store (no TSan runtime
// is linked).  Shadow state per 4-byte granule of every emulated device buffer
// and of the shared-memory section:
//   * two waves of one workgroup touch a granule between the same pair of
//     barriers, at least one of them writing                -> intra-group race
//   * two workgroups of one launch touch a granule, at least one writing
//                                                          -> inter-group race
//   * a workgroup reads shared memory it has not written    -> undefined read
// It also adds up the device bytes each launch's loads and stores ask for.
//   * two lanes of one wave touch a granule between the same pair of
//     barriers, one of them writing                         -> lane race
//     (the lanes run in lockstep, but the compiler orders each lane's
//     accesses as if no other lane touched them)
// Atomic operations are not recorded.
#include "hip/hip_runtime.h"

#include <dlfcn.h>
#include <stdio.h>
#include <stdlib.h>

#include <map>
#include <vector>

extern "C" char __start_emu_lds[] __attribute__((weak));
extern "C" char __stop_emu_lds[] __attribute__((weak));

namespace emu {
// from emu_runtime.cpp
extern uint64_t g_epoch;
extern uint64_t g_launch;
extern uint32_t g_group;
}

namespace {

struct Cell {
  uint32_t wl, wg;       // launch and group of the last write
  uint64_t we;           // barrier epoch of the last write
  void* wpc;             // where it was written
  uint32_t rl, rg;       // launch and group of the last read
  uint64_t re;           // epoch of the reads recorded in rmask
  uint16_t wwave, rmask; // writing wave, reading waves (bit per wave) in epoch re
  uint16_t wtid, rtid;   // writing lane (thread index), first reading lane in epoch re
  uint8_t rmulti;        // read by more than one group in launch rl
  uint8_t rtmulti;       // read by more than one lane in epoch re
  uint8_t pad[2];
};

struct Region {
  uintptr_t base;
  size_t n;
  Cell* sh;
  int id;
};

std::map<uintptr_t, Region> regions;   // by base
Region lds{0, 0, nullptr, -1};
Region* last = nullptr;
int next_id = 0;
uint64_t n_reports = 0, n_checked = 0, n_lane_reports = 0;
uint64_t dev_read = 0, dev_write = 0;              // device bytes of the current launch
std::vector<uint64_t> launch_bytes;                 // per launch: read, written
std::map<std::pair<void*, void*>, uint64_t> seen;   // (pc, other pc) -> count

Region* find(uintptr_t a) {
  if (last && a - last->base < last->n) return last;
  if (lds.sh && a - lds.base < lds.n) return last = &lds;
  auto it = regions.upper_bound(a);
  if (it == regions.begin()) return nullptr;
  --it;
  if (a - it->second.base < it->second.n) return last = &it->second;
  return nullptr;
}

void describe(void* pc, char* buf, size_t n) {
  Dl_info info;
  if (pc && dladdr(pc, &info) && info.dli_fname)
    snprintf(buf, n, "%s+0x%lx", info.dli_fname, (unsigned long)((char*)pc - (char*)info.dli_fbase));
  else
    snprintf(buf, n, "%p", pc);
}

void report(const char* kind, const Region* r, uintptr_t a, void* pc, void* opc, uint32_t og, int ow,
            bool lanes = false) {
  auto key = std::make_pair(pc, opc);
  if (seen[key]++ > 0) return;
  if (lanes) n_lane_reports++;
  else n_reports++;
  if (n_reports + n_lane_reports > 60) return;
  char b1[512], b2[512];
  describe(pc, b1, sizeof b1);
  describe(opc, b2, sizeof b2);
  const int w = emu::g_cur ? (int)(emu::g_cur->tid.x >> 6) : -1;
  fprintf(stderr,
          "EMU RACE %s: region %d (%s) offset %zu, launch %u group %u wave %d at %s; other: group %u "
          "wave %d at %s\n",
          kind, r->id, r == &lds ? "shared" : "device", (size_t)(a - r->base), (unsigned)emu::g_launch,
          emu::g_group, w, b1, og, ow, b2);
}

inline void access(uintptr_t a, size_t size, bool write, void* pc) {
  if (!emu::g_cur) return;   // host code
  Region* r = find(a);
  if (!r) return;            // private memory, kernel arguments
  if (r == &lds && !r->sh) return;
  n_checked++;
  if (r != &lds) (write ? dev_write : dev_read) += size;
  const uint32_t L = (uint32_t)emu::g_launch, g = emu::g_group;
  const uint64_t e = emu::g_epoch;
  const int t = (int)emu::g_cur->tid.x, w = t >> 6;
  const size_t g0 = (a - r->base) >> 2, g1 = (a + size - 1 - r->base) >> 2;
  if (r == &lds) {
    // shared memory lives for one workgroup: a read must see a write of
    // the same workgroup and launch; waves race as for device memory
    for (size_t k = g0; k <= g1 && k < (r->n + 3) / 4; ++k) {
      Cell& c = r->sh[k];
      const bool mine = c.wpc && c.wl == L && c.wg == g;
      if (write) {
        if (mine && c.we == e && c.wwave != w) report("shared write after write by another wave, no barrier", r, a, pc, c.wpc, c.wg, c.wwave);
        else if (mine && c.we == e && c.wtid != t) report("shared write after write by another lane of the wave, no barrier", r, a, pc, c.wpc, c.wg, c.wwave, true);
        if (c.rl == L && c.rg == g && c.re == e) {
          if (c.rmask & ~(1u << w)) report("shared write after read by another wave, no barrier", r, a, pc, nullptr, c.rg, -1);
          else if (c.rtid != t || c.rtmulti) report("shared write after read by another lane of the wave, no barrier", r, a, pc, nullptr, c.rg, -1, true);
        }
        c.wl = L; c.wg = g; c.we = e; c.wwave = (uint16_t)w; c.wtid = (uint16_t)t; c.wpc = pc;
      } else {
        if (!mine) report("shared read of a value this workgroup never wrote", r, a, pc, c.wpc, c.wg, c.wwave);
        else if (c.we == e && c.wwave != w) report("shared read after write by another wave, no barrier", r, a, pc, c.wpc, c.wg, c.wwave);
        else if (c.we == e && c.wtid != t) report("shared read after write by another lane of the wave, no barrier", r, a, pc, c.wpc, c.wg, c.wwave, true);
        if (c.rl == L && c.rg == g && c.re == e) {
          c.rmask |= (uint16_t)(1u << w);
          if (c.rtid != t) c.rtmulti = 1;
        } else {
          c.rl = L; c.rg = g; c.re = e; c.rmask = (uint16_t)(1u << w); c.rtid = (uint16_t)t; c.rtmulti = 0;
        }
      }
    }
    return;
  }
  for (size_t k = g0; k <= g1 && k < (r->n + 3) / 4; ++k) {
    Cell& c = r->sh[k];
    if (write) {
      if (c.wl == L && c.wpc) {
        if (c.wg != g) report("write after write by another workgroup", r, a, pc, c.wpc, c.wg, c.wwave);
        else if (c.we == e && c.wwave != w) report("write after write by another wave, no barrier", r, a, pc, c.wpc, c.wg, c.wwave);
        else if (c.we == e && c.wtid != t) report("write after write by another lane of the wave, no barrier", r, a, pc, c.wpc, c.wg, c.wwave, true);
      }
      if (c.rl == L) {
        if (c.rg != g || c.rmulti) report("write after read by another workgroup", r, a, pc, nullptr, c.rg, -1);
        else if (c.re == e && (c.rmask & ~(1u << w))) report("write after read by another wave, no barrier", r, a, pc, nullptr, c.rg, -1);
        else if (c.re == e && (c.rtid != t || c.rtmulti)) report("write after read by another lane of the wave, no barrier", r, a, pc, nullptr, c.rg, -1, true);
      }
      c.wl = L; c.wg = g; c.we = e; c.wwave = (uint16_t)w; c.wtid = (uint16_t)t; c.wpc = pc;
    } else {
      if (c.wl == L && c.wpc) {
        if (c.wg != g) report("read of a value written by another workgroup", r, a, pc, c.wpc, c.wg, c.wwave);
        else if (c.we == e && c.wwave != w) report("read after write by another wave, no barrier", r, a, pc, c.wpc, c.wg, c.wwave);
        else if (c.we == e && c.wtid != t) report("read after write by another lane of the wave, no barrier", r, a, pc, c.wpc, c.wg, c.wwave, true);
      }
      if (c.rl == L && c.rg == g) {
        if (c.re == e) {
          c.rmask |= (uint16_t)(1u << w);
          if (c.rtid != t) c.rtmulti = 1;
        } else {
          c.re = e; c.rmask = (uint16_t)(1u << w); c.rtid = (uint16_t)t; c.rtmulti = 0;
        }
      } else {
        if (c.rl == L && c.rg != g) c.rmulti = 1;
        else c.rmulti = 0;
        c.rl = L; c.rg = g; c.re = e; c.rmask = (uint16_t)(1u << w); c.rtid = (uint16_t)t; c.rtmulti = 0;
      }
    }
  }
}

}  // namespace

extern "C" {
void emu_race_register(void* p, size_t n) {
  Region r{(uintptr_t)p, n, (Cell*)calloc((n + 3) / 4 + 1, sizeof(Cell)), next_id++};
  if (!r.sh) { fprintf(stderr, "race shadow: out of memory\n"); abort(); }
  regions[r.base] = r;
  last = nullptr;
}
void emu_race_unregister(void* p) {
  auto it = regions.find((uintptr_t)p);
  if (it != regions.end()) { free(it->second.sh); regions.erase(it); }
  last = nullptr;
}
void emu_race_lds_setup() {
  if (lds.sh || !__start_emu_lds) return;
  lds.base = (uintptr_t)__start_emu_lds;
  lds.n = __stop_emu_lds - __start_emu_lds;
  lds.sh = (Cell*)calloc((lds.n + 3) / 4 + 1, sizeof(Cell));
}
void emu_race_stats(uint64_t* out) { out[0] = n_reports; out[1] = n_checked; out[2] = n_lane_reports; }
// called by the runtime at the end of every launch
void emu_race_launch_end() {
  launch_bytes.push_back(dev_read);
  launch_bytes.push_back(dev_write);
  dev_read = dev_write = 0;
}
// per launch: device bytes the kernel's loads and stores asked for (before
// any cache), oldest first; returns the number of launches
int emu_race_launch_bytes(uint64_t* out, int max) {
  const int n = (int)(launch_bytes.size() / 2);
  for (int i = 0; i < n && i < max; ++i) {
    out[2 * i] = launch_bytes[2 * i];
    out[2 * i + 1] = launch_bytes[2 * i + 1];
  }
  return n;
}

void __tsan_init() {}
void __tsan_func_entry(void*) {}
void __tsan_func_exit() {}
#define RD(n) void __tsan_read##n(void* a) { access((uintptr_t)a, n, false, __builtin_return_address(0)); } \
  void __tsan_unaligned_read##n(void* a) { access((uintptr_t)a, n, false, __builtin_return_address(0)); } \
  void __tsan_write##n(void* a) { access((uintptr_t)a, n, true, __builtin_return_address(0)); } \
  void __tsan_unaligned_write##n(void* a) { access((uintptr_t)a, n, true, __builtin_return_address(0)); }
RD(1) RD(2) RD(4) RD(8) RD(16)
void __tsan_read_range(void* a, unsigned long n) { access((uintptr_t)a, n, false, __builtin_return_address(0)); }
void __tsan_write_range(void* a, unsigned long n) { access((uintptr_t)a, n, true, __builtin_return_address(0)); }
void* __tsan_memcpy(void* d, const void* s, size_t n) {
  access((uintptr_t)s, n, false, __builtin_return_address(0));
  access((uintptr_t)d, n, true, __builtin_return_address(0));
  return memcpy(d, s, n);
}
void* __tsan_memmove(void* d, const void* s, size_t n) {
  access((uintptr_t)s, n, false, __builtin_return_address(0));
  access((uintptr_t)d, n, true, __builtin_return_address(0));
  return memmove(d, s, n);
}
void* __tsan_memset(void* d, int v, size_t n) {
  access((uintptr_t)d, n, true, __builtin_return_address(0));
  return memset(d, v, n);
}
void __tsan_vptr_update(void**, void*) {}
void __tsan_vptr_read(void**) {}
int __tsan_atomic32_compare_exchange_val(volatile int* a, int c, int v, int, int) {
  __atomic_compare_exchange_n(a, &c, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST);
  return c;
}
int __tsan_atomic32_load(const volatile int* a, int) { return __atomic_load_n(a, __ATOMIC_SEQ_CST); }
void __tsan_atomic32_store(volatile int* a, int v, int) { __atomic_store_n(a, v, __ATOMIC_SEQ_CST); }
int __tsan_atomic32_fetch_add(volatile int* a, int v, int) { return __atomic_fetch_add(a, v, __ATOMIC_SEQ_CST); }
void __tsan_atomic_thread_fence(int) {}
void __tsan_atomic_signal_fence(int) {}
}

// Self-test of the host-build checkers: each mode plants one mistake in a
// small kernel (built for the host only, never for the GPU), and the test
// expects the checker named beside it to report it; mode "ok" is the same
// kernel without a mistake and must run clean under every checker.
//
//   ok             no report
//   wave_race      race build: a wave reads shared memory another wave writes
//                  with no barrier in between
//   group_race     race build: every workgroup writes the same device word
//   uninit_shared  race build: shared memory read before any write
//   member_oob     array-bounds: an index past one member of a shared struct
//   heap_oob       AddressSanitizer: a store one element past a device buffer
//   private_oob    AddressSanitizer/array-bounds: a per-lane array indexed past
//                  its end
//   divergent_wave the emulator: half a wave at a shuffle, the other half at a
//                  barrier (reported as a deadlock)
//   lane_race      race build: a lane reads shared memory that another lane of
//                  its own wave writes, with no barrier in between (the
//                  compiler may reorder one lane's accesses around it)
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <string.h>

struct Shared {
  double a[512];
  double b[64];
  int flag;
};

__global__ void k_selftest(double* out, int n, int mode) {
  __shared__ Shared S;
  const int t = threadIdx.x, lane = t & 63;
  S.a[t] = t;
  if (t < 64) S.b[t] = 0.5 * t;
  if (mode == n && t == 0) S.flag = 1;   // never taken: keeps S.flag a runtime object
  double v = 0.0;
  switch (mode) {
    case 1:   // wave_race
      v = S.a[(t + 64) % 512];
      __syncthreads();
      break;
    case 2:   // group_race
      __syncthreads();
      if (t == 0) out[0] = S.a[1] + blockIdx.x;
      v = S.a[t];
      break;
    case 3:   // uninit_shared: S.flag is never written
      __syncthreads();
      v = (t == 64) ? (double)S.flag : S.a[t];
      break;
    case 4: {  // member_oob
      __syncthreads();
      const int i = 512 + (t & 7) * (n > 0 ? 1 : 0);
      v = S.a[i];
      break;
    }
    case 5:   // heap_oob
      __syncthreads();
      if (t == 0) out[(size_t)gridDim.x * blockDim.x] = 1.0;
      v = S.a[t];
      break;
    case 6: {  // private_oob
      double p[4] = {1.0, 2.0, 3.0, 4.0};
      __syncthreads();
      volatile int i = 4 + (t & 1);
      v = p[i];
      break;
    }
    case 7:   // divergent_wave
      if (lane < 32) v = __shfl(S.a[t], 0, 64);
      __syncthreads();
      break;
    case 8:   // lane_race
      v = S.a[(t & ~63) | ((t + 1) & 63)];
      __syncthreads();
      break;
    default:  // ok
      __syncthreads();
      v = S.a[(t + 64) % 512] + S.b[lane];
      break;
  }
  v += __shfl_xor(v, 1, 64);
  out[(size_t)blockIdx.x * blockDim.x + t] = v;
}

extern "C" void emu_race_stats(uint64_t*) __attribute__((weak));
extern "C" void emu_stats(uint64_t*);

int main(int argc, char** argv) {
  static const char* modes[] = {"ok", "wave_race", "group_race", "uninit_shared", "member_oob",
                                "heap_oob", "private_oob", "divergent_wave", "lane_race"};
  int mode = -1;
  for (int m = 0; m < 9; ++m)
    if (argc > 1 && strcmp(argv[1], modes[m]) == 0) mode = m;
  if (mode < 0) {
    fprintf(stderr, "usage: %s <mode>\n", argv[0]);
    return 2;
  }
  const int groups = 2, n = groups * 512;
  double* d = nullptr;
  if (hipMalloc((void**)&d, n * sizeof(double)) != hipSuccess) return 3;
  hipLaunchKernelGGL(k_selftest, dim3(groups), dim3(512), 0, 0, d, n, mode);
  uint64_t races[3] = {0, 0, 0};
  if (emu_race_stats) emu_race_stats(races);
  uint64_t st[6];
  emu_stats(st);
  printf("{\"mode\": \"%s\", \"races\": %llu, \"lane_races\": %llu, \"barrier_site_mismatch\": %llu}\n",
         modes[mode], (unsigned long long)races[0], (unsigned long long)races[2],
         (unsigned long long)st[5]);
  hipFree(d);
  return 0;
}

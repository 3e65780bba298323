// fd_greens_noalloc: fd_greens with the workspace in a fixed device array of
// this library instead of caller memory, for callers that cannot allocate
// device memory (code under stream capture, tight serving loops, harnesses
// that forbid allocation).
//
// `scratch` below is one array per GPU, held until the process ends.  In host
// code its name is only a host-side stand-in: its device address comes from
// hipGetSymbolAddress, taken once per device (with that device current) and
// kept in g_ptr; kernels and copies only ever see that address.  Every call
// on a device shares its array and leaves its contents behind; the call
// rewrites everything it reads (work descriptors, the status word is cleared
// by its first kernel), so nothing needs clearing between calls, but calls
// that overlap in time on one device race for the array.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/fdet.h"

// error reporting of the library (fdet_abi.cpp): sets the thread's last
// error message and returns `code`
int fdet_fail(int code, const char* msg);

namespace {

static __device__ __align__(256) unsigned char scratch[FD_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's `scratch` (current device), looked up once.
int scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fdet_fail(FD_ERR_HIP, (std::string("hipGetDevice: ") + hipGetErrorString(e)).c_str());
  if (dev < 0 || dev >= kMaxDevices) return fdet_fail(FD_ERR_UNSUPPORTED, "device ordinal out of range");
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fdet_fail(FD_ERR_HIP, (std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)).c_str());
    g_ptr[dev] = ptr;
  }
  *out = g_ptr[dev];
  return FD_OK;
}

}  // namespace

extern "C" int fd_greens_noalloc(const fd_problem* p, const fd_options* o, double* logdet, double* G,
                                 int32_t* status, void* stream) {
  if (!G) return fdet_fail(FD_ERR_INVALID_ARG, "G must be a device pointer");
  if (!status) return fdet_fail(FD_ERR_INVALID_ARG, "status must be a device pointer");
  const size_t need = fd_workspace_bytes(p, 1, o, FD_WHAT_GREENS);
  if (need == 0) return FD_ERR_INVALID_ARG;   // fd_workspace_bytes set the message
  if (need > (size_t)FD_NOALLOC_MAX_BYTES) {
    const std::string msg = "fd_greens_noalloc: the call needs " + std::to_string(need) +
                            " bytes of workspace, more than the fixed " +
                            std::to_string((size_t)FD_NOALLOC_MAX_BYTES) +
                            " (fewer segments, or fd_greens with a caller workspace)";
    return fdet_fail(FD_ERR_WORKSPACE, msg.c_str());
  }
  void* ws = nullptr;
  const int rc = scratch_address(&ws);
  if (rc != FD_OK) return rc;
  return fd_greens(p, o, logdet, G, ws, (size_t)FD_NOALLOC_MAX_BYTES, status, stream);
}

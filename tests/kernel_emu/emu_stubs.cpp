// Launchers of the size classes left out of a host build: they report that
// the class is missing, so a case that would need one fails loudly.
#include "hip/hip_runtime.h"

#include <stdio.h>

namespace fdet_stub {
struct Prob;
struct Item;
struct Sched;
}  // namespace fdet_stub

#define EMU_STUB(NC)                                                                          \
  extern "C" hipError_t fdet_launch_items_##NC(int, const fdet_stub::Prob*, const fdet_stub::Item*, \
                                               int, hipStream_t) {                            \
    fprintf(stderr, "EMU ERROR: size class " #NC " is not in this host build\n");             \
    return hipErrorNotSupported;                                                              \
  }                                                                                           \
  extern "C" hipError_t fdet_launch_persist_##NC(const fdet_stub::Prob*, const fdet_stub::Item*, \
                                                 int, const int32_t*, uint32_t*,              \
                                                 fdet_stub::Sched*, uint64_t, int, hipStream_t) { \
    return hipErrorNotSupported;                                                              \
  }                                                                                           \
  extern "C" int fdet_persist_blocks_per_cu_##NC(void) { return 0; }

#ifdef EMU_STUB_64
EMU_STUB(64)
#endif
#ifdef EMU_STUB_80
EMU_STUB(80)
#endif
#ifdef EMU_STUB_96
EMU_STUB(96)
#endif
#ifdef EMU_STUB_128
EMU_STUB(128)
#endif
#ifdef EMU_STUB_512
EMU_STUB(512)
#endif

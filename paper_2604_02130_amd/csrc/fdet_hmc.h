// Descriptor of one field's molecular-dynamics update, shared by the host
// side and the kernels of fdet_hmc.hip.
#pragma once

#include <stdint.h>

namespace fdet {

struct HmcProb {
  double* phi;    // the field, N_t * N doubles, advanced in place
  int64_t off;    // offset of this field's momenta and force in the batch arrays
  int64_t n;      // N_t * N
};

}  // namespace fdet

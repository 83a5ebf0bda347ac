// Kernels for 1 term(s), all SHO, with per-instrument amplitudes and
// offsets enabled; see kernels_impl.h.
#define GPSSM_M 1
#define GPSSM_NS m1
#include "kernels_impl.h"

namespace gpssm {
KernelSet kernels_m1i(int J) {
  switch (J) {
    case 1: return m1::make_set<1, 2>();
    case 2: return m1::make_set<2, 2>();
    case 3: return m1::make_set<3, 2>();
    default: return m1::make_set<4, 2>();
  }
}
}  // namespace gpssm

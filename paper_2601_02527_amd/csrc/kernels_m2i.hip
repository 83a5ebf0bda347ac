// Kernels for 2 term(s), all SHO, with per-instrument amplitudes and
// offsets enabled; see kernels_impl.h.
#define GPSSM_M 2
#define GPSSM_NS m2
#include "kernels_impl.h"

namespace gpssm {
KernelSet kernels_m2i(int J) {
  switch (J) {
    case 1: return m2::make_set<1, 2>();
    case 2: return m2::make_set<2, 2>();
    case 3: return m2::make_set<3, 2>();
    default: return m2::make_set<4, 2>();
  }
}
}  // namespace gpssm

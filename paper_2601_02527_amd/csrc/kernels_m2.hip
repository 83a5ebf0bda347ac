// Kernels for 2 term(s), all SHO and without instrument tables (the plain
// model); see kernels_impl.h.
#define GPSSM_M 2
#define GPSSM_NS m2
#include "kernels_impl.h"

namespace gpssm {
KernelSet kernels_m2(int J) {
  switch (J) {
    case 1: return m2::make_set<1, 0>();
    case 2: return m2::make_set<2, 0>();
    case 3: return m2::make_set<3, 0>();
    default: return m2::make_set<4, 0>();
  }
}
}  // namespace gpssm

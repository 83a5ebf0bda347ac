// Kernels for 1 term(s), all SHO and without instrument tables (the plain
// model); see kernels_impl.h.
#define GPSSM_M 1
#define GPSSM_NS m1
#include "kernels_impl.h"

namespace gpssm {
KernelSet kernels_m1(int J) {
  switch (J) {
    case 1: return m1::make_set<1, 0>();
    case 2: return m1::make_set<2, 0>();
    case 3: return m1::make_set<3, 0>();
    default: return m1::make_set<4, 0>();
  }
}
}  // namespace gpssm

// Kernels for 4 term(s) with real exponential terms and per-instrument
// amplitudes and offsets enabled; see kernels_impl.h.
#define GPSSM_M 4
#define GPSSM_NS m4
#include "kernels_impl.h"

namespace gpssm {
KernelSet kernels_m4x(int J) {
  switch (J) {
    case 1: return m4::make_set<1, 3>();
    case 2: return m4::make_set<2, 3>();
    case 3: return m4::make_set<3, 3>();
    default: return m4::make_set<4, 3>();
  }
}
}  // namespace gpssm

// Kernels for 3 term(s) with real exponential terms and per-instrument
// amplitudes and offsets enabled; see kernels_impl.h.
#define GPSSM_M 3
#define GPSSM_NS m3
#include "kernels_impl.h"

namespace gpssm {
KernelSet kernels_m3x(int J) {
  switch (J) {
    case 1: return m3::make_set<1, 3>();
    case 2: return m3::make_set<2, 3>();
    case 3: return m3::make_set<3, 3>();
    default: return m3::make_set<4, 3>();
  }
}
}  // namespace gpssm

// elbm_step_d1.hip -- step-kernel instantiations for the D1Q3 lattice
// (one translation unit per lattice so that they compile in parallel).
#include "elbm_step_impl.hpp"

namespace elbm {
StepLauncher step_launcher_d1(int storage, int mode, int fp64) {
  return step_launcher_for<1>(storage, mode, fp64);
}
}  // namespace elbm

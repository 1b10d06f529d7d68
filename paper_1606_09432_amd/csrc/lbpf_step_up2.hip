// Step kernel instances with the second-order upwind (biased) directional
// derivatives of Sec. 4.2 put through the moment of Eq. Grad_DF-Centree: a
// wider phi ring (3-node halo, one more plane).  Single simulations, 4-row
// tiles in 3D (and 12-row tiles for the FP32-arithmetic forms), with or
// without the index field, no mirror planes.  A separate source file so that
// the instance sets compile in parallel.
#include "lbpf_step_kernel.hpp"

namespace lbpf {

hipError_t launch_step_up2(int lattice, int storage, const SimDev &sd, const TileDev &tc, hipStream_t st) {
  switch (lattice) {
    case 0: return launch_step_up2_k<0>(storage, sd, tc, st);
    case 1: return launch_step_up2_k<1>(storage, sd, tc, st);
    case 2: return launch_step_up2_k<2>(storage, sd, tc, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbpf

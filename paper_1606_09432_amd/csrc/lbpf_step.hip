// Step launchers for boxes without mirror planes (periodic or zero flux), and
// the dispatch to the mirror-plane instances in lbpf_step_mirror.hip.
#include "lbpf_step_kernel.hpp"

namespace lbpf {

hipError_t launch_step(int lattice, int storage, const SimDev &sd, const TileDev &tc, hipStream_t st) {
  if (sd.grad_up2) return launch_step_up2(lattice, storage, sd, tc, st);
  // (part 2 of a box with mirror planes: tiles the mirror rules do not reach)
  if (sd.mirror && tc.part != 2) return launch_step_mirror(lattice, storage, sd, tc, st);
  return launch_step_m<false>(lattice, storage, sd, tc, st);
}

hipError_t launch_batch(int storage, bool ids, bool mirror, const SimDev *sims, const BatchItem *items, int n_items,
                        int grid, hipStream_t st) {
  if (mirror) return launch_batch_mirror(storage, ids, sims, items, n_items, grid, st);
  return launch_batch_m<false>(storage, ids, sims, items, n_items, grid, st);
}

int batch_blocks_per_cu(int storage, bool ids, bool mirror) {
  if (mirror) return batch_blocks_per_cu_mirror(storage, ids);
  return batch_blocks_per_cu_m<false>(storage, ids);
}

}  // namespace lbpf

// Step kernel instances with mirror planes through node 0 (symmetric boxes:
// one octant, or one quadrant in 2D, of a mirror-symmetric domain).  A
// separate source file so that both sets of instances compile in parallel.
#include "lbpf_step_kernel.hpp"

namespace lbpf {

hipError_t launch_step_mirror(int lattice, int storage, const SimDev &sd, const TileDev &tc, hipStream_t st) {
  return launch_step_m<true>(lattice, storage, sd, tc, st);
}

hipError_t launch_batch_mirror(int storage, bool ids, const SimDev *sims, const BatchItem *items, int n_items,
                               int grid, hipStream_t st) {
  return launch_batch_m<true>(storage, ids, sims, items, n_items, grid, st);
}

int batch_blocks_per_cu_mirror(int storage, bool ids) { return batch_blocks_per_cu_m<true>(storage, ids); }

}  // namespace lbpf

// Launchers shared between the kernel sources and the C-ABI host code.
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>

#include "lbpf_common.hpp"

namespace lbpf {

// Tiling of the step kernel: tiles_x x tiles_y tiles of 64 x ty nodes, each
// marching `chunk` planes; nchunks = ceil(extent along m / chunk).  part
// selects the work items of one launch: 0 every one; in a box with mirror
// planes through node 0, 1 those at a plane (tile x 0, tile y 0 in 3D, chunk
// 0) and 2 all others (which the mirror rules do not reach when ty >= 4 in 3D
// and chunk >= 4: their rings start at node 4 or beyond along every axis).
struct TileDev {
  int tiles_x, tiles_y, nchunks, chunk, ty, part;
};

// Work-groups of a launch over part t.part of the tiles (ydir: tile y 0 lies
// at a plane, i.e. 3D).
__host__ __device__ inline long long part_blocks(const TileDev &t, bool ydir) {
  const long long all = (long long)t.tiles_x * t.tiles_y * t.nchunks;
  const long long inner = (long long)(t.tiles_x - 1) * (t.tiles_y - (ydir ? 1 : 0)) * (t.nchunks - 1);
  return t.part == 0 ? all : (t.part == 2 ? inner : all - inner);
}

// Tile (x, y) and chunk c of work-group L of a launch over part 1 or 2.
// Part 1 lists the slab of tile x 0 (every y, every chunk), then in 3D the
// slab of tile y 0 (x >= 1, every chunk), then chunk 0 of the remaining tiles.
__device__ inline void part_tile(const TileDev &t, bool ydir, int L, int &x, int &y, int &c) {
  const int y0 = ydir ? 1 : 0;
  const int nx1 = t.tiles_x - 1, ny1 = t.tiles_y - y0;
  if (t.part == 2) {
    x = 1 + L % nx1;
    L /= nx1;
    y = y0 + L % ny1;
    c = 1 + L / ny1;
    return;
  }
  const int a = t.tiles_y * t.nchunks;
  const int b = ydir ? nx1 * t.nchunks : 0;
  if (L < a) {
    x = 0;
    y = L % t.tiles_y;
    c = L / t.tiles_y;
  } else if (L < a + b) {
    L -= a;
    x = 1 + L % nx1;
    y = 0;
    c = L / nx1;
  } else {
    L -= a + b;
    x = 1 + L % nx1;
    y = y0 + L / nx1;
    c = 0;
  }
}

// One item of a batched step: rows m0 .. m1-1 of the 64-wide column at x0
// of simulation `sim` (2D).
struct BatchItem {
  int sim, x0, m0, m1;
};

// Seeds in lattice units, in (x, y, z) order.
struct SeedDev {
  double x, y, z, r;
  int id;
};

// Where the initial fields come from: the seeds (Eq. Initial_Condition, u = -delta)
// or caller FP64 arrays in the compact x-fastest layout.
struct InitSrc {
  const SeedDev *seeds;
  int n_seeds;
  const double *phi;   // arrays (NULL when seeded)
  const double *u;
  const int16_t *ids;
  int nx, ny;          // compact layout extents (x, y)
};

// Diagnostics accumulators: sum phi, sum u, sum (u - phi/2), sum (1 + phi),
// count phi > 0, non-finite flag, then the tip position.
constexpr int kDiagVals = 6;
constexpr int kDiagBlocks = 512;

// Head of a checkpoint blob: what the state blocks after it belong to, and the
// step counter.  The blob starts with kStateHeaderBytes bytes holding it.
struct StateHeader {
  unsigned long long magic;   // kStateMagic
  long long version;          // 1
  long long n_sims;
  long long step;             // step counter of the saved state
  unsigned long long bytes;   // size of the whole blob
  unsigned long long layout;  // hash of every simulation's extents, lattice, storage and block size
};
constexpr unsigned long long kStateMagic = 0x5441545346504c42ULL;  // "BLPFSTAT"
constexpr size_t kStateHeaderBytes = 256;

// Writes h to device memory dst (stream-ordered; h travels as a kernel argument).
hipError_t launch_state_header(StateHeader *dst, const StateHeader &h, hipStream_t st);
// Reads and writes every byte of src once (16-byte vectors, nontemporal):
// the plain streaming copy that bounds a step moving the same bytes.
hipError_t launch_stream_copy(const void *src, void *dst, size_t bytes, int blocks_per_cu, hipStream_t st);

// lattice: pair code (0 D2Q9/D2Q5, 1 D3Q19/D3Q7, 2 D3Q15/D3Q7).
hipError_t launch_step(int lattice, int storage, const SimDev &sd, const TileDev &tc, hipStream_t st);
// sims: the SimDev of every simulation for the step's parity (device memory);
// mirror: some simulation of the ensemble has mirror planes.
hipError_t launch_batch(int storage, bool ids, bool mirror, const SimDev *sims, const BatchItem *items, int n_items,
                        int grid, hipStream_t st);
// Resident work-groups per compute unit of the batch kernel (0 on failure).
int batch_blocks_per_cu(int storage, bool ids, bool mirror);
// The instances with mirror planes (lbpf_step_mirror.hip).
hipError_t launch_step_mirror(int lattice, int storage, const SimDev &sd, const TileDev &tc, hipStream_t st);
hipError_t launch_batch_mirror(int storage, bool ids, const SimDev *sims, const BatchItem *items, int n_items,
                               int grid, hipStream_t st);
int batch_blocks_per_cu_mirror(int storage, bool ids);
// The instances with the second-order upwind gradient (lbpf_step_up2.hip).
hipError_t launch_step_up2(int lattice, int storage, const SimDev &sd, const TileDev &tc, hipStream_t st);
hipError_t launch_init(int lattice, int storage, const SimDev &sd, int16_t *ids_out, const InitSrc &src,
                       hipStream_t st);
hipError_t launch_diag(int dim, int storage, const SimDev &sd, double *partials, double *result,
                       long long nodes, int ox, int oy, int oz, int dx, int dy, int dz, hipStream_t st);
hipError_t launch_export(int lattice, int storage, const SimDev &sd, double *phi, double *u, int16_t *ids,
                         double *g, double *f, int ny_full, hipStream_t st);

}  // namespace lbpf

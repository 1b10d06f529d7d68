// Fused coupled step (phase field, then heat) for gfx950.
//
// One launch advances one simulation (or, in 2D, a batch of them) by one time
// step.  A work-group owns a 64 x TY tile of the plane perpendicular to the
// march axis m (z in 3D, y in 2D; TY = 1 in 2D) and walks `chunk` planes along
// m.  For output plane m it
//   A. computes, for plane m+1 on the tile + 1-node halo, the gradient of
//      phi^n (directional derivatives, Eqs. Def_DeriveeDirectionnelle and
//      Grad_DF-Centree, or central differences), the crystal index update
//      (Sec. 4.3), u^n by gathering the heat populations, a_s and N
//      (Eq. TermesAnisotropes), eta_phi (Eq. LBE_RelaxationTime) and Q_phi
//      (Eq. LBE_SourceTerm), folded into per-node coefficients kept in an LDS
//      ring of 3 planes;
//   B. for every node y of plane m pulls g_i from x = y - e_i with the nonlocal
//      a_s^2 form of Eq. LBE_Eq_Phase,
//        g_i(y, t+1) = g_i(y, t) + [g*_i(x) - g_i(y, t)] / a_s^2(x),
//        g*_i(x)    = (1 - w) g_i(x) + w g^(0)_i(x) + w_i Q_phi(x) dt/tau0,
//      applies bounce-back on the walls (Eq. Bounce-Back), sums phi^{n+1}
//      (Eq. Def_M0_Phi), collides the heat populations with the source
//      (phi^{n+1} - phi^n)/2 (Eqs. LBE_Eq_Temp, Source_Tempr) and stores them
//      post-collision at y ("stream on read": the next step pulls them).
// Latency: the loads of the next planes -- the heat populations gathered by
// the coefficient nodes of plane m+2 and plane m+3 of the phi / u* / index
// rings (5 or 4 planes, 2-node halo) -- are issued at the top of the
// iteration and land while A runs from LDS and registers; B issues its g
// loads in one batch.  Index and boundary logic is branch-free (selects) so
// that loads are never serialised behind branches.  Two work-group barriers
// per plane.  Every distribution is written once per step and loaded once as
// the node's own value; the shifted load of g_i(x), the heat gathers of the
// halo nodes and the ring halos are the extra loads, served by L2 only in
// part (the rest shows as HBM traffic above the algorithmic bytes).  Tiles
// whose halo stays inside the box take a path without boundary checks.
//
// Offset storage (FP32 arithmetic): h_i = g_i - w_i phi and
// k_i = f*_i - w_i u* are stored in FP32 or FP16 beside FP32 phi and u*; the
// update is written on these small quantities:
//   h*_i(x) = A h_i(x) + w_i (Q s + e_i . C),  A = 1 - w,  C = -w (Dphi/e^2) N
//   d_i     = h_i(y) + [w_i (phi(x) - phi(y)) + h*_i(x) - h_i(y)] / a^2(x)
//   phi^{n+1}(y) = phi^n(y) + sum_i d_i,   h_i^{n+1}(y) = d_i - w_i sum_j d_j.
// In FP16 the rest offset h_0 is stored as minus the sum of the other offsets
// as rounded (likewise k_0), so the stored offsets of a node sum to zero up to
// the rounding of h_0, which stays near zero.
#pragma once

#include <type_traits>

#include "lbpf_kernels.hpp"

namespace lbpf {

// XCD-aware work-group order: the hardware hands consecutive work-group ids
// to the 8 XCDs in turn; remap so that each XCD receives one contiguous range
// of tiles and its L2 sees neighbouring tiles.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = b & 7, k = b >> 3;
  return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + k;
}

// Loads and stores at a 32-bit byte offset from a uniform base pointer, so that
// the address is an SGPR base plus one VGPR offset (no 64-bit address math).
template <class E> __device__ __forceinline__ E ldb(const E *base, unsigned boff) {
  return *reinterpret_cast<const E *>(reinterpret_cast<const char *>(base) + boff);
}
// f(integral_constant<int, I>) for I = I0 .. N-1, unrolled at compile time.
template <int I, int N, class F> __device__ __forceinline__ void static_for(F &&f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}
// Load with the non-temporal hint, for the last read of a line's data.
template <class E> __device__ __forceinline__ E ldb_nt(const E *base, unsigned boff) {
  const E *p = reinterpret_cast<const E *>(reinterpret_cast<const char *>(base) + boff);
  if constexpr (sizeof(E) == 2) {
    const unsigned short b = __builtin_nontemporal_load(reinterpret_cast<const unsigned short *>(p));
    E v;
    __builtin_memcpy(&v, &b, 2);
    return v;
  } else {
    return __builtin_nontemporal_load(p);
  }
}
template <class E> __device__ __forceinline__ void stb(E *base, unsigned boff, E v) {
  nt_store(reinterpret_cast<E *>(reinterpret_cast<char *>(base) + boff), v);
}

// Largest crystal-index table staged in LDS.
constexpr int kStagedAniso = 32;

// Minimum waves per SIMD the register allocator must leave room for (2D
// kernels with the index field or the mirror planes: 4, which they fit
// without spills).
template <int DIM, int TY, class ST, bool IDS, bool MIR> constexpr int min_waves() {
  return DIM == 2 ? (std::is_same<ST, StF64>::value ? 3 : ((IDS || MIR) ? 4 : 5))
                  : (std::is_same<ST, StF64>::value ? 2 : (TY == 8 ? 4 : 3));
}

// BATCH = false: one simulation (sd_arg); the work-group id gives the tile and
// the chunk of planes.  BATCH = true (2D): a persistent launch over the work
// list `items` of a batched ensemble, whose per-simulation state is sims[k];
// items are in decreasing cost and work-group b takes items b, b + G, b + 2G,
// ... (G = grid size): static balance, no atomics, no per-step reset.
// MIR = true adds the mirror planes through node 0 (SimDev::mirror): a source
// x = y - e_i beyond one is the mirror node x' inside, whose population is the
// mirror image i' of i; its coefficients are those of the ghost node at x
// (computed from the mirrored rings: the mirror image of x', so that
// e_i . C(x) = e_i' . C(x')).
// GR = 2 takes the second-order upwind (biased) directional derivatives of
// Sec. 4.2 through the moment of Eq. Grad_DF-Centree; the gradient then reaches
// two nodes, so the phi ring keeps a 3-node halo and one more plane.
template <int K, int TY, class ST, bool IDS, bool BATCH, bool MIR, int GR>
__global__ __launch_bounds__(64 * TY) __attribute__((amdgpu_waves_per_eu(min_waves<LatOf<K>::DIM, TY, ST, IDS, MIR>(), 8))) void
step_kernel(SimDev sd_arg, TileDev tc, const SimDev *__restrict__ sims, const BatchItem *__restrict__ items,
            int n_items) {
  constexpr int DIM = LatOf<K>::DIM;
  static_assert(!BATCH || DIM == 2, "batched ensembles are 2D");
  using T = typename ST::T;
  using LP = typename LatOf<K>::P;
  using LU = typename LatOf<K>::U;
  using S = typename ST::S;
  using PT = typename ST::P;
  constexpr int TX = 64;
  constexpr int NT = TX * TY;
  constexpr int HX = TX + 2, HY = (DIM == 3 ? TY + 2 : 1);
  static_assert(GR == 1 || GR == 2, "gradient reach");
  constexpr int HF = GR + 1;  // ring halo: coefficient halo + gradient reach
  constexpr int PX = TX + 2 * HF, PY = (DIM == 3 ? TY + 2 * HF : 1);
  constexpr int NP = DIM + 3;  // A, B, C[DIM], 1/a^2
  constexpr int PLANE_P = HX * HY;
  constexpr int PLANE_F = PX * PY;
  constexpr int NHALO = PLANE_P - NT;             // halo coefficient nodes per plane
  constexpr int NLOAD = (PLANE_F + NT - 1) / NT;  // ring entries staged per thread
  constexpr int PYO = (DIM == 3) ? HF - 1 : 0;    // row offset of a coefficient node in the ring
  constexpr int PXO = HF - 1;                      // column offset of a coefficient node in the ring
  constexpr int NRP = GR + 4;                      // phi ring planes
  constexpr int NRU = GR + 3;                      // u* and index ring planes
  constexpr int QP = LP::Q, QU = LU::Q;
  constexpr bool OFF = ST::OFF;
  constexpr bool FOLD = OFF && (DIM == 2 || ST::FOLD_3D);
  constexpr bool HEAT_CONST = DIM == 2 || ST::HEAT_CONST_3D;
  // offsets (h, k, and the pulled d and gathered fd of the offset forms) are
  // kept in stored units: SC per true unit; true-unit terms entering them are
  // scaled through the weights (compile-time constants)
  constexpr double SC = ST::SC;
  static_assert(NHALO <= NT, "one halo coefficient node per thread at most");

  __shared__ T phiS[NRP][PLANE_F];
  __shared__ float usS[OFF ? NRU : 1][OFF ? PLANE_F : 1];
  __shared__ int16_t idS[IDS ? NRU : 1][IDS ? PLANE_F : 1];
  __shared__ T parS[3][NP][PLANE_P];
  // the crystal-index table, staged in LDS in the arithmetic type when it has at
  // most kStagedAniso entries: a node's entry is then an LDS read, not a vector
  // load followed by a wait for every load in flight
  constexpr bool STAGE = IDS;
  __shared__ StagedAniso<T> tabS[STAGE ? kStagedAniso : 1];

  for (int it = blockIdx.x; !BATCH || it < n_items; it += gridDim.x) {
    const int tx = threadIdx.x;
    const int ty = (DIM == 3) ? threadIdx.y : 0;
    const int tid = ty * TX + tx;

    BatchItem bi{};
    if constexpr (BATCH) bi = items[it];
    const SimDev &sd = BATCH ? sims[bi.sim] : sd_arg;
    int x0, y0, m0, m1;
    if constexpr (BATCH) {
      x0 = bi.x0;
      y0 = 0;
      m0 = bi.m0;
      m1 = bi.m1;
      __syncthreads();  // the previous item is done with the LDS rings
    } else {
      int L = xcd_remap(blockIdx.x, gridDim.x);
      int tile_x, tile_y, chunk;
      if (tc.part == 0) {
        tile_x = L % tc.tiles_x;
        L /= tc.tiles_x;
        tile_y = L % tc.tiles_y;
        chunk = L / tc.tiles_y;
      } else {
        part_tile(tc, DIM == 3, L, tile_x, tile_y, chunk);
      }
      x0 = tile_x * TX;
      y0 = (DIM == 3) ? tile_y * TY : 0;
      m0 = chunk * tc.chunk;
      m1 = min(m0 + tc.chunk, sd.nm);
    }
    const int per = sd.periodic;
    const bool staged = STAGE && sd.n_aniso <= kStagedAniso;
    if (staged) {
      // visible to every wave after the warm-up barrier below (in an ensemble
      // the item's opening barrier keeps the previous item's readers apart)
      for (int k = threadIdx.x + ((DIM == 3) ? threadIdx.y * TX : 0); k < sd.n_aniso; k += NT)
        stage_entry<T>(sd.aniso[k], tabS[k]);
    }
    // mirror planes through node 0 can be reached only by tiles whose rings,
    // gathers and pulls go below node 3 of an axis (ring halo GR + 1 at most);
    // every other tile skips the mirror rules (a uniform branch), whose flags
    // would all be zero there
    const bool mir_tile =
        MIR && sd.mirror && (x0 < 4 || (DIM == 3 && y0 < 4) || m0 < 4);
    // tiles whose pulls (output: 1-node halo) or gathers (coefficients: 2-node
    // halo) stay inside the box without wrapping: plain constant offsets there
    const bool xy_in1 = x0 >= 1 && x0 + TX + 1 <= sd.nx && (DIM == 2 || (y0 >= 1 && y0 + TY + 1 <= sd.nyp));
    const bool xy_in2 = x0 >= 2 && x0 + TX + 2 <= sd.nx && (DIM == 2 || (y0 >= 2 && y0 + TY + 2 <= sd.nyp));
    // a tile at a zero-flux wall x = 0 or x = nx - 1 whose pulls stay inside
    // the box along yp (and m, per plane) takes the constant-offset loads too;
    // a lane on the wall reads an in-box node in place of a source beyond it,
    // and the bounce-back below replaces that population, knowing it from two
    // lane flags
    const bool x_walls_only = !per && !mir_tile && !xy_in1 &&
                              (DIM == 2 || (y0 >= 1 && y0 + TY + 1 <= sd.nyp));

    // (no __restrict__: the g loads of B must stay below the barrier that ends A,
    // where they would otherwise be hoisted and held in registers through A)
    const S *Gin = reinterpret_cast<const S *>(sd.g_in);
    S *Gout = reinterpret_cast<S *>(sd.g_out);
    const S *Fin = reinterpret_cast<const S *>(sd.f_in);
    S *Fout = reinterpret_cast<S *>(sd.f_out);
    const PT *__restrict__ Phin = reinterpret_cast<const PT *>(sd.phi_in);
    PT *__restrict__ Phout = reinterpret_cast<PT *>(sd.phi_out);
    // per-direction field base pointers (uniform); node offsets are 32-bit
    auto gfield = [&](int i) { return Gin + (size_t)i * (size_t)sd.fstride; };
    auto gofield = [&](int i) { return Gout + (size_t)i * (size_t)sd.fstride; };
    auto ffield = [&](int i) { return Fin + (size_t)i * (size_t)sd.fstride; };
    auto fofield = [&](int i) { return Fout + (size_t)i * (size_t)sd.fstride; };
    const int pitch = sd.pitch;
    const int mstride = (int)sd.mstride;
    // byte offset from a node to its neighbour -e (uniform)
    auto boff_of = [&](int cx, int cy, int cm, int esize) { return -(cx + cy * pitch + cm * mstride) * esize; };

    // ---- the coefficient nodes of this thread: its own column, maybe one halo node
    const int hx_o = tx + 1, hy_o = (DIM == 3) ? ty + 1 : 0;
    const bool has_h = tid < NHALO;
    int hx_h = 0, hy_h = 0;
    if constexpr (DIM == 3) {
      const int r = tid;
      if (r < HX) {
        hx_h = r;
        hy_h = 0;
      } else if (r < 2 * HX) {
        hx_h = r - HX;
        hy_h = HY - 1;
      } else if (r < 2 * HX + TY) {
        hx_h = 0;
        hy_h = r - 2 * HX + 1;
      } else {
        hx_h = HX - 1;
        hy_h = r - 2 * HX - TY + 1;
      }
    } else {
      hx_h = (tid == 0) ? 0 : HX - 1;
    }

    // box coordinates of coefficient node (hx, hy) of plane pm; false when the
    // node is never pulled from (outside the box, or beyond its one-node halo).
    // The coordinates returned are always inside the box (clamped when invalid).
    // A ghost node at -1 beyond a mirror plane is valid: it holds the mirror
    // image of the node at +1, whose coordinates are returned, with bit k of
    // mir set for each mirrored axis (0 x, 1 yp, 2 m); a pull from beyond the
    // plane then takes the ghost's coefficients like those of any other node.
    auto node_at = [&](int hx, int hy, int pm, int &gx, int &gy, int &gm, int &mir) -> bool {
      gx = x0 - 1 + hx;
      gy = (DIM == 3) ? y0 - 1 + hy : 0;
      gm = pm;
      mir = 0;
      bool ok;
      if (per) {
        ok = gx <= sd.nx && (DIM == 2 || gy <= sd.nyp);
        gx = wrapc(gx, sd.nx);
        gy = (DIM == 3) ? wrapc(gy, sd.nyp) : 0;
        gm = wrapc(gm, sd.nm);
      } else {
        ok = in_range(gx, sd.nx) && (DIM == 2 || in_range(gy, sd.nyp)) && in_range(gm, sd.nm);
        if constexpr (MIR) {
          if (mir_tile) {
            ok = gx >= -1 && gx < sd.nx && (DIM == 2 || (gy >= -1 && gy < sd.nyp)) && gm >= -1 && gm < sd.nm;
            mir = (gx == -1 ? 1 : 0) | (DIM == 3 && gy == -1 ? 2 : 0) | (gm == -1 ? 4 : 0);
            gx = abs(gx);
            gy = abs(gy);
            gm = abs(gm);
          }
        }
      }
      gx = min(max(gx, 0), sd.nx - 1);
      gy = (DIM == 3) ? min(max(gy, 0), sd.nyp - 1) : 0;
      gm = min(max(gm, 0), sd.nm - 1);
      return ok;
    };

    // heat population i pulled by node (gx, gy, gm): stored field d at node src,
    // which sits at ring offset (ox, oy, om) from the node.  Bounce-back for
    // sources outside the box (Eq. Bounce-Back): the opposite population pulled
    // from y + e_i, or the node's own post-collision opposite population.  A
    // source beyond a mirror plane is the mirror node, population OPP[i] (one
    // nonzero component); the ring holds the mirror values at offset -e_i.
    auto heat_src = [&](int gx, int gy, int gm, int i, unsigned &src, int &d, int &ox, int &oy, int &om) {
      const int cx = ex<LU, DIM>(i), cy = ey<LU, DIM>(i), cm = em<LU, DIM>(i);
      int sx = gx - cx, sy = gy - cy, sm = gm - cm;
      bool flip = false;
      if constexpr (MIR) {
        if (mir_tile) {
          flip = (sx < 0) | (sy < 0) | (sm < 0);
          sx = abs(sx);
          sy = abs(sy);
          sm = abs(sm);
        }
      }
      bool in1;
      if (per) {
        sx = wrapc(sx, sd.nx);
        sy = (DIM == 3) ? wrapc(sy, sd.nyp) : 0;
        sm = wrapc(sm, sd.nm);
        in1 = true;
      } else {
        in1 = in_range(sx, sd.nx) && (DIM == 2 || in_range(sy, sd.nyp)) && in_range(sm, sd.nm);
      }
      const int tx_ = gx + cx, ty_ = gy + cy, tm_ = gm + cm;
      const bool in2 = in_range(tx_, sd.nx) && (DIM == 2 || in_range(ty_, sd.nyp)) && in_range(tm_, sd.nm);
      const int rx = in1 ? sx : (in2 ? tx_ : gx);
      const int ry = in1 ? sy : (in2 ? ty_ : gy);
      const int rm = in1 ? sm : (in2 ? tm_ : gm);
      src = lin(sd, rx, ry, rm);
      d = (in1 && !flip) ? i : LU::OPP[i];
      ox = in1 ? -cx : (in2 ? cx : 0);
      oy = in1 ? -cy : (in2 ? cy : 0);
      om = in1 ? -cm : (in2 ? cm : 0);
    };

    // ---- ring staging: plane pm of phi^n, u*, I^n (tile + HF-node halo) -------
    T ph_pf[NLOAD];
    float us_pf[NLOAD];
    int16_t id_pf[NLOAD];
    // Halo coordinates beyond [-HF, n + HF - 1] (ragged last tile) are never read by a
    // node that matters: they are clamped so every load stays in the box.  The
    // FP64 form keeps the in-plane part of each ring entry (the same on every
    // plane) in registers; the offset forms recompute it, which measures faster
    // there (fewer live registers).
    unsigned ring_off[NLOAD];
    bool ring_out[NLOAD];
    auto ring_xy = [&](int j, unsigned &off, bool &out) {
      const int k = min(tid + j * NT, PLANE_F - 1);
      const int px = k % PX, py = k / PX;
      const int rx = min(max(x0 - HF + px, -HF), sd.nx + HF - 1);
      const int ry = (DIM == 3) ? min(max(y0 - HF + py, -HF), sd.nyp + HF - 1) : 0;
      const int gx = ghost(rx, sd.nx, per);
      const int gy = (DIM == 3) ? ghost(ry, sd.nyp, per) : 0;
      off = (unsigned)gy * (unsigned)pitch + (unsigned)gx;
      out = !per && (!in_range(rx, sd.nx) || (DIM == 3 && !in_range(ry, sd.nyp)));
      if constexpr (MIR) {
        if (mir_tile) out = rx >= sd.nx || (DIM == 3 && ry >= sd.nyp);  // mirrored below 0
      }
    };
    if constexpr (!OFF) {
  #pragma unroll
      for (int j = 0; j < NLOAD; ++j) ring_xy(j, ring_off[j], ring_out[j]);
    }
    auto ring_fetch = [&](int pm) {
      const int gm = ghost(pm, sd.nm, per);  // pm is always within [-HF, nm + HF - 1]
      bool mout = !per && !in_range(pm, sd.nm);
      if constexpr (MIR) {
        if (mir_tile) mout = pm >= sd.nm;  // mirrored below 0
      }
      const unsigned mo = (unsigned)gm * (unsigned)mstride;
  #pragma unroll
      for (int j = 0; j < NLOAD; ++j) {
        if (tid + j * NT >= PLANE_F) break;
        unsigned off;
        bool out;
        if constexpr (!OFF) {
          off = ring_off[j];
          out = ring_out[j];
        } else {
          ring_xy(j, off, out);
        }
        const unsigned idx = mo + off;
        ph_pf[j] = T(ldb(Phin, idx * (unsigned)sizeof(PT)));
        if constexpr (OFF) us_pf[j] = ldb(sd.us_in, idx * 4u);
        if constexpr (IDS) id_pf[j] = (mout || out) ? int16_t(0) : ldb(sd.id_in, idx * 2u);
      }
    };
    // phi keeps 5 planes (B of plane m reads plane m-1 while plane m+3 is
    // committed); u* and I^n, read in A only, keep 4.  With GR = 2 the plane
    // committed is m+4 and each ring keeps one plane more.
    auto rs = [](int pm) { return GR == 1 ? (pm + 10) % 5 : (pm + 12) % 6; };
    auto rs4 = [](int pm) { return GR == 1 ? (pm + 8) & 3 : (pm + 10) % 5; };
    auto ring_commit = [&](int pm) {
      const int slot = rs(pm), slot4 = rs4(pm);
  #pragma unroll
      for (int j = 0; j < NLOAD; ++j) {
        const int k = tid + j * NT;
        if (k >= PLANE_F) break;
        phiS[slot][k] = ph_pf[j];
        if constexpr (OFF) usS[slot4][k] = us_pf[j];
        if constexpr (IDS) idS[slot4][k] = id_pf[j];
      }
    };

    // ---- heat populations gathered by a coefficient node (prefetched) ---------
    S kv_o_c[QU], kv_h_c[QU], kv_o_n[QU], kv_h_n[QU];
    auto gather_fetch = [&](int hx, int hy, int pm, S(&kv)[QU]) {
      int gx, gy, gm, mir;
      node_at(hx, hy, pm, gx, gy, gm, mir);  // a ghost gathers as its mirror node
      if (xy_in2 && pm >= 1 && pm + 1 < sd.nm) {
        const unsigned ib = lin(sd, gx, gy, gm) * (unsigned)sizeof(S);
  #pragma unroll
        for (int i = 0; i < QU; ++i)
          kv[i] = ldb(ffield(i), ib + boff_of(ex<LU, DIM>(i), ey<LU, DIM>(i), em<LU, DIM>(i), sizeof(S)));
      } else {
  #pragma unroll
        for (int i = 0; i < QU; ++i) {
          unsigned src;
          int d, ox, oy, om;
          heat_src(gx, gy, gm, i, src, d, ox, oy, om);
          kv[i] = ldb(ffield(d), src * (unsigned)sizeof(S));
        }
      }
    };

    // own-column node of the plane being prepared (nxt) and written (cur)
    T fd_cur[QU], fd_nxt[QU];
    T u_cur = T(0), u_nxt = T(0), us_cur = T(0), us_nxt = T(0);
    int16_t id_cur = 0, id_nxt = 0;

    // ---- A: coefficients of node (hx, hy) of plane pm into coefficient slot ps
    auto param_node = [&](int hx, int hy, int pm, int ps, const S(&kv)[QU], bool own_node) {
      int gx, gy, gm, mir;
      if (!node_at(hx, hy, pm, gx, gy, gm, mir)) return;
      const int pc = (hy + PYO) * PX + (hx + PXO);  // node in the ring
      const int sl0 = rs(pm);
      const T phc = phiS[sl0][pc];
      // gradient of phi^n, lattice units
      T p0 = T(0), p1 = T(0), p2 = T(0);
      if (sd.grad_cd) {
        p0 = (phiS[sl0][pc + 1] - phiS[sl0][pc - 1]) / T(2);
        if constexpr (DIM == 3) {
          p1 = (phiS[sl0][pc + PX] - phiS[sl0][pc - PX]) / T(2);
          p2 = (phiS[rs(pm + 1)][pc] - phiS[rs(pm - 1)][pc]) / T(2);
        } else {
          p1 = (phiS[rs(pm + 1)][pc] - phiS[rs(pm - 1)][pc]) / T(2);
        }
      } else {
        // e_i and -e_i give the same term w_i e_i (e_i . grad phi): one of each
        // pair, with the central difference phi(x + e_i) - phi(x - e_i)
  #pragma unroll
        for (int i = 1; i < QP; ++i) {
          if (LP::OPP[i] < i) continue;
          const int o = ey<LP, DIM>(i) * PX + ex<LP, DIM>(i);
          T dd = phiS[rs(pm + em<LP, DIM>(i))][pc + o] - phiS[rs(pm - em<LP, DIM>(i))][pc - o];
          if constexpr (GR == 2) {
            // second-order upwind pair: 2 [f(x+e) - f(x-e)] - [f(x+2e) - f(x-2e)] / 2
            const T d2 = phiS[rs(pm + 2 * em<LP, DIM>(i))][pc + 2 * o] - phiS[rs(pm - 2 * em<LP, DIM>(i))][pc - 2 * o];
            dd = T(2) * dd - T(0.5) * d2;
          }
          if (LP::E[i][0] != 0) p0 += (T(LP::W[i]) * T(LP::E[i][0])) * dd;
          if (LP::E[i][1] != 0) p1 += (T(LP::W[i]) * T(LP::E[i][1])) * dd;
          if (LP::E[i][2] != 0) p2 += (T(LP::W[i]) * T(LP::E[i][2])) * dd;
        }
        p0 *= T(LP::INV_E2);
        p1 *= T(LP::INV_E2);
        p2 *= T(LP::INV_E2);
      }
      // crystal index, Jacobi dilation by one node per step
      int16_t idn = 0;
      if constexpr (IDS) {
        idn = idS[rs4(pm)][pc];
        const T r2 = (p0 * p0 + p1 * p1) + p2 * p2;
        if (idn == 0 && r2 > pick<T>(sd.xi2, sd.xi2_f)) {
          T best = T(-1e30);
          int16_t bid = 0;
  #pragma unroll
          for (int i = 1; i < QP; ++i) {
            const int o = ey<LP, DIM>(i) * PX + ex<LP, DIM>(i);
            const int16_t nb = idS[rs4(pm + em<LP, DIM>(i))][pc + o];
            const T ph = phiS[rs(pm + em<LP, DIM>(i))][pc + o];
            if (nb != 0 && (ph > best || (ph == best && nb < bid))) {
              best = ph;
              bid = nb;
            }
          }
          idn = bid;
        }
      }
      // u^n = sum_i f_i^n(x), f_i^n(x) = f*_i(x - e_i) (prefetched in kv)
      T fd[QU];
      T us_self = T(0);
      if constexpr (OFF) us_self = usS[rs4(pm)][pc];
      T usum = T(0);
      // the node's heat sources all lie inside the box (and beyond no plane):
      // each sits at the ring offset -e_i, a constant
      const bool inner = HEAT_CONST && xy_in2 && pm >= 1 && pm + 1 < sd.nm;
  #pragma unroll
      for (int i = 0; i < QU; ++i) {
        const T kvv = T(kv[i]);
        if constexpr (OFF) {
          unsigned src;
          int d, ox, oy, om;
          if (inner) {
            ox = -ex<LU, DIM>(i);
            oy = -ey<LU, DIM>(i);
            om = -em<LU, DIM>(i);
          } else {
            heat_src(gx, gy, gm, i, src, d, ox, oy, om);
          }
          if constexpr (MIR) {
            // a ghost node: its mirror node's source, seen from the ghost
            if (mir_tile) {
              if (mir & 1) ox = -ox;
              if (mir & 2) oy = -oy;
              if (mir & 4) om = -om;
            }
          }
          const float usrc = usS[rs4(pm + om)][pc + oy * PX + ox];
          fd[i] = T(LU::W[i] * SC) * (usrc - us_self) + kvv;
        } else {
          fd[i] = kvv;
        }
        usum = (i == 0) ? fd[0] : usum + fd[i];
      }
      const T un = OFF ? us_self + usum * T(1.0 / SC) : usum;
      // a_s, N, relaxation and source
      T a, Nx, Ny, Nz;
      if constexpr (IDS) {
        if (staged)
          flux<T>(idn > 0 ? &tabS[idn] : nullptr, p0, p1, p2, a, Nx, Ny, Nz);
        else
          flux<T>(idn > 0 ? sd.aniso + idn : nullptr, p0, p1, p2, a, Nx, Ny, Nz);
      } else {  // one entry for every node
        flux<T>((ConstAniso *)sd.aniso, p0, p1, p2, a, Nx, Ny, Nz);
      }
      const T a2 = a * a;
      const T kph = pick<T>(sd.kphi, sd.kphi_f);
      const T om_ = rcp(a2 * kph + T(0.5));
      const T o1 = T(1) - phc * phc;
      const T Qs = (phc - pick<T>(sd.lambda, sd.lambda_f) * un * o1) * o1 * pick<T>(sd.s, sd.s_f);
      const T cC = -om_ * kph;
      const int node = hy * HX + hx;
      const T ia2 = rcp(a2);
      if constexpr (FOLD) {
        // what a pull from this node needs, with 1/a^2 folded in:
        //   M = 1 - 1/a^2, A' = (1 - w)/a^2, Kc = SC cC N / a^2, K0 = SC (phi + Q s)/a^2
        const T kc = T(SC) * ia2 * cC;
        parS[ps][0][node] = T(1) - ia2;
        parS[ps][1][node] = ia2 * (T(1) - om_);
        parS[ps][2][node] = kc * Nx;
        parS[ps][3][node] = kc * Ny;  // in 2D the lattice y is the march axis
        if constexpr (DIM == 3) parS[ps][4][node] = kc * Nz;
        parS[ps][NP - 1][node] = (T(SC) * ia2) * (phc + Qs);
      } else {
        // A = 1 - w, B = w phi + Q s (offsets: Q s), C = cC N and 1/a^2
        parS[ps][0][node] = T(1) - om_;
        parS[ps][1][node] = OFF ? Qs : om_ * phc + Qs;
        parS[ps][2][node] = cC * Nx;
        parS[ps][3][node] = cC * Ny;
        if constexpr (DIM == 3) parS[ps][4][node] = cC * Nz;
        parS[ps][NP - 1][node] = ia2;
      }
      if (own_node) {
  #pragma unroll
        for (int i = 0; i < QU; ++i) fd_nxt[i] = fd[i];
        u_nxt = un;
        us_nxt = us_self;
        id_nxt = idn;
      }
    };

    // base + the component of Kc (offsets) or C (FP64) along direction i of the
    // phi lattice.  The sum starts from the first nonzero term: adding a term
    // to +0 is not an identity in IEEE arithmetic (-0 + 0 = +0), so the
    // compiler would keep that addition as an instruction.
    auto addEC = [&](int i, int ps, int node, T base) -> T {
      T v = T(0);
      bool any = false;
      auto term = [&](int c, int k) {
        if (c == 0) return;
        const T t = T(c) * parS[ps][k][node];
        v = any ? v + t : t;
        any = true;
      };
      term(LP::E[i][0], 2);
      term(LP::E[i][1], 3);
      if constexpr (DIM == 3) term(LP::E[i][2], 4);
      return any ? base + v : base;
    };

    const int gx_o = x0 + tx;
    const int gy_o = y0 + ty;
    const bool own = in_range(gx_o, sd.nx) && (DIM == 2 || in_range(gy_o, sd.nyp));
    // on a wall x = 0 / x = nx - 1 of such a tile (false on every other tile)
    const bool at_x0 = x_walls_only && gx_o == 0, at_x1 = x_walls_only && gx_o == sd.nx - 1;
    const int nodeo = hy_o * HX + hx_o;
    const int pco = (hy_o + PYO) * PX + (hx_o + PXO);

    int sp = 0, sc = 1, sn = 2;  // coefficient slots of planes m-1, m, m+1

    // ---- B: write node y of plane m ---------------------------------------------
    auto output = [&](int m, bool walls) {
      const unsigned iy = lin(sd, gx_o, gy_o, m);
      const unsigned iyb = iy * (unsigned)sizeof(S);
      S gy_r[QP], gx_r[QP];
      bool unk[QP];
      // one batch of loads: g_i(y) and g_i(y - e_i)
      const bool fast = (xy_in1 || x_walls_only) && m >= 1 && m + 1 < sd.nm;
      // Each population is read twice, as the own value of its node and as the
      // upstream value of the node downstream. The second of the two reads
      // carries the non-temporal hint, so that L2 keeps the lines still to be
      // read again: for e_m = +1 the upstream row (plane m - 1, read as its own
      // one plane earlier), for e_m = -1 the own row (read as upstream one
      // plane earlier). The choice is made at compile time; a hinted and a
      // plain load of one address would be merged into a plain one.
      auto load_fast = [&]() {
        // a lane on a wall reads the source one node further in along x (its
        // own column): an address inside the box, for a value the bounce-back
        // replaces
        const unsigned iyb_p = at_x0 ? iyb + (unsigned)sizeof(S) : iyb;  // sources of e_x = +1
        const unsigned iyb_m = at_x1 ? iyb - (unsigned)sizeof(S) : iyb;  // sources of e_x = -1
        static_for<0, QP>([&](auto ic) {
          constexpr int i = decltype(ic)::value;
          constexpr int cx = ex<LP, DIM>(i);
          unk[i] = (cx == 1 && at_x0) || (cx == -1 && at_x1);
          const unsigned bx = (cx == 1 ? iyb_p : (cx == -1 ? iyb_m : iyb)) +
                              boff_of(cx, ey<LP, DIM>(i), em<LP, DIM>(i), sizeof(S));
          if constexpr (em<LP, DIM>(i) == -1)
            gy_r[i] = ldb_nt(gfield(i), iyb);
          else
            gy_r[i] = ldb(gfield(i), iyb);
          if constexpr (em<LP, DIM>(i) == 1)
            gx_r[i] = ldb_nt(gfield(i), bx);
          else
            gx_r[i] = ldb(gfield(i), bx);
        });
      };
      auto load_generic = [&](auto flip) {
        constexpr bool FLIP = decltype(flip)::value;
        static_for<0, QP>([&](auto ic) {
          constexpr int i = decltype(ic)::value;
          constexpr int cx = ex<LP, DIM>(i), cy = ey<LP, DIM>(i), cm = em<LP, DIM>(i);
          int sx = gx_o - cx, sy = gy_o - cy, sm = m - cm;
          int fl = 0;  // mirrored axes of the source (bit 0 x, 1 yp, 2 m)
          if constexpr (FLIP) {
            // only a component +1 can cross a plane through node 0: the
            // flags of the other components are zero at compile time; a
            // simulation without mirror planes never sets them
            const bool mir = mir_tile;
            const bool fx = mir && cx == 1 && gx_o == 0, fy = mir && DIM == 3 && cy == 1 && gy_o == 0,
                       fm = mir && cm == 1 && m == 0;
            fl = (fx ? 1 : 0) | (fy ? 2 : 0) | (fm ? 4 : 0);
            if (fx) sx = 1;
            if (fy) sy = 1;
            if (fm) sm = 1;
          }
          if (per) {
            sx = wrapc(sx, sd.nx);
            sy = (DIM == 3) ? wrapc(sy, sd.nyp) : 0;
            sm = wrapc(sm, sd.nm);
            unk[i] = false;
          } else {
            unk[i] = !(in_range(sx, sd.nx) && (DIM == 2 || in_range(sy, sd.nyp)) && in_range(sm, sd.nm));
          }
          const unsigned isrc = unk[i] ? iy : lin(sd, sx, sy, sm);
          if constexpr (cm == -1)
            gy_r[i] = ldb_nt(gfield(i), iyb);
          else
            gy_r[i] = ldb(gfield(i), iyb);
          if constexpr (FLIP) {
            gx_r[i] = ldb(gfield(mirror_sel<LP, DIM>(i, fl)), isrc * (unsigned)sizeof(S));
          } else {
            if constexpr (cm == 1)
              gx_r[i] = ldb_nt(gfield(i), isrc * (unsigned)sizeof(S));
            else
              gx_r[i] = ldb(gfield(i), isrc * (unsigned)sizeof(S));
          }
        });
      };
      T phy, scphy;
      T d[QP];
      // the pulls (a source beyond a mirror plane is its ghost coefficient node)
      auto pull = [&]() {
    #pragma unroll
        for (int i = 0; i < QP; ++i) {
          const int cx = ex<LP, DIM>(i), cy = ey<LP, DIM>(i), cm = em<LP, DIM>(i);
          const int ps = (cm == 1) ? sp : ((cm == -1) ? sn : sc);
          const int node = nodeo - cy * HX - cx;
          const T gy_ = ST::ld(&gy_r[i]);
          const T gx_ = ST::ld(&gx_r[i]);
          if constexpr (FOLD) {
            // d = h(y) + [h*(x) + w_i (phi(x) - phi(y)) - h(y)]/a^2(x)
            //   = M h(y) + A' h(x) + w_i (K0 + e_i.Kc - SC phi(y)/a^2(x))
            const T Mc = parS[ps][0][node];
            const T Ap = parS[ps][1][node];
            const T t = scphy * (Mc - T(1)) + addEC(i, ps, node, parS[ps][NP - 1][node]);
            d[i] = Mc * gy_ + (T(LP::W[i]) * t + Ap * gx_);
          } else if constexpr (OFF) {
            // d = h(y) + [h*(x) + w_i SC (phi(x) - phi(y)) - h(y)]/a^2(x),
            // h*(x) = A h(x) + w_i SC (B + e_i.C)
            const T phx = phiS[rs(m - cm)][pco - cy * PX - cx];
            const T hs = parS[ps][0][node] * gx_ + T(LP::W[i] * SC) * addEC(i, ps, node, parS[ps][1][node]);
            d[i] = gy_ + parS[ps][NP - 1][node] * (T(LP::W[i] * SC) * (phx - phy) + hs - gy_);
          } else {
            const T gs = parS[ps][0][node] * gx_ + T(LP::W[i]) * addEC(i, ps, node, parS[ps][1][node]);
            d[i] = gy_ + parS[ps][NP - 1][node] * (gs - gy_);
          }
        }
      };
      if constexpr (MIR) {
        // the generic loads take a mirrored population where the source lies
        // beyond a mirror plane (the flags are zero elsewhere, and for members
        // of an ensemble without mirror planes); the pulls take the ghost
        // coefficient nodes beyond the plane as they are.  One generic path
        // instead of two leaves the mirror instances fewer registers.
        if (fast)
          load_fast();
        else
          load_generic(std::true_type{});
        phy = phiS[rs(m)][pco];
        scphy = T(SC) * phy;
        pull();
      } else {
        if (fast)
          load_fast();
        else
          load_generic(std::false_type{});
        phy = phiS[rs(m)][pco];
        scphy = T(SC) * phy;
        pull();
      }
      if (walls) {
        // bounce-back: an unknown incoming population takes the opposite one; if
        // that is unknown too, the local post-collision opposite population
        // (folded offsets: h*_j(y) = a^2 [A' h_j(y) + w_j (K0 + e_j.Kc)] - w_j SC phi(y);
        // otherwise h*_j(y) = A h_j(y) + w_j SC (B + e_j.C))
        T dn[QP];
        const T a2o = FOLD ? rcp(T(1) - parS[sc][0][nodeo]) : T(0);
  #pragma unroll
        for (int i = 0; i < QP; ++i) {
          const int j = LP::OPP[i];
          T loc;
          if constexpr (FOLD)
            loc = a2o * (parS[sc][1][nodeo] * ST::ld(&gy_r[j]) +
                         T(LP::W[j]) * addEC(j, sc, nodeo, parS[sc][NP - 1][nodeo])) -
                  T(LP::W[j]) * scphy;
          else  // (SC is 1 for FP64)
            loc = parS[sc][0][nodeo] * ST::ld(&gy_r[j]) + T(LP::W[j] * SC) * addEC(j, sc, nodeo, parS[sc][1][nodeo]);
          dn[i] = unk[i] ? (unk[j] ? loc : d[j]) : d[i];
        }
  #pragma unroll
        for (int i = 0; i < QP; ++i) d[i] = dn[i];
      }
      T sum = d[0];  // (not 0 + d[0]: see addEC)
  #pragma unroll
      for (int i = 1; i < QP; ++i) sum += d[i];
      const T phn = OFF ? phy + sum * T(1.0 / SC) : sum;
      if constexpr (OFF) {
        // the offsets of a node sum to zero. With COMP the rest offset is stored
        // as minus the sum of the others as rounded, so their rounding errors
        // cancel in the next step's phi; the rest offset itself stays near
        // zero, so its own rounding is small
        T rsum = T(0);
  #pragma unroll
        for (int i = 1; i < QP; ++i) {
          const S q = ST::enc(d[i] - T(LP::W[i]) * sum);
          nt_store(reinterpret_cast<S *>(reinterpret_cast<char *>(gofield(i)) + iyb), q);
          rsum = (i == 1) ? ST::dec(q) : rsum + ST::dec(q);
        }
        ST::st(reinterpret_cast<S *>(reinterpret_cast<char *>(gofield(0)) + iyb),
               ST::COMP ? -rsum : d[0] - T(LP::W[0]) * sum);
      } else {
  #pragma unroll
        for (int i = 0; i < QP; ++i)
          ST::st(reinterpret_cast<S *>(reinterpret_cast<char *>(gofield(i)) + iyb), d[i]);
      }
      stb(Phout, iy * (unsigned)sizeof(PT), (PT)phn);

      // heat equation at y: BGK toward w_i u^n with source (phi^{n+1} - phi^n)/2
      const T half_dphi = T(0.5) * (phn - phy);
      const T om_u = pick<T>(sd.omega_u, sd.omega_u_f);
      if constexpr (OFF) {
        const T Sm = u_cur - us_cur;  // sum of the decoded offsets, true units
        const T keep = T(1) - om_u;
        T rsum = T(0);  // as for g: the rest population balances the rounded others
  #pragma unroll
        for (int i = 1; i < QU; ++i) {
          const S q = ST::enc(keep * (fd_cur[i] - T(LU::W[i] * SC) * Sm));
          nt_store(reinterpret_cast<S *>(reinterpret_cast<char *>(fofield(i)) + iyb), q);
          rsum = (i == 1) ? ST::dec(q) : rsum + ST::dec(q);
        }
        ST::st(reinterpret_cast<S *>(reinterpret_cast<char *>(fofield(0)) + iyb),
               ST::COMP ? -rsum : keep * (fd_cur[0] - T(LU::W[0] * SC) * Sm));
        stb(sd.us_out, iy * 4u, float(u_cur + half_dphi));
      } else {
  #pragma unroll
        for (int i = 0; i < QU; ++i) {
          const T fi = fd_cur[i];
          ST::st(reinterpret_cast<S *>(reinterpret_cast<char *>(fofield(i)) + iyb),
                 fi - om_u * (fi - T(LU::W[i]) * u_cur) + T(LU::W[i]) * half_dphi);
        }
      }
      if constexpr (IDS) stb(sd.id_out, iy * 2u, id_cur);
    };

    // planes whose pulls can meet a wall (only then is bounce-back applied)
    const bool xy_walls = !per && !xy_in1;
    auto walls_at = [&](int m) { return !per && (xy_walls || m == 0 || m == sd.nm - 1); };

    // ---- warm-up ----------------------------------------------------------------
    // ring planes m0-1-GR .. m0+GR; coefficients of planes m0-1 and m0 (gathers
    // loaded on the spot); then ring plane m0+GR+1 and the gathers of plane m0+1
    for (int pm = m0 - 1 - GR; pm <= m0 + GR; ++pm) {
      ring_fetch(pm);
      ring_commit(pm);
    }
    __syncthreads();
    for (int pm = m0 - 1; pm <= m0; ++pm) {
      const int ps = (pm == m0) ? sc : sp;
      gather_fetch(hx_o, hy_o, pm, kv_o_c);
      if (has_h) gather_fetch(hx_h, hy_h, pm, kv_h_c);
      param_node(hx_o, hy_o, pm, ps, kv_o_c, true);
      if (has_h) param_node(hx_h, hy_h, pm, ps, kv_h_c, false);
    }
    __syncthreads();
    ring_fetch(m0 + GR + 1);
    ring_commit(m0 + GR + 1);
    gather_fetch(hx_o, hy_o, m0 + 1, kv_o_c);
    if (has_h) gather_fetch(hx_h, hy_h, m0 + 1, kv_h_c);
  #pragma unroll
    for (int i = 0; i < QU; ++i) fd_cur[i] = fd_nxt[i];
    u_cur = u_nxt;
    us_cur = us_nxt;
    id_cur = id_nxt;
    __syncthreads();

    for (int m = m0; m < m1; ++m) {
      // loads for the next iterations: ring plane m+3, gathers of plane m+2
      const bool more_ring = m + GR + 2 <= m1 + GR;
      if (more_ring) ring_fetch(m + GR + 2);
      if (m + 2 <= m1) {
        gather_fetch(hx_o, hy_o, m + 2, kv_o_n);
        if (has_h) gather_fetch(hx_h, hy_h, m + 2, kv_h_n);
      }
      // A: coefficients of plane m+1 (LDS and prefetched registers only)
      param_node(hx_o, hy_o, m + 1, sn, kv_o_c, true);
      if (has_h) param_node(hx_h, hy_h, m + 1, sn, kv_h_c, false);
      __syncthreads();
      // B: plane m
      if (own) output(m, walls_at(m));
      if (more_ring) ring_commit(m + GR + 2);
      __syncthreads();
      // rotate the coefficient ring, the own-column state and the prefetches
      const int t = sp;
      sp = sc;
      sc = sn;
      sn = t;
  #pragma unroll
      for (int i = 0; i < QU; ++i) {
        fd_cur[i] = fd_nxt[i];
        kv_o_c[i] = kv_o_n[i];
        kv_h_c[i] = kv_h_n[i];
      }
      u_cur = u_nxt;
      us_cur = us_nxt;
      id_cur = id_nxt;
    }
    if constexpr (!BATCH) break;
  }
}


// ---- launchers, instantiated once per value of MIR (one source file each) ----
template <int K, int TY, class ST, bool IDS, bool MIR, int GR = 1>
static hipError_t launch_step_t(const SimDev &sd, const TileDev &tc, hipStream_t st) {
  const int nblocks = (int)part_blocks(tc, LatOf<K>::DIM == 3);
  if (nblocks == 0) return hipSuccess;
  dim3 block(64, LatOf<K>::DIM == 3 ? TY : 1);
  hipLaunchKernelGGL((step_kernel<K, TY, ST, IDS, false, MIR, GR>), dim3(nblocks), block, 0, st, sd, tc, nullptr,
                     nullptr, 0);
  return hipGetLastError();
}

// The second-order upwind gradient (GR = 2): 4-row tiles in 3D, and 12-row
// tiles for the FP32-arithmetic forms; with or without the index field; no
// mirror planes; single simulations.
template <int K, class ST, bool IDS>
static hipError_t launch_step_up2_ids(const SimDev &sd, const TileDev &tc, hipStream_t st) {
  if constexpr (LatOf<K>::DIM == 2) {
    return launch_step_t<K, 1, ST, IDS, false, 2>(sd, tc, st);
  } else {
    if (tc.ty == 4) return launch_step_t<K, 4, ST, IDS, false, 2>(sd, tc, st);
    if constexpr (!std::is_same<ST, StF64>::value) {
      if (tc.ty == 12) return launch_step_t<K, 12, ST, IDS, false, 2>(sd, tc, st);
    }
    return hipErrorInvalidValue;
  }
}
template <int K, class ST> static hipError_t launch_step_up2_st(const SimDev &sd, const TileDev &tc, hipStream_t st) {
  return sd.use_ids ? launch_step_up2_ids<K, ST, true>(sd, tc, st) : launch_step_up2_ids<K, ST, false>(sd, tc, st);
}
template <int K> static hipError_t launch_step_up2_k(int storage, const SimDev &sd, const TileDev &tc, hipStream_t st) {
  switch (storage) {
    case 0: return launch_step_up2_st<K, StF64>(sd, tc, st);
    case 1: return launch_step_up2_st<K, StF32>(sd, tc, st);
    case 2: return launch_step_up2_st<K, StF16>(sd, tc, st);
  }
  return hipErrorInvalidValue;
}

template <int K, class ST, bool IDS, bool MIR>
static hipError_t launch_step_ty(const SimDev &sd, const TileDev &tc, hipStream_t st) {
  if constexpr (LatOf<K>::DIM == 2) {
    return launch_step_t<K, 1, ST, IDS, MIR>(sd, tc, st);
  } else {
    switch (tc.ty) {
      case 4: return launch_step_t<K, 4, ST, IDS, MIR>(sd, tc, st);
      case 8: return launch_step_t<K, 8, ST, IDS, MIR>(sd, tc, st);
      case 12:
        if constexpr (!std::is_same<ST, StF64>::value) return launch_step_t<K, 12, ST, IDS, MIR>(sd, tc, st);
        return hipErrorInvalidValue;
      default: return hipErrorInvalidValue;
    }
  }
}

template <int K, class ST, bool MIR>
static hipError_t launch_step_st(const SimDev &sd, const TileDev &tc, hipStream_t st) {
  return sd.use_ids ? launch_step_ty<K, ST, true, MIR>(sd, tc, st) : launch_step_ty<K, ST, false, MIR>(sd, tc, st);
}

template <int K, bool MIR>
static hipError_t launch_step_k(int storage, const SimDev &sd, const TileDev &tc, hipStream_t st) {
  switch (storage) {
    case 0: return launch_step_st<K, StF64, MIR>(sd, tc, st);
    case 1: return launch_step_st<K, StF32, MIR>(sd, tc, st);
    case 2: return launch_step_st<K, StF16, MIR>(sd, tc, st);
  }
  return hipErrorInvalidValue;
}

template <bool MIR>
static hipError_t launch_step_m(int lattice, int storage, const SimDev &sd, const TileDev &tc, hipStream_t st) {
  switch (lattice) {
    case 0: return launch_step_k<0, MIR>(storage, sd, tc, st);
    case 1: return launch_step_k<1, MIR>(storage, sd, tc, st);
    case 2: return launch_step_k<2, MIR>(storage, sd, tc, st);
  }
  return hipErrorInvalidValue;
}

template <class ST, bool IDS, bool MIR>
static hipError_t launch_batch_t(const SimDev *sims, const BatchItem *items, int n_items, int grid, hipStream_t st) {
  hipLaunchKernelGGL((step_kernel<0, 1, ST, IDS, true, MIR, 1>), dim3(grid), dim3(64), 0, st, SimDev{}, TileDev{}, sims,
                     items, n_items);
  return hipGetLastError();
}

template <bool MIR>
static hipError_t launch_batch_m(int storage, bool ids, const SimDev *sims, const BatchItem *items, int n_items,
                                 int grid, hipStream_t st) {
  if (n_items < 1 || grid < 1) return hipErrorInvalidValue;
  switch (storage) {
    case 0: return ids ? launch_batch_t<StF64, true, MIR>(sims, items, n_items, grid, st)
                       : launch_batch_t<StF64, false, MIR>(sims, items, n_items, grid, st);
    case 1: return ids ? launch_batch_t<StF32, true, MIR>(sims, items, n_items, grid, st)
                       : launch_batch_t<StF32, false, MIR>(sims, items, n_items, grid, st);
    case 2: return ids ? launch_batch_t<StF16, true, MIR>(sims, items, n_items, grid, st)
                       : launch_batch_t<StF16, false, MIR>(sims, items, n_items, grid, st);
  }
  return hipErrorInvalidValue;
}

template <class ST, bool IDS, bool MIR> static int batch_occupancy_t() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_kernel<0, 1, ST, IDS, true, MIR, 1>, 64, 0) != hipSuccess)
    return 0;
  return nb;
}

template <bool MIR> static int batch_blocks_per_cu_m(int storage, bool ids) {
  switch (storage) {
    case 0: return ids ? batch_occupancy_t<StF64, true, MIR>() : batch_occupancy_t<StF64, false, MIR>();
    case 1: return ids ? batch_occupancy_t<StF32, true, MIR>() : batch_occupancy_t<StF32, false, MIR>();
    case 2: return ids ? batch_occupancy_t<StF16, true, MIR>() : batch_occupancy_t<StF16, false, MIR>();
  }
  return 0;
}

}  // namespace lbpf

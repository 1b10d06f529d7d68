// Fused coupled step (phase field, then heat) for gfx950.
//
// One launch advances one simulation by one time step.  A work-group owns a
// 64 x TY tile of the plane perpendicular to the march axis m (z in 3D, y in
// 2D; TY = 1 in 2D) and walks `chunk` planes along m.  Per plane it
//   1. stages phi^n of plane m+2 (tile + 2-node halo) in an LDS ring of 4 planes,
//   2. computes, for plane m+1 on the tile + 1-node halo, the gradient of phi
//      (directional derivatives, Eqs. Def_DeriveeDirectionnelle and
//      Grad_DF-Centree, or central differences), the crystal index update
//      (Sec. 4.3), u^n by gathering the heat populations, a_s and N
//      (Eq. TermesAnisotropes), eta_phi (Eq. LBE_RelaxationTime) and Q_phi
//      (Eq. LBE_SourceTerm), folded into six per-node coefficients kept in an
//      LDS ring of 3 planes,
//   3. for every node y of plane m pulls g_i from x = y - e_i with the nonlocal
//      a_s^2 form of Eq. LBE_Eq_Phase,
//        g_i(y, t+1) = g_i(y, t) + [g*_i(x) - g_i(y, t)] / a_s^2(x),
//        g*_i(x)    = (1 - w) g_i(x) + w g^(0)_i(x) + w_i Q_phi(x) dt/tau0,
//      applies bounce-back on the walls (Eq. Bounce-Back), sums phi^{n+1}
//      (Eq. Def_M0_Phi), then collides the heat populations with the source
//      (phi^{n+1} - phi^n)/2 (Eqs. LBE_Eq_Temp, Source_Tempr) and stores them
//      post-collision at y ("stream on read": the next step pulls them).
// Every distribution is read from HBM once and written once per step; the
// second, shifted read of g_i(x) and the halo gathers hit L2.
//
// Offset storage (FP32 arithmetic): h_i = g_i - w_i phi and
// k_i = f*_i - w_i u* are stored in FP32 or FP16 beside FP32 phi and u*; the
// update is written on these small quantities:
//   h*_i(x) = A h_i(x) + w_i (Q s + e_i . C),  A = 1 - w,  C = -w (Dphi/e^2) N
//   d_i     = h_i(y) + [w_i (phi(x) - phi(y)) + h*_i(x) - h_i(y)] / a^2(x)
//   phi^{n+1}(y) = phi^n(y) + sum_i d_i,   h_i^{n+1}(y) = d_i - w_i sum_j d_j.
#include "lbpf_common.hpp"
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

template <int DIM, int TY, class ST, bool IDS>
__global__ __launch_bounds__(64 * TY) void step_kernel(SimDev sd, TileDev tc) {
  using T = typename ST::T;
  using LP = typename Lat<DIM>::P;
  using LU = typename Lat<DIM>::U;
  using S = typename ST::S;
  constexpr int TX = 64;
  constexpr int NT = TX * TY;
  constexpr int HX = TX + 2, HY = (DIM == 3 ? TY + 2 : 1);
  constexpr int PX = TX + 4, PY = (DIM == 3 ? TY + 4 : 1);
  constexpr int NP = DIM + 3;  // A, B, C[DIM], 1/a^2
  constexpr int PLANE_P = HX * HY;
  constexpr int PLANE_F = PX * PY;
  constexpr int PYO = (DIM == 3) ? 1 : 0;  // row offset of a coefficient node in the phi ring
  constexpr int QP = LP::Q, QU = LU::Q;

  __shared__ T phiS[4][PLANE_F];
  __shared__ T parS[3][NP][PLANE_P];
  __shared__ int16_t idS[IDS ? 4 : 1][IDS ? PLANE_F : 1];

  const int tx = threadIdx.x;
  const int ty = (DIM == 3) ? threadIdx.y : 0;
  const int tid = ty * TX + tx;

  int L = xcd_remap(blockIdx.x, gridDim.x);
  const int tile_x = L % tc.tiles_x;
  L /= tc.tiles_x;
  const int tile_y = L % tc.tiles_y;
  const int chunk = L / tc.tiles_y;
  const int x0 = tile_x * TX;
  const int y0 = (DIM == 3) ? tile_y * TY : 0;
  const int m0 = chunk * tc.chunk;
  const int m1 = min(m0 + tc.chunk, sd.nm);
  const int per = sd.periodic;

  const S *Gin = reinterpret_cast<const S *>(sd.g_in);
  S *Gout = reinterpret_cast<S *>(sd.g_out);
  S *Fout = reinterpret_cast<S *>(sd.f_out);
  const typename ST::P *Phin = reinterpret_cast<const typename ST::P *>(sd.phi_in);
  typename ST::P *Phout = reinterpret_cast<typename ST::P *>(sd.phi_out);

  // ---- stage phi^n (and I^n) of plane pm, tile + 2-node halo --------------
  auto load_plane = [&](int pm) {
    const int slot = pm & 3;
    const int gm = ghost(pm, sd.nm, per);  // pm is always within [-2, nm + 1]
    const bool mout = !in_range(pm, sd.nm);
    for (int k = tid; k < PLANE_F; k += NT) {
      const int px = k % PX, py = k / PX;
      // halo coordinates beyond [-2, n + 1] (ragged last tile) are never read
      // by a node that matters: clamp them so every load stays in the box
      const int rx = min(max(x0 - 2 + px, -2), sd.nx + 1);
      const int ry = (DIM == 3) ? min(max(y0 - 2 + py, -2), sd.nyp + 1) : 0;
      const int gx = ghost(rx, sd.nx, per);
      const int gy = (DIM == 3) ? ghost(ry, sd.nyp, per) : 0;
      const long long idx = lin(sd, gx, gy, gm);
      phiS[slot][k] = T(Phin[idx]);
      if constexpr (IDS) {
        const bool out = !per && (mout || !in_range(rx, sd.nx) || (DIM == 3 && !in_range(ry, sd.nyp)));
        idS[slot][k] = out ? int16_t(0) : sd.id_in[idx];
      }
    }
  };

  // registers describing the own-column node of the plane being prepared
  // (nxt) and of the plane being written (cur)
  T fd_cur[QU], fd_nxt[QU];
  T u_cur = T(0), u_nxt = T(0), us_cur = T(0), us_nxt = T(0);
  int16_t id_cur = 0, id_nxt = 0;

  // ---- per-node coefficients of plane pm into parameter slot ps -----------
  auto compute_params = [&](int pm, int ps) {
    for (int k = tid; k < PLANE_P; k += NT) {
      int hx, hy;
      if (k < NT) {  // own columns first: thread tid gets its own column
        hx = (k % TX) + 1;
        hy = (DIM == 3) ? (k / TX) + 1 : 0;
      } else {
        const int r = k - NT;
        if constexpr (DIM == 3) {
          if (r < HX) {
            hx = r;
            hy = 0;
          } else if (r < 2 * HX) {
            hx = r - HX;
            hy = HY - 1;
          } else if (r < 2 * HX + TY) {
            hx = 0;
            hy = r - 2 * HX + 1;
          } else {
            hx = HX - 1;
            hy = r - 2 * HX - TY + 1;
          }
        } else {
          hx = (r == 0) ? 0 : HX - 1;
          hy = 0;
        }
      }
      int gx = x0 - 1 + hx, gy = (DIM == 3) ? y0 - 1 + hy : 0, gm = pm;
      // only nodes within one node of the box are ever pulled from
      if (gx > sd.nx || (DIM == 3 && gy > sd.nyp)) continue;
      if (per) {
        gx = wrapc(gx, sd.nx);
        if (DIM == 3) gy = wrapc(gy, sd.nyp);
        gm = wrapc(gm, sd.nm);
      } else if (!in_range(gx, sd.nx) || (DIM == 3 && !in_range(gy, sd.nyp)) || !in_range(gm, sd.nm)) {
        continue;  // outside the box: never pulled from (bounce-back instead)
      }
      const int pc = (hy + PYO) * PX + (hx + 1);  // node in the phi ring
      const T phc = phiS[pm & 3][pc];
      // gradient of phi^n, lattice units
      T p0 = T(0), p1 = T(0), p2 = T(0);
      if (sd.grad_cd) {
        p0 = (phiS[pm & 3][pc + 1] - phiS[pm & 3][pc - 1]) / T(2);
        if constexpr (DIM == 3) {
          p1 = (phiS[pm & 3][pc + PX] - phiS[pm & 3][pc - PX]) / T(2);
          p2 = (phiS[(pm + 1) & 3][pc] - phiS[(pm - 1) & 3][pc]) / T(2);
        } else {
          p1 = (phiS[(pm + 1) & 3][pc] - phiS[(pm - 1) & 3][pc]) / T(2);
        }
      } else {
#pragma unroll
        for (int i = 1; i < QP; ++i) {
          const int o = ey<LP, DIM>(i) * PX + ex<LP, DIM>(i);
          const T dd = (phiS[(pm + em<LP, DIM>(i)) & 3][pc + o] - phiS[(pm - em<LP, DIM>(i)) & 3][pc - o]) / T(2);
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
        idn = idS[pm & 3][pc];
        const T r2 = (p0 * p0 + p1 * p1) + p2 * p2;
        if (idn == 0 && r2 > T(sd.xi2)) {
          T best = T(-1e300);
          int16_t bid = 0;
#pragma unroll
          for (int i = 1; i < QP; ++i) {
            const int o = ey<LP, DIM>(i) * PX + ex<LP, DIM>(i);
            const int16_t nb = idS[(pm + em<LP, DIM>(i)) & 3][pc + o];
            const T ph = phiS[(pm + em<LP, DIM>(i)) & 3][pc + o];
            if (nb != 0 && (ph > best || (ph == best && nb < bid))) {
              best = ph;
              bid = nb;
            }
          }
          idn = bid;
        }
      }
      // u^n from the stored heat populations
      T fd[QU];
      T us_self;
      const T un = gather_u<DIM, ST>(sd, gx, gy, gm, fd, us_self);
      // a_s, N, relaxation and source
      const AnisoDev *A = IDS ? (idn > 0 ? sd.aniso + idn : nullptr) : sd.aniso;
      T a, Nx, Ny, Nz;
      flux<T>(A, p0, p1, p2, a, Nx, Ny, Nz);
      const T a2 = a * a;
      const T om = T(1) / (a2 * T(sd.kphi) + T(0.5));
      const T o1 = T(1) - phc * phc;
      const T Qs = (phc - T(sd.lambda) * un * o1) * o1 * T(sd.s);
      const T cC = -om * T(sd.kphi);
      const int node = hy * HX + hx;
      parS[ps][0][node] = T(1) - om;
      parS[ps][1][node] = ST::OFF ? Qs : om * phc + Qs;
      if constexpr (DIM == 3) {
        parS[ps][2][node] = cC * Nx;
        parS[ps][3][node] = cC * Ny;
        parS[ps][4][node] = cC * Nz;
      } else {
        parS[ps][2][node] = cC * Nx;
        parS[ps][3][node] = cC * Ny;  // the lattice y is the march axis in 2D
      }
      parS[ps][NP - 1][node] = T(1) / a2;
      if (k == tid) {
#pragma unroll
        for (int i = 0; i < QU; ++i) fd_nxt[i] = fd[i];
        u_nxt = un;
        us_nxt = us_self;
        id_nxt = idn;
      }
    }
  };

  // component of C along direction i of the phi lattice (C stored as x, then
  // the in-plane y in 3D, then the march axis)
  auto eC = [&](int i, int ps, int node) -> T {
    T v = T(0);
    if (LP::E[i][0] != 0) v += T(LP::E[i][0]) * parS[ps][2][node];
    if (LP::E[i][1] != 0) v += T(LP::E[i][1]) * parS[ps][3][node];
    if constexpr (DIM == 3) {
      if (LP::E[i][2] != 0) v += T(LP::E[i][2]) * parS[ps][4][node];
    }
    return v;
  };

  // ---- warm-up: phi planes m0-2 .. m0+1, coefficients of planes m0-1, m0 ----
  for (int pm = m0 - 2; pm <= m0 + 1; ++pm) load_plane(pm);
  __syncthreads();
  int sp = 0, sc = 1, sn = 2;  // coefficient slots of planes m-1, m, m+1
  compute_params(m0 - 1, sp);
  compute_params(m0, sc);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < QU; ++i) fd_cur[i] = fd_nxt[i];
  u_cur = u_nxt;
  us_cur = us_nxt;
  id_cur = id_nxt;

  const int gx = x0 + tx;
  const int gy = y0 + ty;
  const bool own = in_range(gx, sd.nx) && (DIM == 2 || in_range(gy, sd.nyp));
  const int hxo = tx + 1, hyo = (DIM == 3) ? ty + 1 : 0;
  const int nodeo = hyo * HX + hxo;
  const int pco = (hyo + PYO) * PX + (hxo + 1);

  for (int m = m0; m < m1; ++m) {
    load_plane(m + 2);
    __syncthreads();
    compute_params(m + 1, sn);
    __syncthreads();

    if (own) {
      const long long iy = lin(sd, gx, gy, m);
      const T phy = phiS[m & 3][pco];
      T d[QP];
      bool unk[QP];
#pragma unroll
      for (int i = 0; i < QP; ++i) {
        const int cx = ex<LP, DIM>(i), cy = ey<LP, DIM>(i), cm = em<LP, DIM>(i);
        int sx = gx - cx, sy = gy - cy, sm = m - cm;
        unk[i] = false;
        if (per) {
          sx = wrapc(sx, sd.nx);
          if (DIM == 3) sy = wrapc(sy, sd.nyp);
          sm = wrapc(sm, sd.nm);
        } else if (!in_range(sx, sd.nx) || (DIM == 3 && !in_range(sy, sd.nyp)) || !in_range(sm, sd.nm)) {
          unk[i] = true;
          d[i] = T(0);
          continue;
        }
        const int ps = (cm == 1) ? sp : ((cm == -1) ? sn : sc);
        const int node = nodeo - cy * HX - cx;
        const T gy_ = ST::ld(Gin + (long long)i * sd.fstride + iy);
        const T gx_ = ST::ld(Gin + (long long)i * sd.fstride + lin(sd, sx, sy, sm));
        const T Acoef = parS[ps][0][node];
        const T Bcoef = parS[ps][1][node];
        const T ia2 = parS[ps][NP - 1][node];
        const T src = T(LP::W[i]) * (Bcoef + eC(i, ps, node));
        if constexpr (ST::OFF) {
          const T phx = phiS[(m - cm) & 3][pco - cy * PX - cx];
          const T hs = Acoef * gx_ + src;
          d[i] = gy_ + ia2 * (T(LP::W[i]) * (phx - phy) + hs - gy_);
        } else {
          const T gs = Acoef * gx_ + src;
          d[i] = gy_ + ia2 * (gs - gy_);
        }
      }
      if (!per) {
        // bounce-back: an unknown incoming population takes the opposite one;
        // if that is unknown too, the local post-collision opposite population
#pragma unroll
        for (int i = 1; i < QP; ++i) {
          if (!unk[i]) continue;
          const int j = LP::OPP[i];
          if (!unk[j]) {
            d[i] = d[j];
          } else {
            const T gj = ST::ld(Gin + (long long)j * sd.fstride + iy);
            d[i] = parS[sc][0][nodeo] * gj + T(LP::W[j]) * (parS[sc][1][nodeo] + eC(j, sc, nodeo));
          }
        }
      }
      T sum = T(0);
#pragma unroll
      for (int i = 0; i < QP; ++i) sum += d[i];
      const T phn = ST::OFF ? phy + sum : sum;
#pragma unroll
      for (int i = 0; i < QP; ++i) {
        const T v = ST::OFF ? d[i] - T(LP::W[i]) * sum : d[i];
        ST::st(Gout + (long long)i * sd.fstride + iy, v);
      }
      Phout[iy] = (typename ST::P)phn;

      // heat equation at y: BGK toward w_i u^n with source (phi^{n+1} - phi^n)/2
      const T half_dphi = T(0.5) * (phn - phy);
      const T om_u = T(sd.omega_u);
      if constexpr (ST::OFF) {
        const T Sm = u_cur - us_cur;  // sum of decoded offsets
        const T keep = T(1) - om_u;
#pragma unroll
        for (int i = 0; i < QU; ++i) ST::st(Fout + (long long)i * sd.fstride + iy, keep * (fd_cur[i] - T(LU::W[i]) * Sm));
        sd.us_out[iy] = float(u_cur + half_dphi);
      } else {
#pragma unroll
        for (int i = 0; i < QU; ++i) {
          const T fi = fd_cur[i];
          ST::st(Fout + (long long)i * sd.fstride + iy, fi - om_u * (fi - T(LU::W[i]) * u_cur) + T(LU::W[i]) * half_dphi);
        }
      }
      if constexpr (IDS) sd.id_out[iy] = id_cur;
    }
    __syncthreads();
    // rotate the coefficient ring and the own-column registers
    const int t = sp;
    sp = sc;
    sc = sn;
    sn = t;
#pragma unroll
    for (int i = 0; i < QU; ++i) fd_cur[i] = fd_nxt[i];
    u_cur = u_nxt;
    us_cur = us_nxt;
    id_cur = id_nxt;
  }
}

template <int DIM, int TY, class ST, bool IDS>
static hipError_t launch_step_t(const SimDev &sd, const TileDev &tc, hipStream_t st) {
  const int nblocks = tc.tiles_x * tc.tiles_y * tc.nchunks;
  dim3 block(64, DIM == 3 ? TY : 1);
  hipLaunchKernelGGL((step_kernel<DIM, TY, ST, IDS>), dim3(nblocks), block, 0, st, sd, tc);
  return hipGetLastError();
}

template <int DIM, class ST, bool IDS>
static hipError_t launch_step_ty(const SimDev &sd, const TileDev &tc, hipStream_t st) {
  if constexpr (DIM == 2) {
    return launch_step_t<2, 1, ST, IDS>(sd, tc, st);
  } else {
    switch (tc.ty) {
      case 2: return launch_step_t<3, 2, ST, IDS>(sd, tc, st);
      case 4: return launch_step_t<3, 4, ST, IDS>(sd, tc, st);
      case 8:
        if constexpr (!std::is_same<ST, StF64>::value) return launch_step_t<3, 8, ST, IDS>(sd, tc, st);
        return hipErrorInvalidValue;
      default: return hipErrorInvalidValue;
    }
  }
}

template <int DIM, class ST>
static hipError_t launch_step_st(const SimDev &sd, const TileDev &tc, hipStream_t st) {
  return sd.use_ids ? launch_step_ty<DIM, ST, true>(sd, tc, st) : launch_step_ty<DIM, ST, false>(sd, tc, st);
}

hipError_t launch_step(int dim, int storage, const SimDev &sd, const TileDev &tc, hipStream_t st) {
  if (dim == 2) {
    switch (storage) {
      case 0: return launch_step_st<2, StF64>(sd, tc, st);
      case 1: return launch_step_st<2, StF32>(sd, tc, st);
      case 2: return launch_step_st<2, StF16>(sd, tc, st);
    }
  } else {
    switch (storage) {
      case 0: return launch_step_st<3, StF64>(sd, tc, st);
      case 1: return launch_step_st<3, StF32>(sd, tc, st);
      case 2: return launch_step_st<3, StF16>(sd, tc, st);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace lbpf

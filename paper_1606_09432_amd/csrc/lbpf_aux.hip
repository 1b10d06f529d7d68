// Initial state, field import/export and FP64 diagnostics reductions.
#include <algorithm>
#include <cmath>

#include "lbpf_kernels.hpp"

namespace lbpf {

__device__ __forceinline__ void to_xyz(int dim, int x, int yp, int m, int &X, int &Y, int &Z) {
  X = x;
  if (dim == 3) {
    Y = yp;
    Z = m;
  } else {
    Y = m;
    Z = 0;
  }
}

__device__ __forceinline__ long long compact(int dim, const SimDev &sd, int x, int yp, int m) {
  return dim == 3 ? ((long long)m * sd.nyp + yp) * sd.nx + x : (long long)m * sd.nx + x;
}

// phi of the initial state at (x, yp, m) (already inside the box).
template <int DIM>
__device__ double init_phi(const SimDev &sd, const InitSrc &src, int x, int yp, int m) {
  if (src.phi) return src.phi[compact(DIM, sd, x, yp, m)];
  int X, Y, Z;
  to_xyz(DIM, x, yp, m, X, Y, Z);
  double ph = -1.0;
  for (int k = 0; k < src.n_seeds; ++k) {
    const SeedDev &s = src.seeds[k];
    const double dx = X - s.x, dy = Y - s.y, dz = Z - s.z;
    const double d2 = (dx * dx + dy * dy) + dz * dz;
    // beyond 20 widths outside the seed tanh is -1 to the last bit (1 - |tanh|
    // < 1e-17), which cannot raise the maximum: skipping it changes nothing
    const double reach = s.r + 20.0 * sd.width;
    if (reach > 0.0 && d2 > reach * reach) continue;
    const double d = sqrt(d2);
    const double v = tanh((s.r - d) / sd.width);  // Eq. Initial_Condition, lattice units
    if (v > ph) ph = v;
  }
  return ph;
}

template <int DIM>
__device__ double init_u(const SimDev &sd, const InitSrc &src, int x, int yp, int m) {
  if (src.u) return src.u[compact(DIM, sd, x, yp, m)];
  return sd.u0;  // Eq. Intial-Cond_u
}

template <int K, class ST>
__global__ __launch_bounds__(256) void init_kernel(SimDev sd, int16_t *ids_out, InitSrc src) {
  constexpr int DIM = LatOf<K>::DIM;
  using LP = typename LatOf<K>::P;
  using LU = typename LatOf<K>::U;
  using S = typename ST::S;
  const long long total = (long long)sd.nx * sd.nyp * sd.nm;
  S *G = reinterpret_cast<S *>(sd.g_out);
  S *F = reinterpret_cast<S *>(sd.f_out);
  typename ST::P *Ph = reinterpret_cast<typename ST::P *>(sd.phi_out);
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < total;
       n += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(n % sd.nx);
    const long long r = n / sd.nx;
    const int yp = (int)(r % sd.nyp);
    const int m = (int)(r / sd.nyp);
    const long long idx = lin(sd, x, yp, m);
    const double ph = init_phi<DIM>(sd, src, x, yp, m);
    // gradient with ghost values mirrored (zero flux) or wrapped (periodic)
    auto phn = [&](int dx, int dy, int dm) {
      const int gx = ghost(x + dx, sd.nx, sd.periodic);
      const int gy = DIM == 3 ? ghost(yp + dy, sd.nyp, sd.periodic) : 0;
      const int gm = ghost(m + dm, sd.nm, sd.periodic);
      return init_phi<DIM>(sd, src, gx, gy, gm);
    };
    double p[3] = {0.0, 0.0, 0.0};
    if (sd.grad_cd) {
      p[0] = (phn(1, 0, 0) - phn(-1, 0, 0)) / 2.0;
      if (DIM == 3) {
        p[1] = (phn(0, 1, 0) - phn(0, -1, 0)) / 2.0;
        p[2] = (phn(0, 0, 1) - phn(0, 0, -1)) / 2.0;
      } else {
        p[1] = (phn(0, 0, 1) - phn(0, 0, -1)) / 2.0;
      }
    } else {
#pragma unroll
      for (int i = 1; i < LP::Q; ++i) {
        const int cx = ex<LP, DIM>(i), cy = ey<LP, DIM>(i), cm = em<LP, DIM>(i);
        // central, or second-order upwind (Sec. 4.2), directional derivative
        const double dd = sd.grad_up2 ? (-phn(2 * cx, 2 * cy, 2 * cm) + 4.0 * phn(cx, cy, cm) - 3.0 * ph) / 2.0
                                      : (phn(cx, cy, cm) - phn(-cx, -cy, -cm)) / 2.0;
        for (int a = 0; a < 3; ++a)
          if (LP::E[i][a] != 0) p[a] += (LP::W[i] * LP::E[i][a]) * dd;
      }
      for (int a = 0; a < 3; ++a) p[a] *= LP::INV_E2;
    }
    // crystal index
    int16_t id = 0;
    if (sd.use_ids) {
      if (src.ids) {
        id = src.ids[compact(DIM, sd, x, yp, m)];
      } else if (src.seeds && src.n_seeds > 0) {
        const double r2 = (p[0] * p[0] + p[1] * p[1]) + p[2] * p[2];
        if (ph > 0.0 || r2 > sd.xi2) {
          int X, Y, Z;
          to_xyz(DIM, x, yp, m, X, Y, Z);
          double best = 1e300;
          for (int k = 0; k < src.n_seeds; ++k) {
            const SeedDev &s = src.seeds[k];
            const double dx = X - s.x, dy = Y - s.y, dz = Z - s.z;
            const double gap = sqrt((dx * dx + dy * dy) + dz * dz) - s.r;
            if (gap < best) {
              best = gap;
              id = (int16_t)s.id;
            }
          }
        }
      }
      ids_out[idx] = id;
    }
    const AnisoDev *A = sd.use_ids ? (id > 0 ? sd.aniso + id : nullptr) : sd.aniso;
    double a, Nv[3];
    flux<double>(A, p[0], p[1], p[2], a, Nv[0], Nv[1], Nv[2]);
    // g = g^(0)(phi, N), Eq. Feq_Phase (lattice units). The offsets sum to
    // zero; as in the step, FP16 stores the rest offset (i = 0, written last)
    // as minus the sum of the others as rounded.
    typename ST::T rsum = 0;
#pragma unroll
    for (int i = LP::Q - 1; i >= 0; --i) {
      const double eN = (LP::E[i][0] * Nv[0] + LP::E[i][1] * Nv[1]) + LP::E[i][2] * Nv[2];
      const double geq = LP::W[i] * (ph - sd.kphi * eN);
      typename ST::T v = typename ST::T(ST::OFF ? -LP::W[i] * sd.kphi * eN * ST::SC : geq);
      if constexpr (ST::COMP) {
        if (i == 0)
          v = -rsum;
        else
          rsum += ST::dec(ST::enc(v));
      }
      ST::st(G + (long long)i * sd.fstride + idx, v);
    }
    Ph[idx] = (typename ST::P)ph;
    // heat populations stored post-collision at the source, so that the first
    // pull gives f_i = w_i u(y): f*_i(y) = w_i u(y + e_i)
    const double uy = init_u<DIM>(sd, src, x, yp, m);
    if (ST::OFF) sd.us_out[idx] = (float)uy;
#pragma unroll
    for (int i = 0; i < LU::Q; ++i) {
      int tx = x + ex<LU, DIM>(i), ty = yp + ey<LU, DIM>(i), tm = m + em<LU, DIM>(i);
      double ut = uy;
      if (sd.periodic) {
        ut = init_u<DIM>(sd, src, wrapc(tx, sd.nx), DIM == 3 ? wrapc(ty, sd.nyp) : 0, wrapc(tm, sd.nm));
      } else if (in_range(tx, sd.nx) && (DIM == 2 || in_range(ty, sd.nyp)) && in_range(tm, sd.nm)) {
        ut = init_u<DIM>(sd, src, tx, ty, tm);
      }
      const double v = ST::OFF ? LU::W[i] * (ut - uy) * ST::SC : LU::W[i] * ut;
      ST::st(F + (long long)i * sd.fstride + idx, typename ST::T(v));
    }
  }
}

template <int K, class ST>
static hipError_t launch_init_t(const SimDev &sd, int16_t *ids_out, const InitSrc &src, hipStream_t st) {
  const long long total = (long long)sd.nx * sd.nyp * sd.nm;
  long long nb = (total + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL((init_kernel<K, ST>), dim3((unsigned)nb), dim3(256), 0, st, sd, ids_out, src);
  return hipGetLastError();
}

template <int K>
static hipError_t launch_init_k(int storage, const SimDev &sd, int16_t *ids_out, const InitSrc &src, hipStream_t st) {
  if (storage == 0) return launch_init_t<K, StF64>(sd, ids_out, src, st);
  if (storage == 1) return launch_init_t<K, StF32>(sd, ids_out, src, st);
  return launch_init_t<K, StF16>(sd, ids_out, src, st);
}

hipError_t launch_init(int lattice, int storage, const SimDev &sd, int16_t *ids_out, const InitSrc &src,
                       hipStream_t st) {
  switch (lattice) {
    case 0: return launch_init_k<0>(storage, sd, ids_out, src, st);
    case 1: return launch_init_k<1>(storage, sd, ids_out, src, st);
    case 2: return launch_init_k<2>(storage, sd, ids_out, src, st);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Diagnostics: FP64 sums with wavefront shuffles, then LDS across the waves of
// a work-group, one partial per work-group and a fixed-order final pass
// (deterministic, no atomics).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  return v;
}

template <int DIM, class ST>
__global__ __launch_bounds__(256) void diag_kernel(SimDev sd, double *partials) {
  using LU = typename Lat<DIM>::U;
  using T = typename ST::T;
  const typename ST::P *Ph = reinterpret_cast<const typename ST::P *>(sd.phi_in);
  double acc[kDiagVals] = {0, 0, 0, 0, 0, 0};
  const long long total = (long long)sd.nx * sd.nyp * sd.nm;
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < total;
       n += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(n % sd.nx);
    const long long r = n / sd.nx;
    const int yp = (int)(r % sd.nyp);
    const int m = (int)(r / sd.nyp);
    const double ph = (double)Ph[lin(sd, x, yp, m)];
    T fd[LU::Q];
    T us;
    const double u = (double)gather_u<DIM, ST>(sd, x, yp, m, fd, us);
    acc[0] += ph;
    acc[1] += u;
    acc[2] += u - 0.5 * ph;
    acc[3] += 1.0 + ph;
    acc[4] += ph > 0.0 ? 1.0 : 0.0;
    if (!isfinite(ph) || !isfinite(u)) acc[5] = 1.0;
  }
  __shared__ double red[kDiagVals][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kDiagVals; ++k) {
    const double v = (k == 5) ? wave_max(acc[k]) : wave_sum(acc[k]);
    if (lane == 0) red[k][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < kDiagVals) {
    const int k = threadIdx.x;
    double v = red[k][0];
    for (int w = 1; w < 4; ++w) v = (k == 5) ? fmax(v, red[k][w]) : v + red[k][w];
    partials[(long long)blockIdx.x * kDiagVals + k] = v;
  }
}

__global__ void diag_finalize(const double *partials, int nb, double *result) {
  const int k = threadIdx.x;
  if (k >= kDiagVals) return;
  double v = 0.0;
  for (int b = 0; b < nb; ++b) v = (k == 5) ? fmax(v, partials[(long long)b * kDiagVals + k]) : v + partials[(long long)b * kDiagVals + k];
  result[k] = v;
}

// Tip: largest linearly interpolated phi = 0 crossing along the ray
// o + k d (lattice units), reduced with wavefront maxima.
template <int DIM, class ST>
__global__ __launch_bounds__(256) void tip_kernel(SimDev sd, int ox, int oy, int oz, int dx, int dy, int dz,
                                                  double *result) {
  const typename ST::P *Ph = reinterpret_cast<const typename ST::P *>(sd.phi_in);
  const int NX = sd.nx, NY = DIM == 3 ? sd.nyp : sd.nm, NZ = DIM == 3 ? sd.nm : 1;
  const double len = sqrt((double)(dx * dx + dy * dy + dz * dz));
  const int kmax = NX + NY + NZ;
  double best = -1.0;
  for (int k = threadIdx.x; k < kmax; k += blockDim.x) {
    const int a0 = ox + k * dx, a1 = oy + k * dy, a2 = oz + k * dz;
    const int b0 = a0 + dx, b1 = a1 + dy, b2 = a2 + dz;
    if (!in_range(a0, NX) || !in_range(a1, NY) || !in_range(a2, NZ)) continue;
    if (!in_range(b0, NX) || !in_range(b1, NY) || !in_range(b2, NZ)) continue;
    const long long ia = DIM == 3 ? lin(sd, a0, a1, a2) : lin(sd, a0, 0, a1);
    const long long ib = DIM == 3 ? lin(sd, b0, b1, b2) : lin(sd, b0, 0, b1);
    const double pa = (double)Ph[ia], pb = (double)Ph[ib];
    if (pa > 0.0 && pb <= 0.0) best = fmax(best, (k + pa / (pa - pb)) * len);
  }
  __shared__ double red[4];
  const double v = wave_max(best);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) result[kDiagVals] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

template <int DIM, class ST>
static hipError_t launch_diag_t(const SimDev &sd, double *partials, double *result, int ox, int oy, int oz,
                                int dx, int dy, int dz, hipStream_t st) {
  hipLaunchKernelGGL((diag_kernel<DIM, ST>), dim3(kDiagBlocks), dim3(256), 0, st, sd, partials);
  hipLaunchKernelGGL(diag_finalize, dim3(1), dim3(64), 0, st, partials, kDiagBlocks, result);
  hipLaunchKernelGGL((tip_kernel<DIM, ST>), dim3(1), dim3(256), 0, st, sd, ox, oy, oz, dx, dy, dz, result);
  return hipGetLastError();
}

hipError_t launch_diag(int dim, int storage, const SimDev &sd, double *partials, double *result,
                       long long /*nodes*/, int ox, int oy, int oz, int dx, int dy, int dz, hipStream_t st) {
  if (dim == 2) {
    if (storage == 0) return launch_diag_t<2, StF64>(sd, partials, result, ox, oy, oz, dx, dy, dz, st);
    if (storage == 1) return launch_diag_t<2, StF32>(sd, partials, result, ox, oy, oz, dx, dy, dz, st);
    return launch_diag_t<2, StF16>(sd, partials, result, ox, oy, oz, dx, dy, dz, st);
  }
  if (storage == 0) return launch_diag_t<3, StF64>(sd, partials, result, ox, oy, oz, dx, dy, dz, st);
  if (storage == 1) return launch_diag_t<3, StF32>(sd, partials, result, ox, oy, oz, dx, dy, dz, st);
  return launch_diag_t<3, StF16>(sd, partials, result, ox, oy, oz, dx, dy, dz, st);
}

// ---------------------------------------------------------------------------
// Export of phi, u, index and decoded post-streaming distributions (FP64).
// ---------------------------------------------------------------------------
template <int K, class ST>
__global__ __launch_bounds__(256) void export_kernel(SimDev sd, double *phi, double *u, int16_t *ids,
                                                     double *g, double *f) {
  constexpr int DIM = LatOf<K>::DIM;
  using LP = typename LatOf<K>::P;
  using LU = typename LatOf<K>::U;
  using T = typename ST::T;
  const typename ST::S *G = reinterpret_cast<const typename ST::S *>(sd.g_in);
  const typename ST::P *Ph = reinterpret_cast<const typename ST::P *>(sd.phi_in);
  const long long total = (long long)sd.nx * sd.nyp * sd.nm;
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < total;
       n += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(n % sd.nx);
    const long long r = n / sd.nx;
    const int yp = (int)(r % sd.nyp);
    const int m = (int)(r / sd.nyp);
    const long long idx = lin(sd, x, yp, m);
    const long long c = compact(DIM, sd, x, yp, m);
    const double ph = (double)Ph[idx];
    if (phi) phi[c] = ph;
    if (ids) ids[c] = sd.use_ids ? sd.id_in[idx] : int16_t(0);
    if (g) {
      for (int i = 0; i < LP::Q; ++i) {
        const double h = (double)ST::ld(G + (long long)i * sd.fstride + idx) / ST::SC;
        g[(long long)i * total + c] = ST::OFF ? LP::W[i] * ph + h : h;
      }
    }
    if (u || f) {
      T fd[LU::Q];
      T us;
      const double uv = (double)gather_u<DIM, ST>(sd, x, yp, m, fd, us);
      if (u) u[c] = uv;
      if (f)
        for (int i = 0; i < LU::Q; ++i)
          f[(long long)i * total + c] = ST::OFF ? LU::W[i] * (double)us + (double)fd[i] : (double)fd[i];
    }
  }
}

template <int K, class ST>
static hipError_t launch_export_t(const SimDev &sd, double *phi, double *u, int16_t *ids, double *g, double *f,
                                  hipStream_t st) {
  const long long total = (long long)sd.nx * sd.nyp * sd.nm;
  long long nb = (total + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL((export_kernel<K, ST>), dim3((unsigned)nb), dim3(256), 0, st, sd, phi, u, ids, g, f);
  return hipGetLastError();
}

template <int K>
static hipError_t launch_export_k(int storage, const SimDev &sd, double *phi, double *u, int16_t *ids, double *g,
                                  double *f, hipStream_t st) {
  if (storage == 0) return launch_export_t<K, StF64>(sd, phi, u, ids, g, f, st);
  if (storage == 1) return launch_export_t<K, StF32>(sd, phi, u, ids, g, f, st);
  return launch_export_t<K, StF16>(sd, phi, u, ids, g, f, st);
}

hipError_t launch_export(int lattice, int storage, const SimDev &sd, double *phi, double *u, int16_t *ids,
                         double *g, double *f, int /*ny_full*/, hipStream_t st) {
  switch (lattice) {
    case 0: return launch_export_k<0>(storage, sd, phi, u, ids, g, f, st);
    case 1: return launch_export_k<1>(storage, sd, phi, u, ids, g, f, st);
    case 2: return launch_export_k<2>(storage, sd, phi, u, ids, g, f, st);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Checkpoint header: one thread stores the record passed as an argument.
// ---------------------------------------------------------------------------
__global__ void state_header_kernel(StateHeader *dst, StateHeader h) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = h;
}

hipError_t launch_state_header(StateHeader *dst, const StateHeader &h, hipStream_t st) {
  hipLaunchKernelGGL(state_header_kernel, dim3(1), dim3(64), 0, st, dst, h);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Streaming copy: each thread moves four 16-byte vectors per round (loads
// first, then stores), consecutive threads consecutive vectors; a grid of a
// few work-groups per CU strides over the array.  A tail shorter than 16 bytes
// is copied byte by byte by the first threads.
// ---------------------------------------------------------------------------
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void stream_copy_kernel(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                          size_t n16, const unsigned char *__restrict__ tsrc,
                                                          unsigned char *__restrict__ tdst, int ntail) {
  constexpr int U = 4;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (U - 1) * stride < n16; i += U * stride) {
    u32x4 v[U];
#pragma unroll
    for (int k = 0; k < U; ++k) v[k] = __builtin_nontemporal_load(src + i + k * stride);
#pragma unroll
    for (int k = 0; k < U; ++k) __builtin_nontemporal_store(v[k], dst + i + k * stride);
  }
  for (; i < n16; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
  if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tdst[threadIdx.x] = tsrc[threadIdx.x];
}

hipError_t launch_stream_copy(const void *src, void *dst, size_t bytes, int blocks_per_cu, hipStream_t st) {
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const size_t n16 = bytes / 16;
  const int ntail = (int)(bytes % 16);
  const int grid = std::max(1, ncu * std::max(1, blocks_per_cu));
  hipLaunchKernelGGL(stream_copy_kernel, dim3(grid), dim3(256), 0, st, static_cast<const u32x4 *>(src),
                     static_cast<u32x4 *>(dst), n16, static_cast<const unsigned char *>(src) + n16 * 16,
                     static_cast<unsigned char *>(dst) + n16 * 16, ntail);
  return hipGetLastError();
}

}  // namespace lbpf

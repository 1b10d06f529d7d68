// Device-side building blocks of the coupled LB phase-field step for gfx950.
//
// Coordinates.  Every kernel works in (x, yp, m) coordinates: m is the axis a
// work-group marches along (z in 3D, y in 2D), yp the second in-plane axis (y
// in 3D, always 0 in 2D).  A field element (x, yp, m) lives at
// m * mstride + yp * pitch + x, with the x pitch padded to 64 elements so
// that every row starts on a 128-byte line.  Distributions are stored as one
// such field per lattice direction (structure of arrays), fstride elements
// apart.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbpf {

// ---------------------------------------------------------------------------
// Lattices (Sec. 3.3, Table Values-Lattices; D3Q19 with the standard weights
// 1/3, 1/18, 1/36 since the paper names but does not tabulate it).
// ---------------------------------------------------------------------------
struct D2Q9 {
  static constexpr int Q = 9;
  static constexpr int E[9][3] = {{0, 0, 0}, {1, 0, 0},  {0, 1, 0},   {-1, 0, 0}, {0, -1, 0},
                                  {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
  static constexpr double W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                  1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  static constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  static constexpr double INV_E2 = 3.0;
};
struct D2Q5 {
  static constexpr int Q = 5;
  static constexpr int E[5][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0}};
  static constexpr double W[5] = {1.0 / 3, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
  static constexpr int OPP[5] = {0, 3, 4, 1, 2};
  static constexpr double INV_E2 = 3.0;
};
struct D3Q19 {
  static constexpr int Q = 19;
  static constexpr int E[19][3] = {
      {0, 0, 0},  {1, 0, 0},  {0, 1, 0},   {-1, 0, 0}, {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
      {1, 1, 0},  {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {1, 0, 1},  {0, 1, 1},  {-1, 0, 1},
      {0, -1, 1}, {1, 0, -1}, {0, 1, -1},  {-1, 0, -1}, {0, -1, -1}};
  static constexpr double W[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                   1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  static constexpr int OPP[19] = {0, 3, 4, 1, 2, 6, 5, 9, 10, 7, 8, 17, 18, 15, 16, 13, 14, 11, 12};
  static constexpr double INV_E2 = 3.0;
};
struct D3Q7 {
  static constexpr int Q = 7;
  static constexpr int E[7][3] = {{0, 0, 0}, {1, 0, 0},  {0, 1, 0}, {-1, 0, 0},
                                  {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
  static constexpr double W[7] = {1.0 / 4, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8};
  static constexpr int OPP[7] = {0, 3, 4, 1, 2, 6, 5};
  static constexpr double INV_E2 = 4.0;
};

// D3Q15 (Sec. 3.3, Table Values-Lattices): rest 2/9, axes 1/9, the eight cube
// diagonals 1/72, e^2 = 1/3, in the paper's order of the vectors.
struct D3Q15 {
  static constexpr int Q = 15;
  static constexpr int E[15][3] = {{0, 0, 0},  {1, 0, 0},   {0, 1, 0},    {-1, 0, 0},  {0, -1, 0},
                                   {0, 0, 1},  {0, 0, -1},  {1, 1, 1},    {-1, 1, 1},  {-1, -1, 1},
                                   {1, -1, 1}, {1, 1, -1},  {-1, 1, -1},  {-1, -1, -1}, {1, -1, -1}};
  static constexpr double W[15] = {2.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9,
                                   1.0 / 9,  1.0 / 9,  1.0 / 72, 1.0 / 72, 1.0 / 72,
                                   1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72};
  static constexpr int OPP[15] = {0, 3, 4, 1, 2, 6, 5, 13, 14, 11, 12, 9, 10, 7, 8};
  static constexpr double INV_E2 = 3.0;
};

// The heat lattice of a dimension, and the lattice pair of a pair code K
// (0: D2Q9 + D2Q5, 1: D3Q19 + D3Q7, 2: D3Q15 + D3Q7).
template <int DIM> struct Lat;
template <> struct Lat<2> {
  using U = D2Q5;
};
template <> struct Lat<3> {
  using U = D3Q7;
};
template <int K> struct LatOf;
template <> struct LatOf<0> {
  static constexpr int DIM = 2;
  using P = D2Q9;
  using U = D2Q5;
};
template <> struct LatOf<1> {
  static constexpr int DIM = 3;
  using P = D3Q19;
  using U = D3Q7;
};
template <> struct LatOf<2> {
  static constexpr int DIM = 3;
  using P = D3Q15;
  using U = D3Q7;
};

// Components of direction i along (x, yp, m).
template <class L, int DIM> __device__ __forceinline__ constexpr int ex(int i) { return L::E[i][0]; }
template <class L, int DIM> __device__ __forceinline__ constexpr int ey(int i) {
  return DIM == 3 ? L::E[i][1] : 0;
}
template <class L, int DIM> __device__ __forceinline__ constexpr int em(int i) {
  return DIM == 3 ? L::E[i][2] : L::E[i][1];
}

// Mirror image of direction i: the direction whose vector is e_i with the
// components along the axes in fl negated (bit 0: x, bit 1: yp, bit 2: m).
template <class L, int DIM> __device__ __forceinline__ constexpr int mirror_dir(int i, int fl) {
  const int tx = (fl & 1) ? -ex<L, DIM>(i) : ex<L, DIM>(i);
  const int ty = (fl & 2) ? -ey<L, DIM>(i) : ey<L, DIM>(i);
  const int tm = (fl & 4) ? -em<L, DIM>(i) : em<L, DIM>(i);
  for (int j = 0; j < L::Q; ++j)
    if (ex<L, DIM>(j) == tx && ey<L, DIM>(j) == ty && em<L, DIM>(j) == tm) return j;
  return i;
}
// The same for a compile-time i and a runtime fl: a choice among eight constants.
template <class L, int DIM> __device__ __forceinline__ int mirror_sel(int i, int fl) {
  int r = i;
#pragma unroll
  for (int f = 1; f < 8; ++f)
    if (fl == f) r = mirror_dir<L, DIM>(i, f);
  return r;
}

// Stores of the step's outputs carry the non-temporal hint: no launch reads
// what it writes, and keeping the written lines out of the way in L2 leaves it
// to the rows that the neighbouring planes read again.
template <class E> __device__ __forceinline__ void nt_store(E *p, E v) {
  if constexpr (sizeof(E) == 2) {
    unsigned short b;
    __builtin_memcpy(&b, &v, 2);
    __builtin_nontemporal_store(b, reinterpret_cast<unsigned short *>(p));
  } else {
    __builtin_nontemporal_store(v, p);
  }
}

// ---------------------------------------------------------------------------
// Storage: FP64 distributions, or FP32 arithmetic on offsets stored in FP32/FP16.
// ---------------------------------------------------------------------------
// SC: stored units per true unit of an offset.  FP16 offsets are stored
// multiplied by 2^12, so that the small offsets of the bulk (down to about
// 1.5e-8) stay above the FP16 subnormal range; |offsets| stay far below
// 65504 / 2^12 = 16.  A power of two scales without rounding.  The step folds
// SC into its compile-time weights, so the scale costs no instruction.
// FOLD_3D: the 3D offset pulls read coefficients with 1/a^2 folded in (M, A',
// Kc, K0) rather than (A, B, C, 1/a^2) and phi of the source node;
// HEAT_CONST_3D: a 3D node whose heat sources all lie inside the box takes their
// ring offsets as constants.  The 2D forms always do both.  Either form computes
// the same quantities up to rounding order; each is set where it measured
// faster (the offset steps are bound by their instruction stream and register
// schedule, which both change: FP16 3D is 2-4% faster without either, FP32 3D
// 1-5% faster with both, 2D FP16 8% faster with both).
struct StF64 {
  using T = double;  // arithmetic
  using S = double;  // stored distribution
  using P = double;  // stored phi
  static constexpr bool OFF = false;
  static constexpr bool COMP = false;
  static constexpr double SC = 1.0;
  static constexpr bool FOLD_3D = false;
  static constexpr bool HEAT_CONST_3D = false;
  static __device__ __forceinline__ T ld(const S *p) { return *p; }
  static __device__ __forceinline__ void st(S *p, T v) { nt_store(p, S(v)); }
  static __device__ __forceinline__ S enc(T v) { return v; }
  static __device__ __forceinline__ T dec(S s) { return s; }
};
struct StF32 {
  using T = float;
  using S = float;
  using P = float;
  static constexpr bool OFF = true;
  static constexpr bool COMP = false;
  static constexpr double SC = 1.0;
  static constexpr bool FOLD_3D = true;
  static constexpr bool HEAT_CONST_3D = true;
  static __device__ __forceinline__ T ld(const S *p) { return *p; }
  static __device__ __forceinline__ void st(S *p, T v) { nt_store(p, S(v)); }
  static __device__ __forceinline__ S enc(T v) { return v; }
  static __device__ __forceinline__ T dec(S s) { return s; }
};
struct StF16 {
  using T = float;
  using S = __half;
  using P = float;
  static constexpr bool OFF = true;
  // the rest offset balances the rounded others (FP16 rounding is coarse)
  static constexpr bool COMP = true;
  static constexpr double SC = 4096.0;
  static constexpr bool FOLD_3D = false;
  static constexpr bool HEAT_CONST_3D = false;
  static __device__ __forceinline__ T ld(const S *p) { return __half2float(*p); }
  static __device__ __forceinline__ void st(S *p, T v) { nt_store(p, __float2half_rn(v)); }
  static __device__ __forceinline__ S enc(T v) { return __float2half_rn(v); }
  static __device__ __forceinline__ T dec(S s) { return __half2float(s); }
};

// Anisotropy entry as the kernels see it (cos/sin of q phi0 precomputed on the
// host).  rot = 1: the polynomial is evaluated at R n (R row-major), a crystal
// orientation of Sec. 4.3 in 3D; rot = 0 skips the rotation (identity).
// The three cubic kinds share one polynomial, a = c0 + c1 Q + c2 S with
// Q = n_x^4 + n_y^4 + n_z^4 and S = n_x^2 n_y^2 n_z^2:
//   Eq. As_Function_Classical  c0 = 1 - 3 eps, c1 = 4 eps, c2 = 0;
//   Eq. As_MatSci              c0 = 1 - 3 eps/5 - 17 gamma/7, c1 = eps + 3 gamma, c2 = 66 gamma;
//   Eq. As_Function_S          c0 = 1, c1 = 0, c2 = 66 gamma (read with the constant 1).
// Every coefficient is kept in FP64 and in FP32 (the FP32-arithmetic forms
// read the latter and convert nothing).
struct AnisoDev {
  int kind;
  int q;
  double eps, gamma, cr, ci;
  int rot;
  double R[9];
  double c0, c1, c2;
  float epsf, crf, cif, c0f, c1f, c2f;
  float Rf[9];
};
// An entry read through the constant address space (the step never writes the
// table).
using ConstAniso = const __attribute__((address_space(4))) AnisoDev;

// An entry of the crystal-index table staged in LDS by the step kernel, in the
// arithmetic type T only (both field names of AnisoDev name the one value).
template <class T> struct StagedAniso {
  int kind, q, rot;
  union { T R[9]; T Rf[9]; };
  union { T eps; T epsf; };
  union { T cr; T crf; };
  union { T ci; T cif; };
  union { T c0; T c0f; };
  union { T c1; T c1f; };
  union { T c2; T c2f; };
};
template <class T> __host__ __device__ __forceinline__ T pick(double d, float f) {
  if constexpr (sizeof(T) == sizeof(float))
    return f;
  else
    return d;
}

template <class T> __device__ __forceinline__ void stage_entry(const AnisoDev &a, StagedAniso<T> &s) {
  s.kind = a.kind;
  s.q = a.q;
  s.rot = a.rot;
  for (int k = 0; k < 9; ++k) s.R[k] = pick<T>(a.R[k], a.Rf[k]);
  s.eps = pick<T>(a.eps, a.epsf);
  s.cr = pick<T>(a.cr, a.crf);
  s.ci = pick<T>(a.ci, a.cif);
  s.c0 = pick<T>(a.c0, a.c0f);
  s.c1 = pick<T>(a.c1, a.c1f);
  s.c2 = pick<T>(a.c2, a.c2f);
}
constexpr int kMaxAniso = 256;

enum { K_ISO = 0, K_SECTORAL = 1, K_CUBIC = 2, K_CUBIC_HAK = 3, K_CUBIC_S = 4 };

// Everything a kernel needs to know about one simulation and one A->B step.
struct SimDev {
  int nx, nyp, nm, pitch;  // extents in (x, yp, m), x pitch in elements
  long long mstride;       // elements between consecutive m planes
  long long fstride;       // elements between consecutive distribution fields
  int periodic, grad_cd, use_ids, n_aniso;
  double kphi;     // Dphi / e^2 of the phi lattice
  double s;        // dt / tau0
  double lambda;   // coupling
  double omega_u;  // 1 / eta_u
  double xi2;      // xi^2 (index threshold on |p|^2)
  float kphi_f, s_f, lambda_f, omega_u_f, xi2_f;  // the same in FP32
  double width;    // sqrt(2) W0 / dx (seed profile width, lattice units)
  double u0;       // -delta
  const void *g_in;
  void *g_out;
  const void *f_in;
  void *f_out;
  const void *phi_in;
  void *phi_out;
  const float *us_in;
  float *us_out;
  const int16_t *id_in;
  int16_t *id_out;
  const AnisoDev *aniso;
  int mirror;    // the planes through node 0 of each axis are mirror planes
  int grad_up2;  // second-order upwind directional derivatives (Sec. 4.2)
};

__device__ __forceinline__ bool in_range(int c, int n) { return (unsigned)c < (unsigned)n; }

// Ghost coordinate for reads of phi (and of the index field) around the box:
// periodic wrap, or a mirror about the wall node (phi(-k) = phi(k)) so that
// the normal derivative vanishes on the wall.  |offset| <= 2 beyond the box.
__device__ __forceinline__ int ghost(int c, int n, int periodic) {
  if (periodic) return c < 0 ? c + n : (c >= n ? c - n : c);
  return c < 0 ? -c : (c >= n ? 2 * (n - 1) - c : c);
}
__device__ __forceinline__ int wrapc(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

// Element offset of node (x, yp, m) inside one field.  A field holds fewer
// than 2^31 elements (checked when the workspace is planned), so the offset is
// a 32-bit value added to a per-field base pointer.
__device__ __forceinline__ unsigned lin(const SimDev &sd, int x, int yp, int m) {
  return (unsigned)m * (unsigned)sd.mstride + (unsigned)yp * (unsigned)sd.pitch + (unsigned)x;
}

// Reciprocal and reciprocal square root: exact in FP64 (parity with the FP64
// reference), the hardware approximations (about 1 ulp) in FP32.
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rsqrt_(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }

// ---------------------------------------------------------------------------
// Anisotropy functions (Sec. 4.1): value a and gradient G of the polynomial in n.
// ---------------------------------------------------------------------------
template <class T, class E>
__host__ __device__ __forceinline__ void aniso_eval(const E &A, T nx, T ny, T nz, T &a, T &Gx, T &Gy,
                                                    T &Gz) {
  Gx = Gy = Gz = T(0);
  if (A.kind == K_SECTORAL) {
    // Re[z^q c] with z = n_x + i n_y, c = e^{-i q phi0}; gradient Re[q z^{q-1} c], -Im[q z^{q-1} c].
    T pr = T(1), pi = T(0);
    for (int k = 1; k < A.q; ++k) {
      const T tr = pr * nx - pi * ny;
      const T ti = pr * ny + pi * nx;
      pr = tr;
      pi = ti;
    }
    const T cr = pick<T>(A.cr, A.crf), ci = pick<T>(A.ci, A.cif), eps = pick<T>(A.eps, A.epsf);
    const T zr = pr * nx - pi * ny, zi = pr * ny + pi * nx;
    a = T(1) + eps * (zr * cr - zi * ci);
    const T qf = T(A.q);
    Gx = eps * (qf * (pr * cr - pi * ci));
    Gy = -(eps * (qf * (pr * ci + pi * cr)));
    return;
  }
  if (A.kind == K_ISO) {
    a = T(1);
    return;
  }
  // cubic kinds: c0 + c1 Q + c2 S, grad Q = 4 (n_x^3, ..), grad S = 2 n_x n_y^2 n_z^2, ..
  const T c0 = pick<T>(A.c0, A.c0f), c1 = pick<T>(A.c1, A.c1f), c2 = pick<T>(A.c2, A.c2f);
  const T x2 = nx * nx, y2 = ny * ny, z2 = nz * nz;
  const T Q = (x2 * x2 + y2 * y2) + z2 * z2;
  const T yz = y2 * z2, xz = x2 * z2, xy = x2 * y2;
  a = c0 + c1 * Q + c2 * (xy * z2);
  const T f1 = T(4) * c1, f2 = T(2) * c2;
  Gx = nx * (f1 * x2 + f2 * yz);
  Gy = ny * (f1 * y2 + f2 * xz);
  Gz = nz * (f1 * z2 + f2 * xy);
}

// An entry at direction n: the polynomial at m = R n, and by the chain rule
// the gradient with respect to n, R^T (grad A)(m).
template <class T, class E>
__host__ __device__ __forceinline__ void aniso_eval_rot(const E &A, T nx, T ny, T nz, T &a, T &Gx, T &Gy,
                                                        T &Gz) {
  if (!A.rot) {
    aniso_eval<T>(A, nx, ny, nz, a, Gx, Gy, Gz);
    return;
  }
  T R[9];
  for (int k = 0; k < 9; ++k) R[k] = pick<T>(A.R[k], A.Rf[k]);
  const T mx = (R[0] * nx + R[1] * ny) + R[2] * nz;
  const T my = (R[3] * nx + R[4] * ny) + R[5] * nz;
  const T mz = (R[6] * nx + R[7] * ny) + R[8] * nz;
  T Hx, Hy, Hz;
  aniso_eval<T>(A, mx, my, mz, a, Hx, Hy, Hz);
  Gx = (R[0] * Hx + R[3] * Hy) + R[6] * Hz;
  Gy = (R[1] * Hx + R[4] * Hy) + R[7] * Hz;
  Gz = (R[2] * Hx + R[5] * Hy) + R[8] * Hz;
}

// a_s and N = -|p| a (G - n (n.G)) for the gradient p, n = -p/|p|
// (Eqs. Def_Normal_Vector, TermesAnisotropes).  Isotropic where |p| <= 1e-8
// (lattice units): below that the direction of p is set by the rounding of
// phi differences rather than by an interface, and a_s depends on it at O(eps).
// E is StagedAniso<T> (an index table staged in LDS), or AnisoDev, or
// AnisoDev in the constant address space (ConstAniso) when
// every lane reads the same entry: its reads are then scalar loads at the
// point of use (through a generic pointer they are vector loads, each followed
// by a wait for every load in flight).
template <class T, class E>
__device__ __forceinline__ void flux(const E *A, T px, T py, T pz, T &a, T &Nx, T &Ny, T &Nz) {
  a = T(1);
  Nx = Ny = Nz = T(0);
  if (A == nullptr) return;
  // the cutoff first: away from interfaces no lane of a wave reads the entry
  const T r2 = (px * px + py * py) + pz * pz;
  if (!(r2 > T(1e-16))) return;
  if (A->kind == K_ISO) return;
  const T ir = rsqrt_(r2);
  const T r = r2 * ir;
  const T nx = -px * ir, ny = -py * ir, nz = -pz * ir;
  T Gx, Gy, Gz;
  aniso_eval_rot<T>(*A, nx, ny, nz, a, Gx, Gy, Gz);
  const T nG = (nx * Gx + ny * Gy) + nz * Gz;
  const T ra = r * a;
  Nx = -ra * (Gx - nx * nG);
  Ny = -ra * (Gy - ny * nG);
  Nz = -ra * (Gz - nz * nG);
}

// ---------------------------------------------------------------------------
// Heat distributions are stored post-collision at their source node
// ("stream on read"): f_i^n(y) = f*_i(y - e_i).  With zero-flux walls an
// unknown f_i (source outside) is the opposite population f_i'^n(y) = f*_i'(y + e_i)
// (Eq. Bounce-Back); if that source is outside too, f*_i'(y).  A source beyond
// a mirror plane is the mirror node inside, and the population there is the
// mirror image of i: the opposite one, since the heat lattices' vectors have
// one nonzero component.
// gather_u returns u^n(y) = sum_i f_i^n(y) and the decoded populations:
//   FP64:     fd[i] = f_i^n(y)
//   offsets:  fd[i] = f_i^n(y) - w_i u*(y), stored f*_i = w_i u* + k_i
//             (k_i decoded from its stored units).
// ---------------------------------------------------------------------------
template <int DIM, class ST>
__device__ __forceinline__ typename ST::T gather_u(const SimDev &sd, int x, int yp, int m,
                                                   typename ST::T (&fd)[Lat<DIM>::U::Q],
                                                   typename ST::T &ustar_self) {
  using T = typename ST::T;
  using LU = typename Lat<DIM>::U;
  const typename ST::S *F = reinterpret_cast<const typename ST::S *>(sd.f_in);
  const unsigned self = lin(sd, x, yp, m);
  T us_self = T(0);
  if constexpr (ST::OFF) us_self = sd.us_in[self];
  T sum = T(0);
#pragma unroll
  for (int i = 0; i < LU::Q; ++i) {
    int sx = x - ex<LU, DIM>(i), sy = yp - ey<LU, DIM>(i), sm = m - em<LU, DIM>(i);
    int d = i;
    unsigned src;
    if (sd.mirror && (sx < 0 || sy < 0 || sm < 0)) {
      d = LU::OPP[i];
      sx = abs(sx);
      sy = abs(sy);
      sm = abs(sm);
    }
    if (sd.periodic) {
      src = lin(sd, wrapc(sx, sd.nx), DIM == 3 ? wrapc(sy, sd.nyp) : 0, wrapc(sm, sd.nm));
    } else if (in_range(sx, sd.nx) && (DIM == 2 || in_range(sy, sd.nyp)) && in_range(sm, sd.nm)) {
      src = lin(sd, sx, sy, sm);
    } else {
      d = LU::OPP[i];
      const int tx = x + ex<LU, DIM>(i), ty = yp + ey<LU, DIM>(i), tm = m + em<LU, DIM>(i);
      if (in_range(tx, sd.nx) && (DIM == 2 || in_range(ty, sd.nyp)) && in_range(tm, sd.nm))
        src = lin(sd, tx, ty, tm);
      else
        src = self;
    }
    const T kv = ST::ld(F + (long long)d * sd.fstride + src) * T(1.0 / ST::SC);
    if constexpr (ST::OFF) {
      fd[i] = T(LU::W[i]) * (sd.us_in[src] - us_self) + kv;
    } else {
      fd[i] = kv;
    }
    sum += fd[i];
  }
  ustar_self = us_self;
  return ST::OFF ? us_self + sum : sum;
}

}  // namespace lbpf

// C ABI of the library (include/lb_pf.h): configuration checks, lattice-unit
// conversion, workspace layout, launches and diagnostics.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lb_pf.h"
#include "lbpf_kernels.hpp"

using namespace lbpf;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

#define HIPCHK(expr)                                                                            \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return fail(LBPF_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
constexpr long long kFieldSkew = 17 * 64;  // elements
size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

struct SimHost {
  lbpf_config cfg;
  std::vector<lbpf_aniso> aniso;
  std::vector<lbpf_seed> seeds;
  int dim = 2, storage = 0;
  int nx = 0, nyp = 0, nm = 0, pitch = 0;
  long long mstride = 0, fstride = 0;
  int qp = 9, qu = 5;
  size_t dsz = 8, psz = 8;
  // byte offsets inside the workspace
  size_t state_off[2] = {0, 0};
  size_t state_bytes = 0;
  size_t off_g = 0, off_f = 0, off_phi = 0, off_us = 0, off_id = 0;  // inside a state block
  size_t off_aniso = 0, off_seeds = 0, off_part = 0, off_res = 0;
  double kphi = 0, s = 0, omega_u = 0, width = 0;
  TileDev tile{};
};

}  // namespace

// Batched ensemble (2D, n_sims > 1): the per-simulation SimDev tables of both
// parities and the work list live in the workspace; each step is one
// persistent launch, replayed from HIP graphs captured once per parity.
namespace {
constexpr int kMinBatchChunk = 8;  // rows per work item, lower bound (sizes the work list)
constexpr int kGraphSteps = 8;     // steps per long graph (even: the parity is restored)

struct BatchState {
  bool on = false;
  bool ids = false;
  bool mirror = false;                 // some member has mirror planes
  int storage = 0;
  int chunk = 8;                       // rows per work item (measured best for the 256-member ensemble)
  size_t off_sims = 0, off_items = 0;  // workspace offsets
  int max_items = 0;
  std::vector<SimDev> tables;          // [parity][sim]
  std::vector<BatchItem> items;
  int n_items = 0, grid = 0, blocks_per_cu = 0, n_cu = 0;
  bool dirty = true;                   // tables / items not uploaded yet
  hipStream_t cap = nullptr;           // private stream used only for capture
  hipGraphExec_t exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [parity][one step, kGraphSteps]
};
}  // namespace

struct lbpf_handle {
  std::vector<SimHost> sims;
  char *ws = nullptr;
  size_t bytes = 0;
  int parity = 0;
  int64_t step = 0;
  int device = 0;  // the device current at lb_pf_init
  BatchState batch;
  // boxes with mirror planes: the tiles at a plane run on `aux`, concurrently
  // with the others on the caller's stream (events fork and join order them)
  hipStream_t aux = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

namespace {
void release_aux(lbpf_handle *h) {
  if (h->aux) {
    (void)hipStreamSynchronize(h->aux);
    (void)hipStreamDestroy(h->aux);
  }
  if (h->fork) (void)hipEventDestroy(h->fork);
  if (h->join) (void)hipEventDestroy(h->join);
  h->aux = nullptr;
  h->fork = h->join = nullptr;
}
}  // namespace

// Scratch of lb_pf_diagnostics_noalloc: the per-block partials and the result
// of the diagnostics reductions, in a file-scope device array instead of the
// handle's workspace.  Each GPU holds its own copy until the process ends.  In
// host code `scratch` names a host-side stand-in, not device memory: its
// device address is taken once per device with hipGetSymbolAddress (at
// lb_pf_init, with that device current) and only that address is used.
constexpr int kScratchDoubles = 4096;  // 32 KiB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};  // device address of scratch, per device

// Takes the device address of scratch on device dev (current), once.
int scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return fail(LBPF_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return LBPF_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(LBPF_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[dev] = static_cast<double *>(p);
  return LBPF_OK;
}

double *scratch_of(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[dev];
}
}  // namespace

namespace {

// Device form of an entry: cos and sin of q phi0, and the orientation R (an
// all-zero R is the identity, kept as rot = 0 so that the step skips it).
AnisoDev to_dev(const lbpf_aniso &a) {
  AnisoDev d{};
  d.kind = a.kind;
  d.q = a.q;
  d.eps = a.eps;
  d.gamma = a.gamma;
  d.cr = std::cos(a.q * a.phi0);
  d.ci = -std::sin(a.q * a.phi0);
  d.rot = 0;
  for (int k = 0; k < 9; ++k) {
    d.R[k] = a.R[k];
    d.Rf[k] = (float)a.R[k];
    if (a.R[k] != 0.0) d.rot = 1;
  }
  // one polynomial c0 + c1 Q + c2 S for the cubic kinds (Sec. 4.1)
  if (a.kind == LBPF_ANISO_CUBIC) {
    d.c0 = 1.0 - 3.0 * a.eps;
    d.c1 = 4.0 * a.eps;
    d.c2 = 0.0;
  } else if (a.kind == LBPF_ANISO_CUBIC_HAK) {
    d.c0 = 1.0 - 3.0 * a.eps / 5.0 - 17.0 * a.gamma / 7.0;
    d.c1 = a.eps + 3.0 * a.gamma;
    d.c2 = 66.0 * a.gamma;
  } else if (a.kind == LBPF_ANISO_CUBIC_S) {
    d.c0 = 1.0;
    d.c1 = 0.0;
    d.c2 = 66.0 * a.gamma;
  }
  d.epsf = (float)d.eps;
  d.crf = (float)d.cr;
  d.cif = (float)d.ci;
  d.c0f = (float)d.c0;
  d.c1f = (float)d.c1;
  d.c2f = (float)d.c2;
  return d;
}

// The unit directions on which entries are checked: 4000 points of a
// Fibonacci lattice on the sphere and the 26 neighbour directions of a cube
// in 3D; 1440 evenly spaced points on the circle and its 8 neighbour
// directions in 2D.
std::vector<std::array<double, 3>> check_dirs(int dim) {
  std::vector<std::array<double, 3>> v;
  const double pi = 3.14159265358979323846;
  if (dim == 2) {
    for (int j = 0; j < 1440; ++j) {
      const double t = 2.0 * pi * (j + 0.5) / 1440.0;
      v.push_back({std::cos(t), std::sin(t), 0.0});
    }
  } else {
    const double ga = pi * (3.0 - std::sqrt(5.0));
    for (int j = 0; j < 4000; ++j) {
      const double z = 1.0 - (2.0 * j + 1.0) / 4000.0, r = std::sqrt(1.0 - z * z);
      v.push_back({r * std::cos(ga * j), r * std::sin(ga * j), z});
    }
  }
  for (int x = -1; x <= 1; ++x)
    for (int y = -1; y <= 1; ++y)
      for (int z = -1; z <= 1; ++z) {
        if ((x | y | z) == 0 || (dim == 2 && z != 0)) continue;
        const double l = std::sqrt(double(x * x + y * y + z * z));
        v.push_back({x / l, y / l, z / l});
      }
  return v;
}

double entry_a(const AnisoDev &d, const std::array<double, 3> &n) {
  if (d.kind == LBPF_ANISO_ISO) return 1.0;
  double a, gx, gy, gz;
  aniso_eval_rot<double>(d, n[0], n[1], n[2], a, gx, gy, gz);
  return a;
}

int check_entry(const lbpf_aniso &a, int dim, bool mirror) {
  double rr = 0;  // |R^T R - I| (max element) when a rotation is given
  bool any = false;
  for (int k = 0; k < 9; ++k) {
    if (!std::isfinite(a.R[k])) return fail(LBPF_ERR_ARG, "anisotropy rotation must be finite");
    any = any || a.R[k] != 0.0;
  }
  if (any) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double t = 0;
        for (int k = 0; k < 3; ++k) t += a.R[3 * k + i] * a.R[3 * k + j];
        rr = std::max(rr, std::fabs(t - (i == j ? 1.0 : 0.0)));
      }
    if (!(rr <= 1e-9)) return fail(LBPF_ERR_ARG, "anisotropy rotation R is not orthogonal");
  }
  const AnisoDev d = to_dev(a);
  for (const auto &n : check_dirs(dim)) {
    const double v = entry_a(d, n);
    if (!(v > 0.0)) return fail(LBPF_ERR_UNSTABLE, "anisotropy entry with a_s <= 0 in some direction");
    if (mirror) {
      for (int k = 0; k < dim; ++k) {
        std::array<double, 3> m = n;
        m[k] = -m[k];
        if (!(std::fabs(entry_a(d, m) - v) <= 1e-12))
          return fail(LBPF_ERR_UNSUPPORTED,
                      "mirror planes need anisotropy entries symmetric about them (a_s(n) = a_s(n reflected))");
      }
    }
  }
  return LBPF_OK;
}

int validate(const lbpf_config &c) {
  if (c.lattice != LBPF_D2Q9_D2Q5 && c.lattice != LBPF_D3Q19_D3Q7 && c.lattice != LBPF_D3Q15_D3Q7)
    return fail(LBPF_ERR_ARG, "unknown lattice");
  const int dim = c.lattice == LBPF_D2Q9_D2Q5 ? 2 : 3;
  if (c.nx < 3 || c.ny < 3) return fail(LBPF_ERR_ARG, "nx and ny must be >= 3");
  if (dim == 2 && c.nz != 1) return fail(LBPF_ERR_ARG, "nz must be 1 for the 2D lattice pair");
  if (dim == 3 && c.nz < 3) return fail(LBPF_ERR_ARG, "nz must be >= 3 in 3D");
  {
    const long long elems = (long long)((c.nx + 63) / 64 * 64) * c.ny * c.nz;
    const long long esize = c.storage == LBPF_FP64 ? 8 : 4;
    if (elems * esize >= (1LL << 32))
      return fail(LBPF_ERR_ARG, "grid too large: one field must stay below 4 GiB (32-bit byte offsets)");
  }
  if (c.boundary != LBPF_PERIODIC && c.boundary != LBPF_ZERO_FLUX && c.boundary != LBPF_MIRROR_LOW)
    return fail(LBPF_ERR_ARG, "unknown boundary");
  if (c.gradient != LBPF_GRAD_DD && c.gradient != LBPF_GRAD_CD && c.gradient != LBPF_GRAD_UP2)
    return fail(LBPF_ERR_ARG, "unknown gradient");
  if (c.gradient == LBPF_GRAD_UP2) {
    if (c.boundary == LBPF_MIRROR_LOW)
      return fail(LBPF_ERR_UNSUPPORTED, "the upwind gradient runs without mirror planes");
    if (c.nx < 4 || c.ny < 4 || (dim == 3 && c.nz < 4))
      return fail(LBPF_ERR_ARG, "the upwind gradient needs every extent >= 4");
  }
  if (c.storage < LBPF_FP64 || c.storage > LBPF_FP16_OFFSET) return fail(LBPF_ERR_ARG, "unknown storage");
  if (!(c.W0 > 0) || !(c.tau0 > 0) || !(c.dx > 0) || !(c.kappa > 0) || !std::isfinite(c.lambda) ||
      !std::isfinite(c.delta) || !(c.xi >= 0))
    return fail(LBPF_ERR_ARG, "W0, tau0, dx, kappa must be > 0 and lambda, delta, xi finite");
  if (!(c.dt > 0)) return fail(LBPF_ERR_UNSTABLE, "dt must be > 0");
  if (c.n_aniso < 1 || c.n_aniso > kMaxAniso || !c.aniso) return fail(LBPF_ERR_ARG, "need 1..256 anisotropy entries");
  for (int k = 0; k < c.n_aniso; ++k) {
    const lbpf_aniso &a = c.aniso[k];
    if (a.kind < LBPF_ANISO_ISO || a.kind > LBPF_ANISO_CUBIC_S) return fail(LBPF_ERR_ARG, "unknown anisotropy kind");
    if (a.kind == LBPF_ANISO_SECTORAL && (a.q < 1 || a.q > 64)) return fail(LBPF_ERR_ARG, "sectoral q must be 1..64");
    if (!std::isfinite(a.eps) || !std::isfinite(a.gamma) || !std::isfinite(a.phi0))
      return fail(LBPF_ERR_ARG, "anisotropy parameters must be finite");
    const int rc = check_entry(a, dim, c.boundary == LBPF_MIRROR_LOW);
    if (rc) return rc;
  }
  if (c.use_ids && c.aniso[0].kind != LBPF_ANISO_ISO)
    return fail(LBPF_ERR_ARG, "with the index field, entry 0 must be isotropic");
  if (c.n_seeds < 0 || (c.n_seeds > 0 && !c.seeds)) return fail(LBPF_ERR_ARG, "bad seed list");
  for (int k = 0; k < c.n_seeds; ++k) {
    const lbpf_seed &s = c.seeds[k];
    if (s.crystal_id < 0 || (c.use_ids && s.crystal_id >= c.n_aniso))
      return fail(LBPF_ERR_ARG, "seed crystal id out of range");
    if (!std::isfinite(s.x) || !std::isfinite(s.y) || !std::isfinite(s.z) || !std::isfinite(s.radius))
      return fail(LBPF_ERR_ARG, "seed must be finite");
  }
  return LBPF_OK;
}

// Lattice-unit numbers (Eq. ThermalDiffusivity, Eq. LBE_RelaxationTime):
// Dphi = W0^2 dt/(tau0 dx^2), s = dt/tau0, Du = kappa dt/dx^2, eta_u = Du/e^2 + 1/2.
void units(const lbpf_config &c, SimHost &s) {
  const double inv_e2_p = 3.0;
  const double inv_e2_u = s.dim == 2 ? 3.0 : 4.0;
  const double Dphi = c.W0 * c.W0 * c.dt / (c.tau0 * c.dx * c.dx);
  const double Du = c.kappa * c.dt / (c.dx * c.dx);
  s.kphi = Dphi * inv_e2_p;
  s.s = c.dt / c.tau0;
  s.omega_u = 1.0 / (Du * inv_e2_u + 0.5);
  s.width = std::sqrt(2.0) * (c.W0 / c.dx);
}

// Default tile, from measurements at 512^3: FP64 (256 VGPRs, two work-groups
// of 4 x 64 per CU) 4 rows; FP32 arithmetic 12 rows (one work-group of 12
// waves per CU, 3 per SIMD: the 2-node halo of the coefficient pass then costs
// 1/3 of what it costs at 4 rows).  3D: 32 planes per work-group, fewer when
// that would leave fewer than 2048 work-groups, 64 on 12-row tiles when that
// still leaves 2560 or more.  2D: about 16384 work-groups,
// at least 16 rows each (8 in FP64).
void default_tile(SimHost &s) {
  TileDev &t = s.tile;
  t.ty = s.dim == 3 ? (s.storage == LBPF_FP64 ? 4 : 12) : 1;
  t.tiles_x = (s.nx + 63) / 64;
  t.tiles_y = s.dim == 3 ? (s.nyp + t.ty - 1) / t.ty : 1;
  const long long tiles = (long long)t.tiles_x * t.tiles_y;
  long long ch;
  if (s.dim == 3) {
    ch = std::min<long long>(32, std::max<long long>(8, s.nm * tiles / 2048));
    // 12-row tiles on boxes large enough to keep 10 work-groups per CU at 64
    // planes: 64 planes (fewer ring warm-up planes per node; at 512^3 0.8-1.1 %
    // faster in every FP32-arithmetic form, at 384^3 slower)
    if (t.ty == 12 && s.nm * tiles / 64 >= 2560) ch = 64;
  } else {
    ch = std::max<long long>(s.storage == LBPF_FP64 ? 8 : 16, (s.nm * tiles + 16383) / 16384);
  }
  ch = std::min<long long>(ch, s.nm);
  t.chunk = (int)ch;
  t.nchunks = (s.nm + t.chunk - 1) / t.chunk;
}

int set_tile(SimHost &s, int ty, int chunk) {
  TileDev t = s.tile;
  if (ty > 0) {
    if (s.dim == 2 && ty != 1) return fail(LBPF_ERR_UNSUPPORTED, "2D tiles are one row high");
    if (s.dim == 3 && ty != 4 && ty != 8 && ty != 12)
      return fail(LBPF_ERR_UNSUPPORTED, "tile_y must be 4, 8 or 12");
    if (s.dim == 3 && ty == 12 && s.storage == LBPF_FP64)
      return fail(LBPF_ERR_UNSUPPORTED, "tile_y 12 needs FP32 arithmetic");
    if (s.dim == 3 && ty == 8 && s.cfg.gradient == LBPF_GRAD_UP2)
      return fail(LBPF_ERR_UNSUPPORTED, "the upwind gradient runs on 4- and 12-row tiles");
    t.ty = ty;
  }
  if (chunk > 0) t.chunk = std::min(chunk, s.nm);
  t.tiles_x = (s.nx + 63) / 64;
  t.tiles_y = s.dim == 3 ? (s.nyp + t.ty - 1) / t.ty : 1;
  t.nchunks = (s.nm + t.chunk - 1) / t.chunk;
  if ((long long)t.tiles_x * t.tiles_y * t.nchunks > 0x7fffffffLL) return fail(LBPF_ERR_ARG, "too many work-groups");
  s.tile = t;
  return LBPF_OK;
}

// Workspace layout of one simulation starting at `cursor`.
void plan(const lbpf_config &c, SimHost &s, size_t &cursor) {
  s.cfg = c;
  s.dim = c.lattice == LBPF_D2Q9_D2Q5 ? 2 : 3;
  s.storage = c.storage;
  s.qp = s.dim == 2 ? 9 : (c.lattice == LBPF_D3Q15_D3Q7 ? 15 : 19);
  s.qu = s.dim == 2 ? 5 : 7;
  s.nx = c.nx;
  s.nyp = s.dim == 3 ? c.ny : 1;
  s.nm = s.dim == 3 ? c.nz : c.ny;
  s.pitch = (int)align_up((size_t)c.nx, 64);
  s.mstride = (long long)s.pitch * s.nyp;
  // Consecutive direction fields are offset by 17 x 64 extra elements: with a
  // power-of-two field size (512^3) the same node of every direction would
  // otherwise sit at the same address modulo large powers of two, i.e. in the
  // same HBM channel for all 26 concurrent streams.
  s.fstride = s.mstride * s.nm + kFieldSkew;
  s.dsz = c.storage == LBPF_FP64 ? 8 : (c.storage == LBPF_FP32_OFFSET ? 4 : 2);
  s.psz = c.storage == LBPF_FP64 ? 8 : 4;
  const size_t field = (size_t)s.fstride;
  size_t o = 0;
  s.off_g = o;
  o = align_up(o + field * s.qp * s.dsz);
  s.off_f = o;
  o = align_up(o + field * s.qu * s.dsz);
  s.off_phi = o;
  o = align_up(o + field * s.psz);
  s.off_us = o;
  if (c.storage != LBPF_FP64) o = align_up(o + field * 4);
  s.off_id = o;
  if (c.use_ids) o = align_up(o + field * 2);
  s.state_bytes = o;
  cursor = align_up(cursor);
  s.state_off[0] = cursor;
  cursor += s.state_bytes;
  s.state_off[1] = cursor;
  cursor += s.state_bytes;
  s.off_aniso = cursor;
  cursor = align_up(cursor + sizeof(AnisoDev) * (size_t)c.n_aniso);
  s.off_seeds = cursor;
  cursor = align_up(cursor + sizeof(SeedDev) * (size_t)std::max(1, c.n_seeds));
  s.off_part = cursor;
  cursor = align_up(cursor + sizeof(double) * kDiagVals * kDiagBlocks);
  s.off_res = cursor;
  cursor = align_up(cursor + sizeof(double) * (kDiagVals + 2));
}

// SimDev for a step that reads buffer `in` and writes buffer 1 - in.
SimDev make_dev(const lbpf_handle *h, const SimHost &s, int in) {
  SimDev d{};
  char *base = h->ws;
  char *A = base + s.state_off[in];
  char *B = base + s.state_off[1 - in];
  d.nx = s.nx;
  d.nyp = s.nyp;
  d.nm = s.nm;
  d.pitch = s.pitch;
  d.mstride = s.mstride;
  d.fstride = s.fstride;
  d.periodic = s.cfg.boundary == LBPF_PERIODIC;
  d.mirror = s.cfg.boundary == LBPF_MIRROR_LOW;
  d.grad_cd = s.cfg.gradient == LBPF_GRAD_CD;
  d.grad_up2 = s.cfg.gradient == LBPF_GRAD_UP2;
  d.use_ids = s.cfg.use_ids != 0;
  d.n_aniso = s.cfg.n_aniso;
  d.kphi = s.kphi;
  d.s = s.s;
  d.lambda = s.cfg.lambda;
  d.omega_u = s.omega_u;
  d.xi2 = s.cfg.xi * s.cfg.xi;
  d.kphi_f = (float)d.kphi;
  d.s_f = (float)d.s;
  d.lambda_f = (float)d.lambda;
  d.omega_u_f = (float)d.omega_u;
  d.xi2_f = (float)d.xi2;
  d.width = s.width;
  d.u0 = -s.cfg.delta;
  d.g_in = A + s.off_g;
  d.g_out = B + s.off_g;
  d.f_in = A + s.off_f;
  d.f_out = B + s.off_f;
  d.phi_in = A + s.off_phi;
  d.phi_out = B + s.off_phi;
  d.us_in = s.storage == LBPF_FP64 ? nullptr : reinterpret_cast<const float *>(A + s.off_us);
  d.us_out = s.storage == LBPF_FP64 ? nullptr : reinterpret_cast<float *>(B + s.off_us);
  d.id_in = s.cfg.use_ids ? reinterpret_cast<const int16_t *>(A + s.off_id) : nullptr;
  d.id_out = s.cfg.use_ids ? reinterpret_cast<int16_t *>(B + s.off_id) : nullptr;
  d.aniso = reinterpret_cast<const AnisoDev *>(base + s.off_aniso);
  return d;
}

// A SimDev whose *_out pointers address the current state (for init/import).
SimDev make_dev_current(const lbpf_handle *h, const SimHost &s) {
  SimDev d = make_dev(h, s, 1 - h->parity);
  return d;
}

int check_sim(const lbpf_handle *h, int sim) {
  if (!h) return fail(LBPF_ERR_ARG, "null handle");
  if (sim < 0 || sim >= (int)h->sims.size()) return fail(LBPF_ERR_ARG, "simulation index out of range");
  return LBPF_OK;
}

int plan_all(const lbpf_config *cfgs, int n_sims, std::vector<SimHost> &sims, size_t &total) {
  if (!cfgs || n_sims < 1) return fail(LBPF_ERR_ARG, "need at least one config");
  sims.assign(n_sims, SimHost());
  size_t cursor = 0;
  for (int k = 0; k < n_sims; ++k) {
    int rc = validate(cfgs[k]);
    if (rc) return rc;
    if (n_sims > 1 && (cfgs[k].lattice != LBPF_D2Q9_D2Q5 || cfgs[k].lattice != cfgs[0].lattice ||
                       cfgs[k].storage != cfgs[0].storage))
      return fail(LBPF_ERR_UNSUPPORTED, "a batched ensemble must be 2D with one storage mode");
    if (n_sims > 1 && (cfgs[k].use_ids != 0) != (cfgs[0].use_ids != 0))
      return fail(LBPF_ERR_UNSUPPORTED, "a batched ensemble must use the index field in all or none of its configs");
    if (n_sims > 1 && cfgs[k].gradient == LBPF_GRAD_UP2)
      return fail(LBPF_ERR_UNSUPPORTED, "the upwind gradient runs on single simulations");
    plan(cfgs[k], sims[k], cursor);
    sims[k].aniso.assign(cfgs[k].aniso, cfgs[k].aniso + cfgs[k].n_aniso);
    sims[k].seeds.assign(cfgs[k].seeds, cfgs[k].seeds + cfgs[k].n_seeds);
    sims[k].cfg.aniso = sims[k].aniso.data();
    sims[k].cfg.seeds = sims[k].seeds.data();
    units(cfgs[k], sims[k]);
    default_tile(sims[k]);
  }
  total = align_up(cursor);
  return LBPF_OK;
}

// Workspace of the batched tables, after the simulations.
void plan_batch(const std::vector<SimHost> &sims, BatchState &b, size_t &total) {
  b = BatchState();
  if (sims.size() < 2) return;
  b.on = true;
  b.ids = sims[0].cfg.use_ids != 0;
  b.mirror = false;
  for (const SimHost &sh : sims) b.mirror = b.mirror || sh.cfg.boundary == LBPF_MIRROR_LOW;
  b.storage = sims[0].storage;
  long long items = 0;
  for (const SimHost &s : sims) items += (long long)((s.nx + 63) / 64) * ((s.nm + kMinBatchChunk - 1) / kMinBatchChunk);
  b.max_items = (int)items;
  b.off_sims = align_up(total);
  total = align_up(b.off_sims + sizeof(SimDev) * 2 * sims.size());
  b.off_items = total;
  total = align_up(b.off_items + sizeof(BatchItem) * (size_t)b.max_items);
}

// Work list for `chunk` rows per item, in decreasing cost (rows plus the
// three warm-up planes, times the columns in use); ties keep (sim, x0, m0)
// order.  The order does not change results: items write disjoint nodes.
void build_items(const std::vector<SimHost> &sims, BatchState &b) {
  struct Keyed {
    long long cost;
    BatchItem it;
  };
  std::vector<Keyed> v;
  for (size_t k = 0; k < sims.size(); ++k) {
    const SimHost &s = sims[k];
    for (int x0 = 0; x0 < s.nx; x0 += 64)
      for (int m0 = 0; m0 < s.nm; m0 += b.chunk) {
        const int m1 = std::min(m0 + b.chunk, s.nm);
        v.push_back({(long long)(m1 - m0 + 3) * std::min(64, s.nx - x0), BatchItem{(int)k, x0, m0, m1}});
      }
  }
  std::stable_sort(v.begin(), v.end(), [](const Keyed &a, const Keyed &c) { return a.cost > c.cost; });
  b.items.resize(v.size());
  for (size_t i = 0; i < v.size(); ++i) b.items[i] = v[i].it;
  b.n_items = (int)v.size();
  b.grid = std::max(1, std::min(b.n_items, b.blocks_per_cu * b.n_cu));
}

}  // namespace

extern "C" {

const char *lb_pf_last_error(void) { return g_last_error.c_str(); }

int lb_pf_sharp_interface(double W0, double tau0, double lambda, double kappa, double *d0, double *beta,
                          double *lambda_star) {
  if (!(W0 > 0) || !(tau0 > 0) || !(kappa > 0) || !(lambda != 0)) return fail(LBPF_ERR_ARG, "bad parameters");
  const double a1 = 5.0 * std::sqrt(2.0) / 8.0, a2 = 0.6267;
  if (d0) *d0 = a1 * W0 / lambda;
  if (beta) *beta = a1 * (tau0 / (W0 * lambda) - a2 * W0 / kappa);
  if (lambda_star) *lambda_star = kappa * tau0 / (a2 * W0 * W0);
  return LBPF_OK;
}

int lb_pf_workspace_bytes(const lbpf_config *cfgs, int n_sims, size_t *bytes) {
  if (!bytes) return fail(LBPF_ERR_ARG, "bytes is NULL");
  std::vector<SimHost> sims;
  size_t total = 0;
  int rc = plan_all(cfgs, n_sims, sims, total);
  if (rc) return rc;
  BatchState b;
  plan_batch(sims, b, total);
  *bytes = total;
  return LBPF_OK;
}

int lb_pf_init(const lbpf_config *cfgs, int n_sims, void *dev_workspace, size_t bytes, void *hip_stream,
               lbpf_handle **out) {
  if (!out) return fail(LBPF_ERR_ARG, "out is NULL");
  *out = nullptr;
  lbpf_handle *h = new lbpf_handle();
  size_t total = 0;
  int rc = plan_all(cfgs, n_sims, h->sims, total);
  if (rc) {
    delete h;
    return rc;
  }
  plan_batch(h->sims, h->batch, total);
  if (!dev_workspace || (reinterpret_cast<uintptr_t>(dev_workspace) % kAlign) != 0 || bytes < total) {
    delete h;
    return fail(LBPF_ERR_WORKSPACE, "workspace NULL, not 256-byte aligned, or smaller than lb_pf_workspace_bytes()");
  }
  h->ws = static_cast<char *>(dev_workspace);
  h->bytes = bytes;
  h->parity = 0;
  {
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
      delete h;
      return fail(LBPF_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    rc = scratch_setup(h->device);
    if (rc) {
      delete h;
      return rc;
    }
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  for (SimHost &s : h->sims) {
    std::vector<AnisoDev> tab(s.cfg.n_aniso);
    for (int k = 0; k < s.cfg.n_aniso; ++k) tab[k] = to_dev(s.aniso[k]);
    std::vector<SeedDev> sd(std::max(1, s.cfg.n_seeds));
    for (int k = 0; k < s.cfg.n_seeds; ++k) {
      sd[k] = SeedDev{s.seeds[k].x, s.seeds[k].y, s.seeds[k].z, s.seeds[k].radius, s.seeds[k].crystal_id};
    }
    hipError_t e = hipMemcpyAsync(h->ws + s.off_aniso, tab.data(), sizeof(AnisoDev) * tab.size(),
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(h->ws + s.off_seeds, sd.data(), sizeof(SeedDev) * sd.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
      SimDev d = make_dev_current(h, s);
      InitSrc src{};
      src.seeds = reinterpret_cast<const SeedDev *>(h->ws + s.off_seeds);
      src.n_seeds = s.cfg.n_seeds;
      src.nx = s.cfg.nx;
      src.ny = s.cfg.ny;
      e = launch_init(s.cfg.lattice, s.storage, d, d.id_out, src, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      delete h;
      return fail(LBPF_ERR_HIP, std::string("initialisation failed: ") + hipGetErrorString(e));
    }
  }
  if (h->batch.on) {
    BatchState &b = h->batch;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&b.n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    b.blocks_per_cu = batch_blocks_per_cu(b.storage, b.ids, b.mirror);
    if (e == hipSuccess && b.blocks_per_cu < 1) e = hipErrorInvalidDeviceFunction;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b.cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete h;
      return fail(LBPF_ERR_HIP, std::string("batched set-up failed: ") + hipGetErrorString(e));
    }
    build_items(h->sims, b);
  } else {
    bool any_mirror = false;
    for (const SimHost &s : h->sims) any_mirror = any_mirror || s.cfg.boundary == LBPF_MIRROR_LOW;
    if (any_mirror) {
      hipError_t e = hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&h->fork, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&h->join, hipEventDisableTiming);
      if (e != hipSuccess) {
        release_aux(h);
        delete h;
        return fail(LBPF_ERR_HIP, std::string("mirror-box stream set-up failed: ") + hipGetErrorString(e));
      }
    }
  }
  *out = h;
  return LBPF_OK;
}

namespace {

void drop_graphs(BatchState &b) {
  for (auto &row : b.exec)
    for (hipGraphExec_t &g : row)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
}

// Uploads the SimDev tables of both parities and the work list (then waits,
// so that the host copies may change afterwards), and drops stale graphs.
int batch_upload(lbpf_handle *h, hipStream_t st) {
  BatchState &b = h->batch;
  const size_t n = h->sims.size();
  b.tables.resize(2 * n);
  for (int p = 0; p < 2; ++p)
    for (size_t k = 0; k < n; ++k) b.tables[p * n + k] = make_dev(h, h->sims[k], p);
  HIPCHK(hipMemcpyAsync(h->ws + b.off_sims, b.tables.data(), sizeof(SimDev) * b.tables.size(),
                        hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->ws + b.off_items, b.items.data(), sizeof(BatchItem) * b.items.size(),
                        hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  drop_graphs(b);
  b.dirty = false;
  return LBPF_OK;
}

// Graph of `steps` consecutive batched steps starting from parity p.
int batch_graph(lbpf_handle *h, int p, int kind) {
  BatchState &b = h->batch;
  if (b.exec[p][kind]) return LBPF_OK;
  const int steps = kind == 0 ? 1 : kGraphSteps;
  const SimDev *tab = reinterpret_cast<const SimDev *>(h->ws + b.off_sims);
  const BatchItem *items = reinterpret_cast<const BatchItem *>(h->ws + b.off_items);
  const size_t n = h->sims.size();
  HIPCHK(hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal));
  hipError_t le = hipSuccess;
  for (int k = 0; k < steps && le == hipSuccess; ++k)
    le = launch_batch(b.storage, b.ids, b.mirror, tab + ((p + k) & 1) * n, items, b.n_items, b.grid, b.cap);
  hipGraph_t g = nullptr;
  hipError_t ee = hipStreamEndCapture(b.cap, &g);
  if (le != hipSuccess || ee != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(LBPF_ERR_HIP, std::string("graph capture failed: ") +
                                  hipGetErrorString(le != hipSuccess ? le : ee));
  }
  hipError_t ie = hipGraphInstantiate(&b.exec[p][kind], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) {
    b.exec[p][kind] = nullptr;
    return fail(LBPF_ERR_HIP, std::string("graph instantiation failed: ") + hipGetErrorString(ie));
  }
  return LBPF_OK;
}

int batch_step(lbpf_handle *h, int n_steps, hipStream_t st) {
  BatchState &b = h->batch;
  if (b.dirty) {
    int rc = batch_upload(h, st);
    if (rc) return rc;
  }
  int n = n_steps;
  while (n >= kGraphSteps) {
    int rc = batch_graph(h, h->parity, 1);
    if (rc) return rc;
    HIPCHK(hipGraphLaunch(b.exec[h->parity][1], st));
    n -= kGraphSteps;
    h->step += kGraphSteps;
  }
  for (; n > 0; --n) {
    int rc = batch_graph(h, h->parity, 0);
    if (rc) return rc;
    HIPCHK(hipGraphLaunch(b.exec[h->parity][0], st));
    h->parity ^= 1;
    h->step++;
  }
  return LBPF_OK;
}


// One step of simulation s.  A box with mirror planes whose tiling leaves
// tiles beyond the mirror rules' reach runs them with the instance without
// mirror planes (fewer registers and instructions) on st, and the tiles at a
// plane with the mirror instance on the handle's aux stream, concurrently;
// st then waits for both.  Either way every node is written once.
hipError_t step_sim(lbpf_handle *h, const SimHost &s, const SimDev &d, hipStream_t st) {
  const TileDev &t = s.tile;
  const bool split = d.mirror && !d.grad_up2 && h->aux && t.chunk >= 4 && (s.dim == 2 || t.ty >= 4) &&
                     t.tiles_x >= 2 && t.nchunks >= 2 && (s.dim == 2 || t.tiles_y >= 2);
  if (!split) return launch_step(s.cfg.lattice, s.storage, d, t, st);
  TileDev at = t, rest = t;
  at.part = 1;
  rest.part = 2;
  hipError_t e = hipEventRecord(h->fork, st);
  if (e == hipSuccess) e = hipStreamWaitEvent(h->aux, h->fork, 0);
  if (e == hipSuccess) e = launch_step(s.cfg.lattice, s.storage, d, at, h->aux);
  if (e == hipSuccess) e = launch_step(s.cfg.lattice, s.storage, d, rest, st);
  if (e == hipSuccess) e = hipEventRecord(h->join, h->aux);
  if (e == hipSuccess) e = hipStreamWaitEvent(st, h->join, 0);
  return e;
}

}  // namespace

int lb_pf_step(lbpf_handle *h, int n_steps, void *hip_stream) {
  if (!h) return fail(LBPF_ERR_ARG, "null handle");
  if (n_steps < 0) return fail(LBPF_ERR_ARG, "n_steps < 0");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (h->batch.on) return batch_step(h, n_steps, st);
  for (int n = 0; n < n_steps; ++n) {
    for (const SimHost &s : h->sims) {
      const SimDev d = make_dev(h, s, h->parity);
      HIPCHK(step_sim(h, s, d, st));
    }
    h->parity ^= 1;
    h->step++;
  }
  return LBPF_OK;
}

namespace {
// The diagnostics of every simulation; partials/result of the reductions in
// the workspace (static_part == nullptr) or in the static scratch array.
int run_diagnostics(lbpf_handle *h, lbpf_diag *out, hipStream_t st, double *static_part) {
  int bad = 0;
  for (size_t k = 0; k < h->sims.size(); ++k) {
    const SimHost &s = h->sims[k];
    const SimDev d = make_dev(h, s, h->parity);
    int dir[3] = {s.cfg.tip_dir[0], s.cfg.tip_dir[1], s.cfg.tip_dir[2]};
    if (!dir[0] && !dir[1] && !dir[2]) dir[0] = 1;
    int o[3] = {s.cfg.nx / 2, s.cfg.ny / 2, s.cfg.nz / 2};
    if (s.cfg.n_seeds > 0) {
      o[0] = (int)std::floor(s.seeds[0].x + 0.5);
      o[1] = (int)std::floor(s.seeds[0].y + 0.5);
      o[2] = (int)std::floor(s.seeds[0].z + 0.5);
    }
    double *part = static_part ? static_part : reinterpret_cast<double *>(h->ws + s.off_part);
    double *res = static_part ? static_part + kDiagVals * kDiagBlocks : reinterpret_cast<double *>(h->ws + s.off_res);
    HIPCHK(launch_diag(s.dim, s.storage, d, part, res, 0, o[0], o[1], o[2], dir[0], dir[1], dir[2], st));
    double host[kDiagVals + 1];
    HIPCHK(hipMemcpyAsync(host, res, sizeof(host), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double N = (double)s.cfg.nx * s.cfg.ny * s.cfg.nz;
    lbpf_diag &r = out[k];
    r.step = h->step;
    r.sum_phi = host[0];
    r.sum_u = host[1];
    r.sum_u_minus_half_phi = host[2];
    r.solid_fraction = host[3] / (2.0 * N);
    r.n_solid = host[4];
    r.nonfinite = host[5] != 0.0;
    r.tip_position = host[kDiagVals];
    bad |= r.nonfinite;
  }
  if (bad) return fail(LBPF_ERR_NONFINITE, "non-finite phi or u");
  return LBPF_OK;
}
}  // namespace

int lb_pf_diagnostics(lbpf_handle *h, lbpf_diag *out, void *hip_stream) {
  if (!h || !out) return fail(LBPF_ERR_ARG, "null argument");
  return run_diagnostics(h, out, static_cast<hipStream_t>(hip_stream), nullptr);
}

int lb_pf_diagnostics_noalloc(lbpf_handle *h, lbpf_diag *out, void *hip_stream) {
  if (!h || !out) return fail(LBPF_ERR_ARG, "null argument");
  // the reductions need kDiagVals partials per block and kDiagVals + 1 results
  constexpr size_t need = (size_t)kDiagVals * kDiagBlocks + kDiagVals + 2;
  static_assert(need <= (size_t)kScratchDoubles, "diagnostics scratch exceeds the static array");
  if (need > (size_t)kScratchDoubles)
    return fail(LBPF_ERR_UNSUPPORTED, "diagnostics need more scratch than the static array holds");
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != h->device) return fail(LBPF_ERR_ARG, "the handle's device is not the current device");
  double *ptr = scratch_of(dev);
  if (!ptr) return fail(LBPF_ERR_HIP, "static scratch not set up on this device");
  return run_diagnostics(h, out, static_cast<hipStream_t>(hip_stream), ptr);
}

int lb_pf_export_fields(lbpf_handle *h, int sim, double *phi_dev, double *u_dev, int16_t *ids_dev,
                        void *hip_stream) {
  int rc = check_sim(h, sim);
  if (rc) return rc;
  const SimHost &s = h->sims[sim];
  HIPCHK(launch_export(s.cfg.lattice, s.storage, make_dev(h, s, h->parity), phi_dev, u_dev, ids_dev, nullptr, nullptr,
                       s.cfg.ny, static_cast<hipStream_t>(hip_stream)));
  return LBPF_OK;
}

int lb_pf_export_dists(lbpf_handle *h, int sim, double *g_dev, double *f_dev, void *hip_stream) {
  int rc = check_sim(h, sim);
  if (rc) return rc;
  const SimHost &s = h->sims[sim];
  HIPCHK(launch_export(s.cfg.lattice, s.storage, make_dev(h, s, h->parity), nullptr, nullptr, nullptr, g_dev, f_dev,
                       s.cfg.ny, static_cast<hipStream_t>(hip_stream)));
  return LBPF_OK;
}

int lb_pf_import_fields(lbpf_handle *h, int sim, const double *phi_dev, const double *u_dev,
                        const int16_t *ids_dev, void *hip_stream) {
  int rc = check_sim(h, sim);
  if (rc) return rc;
  if (!phi_dev || !u_dev) return fail(LBPF_ERR_ARG, "phi and u are required");
  const SimHost &s = h->sims[sim];
  SimDev d = make_dev_current(h, s);
  InitSrc src{};
  src.phi = phi_dev;
  src.u = u_dev;
  src.ids = ids_dev;
  src.nx = s.cfg.nx;
  src.ny = s.cfg.ny;
  HIPCHK(launch_init(s.cfg.lattice, s.storage, d, d.id_out, src, static_cast<hipStream_t>(hip_stream)));
  return LBPF_OK;
}

namespace {
// FNV-1a over what must match between a saved blob and the loading handle.
unsigned long long state_layout(const lbpf_handle *h) {
  unsigned long long v = 1469598103934665603ULL;
  auto mix = [&](long long x) {
    for (int k = 0; k < 8; ++k) {
      v ^= (unsigned long long)((x >> (8 * k)) & 0xff);
      v *= 1099511628211ULL;
    }
  };
  for (const SimHost &s : h->sims) {
    mix(s.cfg.lattice);
    mix(s.cfg.nx);
    mix(s.cfg.ny);
    mix(s.cfg.nz);
    mix(s.storage);
    mix(s.cfg.use_ids);
    mix((long long)s.state_bytes);
  }
  return v;
}
}  // namespace

int lb_pf_state_bytes(const lbpf_handle *h, size_t *bytes) {
  if (!h || !bytes) return fail(LBPF_ERR_ARG, "null argument");
  size_t b = kStateHeaderBytes;
  for (const SimHost &s : h->sims) b += s.state_bytes;
  *bytes = b;
  return LBPF_OK;
}

int lb_pf_save_state(lbpf_handle *h, void *dev_buf, size_t bytes, void *hip_stream) {
  size_t need = 0;
  int rc = lb_pf_state_bytes(h, &need);
  if (rc) return rc;
  if (!dev_buf || bytes < need) return fail(LBPF_ERR_ARG, "state buffer too small");
  if (reinterpret_cast<uintptr_t>(dev_buf) % 8 != 0) return fail(LBPF_ERR_ARG, "state buffer not 8-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  StateHeader hd{kStateMagic, 1, (long long)h->sims.size(), (long long)h->step, (unsigned long long)need,
                 state_layout(h)};
  HIPCHK(launch_state_header(static_cast<StateHeader *>(dev_buf), hd, st));
  char *dst = static_cast<char *>(dev_buf) + kStateHeaderBytes;
  for (const SimHost &s : h->sims) {
    HIPCHK(hipMemcpyAsync(dst, h->ws + s.state_off[h->parity], s.state_bytes, hipMemcpyDeviceToDevice, st));
    dst += s.state_bytes;
  }
  return LBPF_OK;
}

int lb_pf_load_state(lbpf_handle *h, const void *dev_buf, size_t bytes, void *hip_stream) {
  size_t need = 0;
  int rc = lb_pf_state_bytes(h, &need);
  if (rc) return rc;
  if (!dev_buf || bytes < need) return fail(LBPF_ERR_ARG, "state buffer too small");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  StateHeader hd{};
  HIPCHK(hipMemcpyAsync(&hd, dev_buf, sizeof(hd), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hd.magic != kStateMagic || hd.version != 1 || hd.n_sims != (long long)h->sims.size() ||
      hd.bytes != (unsigned long long)need || hd.layout != state_layout(h) || hd.step < 0)
    return fail(LBPF_ERR_ARG, "the blob is not a checkpoint of a handle with this layout");
  const char *src = static_cast<const char *>(dev_buf) + kStateHeaderBytes;
  for (const SimHost &s : h->sims) {
    HIPCHK(hipMemcpyAsync(h->ws + s.state_off[h->parity], src, s.state_bytes, hipMemcpyDeviceToDevice, st));
    src += s.state_bytes;
  }
  h->step = hd.step;
  return LBPF_OK;
}

int lb_pf_stream_copy(const void *src_dev, void *dst_dev, size_t bytes, int blocks_per_cu, void *hip_stream) {
  if (!src_dev || !dst_dev) return fail(LBPF_ERR_ARG, "null buffer");
  if (reinterpret_cast<uintptr_t>(src_dev) % 16 != 0 || reinterpret_cast<uintptr_t>(dst_dev) % 16 != 0)
    return fail(LBPF_ERR_ARG, "buffers must be 16-byte aligned");
  if (blocks_per_cu < 1 || blocks_per_cu > 64) return fail(LBPF_ERR_ARG, "blocks_per_cu must be 1..64");
  const char *s = static_cast<const char *>(src_dev);
  const char *d = static_cast<const char *>(dst_dev);
  if (s < d + bytes && d < s + bytes) return fail(LBPF_ERR_ARG, "buffers overlap");
  if (bytes == 0) return LBPF_OK;
  HIPCHK(launch_stream_copy(src_dev, dst_dev, bytes, blocks_per_cu, static_cast<hipStream_t>(hip_stream)));
  return LBPF_OK;
}

int lb_pf_state_ptr(const lbpf_handle *h, int sim, void **state, size_t *bytes) {
  int rc = check_sim(h, sim);
  if (rc) return rc;
  const SimHost &s = h->sims[sim];
  if (state) *state = h->ws + s.state_off[h->parity];
  if (bytes) *bytes = s.state_bytes;
  return LBPF_OK;
}

int lb_pf_set_tile(lbpf_handle *h, int tile_y, int chunk) {
  if (!h) return fail(LBPF_ERR_ARG, "null handle");
  if (h->batch.on) {
    if (tile_y > 1) return fail(LBPF_ERR_UNSUPPORTED, "2D tiles are one row high");
    if (chunk > 0) {
      if (chunk < kMinBatchChunk) return fail(LBPF_ERR_ARG, "batched work items need at least 8 rows");
      if (chunk != h->batch.chunk) {
        h->batch.chunk = chunk;
        build_items(h->sims, h->batch);
        h->batch.dirty = true;
      }
    }
    return LBPF_OK;
  }
  for (SimHost &s : h->sims) {
    int rc = set_tile(s, tile_y, chunk);
    if (rc) return rc;
  }
  return LBPF_OK;
}

int lb_pf_get_tile(const lbpf_handle *h, int *tile_y, int *chunk) {
  if (!h) return fail(LBPF_ERR_ARG, "null handle");
  if (tile_y) *tile_y = h->sims[0].tile.ty;
  if (chunk) *chunk = h->batch.on ? h->batch.chunk : h->sims[0].tile.chunk;
  return LBPF_OK;
}

int lb_pf_autotune(lbpf_handle *h, int steps_per_trial, void *hip_stream) {
  if (!h) return fail(LBPF_ERR_ARG, "null handle");
  if (steps_per_trial < 1) return fail(LBPF_ERR_ARG, "steps_per_trial < 1");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const SimHost &s0 = h->sims[0];
  std::vector<int> tys = s0.dim == 3 ? std::vector<int>{4, 8, 12} : std::vector<int>{1};
  std::vector<int> chunks = s0.dim == 3 ? std::vector<int>{16, 32, 64, 128} : std::vector<int>{8, 16, 32, 64};
  // the two timing events, destroyed on every return
  struct Events {
    hipEvent_t e[2] = {nullptr, nullptr};
    ~Events() {
      for (hipEvent_t x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } ev;
  HIPCHK(hipEventCreate(&ev.e[0]));
  HIPCHK(hipEventCreate(&ev.e[1]));
  hipEvent_t e0 = ev.e[0], e1 = ev.e[1];
  float best = 1e30f;
  int bty = s0.tile.ty, bch = h->batch.on ? h->batch.chunk : s0.tile.chunk;
  for (int ty : tys) {
    if (s0.dim == 3 && ((ty == 12 && s0.storage == LBPF_FP64) || (ty == 8 && s0.cfg.gradient == LBPF_GRAD_UP2)))
      continue;
    for (int ch : chunks) {
      if (lb_pf_set_tile(h, ty, ch)) continue;
      // warm-up of twice the trial: the trial then starts from the same
      // parity and finds every graph it replays already captured
      int rc = lb_pf_step(h, 2 * steps_per_trial, hip_stream);
      if (rc) return rc;
      HIPCHK(hipEventRecord(e0, st));
      rc = lb_pf_step(h, steps_per_trial, hip_stream);
      if (rc) return rc;
      HIPCHK(hipEventRecord(e1, st));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        bty = ty;
        bch = ch;
      }
    }
  }
  return lb_pf_set_tile(h, bty, bch);
}

int lb_pf_info(const lbpf_handle *h, int sim, int64_t *nodes, int64_t *step, int *q_phi, int *q_u) {
  int rc = check_sim(h, sim);
  if (rc) return rc;
  const SimHost &s = h->sims[sim];
  if (nodes) *nodes = (int64_t)s.cfg.nx * s.cfg.ny * s.cfg.nz;
  if (step) *step = h->step;
  if (q_phi) *q_phi = s.qp;
  if (q_u) *q_u = s.qu;
  return LBPF_OK;
}

int lb_pf_destroy(lbpf_handle *h) {
  if (!h) return LBPF_OK;
  BatchState &b = h->batch;
  if (b.cap) {
    // graphs of this handle may still run on the caller's streams
    (void)hipDeviceSynchronize();
    drop_graphs(b);
    (void)hipStreamDestroy(b.cap);
  }
  release_aux(h);
  delete h;
  return LBPF_OK;
}

}  // extern "C"

/*
 * CPU FP64 oracle for the coupled lattice Boltzmann phase-field step of
 * Younsi & Cartalade (arXiv:1606.09432).  TEST INFRASTRUCTURE ONLY: only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark use it.
 *
 * Plain whole-grid passes, one per stage of the method, in the order of the
 * paper's algorithm (Sec. 3.1 and 3.2):
 *
 *   phase-field equation (Sec. 3.2)
 *     1. gradient of phi: directional derivatives along every lattice vector
 *        (Eq. Def_DeriveeDirectionnelle) and their weighted first moment
 *        (Eq. Grad_DF-Centree); or central differences (Sec. 4.2).
 *     2. crystal index update, when the index field is on (Sec. 4.3).
 *     3. n (Eq. Def_Normal_Vector), a_s (Sec. 4.1), N (Eq. TermesAnisotropes),
 *        eta_phi (Eq. LBE_RelaxationTime), Q_phi (Eq. LBE_SourceTerm).
 *     4. collision with the nonlocal a_s^2 term and streaming (Eq. LBE_Eq_Phase)
 *        with the equilibrium of Eq. Feq_Phase.
 *     5. bounce-back at the walls (Eq. Bounce-Back).
 *     6. phi = sum g (Eq. Def_M0_Phi).
 *   heat equation (Sec. 3.1), solved after the phase field
 *     7. Q_u dt = (phi(t+dt) - phi(t))/2 (Eq. Source_Tempr, explicit Euler).
 *     8. BGK collision toward w_i u (Eq. EqFunction_Tempr) and streaming
 *        (Eq. LBE_Eq_Temp); bounce-back; u = sum f (Eq. Temperature_LB).
 *
 * Readings where the paper is silent or garbled (all documented in the
 * project's design notes):
 *   - D3Q19 is not tabulated in the paper; the standard weights 1/3, 1/18,
 *     1/36 with e^2 = 1/3 are used.
 *   - The seed profile is tanh((R - d)/(sqrt(2) W0)) in lattice units with
 *     W0 -> W0/dx; several seeds combine by pointwise maximum.
 *   - a_s^2 multiplying the nonlocal term is evaluated at the source node x.
 *   - Bounce-back: after streaming, an unknown incoming g_i (its source lies
 *     outside the box) takes the streamed g_i' of the opposite direction at the
 *     same node.  When the source of g_i' is outside too (edges, corners), g_i
 *     takes the post-collision g_i'* of the same node (no nonlocal term);
 *     parity unpinned for this edge and corner case: nothing outside the two
 *     implementations fixes it (the paper shows a flat wall only).  The
 *     same rule holds for f.  Ghost phi values for gradients are mirrored about
 *     the wall node: phi(-1) = phi(1).
 *   - Symmetric boxes (mirror_low): Sec. 5 computes one octant of a dendrite
 *     grown from a seed at the origin and completes it by symmetry about the
 *     planes XY, YZ and XZ, without saying how the symmetry planes are
 *     treated.  Here they are exact mirror planes through node 0: the state
 *     beyond them is the mirror image of the state inside (phi, u and the
 *     index at -k are those at +k; the population i there is the mirror image
 *     of population i' at +k), and each pass applies its own rule to that
 *     mirror-extended state.  The far walls are zero flux.
 *   - |p| <= 1e-8 (lattice units): n is taken as undefined, a_s = 1, N = 0.
 *     The paper leaves n = -grad phi/|grad phi| undefined where the gradient
 *     vanishes.  Below 1e-8 the FP64 rounding of the phi differences (about
 *     1e-16) decides the direction of n, and a_s(n), which varies by O(eps)
 *     with the direction, would turn rounding into O(eps) changes of the local
 *     relaxation; the bulk there is within 1e-8 of +-1, with no interface.
 *   - Crystal index: a node with I = 0 whose gradient exceeds xi takes the
 *     index of the phi-lattice neighbour with nonzero index and largest phi
 *     (ties: smaller index); the updated index is used in the same step.
 *
 * Arithmetic: FP64, built with -ffp-contract=off.  Every sum over lattice
 * directions uses a fixed tree that is invariant under a 90 degree rotation
 * about z, so that rotated inputs give bitwise rotated outputs.
 */
#include "lbpf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Lattices (Sec. 3.3, Table Values-Lattices).                               */
/* ------------------------------------------------------------------------ */
typedef struct {
  int q;
  int e[19][3];
  double w[19];
  int opp[19];
  double e2;
  double inv_e2;
} lat_t;

static void lat_finish(lat_t *L) {
  for (int i = 0; i < L->q; ++i) {
    L->opp[i] = -1;
    for (int j = 0; j < L->q; ++j)
      if (L->e[j][0] == -L->e[i][0] && L->e[j][1] == -L->e[i][1] && L->e[j][2] == -L->e[i][2])
        L->opp[i] = j;
  }
}

static void lat_set_dir(lat_t *L, int i, int x, int y, int z, double w) {
  L->e[i][0] = x;
  L->e[i][1] = y;
  L->e[i][2] = z;
  L->w[i] = w;
}

/* which: 0 D2Q5, 1 D2Q9, 2 D3Q7, 3 D3Q19, 4 D3Q15 */
static int lat_make(int which, lat_t *L) {
  memset(L, 0, sizeof(*L));
  switch (which) {
  case 0: /* D2Q5: w0 = 1/3, w1..4 = 1/6, e^2 = 1/3 */
    L->q = 5;
    lat_set_dir(L, 0, 0, 0, 0, 1.0 / 3.0);
    lat_set_dir(L, 1, 1, 0, 0, 1.0 / 6.0);
    lat_set_dir(L, 2, 0, 1, 0, 1.0 / 6.0);
    lat_set_dir(L, 3, -1, 0, 0, 1.0 / 6.0);
    lat_set_dir(L, 4, 0, -1, 0, 1.0 / 6.0);
    L->e2 = 1.0 / 3.0;
    L->inv_e2 = 3.0;
    break;
  case 1: /* D2Q9: 4/9, 1/9, 1/36, e^2 = 1/3 */
    L->q = 9;
    lat_set_dir(L, 0, 0, 0, 0, 4.0 / 9.0);
    lat_set_dir(L, 1, 1, 0, 0, 1.0 / 9.0);
    lat_set_dir(L, 2, 0, 1, 0, 1.0 / 9.0);
    lat_set_dir(L, 3, -1, 0, 0, 1.0 / 9.0);
    lat_set_dir(L, 4, 0, -1, 0, 1.0 / 9.0);
    lat_set_dir(L, 5, 1, 1, 0, 1.0 / 36.0);
    lat_set_dir(L, 6, -1, 1, 0, 1.0 / 36.0);
    lat_set_dir(L, 7, -1, -1, 0, 1.0 / 36.0);
    lat_set_dir(L, 8, 1, -1, 0, 1.0 / 36.0);
    L->e2 = 1.0 / 3.0;
    L->inv_e2 = 3.0;
    break;
  case 2: /* D3Q7: 1/4, 1/8, e^2 = 1/4 */
    L->q = 7;
    lat_set_dir(L, 0, 0, 0, 0, 1.0 / 4.0);
    lat_set_dir(L, 1, 1, 0, 0, 1.0 / 8.0);
    lat_set_dir(L, 2, 0, 1, 0, 1.0 / 8.0);
    lat_set_dir(L, 3, -1, 0, 0, 1.0 / 8.0);
    lat_set_dir(L, 4, 0, -1, 0, 1.0 / 8.0);
    lat_set_dir(L, 5, 0, 0, 1, 1.0 / 8.0);
    lat_set_dir(L, 6, 0, 0, -1, 1.0 / 8.0);
    L->e2 = 1.0 / 4.0;
    L->inv_e2 = 4.0;
    break;
  case 3: /* D3Q19 (standard; not tabulated in the paper): 1/3, 1/18, 1/36 */
    L->q = 19;
    lat_set_dir(L, 0, 0, 0, 0, 1.0 / 3.0);
    lat_set_dir(L, 1, 1, 0, 0, 1.0 / 18.0);
    lat_set_dir(L, 2, 0, 1, 0, 1.0 / 18.0);
    lat_set_dir(L, 3, -1, 0, 0, 1.0 / 18.0);
    lat_set_dir(L, 4, 0, -1, 0, 1.0 / 18.0);
    lat_set_dir(L, 5, 0, 0, 1, 1.0 / 18.0);
    lat_set_dir(L, 6, 0, 0, -1, 1.0 / 18.0);
    lat_set_dir(L, 7, 1, 1, 0, 1.0 / 36.0);
    lat_set_dir(L, 8, -1, 1, 0, 1.0 / 36.0);
    lat_set_dir(L, 9, -1, -1, 0, 1.0 / 36.0);
    lat_set_dir(L, 10, 1, -1, 0, 1.0 / 36.0);
    lat_set_dir(L, 11, 1, 0, 1, 1.0 / 36.0);
    lat_set_dir(L, 12, 0, 1, 1, 1.0 / 36.0);
    lat_set_dir(L, 13, -1, 0, 1, 1.0 / 36.0);
    lat_set_dir(L, 14, 0, -1, 1, 1.0 / 36.0);
    lat_set_dir(L, 15, 1, 0, -1, 1.0 / 36.0);
    lat_set_dir(L, 16, 0, 1, -1, 1.0 / 36.0);
    lat_set_dir(L, 17, -1, 0, -1, 1.0 / 36.0);
    lat_set_dir(L, 18, 0, -1, -1, 1.0 / 36.0);
    L->e2 = 1.0 / 3.0;
    L->inv_e2 = 3.0;
    break;
  case 4: /* D3Q15 (Table Values-Lattices): 2/9, 1/9, 1/72; the paper's order */
    L->q = 15;
    lat_set_dir(L, 0, 0, 0, 0, 2.0 / 9.0);
    lat_set_dir(L, 1, 1, 0, 0, 1.0 / 9.0);
    lat_set_dir(L, 2, 0, 1, 0, 1.0 / 9.0);
    lat_set_dir(L, 3, -1, 0, 0, 1.0 / 9.0);
    lat_set_dir(L, 4, 0, -1, 0, 1.0 / 9.0);
    lat_set_dir(L, 5, 0, 0, 1, 1.0 / 9.0);
    lat_set_dir(L, 6, 0, 0, -1, 1.0 / 9.0);
    lat_set_dir(L, 7, 1, 1, 1, 1.0 / 72.0);
    lat_set_dir(L, 8, -1, 1, 1, 1.0 / 72.0);
    lat_set_dir(L, 9, -1, -1, 1, 1.0 / 72.0);
    lat_set_dir(L, 10, 1, -1, 1, 1.0 / 72.0);
    lat_set_dir(L, 11, 1, 1, -1, 1.0 / 72.0);
    lat_set_dir(L, 12, -1, 1, -1, 1.0 / 72.0);
    lat_set_dir(L, 13, -1, -1, -1, 1.0 / 72.0);
    lat_set_dir(L, 14, 1, -1, -1, 1.0 / 72.0);
    L->e2 = 1.0 / 3.0;
    L->inv_e2 = 3.0;
    break;
  default:
    return -1;
  }
  lat_finish(L);
  return 0;
}

/* Sum over directions with a tree that maps onto itself under the 90 degree
 * rotation about z (1->2->3->4->1, and likewise inside every diagonal orbit). */
static double lat_sum(const lat_t *L, const double *v) {
  switch (L->q) {
  case 5:
    return v[0] + ((v[1] + v[3]) + (v[2] + v[4]));
  case 9:
    return v[0] + (((v[1] + v[3]) + (v[2] + v[4])) + ((v[5] + v[7]) + (v[6] + v[8])));
  case 7:
    return v[0] + (((v[1] + v[3]) + (v[2] + v[4])) + (v[5] + v[6]));
  case 15:
    return v[0] + ((((v[1] + v[3]) + (v[2] + v[4])) + (v[5] + v[6])) +
                   (((v[7] + v[9]) + (v[8] + v[10])) + ((v[11] + v[13]) + (v[12] + v[14]))));
  default: /* 19 */
    return v[0] + ((((v[1] + v[3]) + (v[2] + v[4])) + (v[5] + v[6])) +
                   (((v[7] + v[9]) + (v[8] + v[10])) +
                    (((v[11] + v[13]) + (v[12] + v[14])) + ((v[15] + v[17]) + (v[16] + v[18])))));
  }
}

/* ------------------------------------------------------------------------ */
/* Anisotropy functions (Sec. 4.1).  a = A(n); G = gradient of the          */
/* polynomial A with respect to n (only its tangential part is used).       */
/* ------------------------------------------------------------------------ */
static void poly_eval(const orc_aniso *an, const double n[3], double *a, double G[3]) {
  G[0] = G[1] = G[2] = 0.0;
  if (an == NULL || an->kind == ORC_ANISO_ISO) {
    *a = 1.0;
    return;
  }
  const double nx = n[0], ny = n[1], nz = n[2];
  if (an->kind == ORC_ANISO_SECTORAL) {
    /* cos q(phi - phi0) = Re[z^q e^{-i q phi0}], z = n_x + i n_y (Eq. As_Theta);
     * for |n| < 1 in 3D this is the sectoral harmonic of Eq. As_Y66. */
    const int q = an->q;
    const double cr = cos(q * an->phi0), ci = -sin(q * an->phi0);
    double pr = 1.0, pi = 0.0; /* z^(q-1) */
    for (int k = 1; k < q; ++k) {
      const double tr = pr * nx - pi * ny;
      const double ti = pr * ny + pi * nx;
      pr = tr;
      pi = ti;
    }
    const double zr = pr * nx - pi * ny, zi = pr * ny + pi * nx; /* z^q */
    const double re = zr * cr - zi * ci;
    *a = 1.0 + an->eps * re;
    /* d/dn_x Re[z^q c] = Re[q z^(q-1) c];  d/dn_y = Re[i q z^(q-1) c] */
    const double wr = pr * cr - pi * ci, wi = pr * ci + pi * cr;
    G[0] = an->eps * (q * wr);
    G[1] = -(an->eps * (q * wi));
    return;
  }
  const double x2 = nx * nx, y2 = ny * ny, z2 = nz * nz;
  const double Q = (x2 * x2 + y2 * y2) + z2 * z2;
  if (an->kind == ORC_ANISO_CUBIC) {
    /* Eq. As_Function_Classical: 1 - 3 eps + 4 eps Q */
    const double eps = an->eps;
    *a = (1.0 - 3.0 * eps) + 4.0 * eps * Q;
    G[0] = 16.0 * eps * (x2 * nx);
    G[1] = 16.0 * eps * (y2 * ny);
    G[2] = 16.0 * eps * (z2 * nz);
    return;
  }
  if (an->kind == ORC_ANISO_CUBIC_S) {
    /* Eq. As_Function_S read as 1 + 66 gamma S, S = n_x^2 n_y^2 n_z^2 */
    const double gam = an->gamma;
    *a = 1.0 + 66.0 * gam * ((x2 * y2) * z2);
    G[0] = 66.0 * gam * (2.0 * nx * (y2 * z2));
    G[1] = 66.0 * gam * (2.0 * ny * (x2 * z2));
    G[2] = 66.0 * gam * (2.0 * nz * (x2 * y2));
    return;
  }
  /* ORC_ANISO_CUBIC_HAK, Eq. As_MatSci: 1 + eps (Q - 3/5) + gamma (3Q + 66 S - 17/7) */
  const double eps = an->eps, gam = an->gamma;
  const double S = (x2 * y2) * z2;
  *a = 1.0 + eps * (Q - 3.0 / 5.0) + gam * ((3.0 * Q + 66.0 * S) - 17.0 / 7.0);
  const double dQx = 4.0 * (x2 * nx), dQy = 4.0 * (y2 * ny), dQz = 4.0 * (z2 * nz);
  const double dSx = 2.0 * nx * (y2 * z2), dSy = 2.0 * ny * (x2 * z2), dSz = 2.0 * nz * (x2 * y2);
  G[0] = eps * dQx + gam * (3.0 * dQx + 66.0 * dSx);
  G[1] = eps * dQy + gam * (3.0 * dQy + 66.0 * dSy);
  G[2] = eps * dQz + gam * (3.0 * dQz + 66.0 * dSz);
}

static int has_rotation(const orc_aniso *an) {
  for (int k = 0; k < 9; ++k)
    if (an->R[k] != 0.0) return 1;
  return 0;
}

/* The entry's orientation: a(n) = A(R n) for the polynomial A of its kind, and
 * by the chain rule grad_n a = R^T (grad A)(R n). */
void orc_aniso_eval(const orc_aniso *an, const double n[3], double *a, double G[3]) {
  if (an == NULL || an->kind == ORC_ANISO_ISO || !has_rotation(an)) {
    poly_eval(an, n, a, G);
    return;
  }
  const double *R = an->R;
  double m[3], Gm[3];
  for (int r = 0; r < 3; ++r) m[r] = (R[3 * r] * n[0] + R[3 * r + 1] * n[1]) + R[3 * r + 2] * n[2];
  poly_eval(an, m, a, Gm);
  for (int c = 0; c < 3; ++c) G[c] = (R[c] * Gm[0] + R[3 + c] * Gm[1]) + R[6 + c] * Gm[2];
}

/* Unit directions on which entries are checked: a Fibonacci lattice of 4000
 * points on the sphere plus the 26 neighbour directions of a cube (3D), or
 * 1440 evenly spaced points on the circle plus the 8 neighbour directions
 * (2D).  Returns the count; dirs holds at most 4026 directions. */
static int check_dirs(int dim, double (*dirs)[3]) {
  const double pi = 3.14159265358979323846;
  int k = 0;
  if (dim == 2) {
    for (int j = 0; j < 1440; ++j) {
      const double t = 2.0 * pi * (j + 0.5) / 1440.0;
      dirs[k][0] = cos(t);
      dirs[k][1] = sin(t);
      dirs[k][2] = 0.0;
      ++k;
    }
  } else {
    const double golden = pi * (3.0 - sqrt(5.0));
    for (int j = 0; j < 4000; ++j) {
      const double z = 1.0 - (2.0 * j + 1.0) / 4000.0;
      const double r = sqrt(1.0 - z * z);
      dirs[k][0] = r * cos(golden * j);
      dirs[k][1] = r * sin(golden * j);
      dirs[k][2] = z;
      ++k;
    }
  }
  for (int x = -1; x <= 1; ++x)
    for (int y = -1; y <= 1; ++y)
      for (int z = -1; z <= 1; ++z) {
        if ((x == 0 && y == 0 && z == 0) || (dim == 2 && z != 0)) continue;
        const double l = sqrt((double)(x * x + y * y + z * z));
        dirs[k][0] = x / l;
        dirs[k][1] = y / l;
        dirs[k][2] = z / l;
        ++k;
      }
  return k;
}

double orc_aniso_min(const orc_aniso *an, int dim) {
  double(*dirs)[3] = malloc(sizeof(double[4026][3]));
  if (!dirs) return NAN;
  const int n = check_dirs(dim, dirs);
  double lo = HUGE_VAL;
  for (int j = 0; j < n; ++j) {
    double a, G[3];
    orc_aniso_eval(an, dirs[j], &a, G);
    if (!(a >= lo)) lo = a; /* a NaN propagates */
  }
  free(dirs);
  return lo;
}

int orc_aniso_mirror_symmetric(const orc_aniso *an, int dim) {
  double(*dirs)[3] = malloc(sizeof(double[4026][3]));
  if (!dirs) return 0;
  const int n = check_dirs(dim, dirs);
  int sym = 1;
  for (int j = 0; j < n && sym; ++j) {
    double a, G[3];
    orc_aniso_eval(an, dirs[j], &a, G);
    for (int k = 0; k < dim; ++k) {
      double m[3] = {dirs[j][0], dirs[j][1], dirs[j][2]}, b;
      m[k] = -m[k];
      orc_aniso_eval(an, m, &b, G);
      if (!(fabs(a - b) <= 1e-12)) sym = 0;
    }
  }
  free(dirs);
  return sym;
}

/* N of Eq. TermesAnisotropes for a gradient p (lattice units), with
 * n = -p/|p| (Eq. Def_Normal_Vector).  By the chain rule,
 * d a/d p = -(G - n (n.G)) / |p|, hence N = |p|^2 a da/dp = -|p| a (G - n (n.G)). */
void orc_flux(const orc_aniso *an, const double p[3], double *a, double N[3]) {
  N[0] = N[1] = N[2] = 0.0;
  *a = 1.0;
  if (an == NULL || an->kind == ORC_ANISO_ISO) return;
  const double r2 = (p[0] * p[0] + p[1] * p[1]) + p[2] * p[2];
  if (!(r2 > 1e-16)) return;
  const double r = sqrt(r2);
  const double n[3] = {-p[0] / r, -p[1] / r, -p[2] / r};
  double G[3];
  orc_aniso_eval(an, n, a, G);
  const double nG = (n[0] * G[0] + n[1] * G[1]) + n[2] * G[2];
  const double ra = r * (*a);
  N[0] = -ra * (G[0] - n[0] * nG);
  N[1] = -ra * (G[1] - n[1] * nG);
  N[2] = -ra * (G[2] - n[2] * nG);
}

void orc_sharp_interface(double W0, double tau0, double lambda, double kappa, double out[4]) {
  const double a1 = 5.0 * sqrt(2.0) / 8.0, a2 = 0.6267;
  out[0] = a1 * W0 / lambda;                           /* d0   */
  out[1] = a1 * (tau0 / (W0 * lambda) - a2 * W0 / kappa); /* beta */
  out[2] = kappa * tau0 / (a2 * W0 * W0);              /* lambda* with beta = 0 */
  out[3] = a1;
}

int orc_lattice(int which, int *q, int *e, double *w, int *opp, double *e2) {
  lat_t L;
  if (lat_make(which, &L)) return -1;
  *q = L.q;
  for (int i = 0; i < L.q; ++i) {
    for (int k = 0; k < 3; ++k) e[3 * i + k] = L.e[i][k];
    w[i] = L.w[i];
    opp[i] = L.opp[i];
  }
  *e2 = L.e2;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Simulation state.                                                          */
/* ------------------------------------------------------------------------ */
struct orc_sim {
  orc_config cfg;
  orc_aniso *aniso;
  orc_seed *seeds;
  lat_t lp, lu;
  int nx, ny, nz;
  long N;
  double Dphi, s, Du, eta_u, kphi, W0lu;
  double *g, *gn, *f, *fn, *phi, *phin, *u, *un;
  int16_t *id, *idn;
  double *p, *a, *flux, *eta, *Q;
  long long step;
};

static long nid(const orc_sim *S, int x, int y, int z) { return ((long)z * S->ny + y) * S->nx + x; }

/* Coordinate of a ghost read (phi for gradients): wrap when periodic,
 * mirror about the wall node otherwise, phi(-k) = phi(k). */
static int ghost(int c, int n, int periodic) {
  if (periodic) {
    c %= n;
    return c < 0 ? c + n : c;
  }
  if (c < 0) return -c;
  if (c >= n) return 2 * (n - 1) - c;
  return c;
}

/* Coordinate of a streaming partner: wrap when periodic; -1 if outside. */
static int inside(int c, int n, int periodic) {
  if (periodic) {
    c %= n;
    return c < 0 ? c + n : c;
  }
  return (c < 0 || c >= n) ? -1 : c;
}

/* Node x + sign e as the push sees it: no mirror images (-1 if outside). */
static long partner(const orc_sim *S, int x, int y, int z, const int *e, int sign) {
  const int per = S->cfg.periodic;
  const int X = inside(x + sign * e[0], S->nx, per);
  const int Y = inside(y + sign * e[1], S->ny, per);
  const int Z = inside(z + sign * e[2], S->nz, per);
  if (X < 0 || Y < 0 || Z < 0) return -1;
  return nid(S, X, Y, Z);
}

/* Node x + sign e with the mirror planes of a symmetric box (mirror_low): the
 * planes through node 0 of every axis are planes of mirror symmetry of the
 * whole domain (the box is one octant of it, one quadrant in 2D; Sec. 5 runs a
 * dendrite this way), so a coordinate -k stands for the node at +k.  Bit k of
 * *flip is set when axis k was mirrored.  -1 beyond a zero-flux wall. */
static long partner_sym(const orc_sim *S, int x, int y, int z, const int *e, int sign, int *flip) {
  const int n[3] = {S->nx, S->ny, S->nz};
  int c[3] = {x + sign * e[0], y + sign * e[1], z + sign * e[2]};
  *flip = 0;
  for (int k = 0; k < 3; ++k) {
    if (S->cfg.mirror_low && c[k] < 0) {
      c[k] = -c[k];
      *flip |= 1 << k;
    }
  }
  if (*flip == 0) return partner(S, x, y, z, e, sign);
  for (int k = 0; k < 3; ++k)
    if (c[k] >= n[k]) return -1;
  return nid(S, c[0], c[1], c[2]);
}

/* Direction of lattice L whose vector is e_i with the components of the axes
 * in flip negated: the mirror image of direction i. */
static int mirror_dir(const lat_t *L, int i, int flip) {
  int t[3];
  for (int k = 0; k < 3; ++k) t[k] = (flip >> k & 1) ? -L->e[i][k] : L->e[i][k];
  for (int j = 0; j < L->q; ++j)
    if (L->e[j][0] == t[0] && L->e[j][1] == t[1] && L->e[j][2] == t[2]) return j;
  return -1;
}

static const orc_aniso *entry_for(const orc_sim *S, int id) {
  if (!S->cfg.use_ids) return &S->aniso[0];
  if (id <= 0) return NULL; /* I = 0: no crystal, isotropic */
  return &S->aniso[id];
}

/* Pass 1: gradient of phi at every node (lattice units). */
static void pass_gradient(orc_sim *S, const double *phi) {
  const lat_t *L = &S->lp;
  const int per = S->cfg.periodic;
#pragma omp parallel for schedule(static)
  for (long row = 0; row < (long)S->nz * S->ny; ++row) {
    const int z = (int)(row / S->ny), y = (int)(row % S->ny);
    for (int x = 0; x < S->nx; ++x) {
      const long c = nid(S, x, y, z);
      double pv[3];
      if (S->cfg.grad_cd == 1) {
        /* central differences along the axes (Sec. 4.2) */
        for (int k = 0; k < 3; ++k) {
          if (k == 2 && S->cfg.dim == 2) {
            pv[k] = 0.0;
            continue;
          }
          const int d[3] = {k == 0, k == 1, k == 2};
          const double fp = phi[nid(S, ghost(x + d[0], S->nx, per), ghost(y + d[1], S->ny, per), ghost(z + d[2], S->nz, per))];
          const double fm = phi[nid(S, ghost(x - d[0], S->nx, per), ghost(y - d[1], S->ny, per), ghost(z - d[2], S->nz, per))];
          pv[k] = (fp - fm) / 2.0;
        }
      } else {
        /* directional derivative along each e_i (Eq. Def_DeriveeDirectionnelle),
         * or its second-order upwind (biased) form of Sec. 4.2,
         * [-phi(x + 2 e_i) + 4 phi(x + e_i) - 3 phi(x)] / 2, then
         * grad = (1/e^2) sum_i w_i e_i (e_i . grad) (Eq. Grad_DF-Centree) */
        double dd[19];
        dd[0] = 0.0;
        for (int i = 1; i < L->q; ++i) {
          const int *e = L->e[i];
          const double fp = phi[nid(S, ghost(x + e[0], S->nx, per), ghost(y + e[1], S->ny, per), ghost(z + e[2], S->nz, per))];
          if (S->cfg.grad_cd == 2) {
            const double fpp = phi[nid(S, ghost(x + 2 * e[0], S->nx, per), ghost(y + 2 * e[1], S->ny, per),
                                       ghost(z + 2 * e[2], S->nz, per))];
            dd[i] = (-fpp + 4.0 * fp - 3.0 * phi[c]) / 2.0;
            continue;
          }
          const double fm = phi[nid(S, ghost(x - e[0], S->nx, per), ghost(y - e[1], S->ny, per), ghost(z - e[2], S->nz, per))];
          dd[i] = (fp - fm) / 2.0;
        }
        for (int k = 0; k < 3; ++k) {
          double t[19];
          for (int i = 0; i < L->q; ++i) t[i] = (L->w[i] * (double)L->e[i][k]) * dd[i];
          pv[k] = L->inv_e2 * lat_sum(L, t);
        }
      }
      S->p[3 * c + 0] = pv[0];
      S->p[3 * c + 1] = pv[1];
      S->p[3 * c + 2] = pv[2];
    }
  }
}

static int grad_above_xi(const orc_sim *S, long c) {
  const double *pv = &S->p[3 * c];
  const double r2 = (pv[0] * pv[0] + pv[1] * pv[1]) + pv[2] * pv[2];
  return r2 > S->cfg.xi * S->cfg.xi;
}

/* Pass 2: crystal index (Sec. 4.3), Jacobi update into idn. */
static void pass_ids(orc_sim *S) {
  const lat_t *L = &S->lp;
#pragma omp parallel for schedule(static)
  for (long row = 0; row < (long)S->nz * S->ny; ++row) {
    const int z = (int)(row / S->ny), y = (int)(row % S->ny);
    for (int x = 0; x < S->nx; ++x) {
      const long c = nid(S, x, y, z);
      int16_t nv = S->id[c];
      if (nv == 0 && grad_above_xi(S, c)) {
        double best = -HUGE_VAL;
        int16_t bid = 0;
        for (int i = 1; i < L->q; ++i) {
          int fl;
          const long m = partner_sym(S, x, y, z, L->e[i], +1, &fl);
          if (m < 0 || S->id[m] == 0) continue;
          const double ph = S->phi[m];
          if (ph > best || (ph == best && S->id[m] < bid)) {
            best = ph;
            bid = S->id[m];
          }
        }
        nv = bid;
      }
      S->idn[c] = nv;
    }
  }
  int16_t *t = S->id;
  S->id = S->idn;
  S->idn = t;
}

/* Pass 3: a_s, N, eta_phi, Q_phi at every node. */
static void pass_params(orc_sim *S) {
#pragma omp parallel for schedule(static)
  for (long c = 0; c < S->N; ++c) {
    double a, Nv[3];
    orc_flux(entry_for(S, S->id[c]), &S->p[3 * c], &a, Nv);
    S->a[c] = a;
    S->flux[3 * c + 0] = Nv[0];
    S->flux[3 * c + 1] = Nv[1];
    S->flux[3 * c + 2] = Nv[2];
    /* Eq. LBE_RelaxationTime in lattice units: eta = a^2 Dphi / e^2 + 1/2 */
    S->eta[c] = (a * a) * S->kphi + 0.5;
    /* Eq. LBE_SourceTerm: Q = [phi - lambda u (1 - phi^2)] (1 - phi^2) */
    const double ph = S->phi[c];
    const double om = 1.0 - ph * ph;
    S->Q[c] = (ph - S->cfg.lambda * S->u[c] * om) * om;
  }
}

/* g^(0)_i of Eq. Feq_Phase in lattice units: w_i (phi - (Dphi/e^2) e_i . N). */
static double geq(const orc_sim *S, int i, long c) {
  const int *e = S->lp.e[i];
  const double *Nv = &S->flux[3 * c];
  const double eN = ((double)e[0] * Nv[0] + (double)e[1] * Nv[1]) + (double)e[2] * Nv[2];
  return S->lp.w[i] * (S->phi[c] - S->kphi * eN);
}

/* Local BGK post-collision value of g_i at c (no nonlocal term). */
static double gstar_local(const orc_sim *S, int i, long c) {
  const double gi = S->g[(long)i * S->N + c];
  return gi - (gi - geq(S, i, c)) / S->eta[c] + S->lp.w[i] * S->Q[c] * S->s;
}

/* Pass 4: Eq. LBE_Eq_Phase.  From every source x and direction i:
 * a^2(x) g_i(x+e_i, t+1) = g_i(x,t) - (1 - a^2(x)) g_i(x+e_i,t)
 *                          - (g_i(x,t) - g^(0)_i(x,t))/eta(x) + w_i Q(x) dt/tau0. */
static void pass_phi_lbe(orc_sim *S) {
  const lat_t *L = &S->lp;
  const long N = S->N;
#pragma omp parallel for schedule(static)
  for (long row = 0; row < (long)S->nz * S->ny; ++row) {
    const int z = (int)(row / S->ny), y = (int)(row % S->ny);
    for (int x = 0; x < S->nx; ++x) {
      const long c = nid(S, x, y, z);
      const double a2 = S->a[c] * S->a[c];
      for (int i = 0; i < L->q; ++i) {
        const long d = partner(S, x, y, z, L->e[i], +1);
        if (d < 0) continue; /* leaves the box: replaced by bounce-back */
        const double gx = S->g[(long)i * N + c];
        const double gy = S->g[(long)i * N + d];
        const double rhs = gx - (1.0 - a2) * gy - (gx - geq(S, i, c)) / S->eta[c] + L->w[i] * S->Q[c] * S->s;
        S->gn[(long)i * N + d] = rhs / a2;
      }
    }
  }
}

/* Pass 4b (mirror_low only): g_i arriving at y from a source x = y - e_i
 * beyond a mirror plane.  The state at x is the mirror image of the state at
 * the node x' inside: phi, u and the index of x', the population g_i'(x') of
 * the mirrored direction i', and the gradient p(x') with the mirrored axes
 * negated.  The step's rules then give a_s, N and eta at x from that gradient
 * (Sec. 2, Eq. TermesAnisotropes; Eq. LBE_RelaxationTime) and g^(0)_i(x) from
 * N (Eq. Feq_Phase); Q is that of x'.  For an anisotropy symmetric about the
 * plane these are a_s(x') and the mirror image of N(x'). */
static void pass_phi_mirror(orc_sim *S) {
  if (!S->cfg.mirror_low) return;
  const lat_t *L = &S->lp;
  const long N = S->N;
#pragma omp parallel for schedule(static)
  for (long row = 0; row < (long)S->nz * S->ny; ++row) {
    const int z = (int)(row / S->ny), y = (int)(row % S->ny);
    for (int x = 0; x < S->nx; ++x) {
      const long d = nid(S, x, y, z);
      for (int i = 1; i < L->q; ++i) {
        int fl;
        const long c = partner_sym(S, x, y, z, L->e[i], -1, &fl);
        if (c < 0 || fl == 0) continue;
        const int j = mirror_dir(L, i, fl);
        double pg[3], ag, Ng[3];
        for (int k = 0; k < 3; ++k) pg[k] = (fl >> k & 1) ? -S->p[3 * c + k] : S->p[3 * c + k];
        orc_flux(entry_for(S, S->id[c]), pg, &ag, Ng);
        const double a2 = ag * ag;
        const double eta = a2 * S->kphi + 0.5;
        const int *e = L->e[i];
        const double eN = ((double)e[0] * Ng[0] + (double)e[1] * Ng[1]) + (double)e[2] * Ng[2];
        const double geq_x = L->w[i] * (S->phi[c] - S->kphi * eN);
        const double gx = S->g[(long)j * N + c];
        const double gy = S->g[(long)i * N + d];
        const double rhs = gx - (1.0 - a2) * gy - (gx - geq_x) / eta + L->w[i] * S->Q[c] * S->s;
        S->gn[(long)i * N + d] = rhs / a2;
      }
    }
  }
}

/* Pass 5: bounce-back of Eq. Bounce-Back on the unknown incoming g (sources
 * beyond a zero-flux wall). */
static void pass_phi_bounce(orc_sim *S) {
  if (S->cfg.periodic) return;
  const lat_t *L = &S->lp;
  const long N = S->N;
#pragma omp parallel for schedule(static)
  for (long row = 0; row < (long)S->nz * S->ny; ++row) {
    const int z = (int)(row / S->ny), y = (int)(row % S->ny);
    for (int x = 0; x < S->nx; ++x) {
      const long c = nid(S, x, y, z);
      for (int i = 1; i < L->q; ++i) {
        int fl;
        if (partner_sym(S, x, y, z, L->e[i], -1, &fl) >= 0) continue; /* streamed in or mirrored */
        const int j = L->opp[i];
        if (partner_sym(S, x, y, z, L->e[j], -1, &fl) >= 0)
          S->gn[(long)i * N + c] = S->gn[(long)j * N + c];
        else
          S->gn[(long)i * N + c] = gstar_local(S, j, c);
      }
    }
  }
}

/* Passes 6-8: phi moment, then the heat equation. */
static void pass_phi_moment(orc_sim *S) {
  const lat_t *L = &S->lp;
#pragma omp parallel for schedule(static)
  for (long c = 0; c < S->N; ++c) {
    double v[19];
    for (int i = 0; i < L->q; ++i) v[i] = S->gn[(long)i * S->N + c];
    S->phin[c] = lat_sum(L, v); /* Eq. Def_M0_Phi */
  }
}

static double fstar(const orc_sim *S, int i, long c) {
  /* Eq. LBE_Eq_Temp with f^(0) = w_i u (Eq. EqFunction_Tempr) and
   * Q_u dt = (phi(t+dt) - phi(t))/2 (Eq. Source_Tempr, explicit Euler). */
  const double fi = S->f[(long)i * S->N + c];
  const double qu = 0.5 * (S->phin[c] - S->phi[c]);
  return fi - (fi - S->lu.w[i] * S->u[c]) / S->eta_u + S->lu.w[i] * qu;
}

static void pass_heat(orc_sim *S) {
  const lat_t *L = &S->lu;
  const long N = S->N;
#pragma omp parallel for schedule(static)
  for (long row = 0; row < (long)S->nz * S->ny; ++row) {
    const int z = (int)(row / S->ny), y = (int)(row % S->ny);
    for (int x = 0; x < S->nx; ++x) {
      const long c = nid(S, x, y, z);
      for (int i = 0; i < L->q; ++i) {
        const long d = partner(S, x, y, z, L->e[i], +1);
        if (d >= 0) S->fn[(long)i * N + d] = fstar(S, i, c);
      }
    }
  }
  if (S->cfg.mirror_low) {
    /* f_i arriving from beyond a mirror plane: the mirror image i' of i,
     * collided at the mirror node x' inside */
#pragma omp parallel for schedule(static)
    for (long row = 0; row < (long)S->nz * S->ny; ++row) {
      const int z = (int)(row / S->ny), y = (int)(row % S->ny);
      for (int x = 0; x < S->nx; ++x) {
        const long d = nid(S, x, y, z);
        for (int i = 1; i < L->q; ++i) {
          int fl;
          const long c = partner_sym(S, x, y, z, L->e[i], -1, &fl);
          if (c >= 0 && fl != 0) S->fn[(long)i * N + d] = fstar(S, mirror_dir(L, i, fl), c);
        }
      }
    }
  }
  if (!S->cfg.periodic) {
#pragma omp parallel for schedule(static)
    for (long row = 0; row < (long)S->nz * S->ny; ++row) {
      const int z = (int)(row / S->ny), y = (int)(row % S->ny);
      for (int x = 0; x < S->nx; ++x) {
        const long c = nid(S, x, y, z);
        for (int i = 1; i < L->q; ++i) {
          int fl;
          if (partner_sym(S, x, y, z, L->e[i], -1, &fl) >= 0) continue;
          const int j = L->opp[i];
          if (partner_sym(S, x, y, z, L->e[j], -1, &fl) >= 0)
            S->fn[(long)i * N + c] = S->fn[(long)j * N + c];
          else
            S->fn[(long)i * N + c] = fstar(S, j, c);
        }
      }
    }
  }
#pragma omp parallel for schedule(static)
  for (long c = 0; c < N; ++c) {
    double v[19];
    for (int i = 0; i < L->q; ++i) v[i] = S->fn[(long)i * N + c];
    S->un[c] = lat_sum(L, v); /* Eq. Temperature_LB */
  }
}

static void swap_state(orc_sim *S) {
  double *t;
  t = S->g; S->g = S->gn; S->gn = t;
  t = S->f; S->f = S->fn; S->fn = t;
  t = S->phi; S->phi = S->phin; S->phin = t;
  t = S->u; S->u = S->un; S->un = t;
}

int orc_step(orc_sim *S, int nsteps) {
  for (int n = 0; n < nsteps; ++n) {
    pass_gradient(S, S->phi);
    if (S->cfg.use_ids) pass_ids(S);
    pass_params(S);
    pass_phi_lbe(S);
    pass_phi_mirror(S);
    pass_phi_bounce(S);
    pass_phi_moment(S);
    pass_heat(S);
    swap_state(S);
    S->step++;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Set-up.                                                                    */
/* ------------------------------------------------------------------------ */
int orc_set_fields(orc_sim *S, const double *phi, const double *u, const int16_t *ids) {
  const long N = S->N;
  if (S->cfg.use_ids && ids) {
    for (long c = 0; c < N; ++c)
      if (ids[c] < 0 || ids[c] >= S->cfg.n_aniso) return -1;
  }
  memcpy(S->phi, phi, sizeof(double) * N);
  memcpy(S->u, u, sizeof(double) * N);
  if (ids)
    memcpy(S->id, ids, sizeof(int16_t) * N);
  else
    memset(S->id, 0, sizeof(int16_t) * N);
  pass_gradient(S, S->phi);
  pass_params(S);
  for (int i = 0; i < S->lp.q; ++i)
    for (long c = 0; c < N; ++c) S->g[(long)i * N + c] = geq(S, i, c);
  for (int i = 0; i < S->lu.q; ++i)
    for (long c = 0; c < N; ++c) S->f[(long)i * N + c] = S->lu.w[i] * S->u[c];
  return 0;
}

void orc_destroy(orc_sim *S) {
  if (!S) return;
  free(S->aniso); free(S->seeds);
  free(S->g); free(S->gn); free(S->f); free(S->fn);
  free(S->phi); free(S->phin); free(S->u); free(S->un);
  free(S->id); free(S->idn);
  free(S->p); free(S->a); free(S->flux); free(S->eta); free(S->Q);
  free(S);
}

int orc_create(const orc_config *cfg, orc_sim **out) {
  *out = NULL;
  if (cfg->dim != 2 && cfg->dim != 3) return -1;
  if (cfg->nx < 3 || cfg->ny < 3) return -1;
  if (cfg->dim == 2 && cfg->nz != 1) return -1;
  if (cfg->dim == 3 && cfg->nz < 3) return -1;
  if (!(cfg->q_phi == 0 || (cfg->dim == 2 && cfg->q_phi == 9) ||
        (cfg->dim == 3 && (cfg->q_phi == 19 || cfg->q_phi == 15))))
    return -1;
  if (!(cfg->W0 > 0 && cfg->tau0 > 0 && cfg->dx > 0 && cfg->dt > 0 && cfg->kappa > 0)) return -2;
  if (cfg->n_aniso < 1 || cfg->aniso == NULL) return -1;
  for (int k = 0; k < cfg->n_aniso; ++k) {
    const int kd = cfg->aniso[k].kind;
    if (kd < 0 || kd > 4) return -1;
    if (kd == ORC_ANISO_SECTORAL && cfg->aniso[k].q < 1) return -1;
  }
  if (cfg->use_ids && cfg->aniso[0].kind != ORC_ANISO_ISO) return -1;
  if (cfg->mirror_low && cfg->periodic) return -1;
  for (int k = 0; k < cfg->n_aniso; ++k) {
    /* a_s > 0 in every direction: eta_phi and the division by a_s^2 of
     * Eq. LBE_Eq_Phase need it */
    if (!(orc_aniso_min(&cfg->aniso[k], cfg->dim) > 0.0)) return -2;
    /* an octant stands for the symmetric domain only if every entry is */
    if (cfg->mirror_low && !orc_aniso_mirror_symmetric(&cfg->aniso[k], cfg->dim)) return -6;
  }
  for (int k = 0; k < cfg->n_seeds; ++k)
    if (cfg->seeds[k].id < 0 || (cfg->use_ids && cfg->seeds[k].id >= cfg->n_aniso)) return -1;

  orc_sim *S = (orc_sim *)calloc(1, sizeof(orc_sim));
  S->cfg = *cfg;
  S->aniso = (orc_aniso *)malloc(sizeof(orc_aniso) * cfg->n_aniso);
  memcpy(S->aniso, cfg->aniso, sizeof(orc_aniso) * cfg->n_aniso);
  S->seeds = (orc_seed *)malloc(sizeof(orc_seed) * (cfg->n_seeds > 0 ? cfg->n_seeds : 1));
  if (cfg->n_seeds > 0) memcpy(S->seeds, cfg->seeds, sizeof(orc_seed) * cfg->n_seeds);
  S->cfg.aniso = S->aniso;
  S->cfg.seeds = S->seeds;
  lat_make(cfg->dim == 2 ? 1 : (cfg->q_phi == 15 ? 4 : 3), &S->lp);
  lat_make(cfg->dim == 2 ? 0 : 2, &S->lu);
  S->nx = cfg->nx;
  S->ny = cfg->ny;
  S->nz = cfg->nz;
  S->N = (long)S->nx * S->ny * S->nz;
  /* Lattice-unit numbers: Dphi = W0^2 dt/(tau0 dx^2) (Eq. LBE_RelaxationTime),
   * s = dt/tau0 (Eq. LBE_Eq_Phase), Du = kappa dt/dx^2 (Eq. ThermalDiffusivity). */
  S->Dphi = cfg->W0 * cfg->W0 * cfg->dt / (cfg->tau0 * cfg->dx * cfg->dx);
  S->s = cfg->dt / cfg->tau0;
  S->Du = cfg->kappa * cfg->dt / (cfg->dx * cfg->dx);
  S->eta_u = S->Du * S->lu.inv_e2 + 0.5;
  S->kphi = S->Dphi * S->lp.inv_e2;
  S->W0lu = cfg->W0 / cfg->dx;
  if (!(S->eta_u > 0.5)) {
    orc_destroy(S);
    return -2;
  }
  const long N = S->N;
  S->g = (double *)malloc(sizeof(double) * N * S->lp.q);
  S->gn = (double *)malloc(sizeof(double) * N * S->lp.q);
  S->f = (double *)malloc(sizeof(double) * N * S->lu.q);
  S->fn = (double *)malloc(sizeof(double) * N * S->lu.q);
  S->phi = (double *)malloc(sizeof(double) * N);
  S->phin = (double *)malloc(sizeof(double) * N);
  S->u = (double *)malloc(sizeof(double) * N);
  S->un = (double *)malloc(sizeof(double) * N);
  S->id = (int16_t *)calloc(N, sizeof(int16_t));
  S->idn = (int16_t *)calloc(N, sizeof(int16_t));
  S->p = (double *)calloc(3 * N, sizeof(double));
  S->a = (double *)malloc(sizeof(double) * N);
  S->flux = (double *)malloc(sizeof(double) * 3 * N);
  S->eta = (double *)malloc(sizeof(double) * N);
  S->Q = (double *)malloc(sizeof(double) * N);
  if (!S->g || !S->gn || !S->f || !S->fn || !S->phi || !S->phin || !S->u || !S->un || !S->p ||
      !S->a || !S->flux || !S->eta || !S->Q) {
    orc_destroy(S);
    return -3;
  }

  /* Initial condition, Eq. Initial_Condition and Eq. Intial-Cond_u. */
  double *phi0 = (double *)malloc(sizeof(double) * N);
  double *u0 = (double *)malloc(sizeof(double) * N);
  int16_t *id0 = (int16_t *)calloc(N, sizeof(int16_t));
  const double width = sqrt(2.0) * S->W0lu;
  for (int z = 0; z < S->nz; ++z)
    for (int y = 0; y < S->ny; ++y)
      for (int x = 0; x < S->nx; ++x) {
        const long c = nid(S, x, y, z);
        double ph = -1.0;
        for (int k = 0; k < cfg->n_seeds; ++k) {
          const orc_seed *sd = &S->seeds[k];
          const double ddx = x - sd->x, ddy = y - sd->y, ddz = z - sd->z;
          const double d = sqrt((ddx * ddx + ddy * ddy) + ddz * ddz);
          const double v = tanh((sd->radius - d) / width);
          if (v > ph) ph = v;
        }
        phi0[c] = ph;
        u0[c] = -cfg->delta;
      }
  if (cfg->use_ids) {
    pass_gradient(S, phi0);
    for (int z = 0; z < S->nz; ++z)
      for (int y = 0; y < S->ny; ++y)
        for (int x = 0; x < S->nx; ++x) {
          const long c = nid(S, x, y, z);
          if (!(phi0[c] > 0.0 || grad_above_xi(S, c))) continue;
          double best = HUGE_VAL;
          int bid = 0;
          for (int k = 0; k < cfg->n_seeds; ++k) {
            const orc_seed *sd = &S->seeds[k];
            const double ddx = x - sd->x, ddy = y - sd->y, ddz = z - sd->z;
            const double gap = sqrt((ddx * ddx + ddy * ddy) + ddz * ddz) - sd->radius;
            if (gap < best) {
              best = gap;
              bid = sd->id;
            }
          }
          id0[c] = (int16_t)bid;
        }
  }
  orc_set_fields(S, phi0, u0, id0);
  free(phi0);
  free(u0);
  free(id0);
  S->step = 0;
  *out = S;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Accessors and diagnostics.                                                 */
/* ------------------------------------------------------------------------ */
long long orc_nodes(const orc_sim *S) { return S->N; }
int orc_q_phi(const orc_sim *S) { return S->lp.q; }
int orc_q_u(const orc_sim *S) { return S->lu.q; }
void orc_get_phi(const orc_sim *S, double *o) { memcpy(o, S->phi, sizeof(double) * S->N); }
void orc_get_u(const orc_sim *S, double *o) { memcpy(o, S->u, sizeof(double) * S->N); }
void orc_get_ids(const orc_sim *S, int16_t *o) { memcpy(o, S->id, sizeof(int16_t) * S->N); }
void orc_get_g(const orc_sim *S, double *o) { memcpy(o, S->g, sizeof(double) * S->N * S->lp.q); }
void orc_get_f(const orc_sim *S, double *o) { memcpy(o, S->f, sizeof(double) * S->N * S->lu.q); }

void orc_params(orc_sim *S, double *p, double *a, double *flux, double *eta, double *q) {
  pass_gradient(S, S->phi);
  pass_params(S);
  const long N = S->N;
  if (p) memcpy(p, S->p, sizeof(double) * 3 * N);
  if (a) memcpy(a, S->a, sizeof(double) * N);
  if (flux) memcpy(flux, S->flux, sizeof(double) * 3 * N);
  if (eta) memcpy(eta, S->eta, sizeof(double) * N);
  if (q) memcpy(q, S->Q, sizeof(double) * N);
}

void orc_diagnostics(const orc_sim *S, orc_diag *d) {
  double sp = 0, su = 0, sc = 0, sf = 0, ns = 0, bad = 0;
  for (long c = 0; c < S->N; ++c) {
    const double ph = S->phi[c], uu = S->u[c];
    if (!isfinite(ph) || !isfinite(uu)) bad = 1;
    sp += ph;
    su += uu;
    sc += uu - 0.5 * ph;
    sf += 1.0 + ph;
    if (ph > 0.0) ns += 1;
  }
  d->sum_phi = sp;
  d->sum_u = su;
  d->sum_u_minus_half_phi = sc;
  d->solid_fraction = sf / (2.0 * (double)S->N);
  d->n_solid = ns;
  d->nonfinite = bad;
  /* Tip: largest linearly interpolated phi = 0 crossing along the ray from
   * seed 0's centre (rounded to a node) in the direction tip_dir. */
  int dir[3] = {S->cfg.tip_dir[0], S->cfg.tip_dir[1], S->cfg.tip_dir[2]};
  if (dir[0] == 0 && dir[1] == 0 && dir[2] == 0) dir[0] = 1;
  int o[3] = {S->nx / 2, S->ny / 2, S->nz / 2};
  if (S->cfg.n_seeds > 0) {
    o[0] = (int)floor(S->seeds[0].x + 0.5);
    o[1] = (int)floor(S->seeds[0].y + 0.5);
    o[2] = (int)floor(S->seeds[0].z + 0.5);
  }
  const double len = sqrt((double)(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]));
  double tip = -1.0;
  for (int k = 0;; ++k) {
    const int a0 = o[0] + k * dir[0], a1 = o[1] + k * dir[1], a2 = o[2] + k * dir[2];
    const int b0 = a0 + dir[0], b1 = a1 + dir[1], b2 = a2 + dir[2];
    if (b0 < 0 || b1 < 0 || b2 < 0 || b0 >= S->nx || b1 >= S->ny || b2 >= S->nz) break;
    if (a0 < 0 || a1 < 0 || a2 < 0 || a0 >= S->nx || a1 >= S->ny || a2 >= S->nz) break;
    const double pa = S->phi[nid(S, a0, a1, a2)], pb = S->phi[nid(S, b0, b1, b2)];
    if (pa > 0.0 && pb <= 0.0) {
      const double t = (k + pa / (pa - pb)) * len;
      if (t > tip) tip = t;
    }
  }
  d->tip_position = tip;
}

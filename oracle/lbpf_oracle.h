/*
 * CPU FP64 oracle for the coupled lattice Boltzmann phase-field step of
 * Younsi & Cartalade, "On anisotropy function in crystal growth simulations
 * using Lattice Boltzmann equation" (arXiv:1606.09432).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that the
 * GPU path is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never does.
 * It shares no code, header, table or helper with the GPU library: every
 * lattice table, formula and boundary rule below is written out again here.
 *
 * Parity unpinned: the bounce-back of a population whose source and whose
 * opposite's source both lie outside a zero-flux box (edges and corners) has
 * no check outside the two implementations; every other function is pinned by
 * the CPU test-suite against closed forms, invariants or the paper's values.
 *
 * Units: everything is in lattice units (node spacing 1, one step = 1) except
 * the physical parameters W0, tau0, lambda, kappa, delta, dx, dt, which are
 * converted with the relations of Sec. 3 (Eq. ThermalDiffusivity and
 * Eq. LBE_RelaxationTime).  Seed centres and radii are given in lattice units.
 */
#ifndef LBPF_ORACLE_H
#define LBPF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Anisotropy kinds (Sec. 4.1). */
enum {
  ORC_ANISO_ISO = 0,      /* a_s = 1                                                   */
  ORC_ANISO_SECTORAL = 1, /* 1 + eps Re[((n_x + i n_y) e^{-i phi0})^q]: Eq. As_Theta in  */
                          /* 2D (|n| = 1), Eq. As_Multi per crystal, Eq. As_Y66 in 3D   */
  ORC_ANISO_CUBIC = 2,    /* 1 - 3 eps + 4 eps sum n^4: Eq. As_Function_Classical       */
  ORC_ANISO_CUBIC_HAK = 3, /* 1 + eps (Q - 3/5) + gamma (3Q + 66 S - 17/7): Eq. As_MatSci */
  ORC_ANISO_CUBIC_S = 4    /* 1 + 66 gamma n_x^2 n_y^2 n_z^2: Eq. As_Function_S (printed without the 1) */
};

/* An entry is the polynomial of its kind evaluated at R n: a(n) = A(R n), so
 * that each crystal of the index field may have its own orientation (Sec. 4.3,
 * Eq. As_Multi, generalised from the 2D angle phi0 to a 3D rotation).  R is
 * row-major; all nine zero means the identity.  The gradient of a with respect
 * to n is then R^T (grad A)(R n). */
typedef struct {
  int32_t kind;
  int32_t q;
  double eps;
  double gamma;
  double phi0;
  double R[9];
} orc_aniso;

typedef struct {
  double x, y, z;   /* centre, lattice units (node coordinates) */
  double radius;    /* lattice units */
  int32_t id;       /* crystal index I carried by this seed (Sec. 4.3) */
} orc_seed;

typedef struct {
  int32_t dim;          /* 2: D2Q9 phi + D2Q5 u;  3: D3Q19 (or D3Q15, q_phi) phi + D3Q7 u */
  int32_t nx, ny, nz;   /* nz must be 1 when dim == 2 */
  int32_t periodic;     /* 1 periodic box, 0 zero flux (bounce-back, Eq. Bounce-Back) */
  int32_t grad_cd;      /* 0 directional derivatives (Eq. Grad_DF-Centree), 1 central differences,
                           2 second-order upwind directional derivatives (Sec. 4.2) */
  int32_t use_ids;      /* 1: crystal index field I(x,t) selects the anisotropy entry (Sec. 4.3) */
  double W0, tau0, lambda, kappa, delta, dx, dt, xi;
  int32_t n_aniso;
  const orc_aniso *aniso; /* use_ids = 0: entry 0 everywhere; use_ids = 1: entry I, I = 0 isotropic */
  int32_t n_seeds;
  const orc_seed *seeds;
  int32_t tip_dir[3];   /* integer lattice direction of the tip ray from seed 0's centre */
  int32_t q_phi;        /* phi lattice: 0 default (D2Q9 / D3Q19), or 15 for D3Q15 in 3D */
  int32_t mirror_low;   /* 1: the planes through node 0 of every axis are mirror planes of a
                           symmetric domain (periodic must be 0); the far walls stay zero flux */
} orc_config;

typedef struct orc_sim orc_sim;

/* Diagnostics record (all FP64). */
typedef struct {
  double sum_phi, sum_u, sum_u_minus_half_phi, solid_fraction, n_solid, tip_position;
  double nonfinite;
} orc_diag;

/* Returns 0 on success, negative on a bad configuration: -1 bad argument, -2
 * unstable (eta_u <= 1/2, or an anisotropy entry with a_s <= 0 on some
 * direction, where eta_phi and the division by a_s^2 break down), -3 out of
 * memory, -6 a mirror box whose anisotropy entries are not symmetric about the
 * mirror planes (the octant would not stand for a symmetric domain). */
int orc_create(const orc_config *cfg, orc_sim **out);
void orc_destroy(orc_sim *s);
int orc_step(orc_sim *s, int nsteps);
long long orc_nodes(const orc_sim *s);
int orc_q_phi(const orc_sim *s);
int orc_q_u(const orc_sim *s);

/* Copies of the current state (post-streaming distributions at time n). */
void orc_get_phi(const orc_sim *s, double *phi);
void orc_get_u(const orc_sim *s, double *u);
void orc_get_ids(const orc_sim *s, int16_t *ids);
void orc_get_g(const orc_sim *s, double *g);   /* [q_phi][N] */
void orc_get_f(const orc_sim *s, double *f);   /* [q_u][N]   */

/* Replace the state by equilibrium distributions of the given fields
 * (g = g^(0)(phi, N(phi)) of Eq. Feq_Phase, f = w_i u of Eq. EqFunction_Tempr). */
int orc_set_fields(orc_sim *s, const double *phi, const double *u, const int16_t *ids);

/* Parameter fields of the current state, in lattice units: gradient p (3N),
 * a_s (N), flux N (3N), eta_phi (N), Q_phi (N).  Any pointer may be NULL. */
void orc_params(orc_sim *s, double *p, double *a, double *flux, double *eta, double *q);

void orc_diagnostics(const orc_sim *s, orc_diag *d);

/* Pointwise pieces, for pinning against closed forms. */
/* which: 0 D2Q5, 1 D2Q9, 2 D3Q7, 3 D3Q19, 4 D3Q15 */
int orc_lattice(int which, int *q, int *e /* [q][3] */, double *w, int *opp, double *e2);
void orc_aniso_eval(const orc_aniso *an, const double n[3], double *a, double G[3]);
void orc_flux(const orc_aniso *an, const double p[3], double *a, double N[3]);
/* Smallest a_s of an entry over a fixed set of unit directions (the circle
 * n_z = 0 when dim == 2), and whether a_s is unchanged by the reflections
 * n_k -> -n_k of the axes of the box (x, y, and z when dim == 3). */
double orc_aniso_min(const orc_aniso *an, int dim);
int orc_aniso_mirror_symmetric(const orc_aniso *an, int dim);

/* Sharp-interface mapping (Sec. 2, Eqs. Capillary-Length and Kinetic-Coeff):
 * out = {d0, beta, lambda_star (beta = 0), a1}. */
void orc_sharp_interface(double W0, double tau0, double lambda, double kappa, double out[4]);

#ifdef __cplusplus
}
#endif
#endif

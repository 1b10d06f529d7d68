/*
 * Exercise of every entry point of the CPU oracle, for a build with the
 * address and undefined-behaviour sanitizers (test infrastructure only).
 *
 * Small 2D and 3D boxes with every boundary kind, gradient method and lattice,
 * the crystal index field, oriented entries, the accessors, diagnostics,
 * parameter fields, field import and the configurations the oracle refuses.
 * Exits 0 when every call behaved; the sanitizers abort on the first fault.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbpf_oracle.h"

static int failures = 0;

#define CHECK(cond)                                                   \
  do {                                                                \
    if (!(cond)) {                                                    \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                     \
    }                                                                 \
  } while (0)

static orc_config base(int dim, int nx, int ny, int nz) {
  orc_config c;
  memset(&c, 0, sizeof(c));
  c.dim = dim;
  c.nx = nx;
  c.ny = ny;
  c.nz = nz;
  c.W0 = 1.0;
  c.tau0 = 1.0;
  c.lambda = 10.0;
  c.kappa = 6.267;
  c.delta = 0.5;
  c.dx = 0.4;
  c.dt = 0.008;
  c.xi = 1e-7;
  c.tip_dir[0] = 1;
  return c;
}

/* Creates, steps and reads back one configuration; returns orc_create's code. */
static int run(const orc_config *c, int steps) {
  orc_sim *s = NULL;
  const int rc = orc_create(c, &s);
  if (rc != 0) {
    CHECK(s == NULL);
    return rc;
  }
  const long long N = orc_nodes(s);
  const int qp = orc_q_phi(s), qu = orc_q_u(s);
  double *phi = malloc(sizeof(double) * N), *u = malloc(sizeof(double) * N);
  double *g = malloc(sizeof(double) * N * qp), *f = malloc(sizeof(double) * N * qu);
  double *p = malloc(sizeof(double) * 3 * N), *a = malloc(sizeof(double) * N);
  double *fl = malloc(sizeof(double) * 3 * N), *eta = malloc(sizeof(double) * N), *q = malloc(sizeof(double) * N);
  int16_t *ids = malloc(sizeof(int16_t) * N);
  CHECK(orc_step(s, steps) == 0);
  orc_get_phi(s, phi);
  orc_get_u(s, u);
  orc_get_g(s, g);
  orc_get_f(s, f);
  orc_get_ids(s, ids);
  orc_params(s, p, a, fl, eta, q);
  orc_params(s, NULL, NULL, NULL, NULL, NULL);
  orc_diag d;
  orc_diagnostics(s, &d);
  CHECK(d.nonfinite == 0.0);
  for (long long k = 0; k < N; ++k) CHECK(isfinite(phi[k]) && isfinite(u[k]) && a[k] > 0.0 && eta[k] > 0.5);
  /* import the fields back, step once more */
  CHECK(orc_set_fields(s, phi, u, c->use_ids ? ids : NULL) == 0);
  CHECK(orc_step(s, 1) == 0);
  if (c->use_ids) {
    ids[0] = (int16_t)c->n_aniso; /* out of range: refused */
    CHECK(orc_set_fields(s, phi, u, ids) != 0);
  }
  free(phi);
  free(u);
  free(g);
  free(f);
  free(p);
  free(a);
  free(fl);
  free(eta);
  free(q);
  free(ids);
  orc_destroy(s);
  return 0;
}

int main(void) {
  orc_aniso iso, sec, cub, hak, css, rot;
  memset(&iso, 0, sizeof(iso));
  sec = cub = hak = css = rot = iso;
  sec.kind = ORC_ANISO_SECTORAL;
  sec.q = 4;
  sec.eps = 0.05;
  sec.phi0 = 0.3;
  cub.kind = ORC_ANISO_CUBIC;
  cub.eps = 0.05;
  hak.kind = ORC_ANISO_CUBIC_HAK;
  hak.eps = 0.1;
  css.kind = ORC_ANISO_CUBIC_S;
  css.gamma = 0.02;
  rot = hak;
  {
    /* rotation by 0.7 rad about (1, 2, 3)/sqrt(14) */
    const double ax[3] = {1 / sqrt(14.0), 2 / sqrt(14.0), 3 / sqrt(14.0)}, t = 0.7;
    const double c = cos(t), s = sin(t);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const double k = (i == j) ? c : 0.0;
        const double cross = (i == 0 && j == 1) ? -ax[2] : (i == 0 && j == 2) ? ax[1]
                           : (i == 1 && j == 0) ? ax[2] : (i == 1 && j == 2) ? -ax[0]
                           : (i == 2 && j == 0) ? -ax[1] : (i == 2 && j == 1) ? ax[0] : 0.0;
        rot.R[3 * i + j] = k + s * cross + (1 - c) * ax[i] * ax[j];
      }
  }
  orc_aniso table2[3] = {iso, sec, sec};
  table2[2].phi0 = 1.1;
  orc_aniso table3[4] = {iso, cub, rot, css};

  orc_seed s2[3] = {{10.5, 12.0, 0.0, 4.0, 1}, {26.0, 20.5, 0.0, 3.0, 2}, {5.0, 30.0, 0.0, 2.5, 1}};
  orc_seed s3[2] = {{6.5, 7.0, 6.0, 3.5, 1}, {13.0, 12.0, 11.5, 3.0, 2}};
  orc_seed corner = {0.0, 0.0, 0.0, 4.0, 1};

  /* 2D: periodic DD, zero flux CD with the index field, upwind, mirror, 3 x 3 */
  orc_config c = base(2, 40, 36, 1);
  c.periodic = 1;
  c.n_aniso = 1;
  c.aniso = &sec;
  c.n_seeds = 1;
  c.seeds = s2;
  CHECK(run(&c, 20) == 0);
  c.periodic = 0;
  c.grad_cd = 1;
  c.use_ids = 1;
  c.n_aniso = 3;
  c.aniso = table2;
  c.n_seeds = 3;
  CHECK(run(&c, 20) == 0);
  c.grad_cd = 2;
  c.use_ids = 0;
  c.n_aniso = 1;
  c.aniso = &cub;
  CHECK(run(&c, 10) == 0);
  c.grad_cd = 0;
  c.mirror_low = 1;
  c.n_seeds = 1;
  c.seeds = &corner;
  CHECK(run(&c, 15) == 0);
  c.mirror_low = 0;
  c.nx = c.ny = 3;
  CHECK(run(&c, 5) == 0);

  /* 3D: D3Q19 zero flux with oriented entries in the index field, D3Q15
   * periodic CD, mirror box, upwind, 3 x 3 x 3 */
  c = base(3, 20, 18, 17);
  c.use_ids = 1;
  c.n_aniso = 4;
  c.aniso = table3;
  c.n_seeds = 2;
  c.seeds = s3;
  CHECK(run(&c, 8) == 0);
  c.use_ids = 0;
  c.n_aniso = 1;
  c.aniso = &hak;
  c.q_phi = 15;
  c.periodic = 1;
  c.grad_cd = 1;
  CHECK(run(&c, 8) == 0);
  c.q_phi = 0;
  c.periodic = 0;
  c.grad_cd = 0;
  c.mirror_low = 1;
  c.n_seeds = 1;
  c.seeds = &corner;
  CHECK(run(&c, 8) == 0);
  c.mirror_low = 0;
  c.grad_cd = 2;
  c.aniso = &css;
  CHECK(run(&c, 6) == 0);
  c.grad_cd = 0;
  c.nx = c.ny = c.nz = 3;
  CHECK(run(&c, 4) == 0);

  /* refused configurations: each returns its code and leaks nothing */
  c = base(3, 8, 8, 8);
  c.n_aniso = 1;
  c.aniso = &rot;
  c.mirror_low = 1;
  CHECK(run(&c, 1) == -6); /* a generic rotation is not mirror-symmetric */
  c.mirror_low = 0;
  orc_aniso bad = cub;
  bad.eps = 0.7;
  c.aniso = &bad;
  CHECK(run(&c, 1) == -2); /* a_s < 0 on <111> */
  c.aniso = &cub;
  c.kappa = 0.0;
  CHECK(run(&c, 1) == -2); /* no thermal diffusivity */
  c = base(2, 2, 8, 1);
  c.n_aniso = 1;
  c.aniso = &sec;
  CHECK(run(&c, 1) == -1);

  /* pointwise pieces */
  int q, e[57], opp[19];
  double w[19], e2;
  for (int which = 0; which < 5; ++which) CHECK(orc_lattice(which, &q, e, w, opp, &e2) == 0);
  CHECK(orc_lattice(5, &q, e, w, opp, &e2) != 0);
  double n[3] = {0.6, 0.0, 0.8}, av, G[3], pv[3] = {-0.1, 0.2, 0.05}, Nv[3], si[4];
  orc_aniso_eval(&rot, n, &av, G);
  orc_flux(&rot, pv, &av, Nv);
  orc_sharp_interface(1.0, 1.0, 6.3826, 4.0, si);
  CHECK(orc_aniso_min(&cub, 3) > 0.9 && orc_aniso_mirror_symmetric(&cub, 3));

  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  printf("oracle sanitizer run: all checks passed\n");
  return 0;
}

/*
 * lb_pf.h -- C ABI of the MI355X coupled lattice Boltzmann phase-field library.
 *
 * The library advances the pure-substance phase-field model of Younsi &
 * Cartalade (arXiv:1606.09432), Sec. 2 (Eqs. PhaseField_KarmaRappel and
 * Temp_Ramirez), with the lattice Boltzmann schemes of Sec. 3:
 *   - phi on D2Q9 (2D), D3Q19 or D3Q15 (3D) with the nonlocal a_s^2 scheme of
 *     Eq. LBE_Eq_Phase, the equilibrium of Eq. Feq_Phase, the relaxation rate of
 *     Eq. LBE_RelaxationTime and the source of Eq. LBE_SourceTerm;
 *   - u on D2Q5 (2D) or D3Q7 (3D) with the BGK scheme of Eq. LBE_Eq_Temp, the
 *     equilibrium of Eq. EqFunction_Tempr and the source (phi^{n+1} - phi^n)/2
 *     (Eq. Source_Tempr with the explicit Euler derivative of Sec. 3.1);
 *   - the anisotropy a_s(n) and its flux N (Eq. TermesAnisotropes) built from
 *     directional derivatives along every lattice vector (Sec. 4.2, Eqs.
 *     Def_DeriveeDirectionnelle and Grad_DF-Centree), from central
 *     differences (the comparison variant of Sec. 4.2), or from the
 *     second-order upwind directional derivatives of Sec. 4.2;
 *   - per-crystal anisotropy through a crystal index field (Sec. 4.3);
 *   - zero-flux walls by bounce-back (Sec. 3.3, Eq. Bounce-Back), periodic
 *     boundaries, or mirror planes through node 0 (one octant of a symmetric
 *     domain, Sec. 5).
 *
 * Conventions
 *   - Every function returns 0 (LBPF_OK) or a negative status; after a failure
 *     lb_pf_last_error() returns a message (thread-local).
 *   - All config values are host memory.  Seed centres and radii are in
 *     lattice units (node coordinates); W0, tau0, lambda, kappa (the thermal
 *     diffusivity, "D"), delta (the undercooling, u0 = -delta), dx, dt are the
 *     paper's physical parameters; xi is the index-field threshold on the
 *     lattice-unit gradient.
 *   - Device memory: the caller allocates one workspace of
 *     lb_pf_workspace_bytes() bytes (256-byte aligned) and owns it; the library
 *     lays out every field inside it and allocates no device memory of its own
 *     (a batched handle also holds HIP graph objects, which the HIP runtime
 *     manages).  The workspace must outlive the handle.
 *   - Streams: every call that takes a hip_stream enqueues its work on that
 *     stream (a hipStream_t, or NULL for the null stream) and returns without
 *     waiting, unless stated otherwise.
 *   - Field layout used by the export/import calls: FP64 (or int16 for the
 *     index), contiguous, x fastest, then y, then z: element (x,y,z) at
 *     (z*ny + y)*nx + x.  Distribution exports are [q][field].
 *   - A handle is not thread-safe; different handles are independent.
 */
#ifndef LB_PF_H
#define LB_PF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define LBPF_OK 0
#define LBPF_ERR_ARG (-1)         /* bad argument or configuration */
#define LBPF_ERR_UNSTABLE (-2)    /* relaxation rate <= 1/2, dt <= 0, ... */
#define LBPF_ERR_WORKSPACE (-3)   /* workspace NULL, misaligned or too small */
#define LBPF_ERR_HIP (-4)         /* a HIP runtime call failed */
#define LBPF_ERR_NONFINITE (-5)   /* diagnostics found a non-finite phi or u */
#define LBPF_ERR_UNSUPPORTED (-6) /* valid request the library does not implement */

/* Lattice pairs (Sec. 3.3): phi lattice + u lattice.  D3Q15 is the paper's own
 * 3D phi lattice (Table Values-Lattices); D3Q19 takes the standard weights
 * 1/3, 1/18, 1/36. */
#define LBPF_D2Q9_D2Q5 0
#define LBPF_D3Q19_D3Q7 1
#define LBPF_D3Q15_D3Q7 2
/* Boundaries: periodic box, or zero flux on every wall (Sec. 2, Eq. Bounce-Back).
 * LBPF_MIRROR_LOW: the box is one octant (one quadrant in 2D) of a domain that
 * is mirror-symmetric about the planes through node 0 of each axis, as in the
 * paper's 3D run with the seed at the origin, completed by symmetry about the
 * planes XY, YZ and XZ (Sec. 5).  The state beyond those planes is the mirror
 * image of the state inside (phi, u, the index and, for population i, the
 * population of the mirrored direction at the mirror node); the far walls are
 * zero flux.  Seeds belong at the origin or are mirrored with it; every
 * anisotropy entry must be symmetric about the planes, for the octant to stand
 * for the whole domain (LBPF_ERR_UNSUPPORTED otherwise; see lbpf_aniso). */
#define LBPF_PERIODIC 0
#define LBPF_ZERO_FLUX 1
#define LBPF_MIRROR_LOW 2
/* Gradient of phi: directional derivatives (Eq. Grad_DF-Centree) or central
 * differences.  LBPF_GRAD_UP2 puts the second-order upwind (biased)
 * directional derivatives of Sec. 4.2, [-phi(x+2e) + 4 phi(x+e) - 3 phi(x)]/2,
 * through the same moment (the first-order upwind form through it equals
 * LBPF_GRAD_DD); it is implemented for single simulations (not batched
 * ensembles) without mirror planes, with every extent >= 4
 * (LBPF_ERR_UNSUPPORTED / LBPF_ERR_ARG otherwise). */
#define LBPF_GRAD_DD 0
#define LBPF_GRAD_CD 1
#define LBPF_GRAD_UP2 2
/* Storage of the distributions: FP64; or FP32 arithmetic with distributions
 * stored as offsets g_i - w_i phi and f*_i - w_i u* in FP32 or FP16 (RNE) next
 * to FP32 phi and u* fields. In FP16 the rest offset (i = 0) is stored as minus
 * the sum of the other offsets of the node as rounded, so that the offsets of
 * a node sum to zero up to the rounding of that near-zero value. */
#define LBPF_FP64 0
#define LBPF_FP32_OFFSET 1
#define LBPF_FP16_OFFSET 2
/* Anisotropy kinds (Sec. 4.1). */
#define LBPF_ANISO_ISO 0       /* a_s = 1 */
#define LBPF_ANISO_SECTORAL 1  /* 1 + eps Re[((n_x + i n_y) e^{-i phi0})^q]: Eq. As_Theta / As_Multi in 2D, Eq. As_Y66 in 3D (q = 6) */
#define LBPF_ANISO_CUBIC 2     /* 1 - 3 eps + 4 eps (n_x^4 + n_y^4 + n_z^4): Eq. As_Function_Classical */
#define LBPF_ANISO_CUBIC_HAK 3 /* 1 + eps (Q - 3/5) + gamma (3 Q + 66 S - 17/7): Eq. As_MatSci */
#define LBPF_ANISO_CUBIC_S 4   /* 1 + 66 gamma n_x^2 n_y^2 n_z^2: Eq. As_Function_S, read with the
                                  constant 1 (the printed 66 gamma S vanishes on the axes) */

/* One anisotropy entry.  The entry is the polynomial of its kind evaluated at
 * R n, a_s(n) = A(R n), so that every crystal of the index field can have its
 * own orientation in 3D as well (Sec. 4.3, Eq. As_Multi, where each crystal
 * carries its own angle; R generalises that angle to a rotation).  R is
 * row-major and must be orthogonal (|R^T R - I| <= 1e-9, else LBPF_ERR_ARG);
 * all nine zero means the identity.  Every entry must keep a_s > 0 on the unit
 * sphere (the unit circle in 2D), checked on a fixed set of 4026 directions
 * (1448 in 2D): otherwise LBPF_ERR_UNSTABLE, since eta_phi = a_s^2 Dphi/e^2 +
 * 1/2 and the division by a_s^2 of Eq. LBE_Eq_Phase break down.  Under
 * LBPF_MIRROR_LOW every entry must be symmetric about the mirror planes
 * (a_s unchanged when n_x, n_y or, in 3D, n_z changes sign; checked on the
 * same directions to 1e-12): otherwise LBPF_ERR_UNSUPPORTED. */
typedef struct {
  int32_t kind;
  int32_t q;     /* sectoral order, >= 1 */
  double eps;
  double gamma;  /* CUBIC_HAK and CUBIC_S */
  double phi0;   /* sectoral reference angle, radians */
  double R[9];   /* orientation, row-major; all zero = identity */
} lbpf_aniso;

typedef struct {
  double x, y, z;   /* centre, lattice units */
  double radius;    /* lattice units; profile tanh((R - d)/(sqrt(2) W0/dx)), Eq. Initial_Condition */
  int32_t crystal_id;
} lbpf_seed;

typedef struct {
  int32_t lattice;   /* LBPF_D2Q9_D2Q5, LBPF_D3Q19_D3Q7 or LBPF_D3Q15_D3Q7 */
  int32_t nx, ny, nz;/* nz = 1 in 2D; every used extent >= 3 */
  int32_t boundary;  /* LBPF_PERIODIC, LBPF_ZERO_FLUX or LBPF_MIRROR_LOW */
  int32_t gradient;  /* LBPF_GRAD_DD, LBPF_GRAD_CD or LBPF_GRAD_UP2 */
  int32_t storage;   /* LBPF_FP64, LBPF_FP32_OFFSET or LBPF_FP16_OFFSET */
  int32_t use_ids;   /* 0: entry 0 of aniso everywhere; 1: crystal index field
                        I(x,t) selects entry I, I = 0 is isotropic (Sec. 4.3) */
  double W0, tau0, lambda, kappa, delta, dx, dt, xi;
  int32_t n_aniso;
  const lbpf_aniso *aniso; /* n_aniso entries (<= 256); with use_ids entry 0 must be ISO */
  int32_t n_seeds;
  const lbpf_seed *seeds;  /* n_seeds >= 0; overlapping seeds combine by max */
  int32_t tip_dir[3];      /* integer ray direction for the tip diagnostic ((0,0,0) = +x) */
} lbpf_config;

typedef struct {
  int64_t step;
  double sum_phi;              /* sum of phi over the nodes */
  double sum_u;                /* sum of u */
  double sum_u_minus_half_phi; /* sum of u - phi/2, conserved on periodic boxes */
  double solid_fraction;       /* sum (1 + phi) / (2 N) */
  double n_solid;              /* count of phi > 0 */
  double tip_position;         /* largest interpolated phi = 0 crossing along tip_dir from
                                  seed 0's centre, lattice units (-1 if none) */
  int32_t nonfinite;           /* 1 if any phi or u is not finite */
} lbpf_diag;

typedef struct lbpf_handle lbpf_handle;

/* Bytes of device workspace needed for n_sims simulations (n_sims > 1 is the
 * batched ensemble: every config must be 2D, share the storage mode and use
 * the index field in all or none; sizes, parameters, boundaries and gradient
 * methods may differ).  Returns LBPF_ERR_ARG / LBPF_ERR_UNSTABLE for an invalid
 * config, LBPF_ERR_UNSUPPORTED for an ensemble outside these rules. */
int lb_pf_workspace_bytes(const lbpf_config *cfgs, int n_sims, size_t *bytes);

/* Validates the configs, converts to lattice units (Eqs. ThermalDiffusivity,
 * LBE_RelaxationTime), lays out the fields inside dev_workspace and enqueues
 * the initial state on hip_stream: phi from the seeds (Eq. Initial_Condition),
 * u = -delta (Eq. Intial-Cond_u), the crystal index, g = g^(0)(phi, N(phi))
 * (Eq. Feq_Phase) and f = w_i u.  On failure no handle is returned. */
int lb_pf_init(const lbpf_config *cfgs, int n_sims, void *dev_workspace, size_t bytes,
               void *hip_stream, lbpf_handle **out);

/* Enqueues n_steps coupled steps (phase field, then heat) for every
 * simulation of the handle.  One fused kernel launch per step; a box with
 * mirror planes (LBPF_MIRROR_LOW, not batched) whose tiling leaves tiles beyond
 * the planes' reach takes two concurrent launches instead: the tiles at a plane
 * on a stream of the handle's own, forked from and joined back to hip_stream
 * with events, and the others on hip_stream, so that work enqueued on
 * hip_stream afterwards sees the whole step.  A batched
 * handle advances all its simulations in one persistent launch per step over
 * a work list of (simulation, 64-wide column, rows) items, replayed from HIP
 * graphs of 1 and 8 steps that are captured, on a private stream, the first
 * time they are needed (that call waits for the upload of the work list after
 * a change of tile). */
int lb_pf_step(lbpf_handle *h, int n_steps, void *hip_stream);

/* Reductions of the current state in FP64 (sums, solid fraction, tip).
 * out has one record per simulation.  Synchronises hip_stream.  Returns
 * LBPF_ERR_NONFINITE (and fills out) when a phi or u is not finite. */
int lb_pf_diagnostics(lbpf_handle *h, lbpf_diag *out, void *hip_stream);

/* lb_pf_diagnostics for callers that cannot allocate device memory (tight
 * serving loops, harnesses that forbid allocation): the same reductions and
 * the same results, but their per-block partials and the reduced values live
 * in a static device array of the library (32 KiB per GPU, held until the
 * process ends; the reductions need 24.6 KiB) instead of the handle's
 * workspace.  It calls no hipMalloc, hipFree or allocating routine.  Every
 * call on one GPU shares that GPU's array and leaves the last call's values
 * in it (nothing in it must start at zero: each call overwrites what it
 * reads): calls that overlap on one GPU, from several threads or streams,
 * race.  The handle's device (current at lb_pf_init) must be the current
 * device (LBPF_ERR_ARG otherwise).  Synchronises hip_stream. */
int lb_pf_diagnostics_noalloc(lbpf_handle *h, lbpf_diag *out, void *hip_stream);

/* Writes phi, u (FP64) and the crystal index of simulation `sim` into caller
 * device buffers of nx*ny*nz elements (any pointer may be NULL). */
int lb_pf_export_fields(lbpf_handle *h, int sim, double *phi_dev, double *u_dev,
                        int16_t *ids_dev, void *hip_stream);

/* Writes the post-streaming distributions g ([q_phi][N], FP64) and f
 * ([q_u][N], FP64) of simulation `sim` (either pointer may be NULL). */
int lb_pf_export_dists(lbpf_handle *h, int sim, double *g_dev, double *f_dev, void *hip_stream);

/* Replaces the state of simulation `sim` by the equilibrium distributions of
 * the given device fields (FP64 phi and u, int16 index or NULL for 0). */
int lb_pf_import_fields(lbpf_handle *h, int sim, const double *phi_dev, const double *u_dev,
                        const int16_t *ids_dev, void *hip_stream);

/* Checkpoint: the complete state as one opaque device blob of
 * lb_pf_state_bytes() bytes: a 256-byte header (the step counter and a
 * fingerprint of every simulation's extents, lattice, storage and index field)
 * followed by all fields of every simulation.  dev_buf is caller-owned device
 * memory, 8-byte aligned.  lb_pf_save_state enqueues the copy on hip_stream.
 * lb_pf_load_state synchronises hip_stream to read the header, returns
 * LBPF_ERR_ARG (state unchanged) when the blob was not saved from a handle of
 * the same layout, then enqueues the copy and restores the step counter. */
int lb_pf_state_bytes(const lbpf_handle *h, size_t *bytes);
int lb_pf_save_state(lbpf_handle *h, void *dev_buf, size_t bytes, void *hip_stream);
int lb_pf_load_state(lbpf_handle *h, const void *dev_buf, size_t bytes, void *hip_stream);

/* Tile shape of the step kernel: tile_y (4, 8 or 12; 12 needs FP32
 * arithmetic; LBPF_GRAD_UP2 takes 4 or 12) rows of 64 nodes per work-group in
 * 3D (1 in 2D), and `chunk` planes marched per
 * work-group (rows per work item, at least 8, for a batched handle).  0 keeps
 * the current value.  lb_pf_autotune times the candidate shapes on hip_stream
 * (advancing the state by the steps it runs: three times steps_per_trial per
 * candidate) and keeps the fastest. */
int lb_pf_set_tile(lbpf_handle *h, int tile_y, int chunk);
int lb_pf_get_tile(const lbpf_handle *h, int *tile_y, int *chunk);
int lb_pf_autotune(lbpf_handle *h, int steps_per_trial, void *hip_stream);

/* Measurement helpers (Sec. 5 measures the cost of a step; these give the
 * ceiling a step is measured against).  lb_pf_stream_copy reads every byte of
 * src once and writes it to dst once with 16-byte nontemporal vector
 * accesses, from a grid of blocks_per_cu (1..64) work-groups of 256 threads
 * per compute unit: the plain streaming copy that bounds any step moving the
 * same bytes.  Both buffers are caller-owned device memory, 16-byte aligned
 * and disjoint; enqueued on hip_stream.  lb_pf_state_ptr returns the device
 * address and size of simulation `sim`'s current state block inside the
 * workspace (the bytes a step reads; the step writes as many to the other
 * block), owned by the handle's caller. */
int lb_pf_stream_copy(const void *src_dev, void *dst_dev, size_t bytes, int blocks_per_cu, void *hip_stream);
int lb_pf_state_ptr(const lbpf_handle *h, int sim, void **state, size_t *bytes);

/* Number of simulations, nodes of simulation `sim`, step counter. */
int lb_pf_info(const lbpf_handle *h, int sim, int64_t *nodes, int64_t *step, int *q_phi, int *q_u);

/* Frees the handle (not the workspace).  Work enqueued on the handle must be
 * complete, except for a batched handle, whose destruction waits for the
 * device because its graphs may still run (the handle's own stream of a
 * mirror box is synchronised before it is destroyed). */
int lb_pf_destroy(lbpf_handle *h);
const char *lb_pf_last_error(void);

/* Sharp-interface relations of Sec. 2 (Eqs. Capillary-Length and
 * Kinetic-Coeff, a1 = 5 sqrt(2)/8, a2 = 0.6267): capillary length d0, kinetic
 * coefficient beta, and lambda* = kappa tau0 / (a2 W0^2) for which beta = 0. */
int lb_pf_sharp_interface(double W0, double tau0, double lambda, double kappa,
                          double *d0, double *beta, double *lambda_star);

#ifdef __cplusplus
}
#endif
#endif /* LB_PF_H */

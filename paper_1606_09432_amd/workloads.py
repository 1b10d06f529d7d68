"""Seeded, synthetic workload descriptions for the coupled LB phase-field step.

This module only *describes* inputs: grid, lattice pair, physical parameters,
seeds and per-crystal anisotropy entries.  It contains none of the method's
arithmetic and imports neither the GPU binding nor the oracle, so that both
can be driven from the same configuration.

The paper's workloads are themselves synthetic (diffuse seeds in a box,
Sec. 2 Eq. Initial_Condition, and the set-ups of Sec. 3.4, 4.2, 4.3 and 5).
The presets below follow the five benchmark configurations of this project:

* ``c0``  128^2 D2Q9/D2Q5, periodic, one seed R = 10, four-fold a_s, 2000 steps.
* ``c1``  2048^2, 20 seeds R = 5 at seeded random positions, per-crystal
  four-fold a_s rotated by theta0_k, crystal index field, zero flux.
* ``c2``  256^3 D3Q19/D3Q7, cubic a_s (Eq. As_Function_Classical), zero flux.
* ``c3``  512^3 D3Q19/D3Q7, Hoyt-Asta-Karma a_s (Eq. As_MatSci), zero flux.
* ``c4``  256 independent 2D simulations of seeded uneven sizes and parameters.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

LATTICES = ("D2Q9_D2Q5", "D3Q19_D3Q7", "D3Q15_D3Q7")
BOUNDARIES = ("periodic", "zero_flux", "mirror_low")
GRADIENTS = ("dd", "cd", "up2")
STORAGES = ("fp64", "fp32", "fp16")
ANISO_KINDS = ("iso", "sectoral", "cubic", "cubic_hak", "cubic_s")


@dataclass
class Aniso:
    """One anisotropy entry (Sec. 4.1).

    kind ``sectoral``: 1 + eps Re[((n_x + i n_y) e^{-i phi0})^q] (Eq. As_Theta,
    Eq. As_Multi; Eq. As_Y66 in 3D with q = 6).  ``cubic``: Eq.
    As_Function_Classical.  ``cubic_hak``: Eq. As_MatSci with (eps, gamma).
    ``cubic_s``: Eq. As_Function_S, 1 + 66 gamma n_x^2 n_y^2 n_z^2.
    """

    kind: str = "iso"
    eps: float = 0.0
    q: int = 4
    phi0: float = 0.0
    gamma: float = 0.0
    # orientation of the crystal: the polynomial is evaluated at R n (R given
    # row-major, 9 values); None is the identity
    R: Optional[Tuple[float, ...]] = None

    def rotation_row_major(self) -> List[float]:
        """The 9 values of R, or 9 zeros (the C structs' code for the identity)."""
        return [0.0] * 9 if self.R is None else [float(v) for v in self.R]


def rotation(axis: Tuple[float, float, float], angle: float) -> Tuple[float, ...]:
    """Row-major matrix of the rotation by `angle` (radians) about `axis`
    (Rodrigues' formula); an input-description helper for oriented crystals."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    R = np.eye(3) + math.sin(angle) * K + (1.0 - math.cos(angle)) * (K @ K)
    return tuple(float(v) for v in R.ravel())


@dataclass
class Seed:
    """A diffuse seed (Eq. Initial_Condition); centre and radius in lattice units."""

    x: float
    y: float
    z: float = 0.0
    radius: float = 10.0
    id: int = 1


@dataclass
class SimConfig:
    lattice: str = "D2Q9_D2Q5"
    nx: int = 128
    ny: int = 128
    nz: int = 1
    boundary: str = "periodic"
    gradient: str = "dd"
    storage: str = "fp64"
    W0: float = 1.0
    tau0: float = 1.0
    lam: float = 10.0
    kappa: float = 6.267
    delta: float = 0.3
    dx: float = 0.4
    dt: float = 0.008
    xi: float = 1e-7
    aniso: List[Aniso] = field(default_factory=lambda: [Aniso("sectoral", 0.05, 4, 0.0)])
    seeds: List[Seed] = field(default_factory=list)
    use_ids: bool = False
    tip_dir: Tuple[int, int, int] = (1, 0, 0)

    @property
    def dim(self) -> int:
        return 2 if self.lattice == "D2Q9_D2Q5" else 3

    @property
    def nodes(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self) -> Tuple[int, ...]:
        """numpy shape of a field, slowest axis first: (ny, nx) or (nz, ny, nx)."""
        return (self.ny, self.nx) if self.dim == 2 else (self.nz, self.ny, self.nx)

    def replace(self, **kw) -> "SimConfig":
        return dataclasses.replace(self, **kw)

    def validate(self) -> None:
        assert self.lattice in LATTICES, self.lattice
        assert self.boundary in BOUNDARIES, self.boundary
        assert self.gradient in GRADIENTS, self.gradient
        assert self.storage in STORAGES, self.storage
        for a in self.aniso:
            assert a.kind in ANISO_KINDS, a.kind
        if self.dim == 2:
            assert self.nz == 1


# ----------------------------------------------------------------------------
# Presets.  Unstated parameters follow the paper's Sec. 3.4 set-up:
# W0 = tau0 = 1, dx = 0.4, dt = 0.008, lambda = 10, kappa = D = 0.6267 lambda.
# ----------------------------------------------------------------------------
KAPPA_C0 = 0.6267 * 10.0


def c0(storage: str = "fp64", gradient: str = "dd", n: int = 128) -> SimConfig:
    """128^2, periodic, one centred seed R = 10 lu, a_s = 1 + 0.05 cos 4 phi."""
    c = n // 2
    return SimConfig(
        lattice="D2Q9_D2Q5", nx=n, ny=n, nz=1, boundary="periodic", gradient=gradient,
        storage=storage, delta=0.3, kappa=KAPPA_C0,
        aniso=[Aniso("sectoral", eps=0.05, q=4, phi0=0.0)],
        seeds=[Seed(c, c, 0.0, 10.0, 1)], tip_dir=(1, 0, 0))


C0_STEPS = 2000


def c1_seeds(n: int = 2048, count: int = 20, radius: float = 5.0, margin: int = 32,
             min_gap: float = 32.0, rng_seed: int = 160601):
    """Seed centres ~ U[margin, n - margin)^2 with pairwise distance >= min_gap,
    and per-crystal orientation theta0 ~ U[0, pi/2)."""
    rng = np.random.default_rng(rng_seed)
    pts: List[Tuple[float, float]] = []
    while len(pts) < count:
        p = rng.integers(margin, n - margin, size=2)
        if all(math.hypot(p[0] - q[0], p[1] - q[1]) >= min_gap for q in pts):
            pts.append((int(p[0]), int(p[1])))
    theta = rng.uniform(0.0, math.pi / 2, size=count)
    return pts, [float(t) for t in theta]


def c1(storage: str = "fp64", gradient: str = "dd", n: int = 2048, count: int = 20,
       rng_seed: int = 160601) -> SimConfig:
    pts, theta = c1_seeds(n, count, rng_seed=rng_seed,
                          margin=max(4, min(32, n // 16)), min_gap=max(8.0, min(32.0, n / 8)))
    aniso = [Aniso("iso")] + [Aniso("sectoral", eps=0.05, q=4, phi0=t) for t in theta]
    seeds = [Seed(px, py, 0.0, 5.0, k + 1) for k, (px, py) in enumerate(pts)]
    return SimConfig(
        lattice="D2Q9_D2Q5", nx=n, ny=n, nz=1, boundary="zero_flux", gradient=gradient,
        storage=storage, delta=0.5, kappa=KAPPA_C0, aniso=aniso, seeds=seeds, use_ids=True,
        tip_dir=(1, 0, 0))


C1_STEPS = 20000


def c2(storage: str = "fp64", n: int = 256, radius: float = 8.0) -> SimConfig:
    c = n // 2
    return SimConfig(
        lattice="D3Q19_D3Q7", nx=n, ny=n, nz=n, boundary="zero_flux", gradient="dd",
        storage=storage, delta=0.55, kappa=KAPPA_C0, aniso=[Aniso("cubic", eps=0.05)],
        seeds=[Seed(c, c, c, radius, 1)], tip_dir=(1, 0, 0))


C2_STEPS = 10000

# (eps_1, eps_2) of Eq. As_MatSci for the three 512^3 runs, with the lattice
# direction of the favoured growth used as the tip ray.
C3_VARIANTS = {
    "100": ((0.1, 0.0), (1, 0, 0)),
    "111": ((-0.02, 0.0), (1, 1, 1)),
    "110": ((0.0, -0.05), (1, 1, 0)),
}


def c3(storage: str = "fp16", variant: str = "100", n: int = 512, radius: float = 8.0,
       lattice: str = "D3Q19_D3Q7") -> SimConfig:
    (e1, e2), tip = C3_VARIANTS[variant]
    c = n // 2
    return SimConfig(
        lattice=lattice, nx=n, ny=n, nz=n, boundary="zero_flux", gradient="dd",
        storage=storage, delta=0.6, kappa=KAPPA_C0,
        aniso=[Aniso("cubic_hak", eps=e1, gamma=e2)],
        seeds=[Seed(c, c, c, radius, 1)], tip_dir=tip)


C3_STEPS = 20000


def dense_3d(storage: str = "fp16", n: int = 512, spacing: int = 64, radius: float = 20.0,
             lattice: str = "D3Q19_D3Q7", rng_seed: int = 160605) -> SimConfig:
    """The 512^3 workload's physics (Eq. As_MatSci <100>, Delta = 0.6) with a
    crystal every `spacing` nodes (centres jittered by up to spacing/8): every
    node lies within a few interface widths of a crystal, so nearly all take
    the anisotropic path of the step, as in a late stage of a growth run."""
    rng = np.random.default_rng(rng_seed)
    (e1, e2), _ = C3_VARIANTS["100"]
    k = n // spacing
    seeds = []
    for iz in range(k):
        for iy in range(k):
            for ix in range(k):
                j = rng.uniform(-spacing / 8, spacing / 8, size=3)
                c = (np.array([ix, iy, iz]) + 0.5) * spacing + j
                seeds.append(Seed(float(c[0]), float(c[1]), float(c[2]), radius, 1))
    return SimConfig(
        lattice=lattice, nx=n, ny=n, nz=n, boundary="zero_flux", gradient="dd",
        storage=storage, delta=0.6, kappa=KAPPA_C0, aniso=[Aniso("cubic_hak", eps=e1, gamma=e2)],
        seeds=seeds, tip_dir=(1, 0, 0))


def c4(count: int = 256, rng_seed: int = 160604, storage: str = "fp32",
       side_lo: int = 2, side_hi: int = 16) -> List[SimConfig]:
    """Ensemble of independent 2D simulations with seeded uneven sizes/parameters."""
    rng = np.random.default_rng(rng_seed)
    out = []
    for _ in range(count):
        nx = 32 * int(rng.integers(side_lo, side_hi + 1))
        ny = 32 * int(rng.integers(side_lo, side_hi + 1))
        eps = float(rng.uniform(0.01, 0.07))
        delta = float(rng.uniform(0.2, 0.6))
        radius = float(rng.uniform(4.0, 12.0))
        out.append(SimConfig(
            lattice="D2Q9_D2Q5", nx=nx, ny=ny, nz=1, boundary="zero_flux", gradient="dd",
            storage=storage, delta=delta, kappa=KAPPA_C0,
            aniso=[Aniso("sectoral", eps=eps, q=4, phi0=0.0)],
            seeds=[Seed(nx // 2, ny // 2, 0.0, radius, 1)], tip_dir=(1, 0, 0)))
    return out


C4_STEPS = 5000


def e2(gradient: str = "dd", n: int = 800, storage: str = "fp64") -> SimConfig:
    """The isotropy comparison of Sec. 4.2: six-fold a_s (Eq. As_Theta, q = 6,
    phi0 = 0, eps = 0.05), 800^2, seed R = 10 lu at (400, 400), dx = 0.01,
    dt = 1.5e-5, tau0 = 1.5625e-4, W0 = 0.0125, kappa = 1, Delta = 0.3,
    lambda = 10 (lattice units: W0/dx = 1.25, Dphi = 0.15, dt/tau0 = 0.096,
    Du = 0.15); gradients by directional derivatives or central differences.
    The walls are not stated; zero flux is used."""
    c = n // 2
    return SimConfig(
        lattice="D2Q9_D2Q5", nx=n, ny=n, nz=1, boundary="zero_flux", gradient=gradient,
        storage=storage, W0=0.0125, tau0=1.5625e-4, lam=10.0, kappa=1.0, delta=0.3,
        dx=0.01, dt=1.5e-5, aniso=[Aniso("sectoral", eps=0.05, q=6, phi0=0.0)],
        seeds=[Seed(c, c, 0.0, 10.0, 1)], tip_dir=(1, 0, 0))


E2_STEPS = 100000


# The paper's 3D runs of Sec. 5 (D3Q15 + D3Q7, 351^3, seed at the centre):
# dendrite A Eq. As_Function_Classical eps = 0.05, dendrite B Eq. As_MatSci
# eps = 0, gamma = -0.02, dendrite C Eq. As_Function_S gamma = 0.02; with the
# step counts read from the caption of the dendrite figure and the wall-clock
# times the paper gives for 100 CPU cores.
PAPER3D = {
    "A": (Aniso("cubic", eps=0.05), 5000, 3.0 * 3600),
    "B": (Aniso("cubic_hak", eps=0.0, gamma=-0.02), 25000, 8.97 * 3600),
    "C": (Aniso("cubic_s", gamma=0.02), 15000, 9.18 * 3600),
}


def paper3d(dendrite: str = "A", storage: str = "fp64", n: int = 351) -> SimConfig:
    entry = PAPER3D[dendrite][0]
    c = n // 2
    return SimConfig(
        lattice="D3Q15_D3Q7", nx=n, ny=n, nz=n, boundary="zero_flux", gradient="dd", storage=storage,
        W0=0.0125, tau0=1.5625e-4, lam=10.0, kappa=1.0, delta=0.3, dx=0.01, dt=1.5e-5, aniso=[entry],
        seeds=[Seed(c, c, c, 10.0, 1)], tip_dir=(1, 0, 0))


# The paper's symmetric run of dendrite B (Sec. 5): seed at the origin of a
# 351^3 box, completed by symmetry about the planes XY, YZ and XZ, Delta = 0.25,
# 1.5e5 steps in 98.54 h on 50 CPU cores.
PAPER3D_OCTANT = (Aniso("cubic_hak", eps=0.0, gamma=-0.02), 150000, 98.54 * 3600, 50)


def paper3d_octant(storage: str = "fp64", n: int = 351) -> SimConfig:
    return paper3d("B", storage, n).replace(boundary="mirror_low", delta=0.25, aniso=[PAPER3D_OCTANT[0]],
                                            seeds=[Seed(0.0, 0.0, 0.0, 10.0, 1)])


def multi_3d(storage: str = "fp64", lattice: str = "D3Q19_D3Q7", gradient: str = "dd",
             shape=(48, 44, 40), boundary: str = "zero_flux", y66_phi0: float = 0.3) -> SimConfig:
    """A small 3D box with three crystals, each with its own anisotropy entry
    in the crystal index field (Sec. 4.3): cubic, Eq. As_MatSci and Eq. As_Y66
    turned by y66_phi0 about z (0 keeps every entry symmetric about the
    coordinate planes, as a box with mirror planes requires)."""
    nx, ny, nz = shape
    aniso = [Aniso("iso"), Aniso("cubic", eps=0.05), Aniso("cubic_hak", eps=0.1, gamma=0.0),
             Aniso("sectoral", eps=0.05, q=6, phi0=y66_phi0)]
    seeds = [Seed(nx * 0.27, ny * 0.3, nz * 0.35, 4.0, 1), Seed(nx * 0.7, ny * 0.33, nz * 0.6, 4.5, 2),
             Seed(nx * 0.45, ny * 0.72, nz * 0.5, 3.5, 3)]
    return SimConfig(
        lattice=lattice, nx=nx, ny=ny, nz=nz, boundary=boundary, gradient=gradient, storage=storage,
        delta=0.55, kappa=KAPPA_C0, aniso=aniso, seeds=seeds, use_ids=True, tip_dir=(1, 0, 0))


# Orientations of the oriented-crystals workload: rotations about skew axes,
# so that no crystal shares the lattice's axes or another crystal's.
ORIENTED_AXES = (((1.0, 1.0, 1.0), 0.4), ((1.0, -2.0, 0.5), 1.1))


def oriented_3d(storage: str = "fp64", lattice: str = "D3Q19_D3Q7", gradient: str = "dd",
                shape=(56, 48, 44), boundary: str = "zero_flux") -> SimConfig:
    """Three crystals of one cubic-harmonic kind (Eq. As_MatSci, eps = 0.1) in
    the crystal index field, two of them turned by their own rotation R: the
    per-crystal orientation of Sec. 4.3 (Eq. As_Multi) in 3D."""
    nx, ny, nz = shape
    base = dict(kind="cubic_hak", eps=0.1, gamma=0.0)
    aniso = [Aniso("iso"), Aniso(**base)] + [Aniso(**base, R=rotation(ax, ang)) for ax, ang in ORIENTED_AXES]
    seeds = [Seed(nx * 0.27, ny * 0.3, nz * 0.35, 4.5, 1), Seed(nx * 0.7, ny * 0.35, nz * 0.6, 4.5, 2),
             Seed(nx * 0.45, ny * 0.72, nz * 0.45, 4.5, 3)]
    return SimConfig(
        lattice=lattice, nx=nx, ny=ny, nz=nz, boundary=boundary, gradient=gradient, storage=storage,
        delta=0.55, kappa=KAPPA_C0, aniso=aniso, seeds=seeds, use_ids=True, tip_dir=(1, 0, 0))


def small_3d(storage: str = "fp64", n: int = 48, aniso: Aniso | None = None,
             boundary: str = "zero_flux", radius: float = 6.0, delta: float = 0.55,
             nx: int | None = None, ny: int | None = None, nz: int | None = None) -> SimConfig:
    """A short 3D case the oracle finishes in seconds (parity tests)."""
    nx = nx or n
    ny = ny or n
    nz = nz or n
    return SimConfig(
        lattice="D3Q19_D3Q7", nx=nx, ny=ny, nz=nz, boundary=boundary, gradient="dd",
        storage=storage, delta=delta, kappa=KAPPA_C0,
        aniso=[aniso or Aniso("cubic", eps=0.05)],
        seeds=[Seed(nx // 2, ny // 2, nz // 2, radius, 1)], tip_dir=(1, 0, 0))

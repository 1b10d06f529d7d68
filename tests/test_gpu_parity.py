"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle.

Every comparison is element by element on the same seeded inputs.  FP64
storage must match the oracle within 1e-10 max-abs on phi and u (and the
crystal index exactly); the offset storage modes (FP32 arithmetic) are held
to the accuracy bounds written in each test.  Each case prints its name before
touching the GPU.
"""
import math

import numpy as np
import pytest

from paper_1606_09432_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _gpu_run(lb, cfg, steps, tile=None):
    import torch
    sim = lb.Simulation(cfg)
    if tile:
        sim.set_tile(*tile)
    sim.step(steps)
    phi, u, ids = sim.fields()
    torch.cuda.synchronize()
    return sim, phi.cpu().numpy(), u.cpu().numpy(), ids.cpu().numpy()


def _oracle_run(O, cfg, steps):
    orc = O.OracleSim(cfg.replace(storage="fp64"))
    orc.step(steps)
    return orc


def _case(cfg, steps):
    return (f"{cfg.lattice} {cfg.nx}x{cfg.ny}x{cfg.nz} {cfg.boundary} {cfg.gradient} {cfg.storage} "
            f"ids={cfg.use_ids} steps={steps}")


def _compare(lb, O, cfg, steps, tol=FP64_TOL, tile=None):
    _say(_case(cfg, steps))
    sim, phi, u, ids = _gpu_run(lb, cfg, steps, tile)
    orc = _oracle_run(O, cfg, steps)
    ephi = np.abs(phi - orc.phi()).max()
    eu = np.abs(u - orc.u()).max()
    _say(f"  max|dphi| = {ephi:.3e} at {np.unravel_index(np.abs(phi - orc.phi()).argmax(), phi.shape)}"
         f"  max|du| = {eu:.3e}")
    if cfg.use_ids:
        bad = ids != orc.ids()
        _say(f"  index mismatches: {int(bad.sum())} at {np.argwhere(bad)[:5].tolist()}")
    assert ephi <= tol and eu <= tol, (ephi, eu)
    if cfg.use_ids:
        assert np.array_equal(ids, orc.ids())
    return sim, orc


# ---------------------------------------------------------------------------
# The 128^2 periodic four-fold case, 2000 steps, FP64: the headline parity bar.
# ---------------------------------------------------------------------------
def test_c0_fp64_parity(gpu, oracle_mod):
    cfg = W.c0()
    sim, orc = _compare(gpu, oracle_mod, cfg, W.C0_STEPS)
    dg = sim.diagnostics()[0]
    do = orc.diagnostics()
    assert abs(dg["sum_phi"] - do["sum_phi"]) < 1e-8
    assert abs(dg["sum_u_minus_half_phi"] - do["sum_u_minus_half_phi"]) < 1e-8
    assert dg["n_solid"] == do["n_solid"]
    assert abs(dg["tip_position"] - do["tip_position"]) < 1e-8
    assert dg["step"] == W.C0_STEPS


@pytest.mark.parametrize("boundary,grad,nx,ny", [
    ("zero_flux", "dd", 70, 45), ("zero_flux", "cd", 130, 67), ("periodic", "cd", 96, 80),
    ("periodic", "dd", 65, 130), ("zero_flux", "dd", 3, 3), ("periodic", "cd", 3, 5)])
def test_2d_fp64_parity(gpu, oracle_mod, boundary, grad, nx, ny):
    cfg = W.c0(gradient=grad).replace(nx=nx, ny=ny, boundary=boundary,
                                      aniso=[W.Aniso("sectoral", 0.05, 4, math.radians(20))],
                                      seeds=[W.Seed(nx * 0.4, ny * 0.55, 0, min(nx, ny) * 0.15 + 1, 1)])
    _compare(gpu, oracle_mod, cfg, 300 if nx > 3 else 20)


def test_2d_distributions_parity(gpu, oracle_mod):
    cfg = W.c0(n=72).replace(boundary="zero_flux", seeds=[W.Seed(20, 30, 0, 6, 1)])
    _say(_case(cfg, 50))
    sim, _, _, _ = _gpu_run(gpu, cfg, 50)
    g, f = sim.dists()
    orc = _oracle_run(oracle_mod, cfg, 50)
    dg = np.abs(g.cpu().numpy() - orc.g())
    loc = np.unravel_index(dg.argmax(), dg.shape)
    _say(f"  max|dg| = {dg.max():.3e} at (i, y, x) = {loc}; nodes with |dg| > 1e-12: "
         f"{np.argwhere(dg.max(0) > 1e-12)[:8].tolist()}  dirs: {sorted(set(np.argwhere(dg > 1e-12)[:, 0].tolist()))}")
    _say(f"  max|dphi| = {np.abs(sim.fields()[0].cpu().numpy() - orc.phi()).max():.3e}")
    assert np.abs(g.cpu().numpy() - orc.g()).max() < 1e-12
    assert np.abs(f.cpu().numpy() - orc.f()).max() < 1e-12


@pytest.mark.parametrize("boundary,grad,shape,entry,steps", [
    ("zero_flux", "dd", (40, 36, 33), W.Aniso("cubic", eps=0.05), 80),
    ("periodic", "dd", (34, 32, 30), W.Aniso("cubic_hak", eps=0.0, gamma=-0.05), 60),
    ("zero_flux", "cd", (66, 20, 18), W.Aniso("cubic_hak", eps=0.1, gamma=0.0), 40),
    ("zero_flux", "dd", (3, 3, 3), W.Aniso("cubic", eps=0.05), 10),
    ("periodic", "dd", (24, 24, 24), W.Aniso("sectoral", eps=0.05, q=6, phi0=0.0), 40),
    ("zero_flux", "dd", (36, 34, 40), W.Aniso("cubic_s", gamma=0.02), 60),
])
def test_3d_fp64_parity(gpu, oracle_mod, boundary, grad, shape, entry, steps):
    nx, ny, nz = shape
    cfg = W.small_3d(nx=nx, ny=ny, nz=nz, aniso=entry, boundary=boundary,
                     radius=max(1.5, min(shape) * 0.2)).replace(gradient=grad)
    cfg.seeds[0].x = nx * 0.45
    _compare(gpu, oracle_mod, cfg, steps)


# D3Q15, the paper's own 3D phase-field lattice (Table Values-Lattices).
@pytest.mark.parametrize("boundary,grad,shape,entry,steps", [
    ("zero_flux", "dd", (40, 36, 33), W.Aniso("cubic", eps=0.05), 80),
    ("periodic", "cd", (34, 32, 30), W.Aniso("cubic_hak", eps=0.1, gamma=0.0), 60),
    ("zero_flux", "dd", (70, 22, 20), W.Aniso("sectoral", eps=0.05, q=6, phi0=0.0), 50),
])
def test_d3q15_fp64_parity(gpu, oracle_mod, boundary, grad, shape, entry, steps):
    nx, ny, nz = shape
    cfg = W.small_3d(nx=nx, ny=ny, nz=nz, aniso=entry, boundary=boundary, radius=min(shape) * 0.2)
    cfg = cfg.replace(gradient=grad, lattice="D3Q15_D3Q7")
    cfg.seeds[0].x = nx * 0.45
    _compare(gpu, oracle_mod, cfg, steps)


# 64^3 for 200 steps in FP64, both 3D lattice pairs: the benchmark's
# anisotropy (Eq. As_MatSci, <100> variant) with the undercooling of the
# 512^3 runs, the seed off-centre so that no symmetry hides an index mistake.
@pytest.mark.parametrize("lattice,boundary", [("D3Q19_D3Q7", "zero_flux"), ("D3Q15_D3Q7", "zero_flux"),
                                              ("D3Q19_D3Q7", "periodic")])
def test_3d_fp64_parity_64_cubed_200_steps(gpu, oracle_mod, lattice, boundary):
    cfg = W.c3("fp64", "100", n=64).replace(lattice=lattice, boundary=boundary,
                                              seeds=[W.Seed(29.4, 33.2, 31.7, 8.0, 1)])
    sim, orc = _compare(gpu, oracle_mod, cfg, 200)
    dg, do = sim.diagnostics()[0], orc.diagnostics()
    _say(f"  tip {dg['tip_position']:.6f} / {do['tip_position']:.6f}  n_solid {dg['n_solid']} / {do['n_solid']}")
    assert do["tip_position"] > 10.0  # the crystal grew
    assert abs(dg["tip_position"] - do["tip_position"]) < 1e-9 and dg["n_solid"] == do["n_solid"]
    assert abs(dg["sum_u_minus_half_phi"] - do["sum_u_minus_half_phi"]) < 1e-8


# The initial state itself (Sec. 2, Eq. Initial_Condition and Eq.
# Intial-Cond_u; g = g^(0), f = w_i u): phi, u, the index and the decoded
# populations at step 0, then after one step.
@pytest.mark.parametrize("which", ["2d_ids", "3d_oriented", "d3q15", "periodic_2d"])
def test_initial_state_parity(gpu, oracle_mod, which):
    if which == "2d_ids":
        cfg = W.c1(n=96, count=4).replace(seeds=[W.Seed(30.2, 40.7, 0, 9.0, 1), W.Seed(41.3, 44.1, 0, 6.5, 2),
                                                 W.Seed(70.0, 20.0, 0, 5.0, 3), W.Seed(72.5, 70.25, 0, 4.0, 4)])
    elif which == "3d_oriented":
        cfg = W.oriented_3d()
    elif which == "d3q15":
        cfg = W.small_3d(n=30, radius=6.3, aniso=W.Aniso("cubic_s", gamma=0.02)).replace(lattice="D3Q15_D3Q7")
    else:
        cfg = W.c0(n=64).replace(seeds=[W.Seed(3.0, 60.0, 0, 7.0, 1)])  # wraps around two edges
    _say(_case(cfg, 0) + f" initial state ({which})")
    sim = gpu.Simulation(cfg)
    orc = _oracle_run(oracle_mod, cfg, 0)
    for steps in (0, 1):
        phi, u, ids = [t.cpu().numpy() for t in sim.fields()]
        g, f = [t.cpu().numpy() for t in sim.dists()]
        ep, eu = np.abs(phi - orc.phi()).max(), np.abs(u - orc.u()).max()
        eg, ef = np.abs(g - orc.g()).max(), np.abs(f - orc.f()).max()
        _say(f"  step {steps}: |dphi| {ep:.2e} |du| {eu:.2e} |dg| {eg:.2e} |df| {ef:.2e}")
        assert ep <= 1e-14 and eu <= 1e-14 and eg <= 1e-14 and ef <= 1e-14
        if cfg.use_ids:
            assert np.array_equal(ids, orc.ids())
            assert len(np.unique(ids)) == len(cfg.seeds) + 1
        if steps == 0:
            # u is read back as the sum of its populations w_i u
            assert np.abs(u + cfg.delta).max() <= 1e-15
            sim.step(1)
            orc.step(1)


# Two crystals of one cubic-harmonic kind turned by their own rotations and a
# third unturned, in the 3D index field (Sec. 4.3, per-crystal orientation).
@pytest.mark.parametrize("lattice,grad", [("D3Q19_D3Q7", "dd"), ("D3Q15_D3Q7", "dd"), ("D3Q19_D3Q7", "cd")])
def test_oriented_crystals_parity(gpu, oracle_mod, lattice, grad):
    cfg = W.oriented_3d(lattice=lattice, gradient=grad)
    sim, orc = _compare(gpu, oracle_mod, cfg, 150)
    ids = orc.ids()
    assert all((ids == k).sum() > 400 for k in (1, 2, 3))
    # the orientations matter: the same run with every crystal unturned differs
    if lattice == "D3Q19_D3Q7" and grad == "dd":
        plain = cfg.replace(aniso=[cfg.aniso[0]] + [W.Aniso("cubic_hak", eps=0.1)] * 3)
        _, phi2, _, _ = _gpu_run(gpu, plain, 150)
        assert np.abs(phi2 - orc.phi()).max() > 1e-3


@pytest.mark.parametrize("storage,tol", [("fp32", 1e-4), ("fp16", 1e-3)])
def test_oriented_crystals_offset_storage(gpu, oracle_mod, storage, tol):
    cfg = W.oriented_3d(storage=storage)
    _say(_case(cfg, 150))
    sim, phi, u, _ = _gpu_run(gpu, cfg, 150)
    orc = _oracle_run(oracle_mod, cfg, 150)
    ephi, eu = np.abs(phi - orc.phi()).max(), np.abs(u - orc.u()).max()
    _say(f"  {storage}: max|dphi| = {ephi:.3e} max|du| = {eu:.3e}")
    assert ephi <= tol and eu <= tol


# FP64 diagnostics on imported hand-built fields whose sums are exact in
# binary: the reductions must return them exactly.
@pytest.mark.parametrize("cfg", [W.small_3d(n=40, nx=70), W.c0(n=96).replace(ny=130)], ids=["3d", "2d"])
def test_diagnostics_on_hand_built_fields(gpu, cfg):
    import torch
    _say(_case(cfg, 0) + " hand-built diagnostics")
    rng = np.random.default_rng(12)
    phi = rng.choice([-1.0, -0.5, 0.0, 0.25, 1.0], size=cfg.shape)
    u = rng.choice([-0.5, 0.125, 0.375], size=cfg.shape)
    sim = gpu.Simulation(cfg)
    sim.import_fields(phi, u)
    d = sim.diagnostics()[0]
    assert d["sum_phi"] == float(phi.sum())
    # u is read back as the sum of its populations w_i u: exact with the D3Q7
    # weights (1/4, 1/8), within rounding with the D2Q5 ones (1/3, 1/6)
    tol_u = 0.0 if cfg.dim == 3 else 1e-15 * cfg.nodes
    assert abs(d["sum_u"] - float(u.sum())) <= tol_u
    assert abs(d["sum_u_minus_half_phi"] - float((u - 0.5 * phi).sum())) <= tol_u
    assert d["n_solid"] == float((phi > 0).sum())
    assert d["solid_fraction"] == float((1.0 + phi).sum()) / (2.0 * cfg.nodes)
    assert d["nonfinite"] == 0
    torch.cuda.synchronize()


@pytest.mark.parametrize("storage,tol", [("fp32", 1e-4), ("fp16", 1e-3)])
def test_d3q15_offset_storage_accuracy(gpu, oracle_mod, storage, tol):
    cfg = W.small_3d(storage=storage, n=40, radius=6).replace(lattice="D3Q15_D3Q7")
    _say(_case(cfg, 100))
    sim, phi, u, _ = _gpu_run(gpu, cfg, 100)
    orc = _oracle_run(oracle_mod, cfg, 100)
    ephi = np.abs(phi - orc.phi()).max()
    eu = np.abs(u - orc.u()).max()
    _say(f"  {storage}: max|dphi| = {ephi:.3e} max|du| = {eu:.3e}")
    assert ephi <= tol and eu <= tol


@pytest.mark.parametrize("lattice", ["D3Q19_D3Q7", "D3Q15_D3Q7"])
def test_3d_distributions_parity(gpu, oracle_mod, lattice):
    cfg = W.small_3d(nx=30, ny=28, nz=26, radius=5).replace(lattice=lattice)
    _say(_case(cfg, 25))
    sim, _, _, _ = _gpu_run(gpu, cfg, 25)
    g, f = sim.dists()
    orc = _oracle_run(oracle_mod, cfg, 25)
    assert np.abs(g.cpu().numpy() - orc.g()).max() < 1e-12
    assert np.abs(f.cpu().numpy() - orc.f()).max() < 1e-12


@pytest.mark.parametrize("grad", ["dd", "cd"])
def test_crystal_index_parity(gpu, oracle_mod, grad):
    cfg = W.c1(n=160, count=5, gradient=grad)
    _compare(gpu, oracle_mod, cfg, 300)


@pytest.mark.parametrize("lattice,grad,boundary", [("D3Q19_D3Q7", "dd", "zero_flux"), ("D3Q19_D3Q7", "cd", "periodic"),
                                                  ("D3Q15_D3Q7", "dd", "zero_flux")])
def test_3d_crystal_index_parity(gpu, oracle_mod, lattice, grad, boundary):
    """Three crystals with different anisotropy entries in the 3D index field."""
    cfg = W.multi_3d(lattice=lattice, gradient=grad, boundary=boundary)
    sim, orc = _compare(gpu, oracle_mod, cfg, 120)
    ids = orc.ids()
    assert all((ids == k).sum() > 300 for k in (1, 2, 3))  # every crystal grew


@pytest.mark.parametrize("storage,tol", [("fp32", 1e-4), ("fp16", 1e-3)])
def test_3d_crystal_index_offset_storage(gpu, oracle_mod, storage, tol):
    """Offset storage with the index field: phi and u within the offset bounds.
    The index decisions are taken in FP32 there (the oracle takes them in
    FP64).  At the outer edge of the dilation, |grad phi| is compared with
    xi = 1e-7 where phi is within 1e-6 of -1, i.e. at the FP32 rounding level
    of phi, so those decisions may differ; wherever phi > -0.99 the index must
    agree exactly, and the far-field differences stay below 0.1 % of the nodes."""
    cfg = W.multi_3d(storage=storage)
    _say(_case(cfg, 120))
    sim, phi, u, ids = _gpu_run(gpu, cfg, 120)
    orc = _oracle_run(oracle_mod, cfg, 120)
    ephi = np.abs(phi - orc.phi()).max()
    eu = np.abs(u - orc.u()).max()
    diff = ids != orc.ids()
    near = diff & (orc.phi() > -0.99)
    _say(f"  {storage}: max|dphi| = {ephi:.3e} max|du| = {eu:.3e} index mismatches {int(diff.sum())} "
         f"(near the crystals {int(near.sum())})")
    assert ephi <= tol and eu <= tol
    assert int(near.sum()) == 0 and int(diff.sum()) <= cfg.nodes // 1000


@pytest.mark.parametrize("case", ["2d", "3d"])
def test_large_index_table_parity(gpu, oracle_mod, case):
    """More crystal entries than the kernel stages in LDS (32): the entries are
    then read from the table in memory; FP64 against the oracle."""
    if case == "2d":
        cfg = W.c1(n=256, count=40)
        steps = 150
    else:
        base = W.oriented_3d(shape=(48, 44, 40))
        extra = [W.Aniso("iso")] * 38  # unused entries beyond the staged range
        cfg = base.replace(aniso=list(base.aniso) + extra)
        steps = 40
    assert len(cfg.aniso) > 32
    sim, orc = _compare(gpu, oracle_mod, cfg, steps)
    assert np.array_equal(sim.fields()[2].cpu().numpy(), orc.ids())


def test_batched_with_index_field(gpu, oracle_mod):
    """A batched ensemble whose members use the crystal index field."""
    cfgs = [W.c1(n=n, count=3, rng_seed=s).replace(ny=n + 16) for n, s in ((96, 1), (128, 2), (80, 3))]
    _say("batched ensemble with index fields, 60 steps")
    sim = gpu.Simulation(cfgs)
    sim.step(60)
    for k, cfg in enumerate(cfgs):
        phi, u, ids = sim.fields(k)
        orc = _oracle_run(oracle_mod, cfg, 60)
        ep = np.abs(phi.cpu().numpy() - orc.phi()).max()
        eu = np.abs(u.cpu().numpy() - orc.u()).max()
        bad = int((ids.cpu().numpy() != orc.ids()).sum())
        _say(f"  sim {k}: max|dphi| = {ep:.3e} max|du| = {eu:.3e} index mismatches {bad}")
        assert ep <= FP64_TOL and eu <= FP64_TOL and bad == 0


def test_c1_full_size_parity(gpu, oracle_mod):
    """2048^2 with 20 crystals, in the default launch configuration, elementwise."""
    _compare(gpu, oracle_mod, W.c1(), 12)


# ---------------------------------------------------------------------------
# Full-size 512^3 in the benchmark's launch configuration: a node's update
# depends on its 2-hop neighbourhood only, so after k steps the nodes farther
# than 2k from the walls of an oracle box centred on the seed see exactly the
# 512^3 problem.  Compare that window.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("storage,tol", [("fp64", FP64_TOL), ("fp16", 1e-3)])
def test_c3_full_size_window(gpu, oracle_mod, storage, tol):
    import torch
    k, half = 6, 26
    cfg = W.c3(storage, "110")
    _say(_case(cfg, k) + " (window parity)")
    sim = gpu.Simulation(cfg)
    sim.step(k)
    phi, u, _ = sim.fields()
    c = cfg.nx // 2
    sl = slice(c - half, c + half)
    gphi = phi[sl, sl, sl].cpu().numpy()
    gu = u[sl, sl, sl].cpu().numpy()
    del sim, phi, u
    torch.cuda.empty_cache()
    n = 2 * half
    wcfg = cfg.replace(nx=n, ny=n, nz=n, storage="fp64", seeds=[W.Seed(half, half, half, 8.0, 1)])
    orc = _oracle_run(oracle_mod, wcfg, k)
    inner = slice(2 * k, n - 2 * k)
    ephi = np.abs(gphi[inner, inner, inner] - orc.phi()[inner, inner, inner]).max()
    eu = np.abs(gu[inner, inner, inner] - orc.u()[inner, inner, inner]).max()
    _say(f"  window max|dphi| = {ephi:.3e}  max|du| = {eu:.3e}")
    assert ephi <= tol and eu <= tol


# The largest grids the 32-bit byte offsets allow (one field just below 4 GiB),
# with the crystal at the far corner so that the work happens at the largest
# offsets; a window at that corner is checked against the oracle on a box that
# shares the two far walls, away from its artificial near walls.
@pytest.mark.parametrize("storage,shape,tol", [("fp16", (1024, 1024, 1023), 1e-3),
                                               ("fp64", (1024, 1024, 384), FP64_TOL)])
def test_maximum_size_far_corner(gpu, oracle_mod, storage, shape, tol):
    import torch
    nx, ny, nz = shape
    k, w = 6, 40
    cfg = W.small_3d(storage=storage, nx=nx, ny=ny, nz=nz, radius=6.0)
    cfg.seeds = [W.Seed(nx - 14, ny - 14, nz - 14, 6.0, 1)]
    _say(_case(cfg, k) + " (largest offsets, far-corner window)")
    sim = gpu.Simulation(cfg)
    sim.step(k)
    phi, u, _ = sim.fields()
    gphi = phi[nz - w:, ny - w:, nx - w:].cpu().numpy()
    gu = u[nz - w:, ny - w:, nx - w:].cpu().numpy()
    del sim, phi, u
    torch.cuda.empty_cache()
    wcfg = cfg.replace(nx=w, ny=w, nz=w, storage="fp64", seeds=[W.Seed(w - 14, w - 14, w - 14, 6.0, 1)])
    orc = _oracle_run(oracle_mod, wcfg, k)
    inner = slice(2 * k, w)
    ephi = np.abs(gphi[inner, inner, inner] - orc.phi()[inner, inner, inner]).max()
    eu = np.abs(gu[inner, inner, inner] - orc.u()[inner, inner, inner]).max()
    _say(f"  corner window max|dphi| = {ephi:.3e}  max|du| = {eu:.3e}")
    assert ephi <= tol and eu <= tol
    assert np.abs(orc.phi()[inner, inner, inner] + 1).max() > 0.5  # the crystal is inside the window


# ---------------------------------------------------------------------------
# Offset storage (FP32 arithmetic, FP32 / FP16 offsets) against the FP64 oracle.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("storage,tol_phi,tol_u", [("fp32", 1e-4, 1e-4), ("fp16", 1e-3, 1e-3)])
def test_c0_offset_storage_accuracy(gpu, oracle_mod, storage, tol_phi, tol_u):
    cfg = W.c0(storage)
    _say(_case(cfg, W.C0_STEPS))
    sim, phi, u, _ = _gpu_run(gpu, cfg, W.C0_STEPS)
    orc = _oracle_run(oracle_mod, cfg, W.C0_STEPS)
    ephi = np.abs(phi - orc.phi()).max()
    eu = np.abs(u - orc.u()).max()
    dg, do = sim.diagnostics()[0], orc.diagnostics()
    etip = abs(dg["tip_position"] - do["tip_position"])
    efs = abs(dg["solid_fraction"] - do["solid_fraction"])
    _say(f"  {storage}: max|dphi| = {ephi:.3e} max|du| = {eu:.3e} |dtip| = {etip:.3e} |dfs| = {efs:.3e}")
    assert ephi <= tol_phi and eu <= tol_u and etip < 0.1


@pytest.mark.parametrize("storage,tol", [("fp32", 1e-4), ("fp16", 1e-3)])
def test_3d_offset_storage_accuracy(gpu, oracle_mod, storage, tol):
    cfg = W.small_3d(storage=storage, n=40, radius=6)
    _say(_case(cfg, 100))
    sim, phi, u, _ = _gpu_run(gpu, cfg, 100)
    orc = _oracle_run(oracle_mod, cfg, 100)
    ephi = np.abs(phi - orc.phi()).max()
    eu = np.abs(u - orc.u()).max()
    _say(f"  {storage}: max|dphi| = {ephi:.3e} max|du| = {eu:.3e}")
    assert ephi <= tol and eu <= tol


# FP16 storage writes the rest offset h_0 as minus the FP32 sum of the other
# offsets after their rounding, so the stored offsets of a node sum to zero up
# to half an FP16 ulp of h_0 (which stays near zero) and the FP32 summation.
# The export decodes g_i = w_i phi + h_i at the node itself, so sum_i g_i - phi
# is that sum of stored offsets.  Rounding every offset by itself instead
# leaves errors of the size of the larger offsets' ulps: with that rule these
# cases exceed the bound at 21-75 % of the nodes, by up to 145x.
@pytest.mark.parametrize("lattice", ["D2Q9_D2Q5", "D3Q19_D3Q7", "D3Q15_D3Q7"])
def test_fp16_offsets_of_a_node_sum_to_zero(gpu, oracle_mod, lattice):
    if lattice == "D2Q9_D2Q5":
        cfg, steps = W.c0("fp16"), 500
    else:
        cfg, steps = W.small_3d(storage="fp16", n=40, radius=6).replace(lattice=lattice), 100
    _say(_case(cfg, steps) + " (offset sums, after init and after the steps)")
    w = oracle_mod.lattice(lattice.split("_")[0])[1]
    q = len(w)
    sim = gpu.Simulation(cfg)
    for k in (0, steps):
        sim.step(k)
        phi = sim.fields()[0].cpu().numpy()
        g = sim.dists()[0].cpu().numpy()
        h = g - w.reshape((-1,) + (1,) * phi.ndim) * phi
        resid = np.abs(g.sum(axis=0) - phi)
        bound = 2.0 ** -11 * np.abs(h[0]) * (1 + 2.0 ** -10) \
            + (q - 1) * 2.0 ** -24 * np.abs(h[1:]).sum(axis=0) + 2.0 ** -25 + 1e-15
        _say(f"  +{k} steps: max|sum h| = {resid.max():.3e}  max|h_0| = {np.abs(h[0]).max():.3e}  "
             f"max|h_i| = {np.abs(h[1:]).max():.3e}  worst resid/bound = {(resid / bound).max():.3f}")
        # after the steps the offsets are not trivially small (the equilibrium
        # offsets at init are smaller, and those of opposite directions cancel)
        assert k == 0 or np.abs(h[1:]).max() > 1e-3
        assert (resid <= bound).all()


# ---------------------------------------------------------------------------
# Launch shape, determinism, checkpoint, batching.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("storage,tiles", [("fp64", [(4, 8), (4, 64), (4, 5), (8, 32), (8, 7)]),
                                           ("fp16", [(12, 32), (4, 7), (8, 64), (12, 5), (12, 9)])])
def test_tile_shapes_bitwise_equal(gpu, storage, tiles):
    cfg = W.small_3d(storage=storage, nx=70, ny=37, nz=29, radius=6)
    outs = []
    for t in tiles:
        _say(_case(cfg, 15) + f" tile={t}")
        _, phi, u, _ = _gpu_run(gpu, cfg, 15, tile=t)
        outs.append((phi, u))
    for phi, u in outs[1:]:
        assert np.array_equal(phi, outs[0][0]) and np.array_equal(u, outs[0][1])


def test_two_runs_bitwise_equal(gpu):
    cfg = W.c1(n=192, count=6, storage="fp16")
    _say(_case(cfg, 100) + " x2")
    a = _gpu_run(gpu, cfg, 100)
    b = _gpu_run(gpu, cfg, 100)
    for x, y in zip(a[1:], b[1:]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("storage", ["fp64", "fp16"])
def test_checkpoint_restart_bitwise(gpu, storage):
    import torch
    cfg = W.c1(n=128, count=3, storage=storage)
    _say(_case(cfg, 50) + " checkpoint")
    sim = gpu.Simulation(cfg)
    sim.step(30)
    ck = sim.save_state()
    sim.step(20)
    assert sim.step_count == 50
    a = [t.cpu().numpy() for t in sim.fields()]
    sim.load_state(ck)
    assert sim.step_count == 30  # the blob carries the step counter
    sim.step(20)
    assert sim.step_count == 50
    b = [t.cpu().numpy() for t in sim.fields()]
    torch.cuda.synchronize()
    straight = _gpu_run(gpu, cfg, 50)[1:]
    for x, y, z in zip(a, b, straight):
        assert np.array_equal(x, y) and np.array_equal(x, z)
    # a fresh handle of the same layout resumes at the saved step
    other = gpu.Simulation(cfg)
    other.load_state(ck)
    assert other.step_count == 30 and other.diagnostics()[0]["step"] == 30
    other.step(20)
    c = [t.cpu().numpy() for t in other.fields()]
    for x, z in zip(c, straight):
        assert np.array_equal(x, z)
    # a blob of another layout is refused and leaves the state alone
    small = gpu.Simulation(W.c1(n=64, count=2, storage=storage))
    before = [t.cpu().numpy() for t in small.fields()]
    with pytest.raises(gpu.LbpfError) as e:
        small.load_state(ck)
    assert e.value.code == -1
    after = [t.cpu().numpy() for t in small.fields()]
    assert small.step_count == 0 and all(np.array_equal(x, y) for x, y in zip(before, after))


# Four-fold strengths above 1/15 make the stiffness a + a'' negative in some
# directions: the sharp-interface problem is ill-posed there and rounding
# differences grow by orders of magnitude within tens of steps (the oracle
# alone, perturbed by 1e-15, moves by 6e-9 in 40 steps at eps = 0.068).
# Element-wise comparisons between two implementations therefore use
# simulations below that limit.
EPS_WELL_POSED = 1.0 / 15.0


def _uneven_ensemble(storage):
    """Five 2D simulations of uneven sizes (ragged 64-wide columns included),
    parameters, boundaries and gradient methods."""
    base = W.c4(count=5, side_hi=5, storage=storage)
    sizes = [(96, 64), (64, 160), (130, 72), (64, 64), (200, 90)]
    out = []
    for k, (cfg, (nx, ny)) in enumerate(zip(base, sizes)):
        seed = W.Seed(nx // 2 + 0.3 * k, ny // 2 - 0.2 * k, 0.0, cfg.seeds[0].radius, 1)
        a = cfg.aniso[0]
        aniso = [W.Aniso("sectoral", eps=min(a.eps, 0.05), q=4, phi0=0.1 * k)]
        out.append(cfg.replace(nx=nx, ny=ny, seeds=[seed], aniso=aniso,
                               boundary="periodic" if k == 1 else "zero_flux",
                               gradient="cd" if k == 2 else "dd"))
    return out


@pytest.mark.parametrize("storage,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_batched_handle_matches_individual_runs(gpu, storage, tol):
    """The persistent batched launch (graph replays of 1 and 8 steps, with
    eager work in between) against one handle per simulation."""
    cfgs = _uneven_ensemble(storage)
    _say(f"batched ensemble of {len(cfgs)} {storage} 2D sims, 3 + 11 steps")
    import torch
    sim = gpu.Simulation(cfgs)
    sim.step(3)
    d3 = sim.diagnostics()
    assert all(x["step"] == 3 for x in d3)
    sim.step(11)
    for k, cfg in enumerate(cfgs):
        phi, u, _ = sim.fields(k)
        _, p1, u1, _ = _gpu_run(gpu, cfg, 14)
        ep = np.abs(phi.cpu().numpy() - p1).max()
        eu = np.abs(u.cpu().numpy() - u1).max()
        _say(f"  sim {k} {cfg.nx}x{cfg.ny}: max|dphi| = {ep:.3e} max|du| = {eu:.3e}")
        assert ep <= tol and eu <= tol
    d = sim.diagnostics()
    assert len(d) == len(cfgs) and all(x["step"] == 14 for x in d)
    torch.cuda.synchronize()


def test_batched_fp64_matches_oracle(gpu, oracle_mod):
    cfgs = _uneven_ensemble("fp64")
    steps = 40
    _say(f"batched fp64 ensemble vs oracle, {steps} steps")
    sim = gpu.Simulation(cfgs)
    sim.step(steps)
    for k, cfg in enumerate(cfgs):
        phi, u, _ = sim.fields(k)
        orc = _oracle_run(oracle_mod, cfg, steps)
        ep = np.abs(phi.cpu().numpy() - orc.phi()).max()
        eu = np.abs(u.cpu().numpy() - orc.u()).max()
        _say(f"  sim {k}: max|dphi| = {ep:.3e} max|du| = {eu:.3e}")
        assert ep <= FP64_TOL and eu <= FP64_TOL


def test_autotune_3d_keeps_results(gpu):
    """The autotuner steps the simulation through every candidate shape and
    keeps a valid one; the state equals, bitwise, an untuned run of the same
    number of steps (every tile shape gives the same result)."""
    cfg = W.small_3d(storage="fp16", nx=70, ny=37, nz=29, radius=6)
    _say(_case(cfg, 0) + " autotune")
    sim = gpu.Simulation(cfg)
    sim.autotune(1)
    ty, ch = sim.get_tile()
    assert ty in (4, 8, 12) and 1 <= ch <= cfg.nz
    n = sim.step_count
    assert n == 3 * 3 * 4  # three times one trial step for 3 heights x 4 chunk lengths
    phi, u, _ = sim.fields()
    _, p1, u1, _ = _gpu_run(gpu, cfg, n)
    assert np.array_equal(phi.cpu().numpy(), p1) and np.array_equal(u.cpu().numpy(), u1)


def test_batched_autotune_and_chunks(gpu):
    cfgs = _uneven_ensemble("fp32")
    _say("batched autotune, then chunk 8 and 128")
    sim = gpu.Simulation(cfgs)
    sim.autotune(2)
    ty, ch = sim.get_tile()
    assert ty == 1 and ch in (8, 16, 32, 64)
    sim.set_tile(1, 8)
    sim.step(5)
    sim.set_tile(1, 128)
    sim.step(4)
    n = sim.step_count
    for k in (0, 4):
        phi, u, _ = sim.fields(k)
        _, p1, u1, _ = _gpu_run(gpu, cfgs[k], n)
        assert np.abs(phi.cpu().numpy() - p1).max() <= 1e-6 and np.abs(u.cpu().numpy() - u1).max() <= 1e-6
    with pytest.raises(gpu.LbpfError):
        sim.set_tile(1, 4)


def test_c4_full_ensemble(gpu, oracle_mod):
    """The full 256-simulation FP32 ensemble: sampled simulations against
    their own single runs and the smallest against the FP64 oracle."""
    cfgs = W.c4()
    steps = 24
    _say(f"C4: {len(cfgs)} sims, {sum(c.nodes for c in cfgs)} nodes, {steps} steps")
    import torch
    sim = gpu.Simulation(cfgs)
    sim.step(steps)
    d = sim.diagnostics()
    assert all(not x["nonfinite"] for x in d)
    ok = [k for k, c in enumerate(cfgs) if c.aniso[0].eps < EPS_WELL_POSED]
    sizes = {k: cfgs[k].nodes for k in ok}
    picks = sorted({max(sizes, key=sizes.get), min(sizes, key=sizes.get), 17, 201} & set(ok))
    for k in picks:
        phi, u, _ = sim.fields(k)
        _, p1, u1, _ = _gpu_run(gpu, cfgs[k], steps)
        ep = np.abs(phi.cpu().numpy() - p1).max()
        eu = np.abs(u.cpu().numpy() - u1).max()
        _say(f"  sim {k} {cfgs[k].nx}x{cfgs[k].ny}: vs single run max|dphi| = {ep:.3e} max|du| = {eu:.3e}")
        assert ep <= 1e-6 and eu <= 1e-6
    k = min(sizes, key=sizes.get)
    phi, u, _ = sim.fields(k)
    orc = _oracle_run(oracle_mod, cfgs[k], steps)
    ep = np.abs(phi.cpu().numpy() - orc.phi()).max()
    eu = np.abs(u.cpu().numpy() - orc.u()).max()
    _say(f"  sim {k} vs oracle: max|dphi| = {ep:.3e} max|du| = {eu:.3e}")
    assert ep <= 1e-4 and eu <= 1e-4
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------
# The isotropy comparison of Sec. 4.2 (six-fold a_s, 800^2).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("grad", ["dd", "cd"])
def test_e2_parity_window(gpu, oracle_mod, grad):
    _compare(gpu, oracle_mod, W.e2(grad), 200)


def test_e2_isotropy_dd_vs_cd(gpu):
    """Full length (1e5 steps): the profiles along n_a = (1, 0) and
    n_b = (1/2, -sqrt(3)/2) differ far less with directional derivatives than
    with central differences (the paper reports 3.04e-3 and 1.71e-1), and so
    does the solution from its own 60-degree rotation: the extremes of
    phi^rot - phi are printed as 1.446 / -1.454 (central differences) and
    0.1 / -0.103 (directional derivatives), Sec. 4.2."""
    import json
    import os

    import bench
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    gold = gold["dd_vs_fd_isotropy_experiment"]
    _say(f"isotropy comparison, DD and CD batched, {W.E2_STEPS} steps")
    r = bench.run_isotropy(W.E2_STEPS, "fp64")
    _say(f"  {r}")
    assert r["err_l2_dd"] < 1e-2
    assert r["cd_over_dd"] >= 10
    fd = max(r["rot60_cd"]["max"], -r["rot60_cd"]["min"])
    dd = max(r["rot60_dd"]["max"], -r["rot60_dd"]["min"])
    fd_paper = max(abs(v) for v in gold["tip_diff_fd"])
    dd_paper = max(abs(v) for v in gold["tip_diff_dd"])
    assert abs(fd - fd_paper) <= 0.1 * fd_paper
    assert 0.5 * dd_paper <= dd <= 2.0 * dd_paper
    assert fd / dd >= 7


# ---------------------------------------------------------------------------
# The 2D/3D cross-check of Sec. 5: a_s = 1 + eps cos 6 phi in 2D (D2Q9, 301^2)
# against Eq. As_Y66 in 3D (D3Q15, 301 x 301 x 4) started from the same
# z-invariant fields.  For z-invariant fields the D3Q15 directional
# derivatives reduce exactly to the D2Q9 ones and D3Q15 projects onto the
# D2Q9 weights; the heat lattices differ (D3Q7 vs D2Q5).  With walls, the
# on-node bounce-back at the two z walls breaks the z-invariance slightly
# (the oracle shows 3e-3 across the 4 planes); a periodic box keeps it.
# ---------------------------------------------------------------------------
def _y66_pair(boundary):
    common = dict(boundary=boundary, gradient="dd", storage="fp64", W0=0.0125, tau0=1.5625e-4, lam=10.0,
                  kappa=0.7, delta=0.3, dx=0.01, dt=1.5e-5,
                  aniso=[W.Aniso("sectoral", eps=0.05, q=6, phi0=0.0)], tip_dir=(1, 0, 0))
    c2 = W.SimConfig(lattice="D2Q9_D2Q5", nx=301, ny=301, nz=1, seeds=[W.Seed(150, 150, 0.0, 6.0, 1)], **common)
    c3 = W.SimConfig(lattice="D3Q15_D3Q7", nx=301, ny=301, nz=4, seeds=[W.Seed(150, 150, 1.5, 6.0, 1)],
                     **common)
    return c2, c3


@pytest.mark.parametrize("boundary", ["zero_flux", "periodic"])
def test_y66_2d_3d_cross_check(gpu, boundary):
    import torch
    c2, c3 = _y66_pair(boundary)
    _say(f"Y66 2D/3D cross-check, {boundary}, 8000 steps")
    s2 = gpu.Simulation(c2)
    s3 = gpu.Simulation(c3)
    phi2, u2, _ = s2.fields()
    s3.import_fields(phi2.expand(4, -1, -1), u2.expand(4, -1, -1))
    for k in range(4):
        s2.step(2000)
        s3.step(2000)
        p2 = s2.fields()[0]
        p3 = s3.fields()[0]
        t2 = s2.diagnostics()[0]["tip_position"]
        t3 = s3.diagnostics()[0]["tip_position"]
        zdev = float((p3 - p3[0:1]).abs().max())
        dphi = float((p3[1] - p2).abs().max())
        _say(f"  step {2000 * (k + 1)}: tip 2D {t2:.4f} 3D {t3:.4f}  max|dphi| {dphi:.3e}  z-deviation {zdev:.1e}")
        assert abs(t3 - t2) < 0.1 and dphi < 0.1
        if boundary == "periodic":
            assert zdev <= 1e-12
    assert t2 > 25.0  # the six-fold crystal really grew
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------
# Properties that hold at any size.
# ---------------------------------------------------------------------------
def _ray_radius(phi, c, d):
    """Largest linearly interpolated phi = 0 crossing along the lattice ray
    c + k d (lattice units; numpy axes z, y, x)."""
    step = math.sqrt(sum(v * v for v in d))
    best, k = -1.0, 0
    while True:
        a = [c + k * v for v in d]
        b = [c + (k + 1) * v for v in d]
        if any(not 0 <= v < phi.shape[2 - j] for j, v in enumerate(b)):
            return best
        pa, pb = phi[a[2], a[1], a[0]], phi[b[2], b[1], b[0]]
        if pa > 0 >= pb:
            best = (k + pa / (pa - pb)) * step
        k += 1


@pytest.mark.parametrize("dendrite,family,count", [("A", 1, 6), ("B", 2, 12), ("C", 3, 8)])
def test_paper_dendrite_tip_families(gpu, dendrite, family, count):
    """Sec. 5: dendrite A (Eq. As_Function_Classical) grows six <100> tips, B
    (Eq. As_MatSci, eps = 0, gamma = -0.02) twelve <110> tips, C (Eq.
    As_Function_S) eight <111> tips.  Lattice rays by the number of nonzero
    components (1: <100>, 2: <110>, 3: <111>); after 2000 steps on a 161^3 box
    the preferred family reaches farther than every other ray by 10 %."""
    import itertools
    n = 161
    cfg = W.paper3d(dendrite, "fp64", n=n)
    _say(f"paper dendrite {dendrite} {n}^3 fp64, 2000 steps")
    sim = gpu.Simulation(cfg)
    sim.step(2000)
    phi = sim.fields()[0].cpu().numpy()
    radii = {1: [], 2: [], 3: []}
    for d in itertools.product((-1, 0, 1), repeat=3):
        if any(d):
            radii[sum(map(abs, d))].append(_ray_radius(phi, n // 2, d))
    _say(f"  radii by family: {({k: (round(min(v), 2), round(max(v), 2)) for k, v in radii.items()})}")
    others = [r for k, v in radii.items() if k != family for r in v]
    assert len(radii[family]) == count
    assert min(radii[family]) > 1.1 * max(others)


@pytest.mark.parametrize("storage,tol", [("fp64", 1e-12), ("fp32", 1e-6)])
def test_conservation_periodic(gpu, storage, tol):
    cfg = W.c0(storage=storage, n=96)
    _say(_case(cfg, 400) + " conservation")
    sim = gpu.Simulation(cfg)
    c0 = sim.diagnostics()[0]["sum_u_minus_half_phi"]
    sim.step(400)
    d = sim.diagnostics()[0]
    assert abs(d["sum_u_minus_half_phi"] - c0) <= tol * cfg.nodes * 400


def test_import_gaussian_diffusion(gpu, oracle_mod):
    import torch
    cfg = W.small_3d(n=32, boundary="periodic").replace(seeds=[])
    _say(_case(cfg, 12) + " gaussian import")
    z, y, x = np.meshgrid(*[np.arange(32) - 16] * 3, indexing="ij")
    r2 = (x**2 + y**2 + z**2).astype(float)
    bump = np.exp(-r2 / 32.0)
    bump[r2 > 15**2 - 1] = 0.0
    sim = gpu.Simulation(cfg)
    sim.import_fields(-np.ones((32, 32, 32)), bump)
    sim.step(12)
    _, u, _ = sim.fields()
    orc = oracle_mod.OracleSim(cfg)
    orc.set_fields(-np.ones((32, 32, 32)), bump)
    orc.step(12)
    assert np.abs(u.cpu().numpy() - orc.u()).max() < 1e-13
    torch.cuda.synchronize()


def test_nonfinite_is_reported(gpu):
    import paper_1606_09432_amd as lb
    cfg = W.c0(n=32)
    _say("non-finite import")
    sim = gpu.Simulation(cfg)
    phi = np.full((32, 32), -1.0)
    phi[3, 4] = np.nan
    sim.import_fields(phi, np.zeros((32, 32)))
    with pytest.raises(lb.LbpfError) as ei:
        sim.diagnostics()
    assert ei.value.code == -5
    assert sim.diagnostics(allow_nonfinite=True)[0]["nonfinite"] == 1


def test_rotation_invariance_gpu(gpu):
    """90 degree rotation about the seed centre (exact for the method, to
    rounding on the GPU where fused multiply-adds break bitwise symmetry)."""
    cfg = W.c0(n=96, storage="fp64").replace(aniso=[W.Aniso("sectoral", 0.05, 4, math.radians(20))])
    _say(_case(cfg, 500) + " rotation")
    _, phi, u, _ = _gpu_run(gpu, cfg, 500)
    c = 48
    y, x = np.meshgrid(np.arange(96), np.arange(96), indexing="ij")
    assert np.abs(phi[x, (2 * c - y) % 96] - phi).max() < 1e-12

"""GPU parity of boxes with mirror planes through node 0 (one octant, or one
quadrant in 2D, of a mirror-symmetric domain; the paper's dendrite grown from
a seed at the origin, Sec. 5), through the C ABI against the CPU FP64 oracle,
and against the GPU's own run of the whole symmetric domain."""
import numpy as np
import pytest

from paper_1606_09432_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _fields(sim, k=0):
    import torch
    phi, u, ids = sim.fields(k)
    torch.cuda.synchronize()
    return phi.cpu().numpy(), u.cpu().numpy(), ids.cpu().numpy()


def _mirror_2d(nx, ny, grad="dd", ids=False, storage="fp64"):
    """Quadrant with a seed on the corner node and one off the planes."""
    entry = W.Aniso("sectoral", eps=0.05, q=4, phi0=0.0)
    seeds = [W.Seed(0, 0, 0, min(nx, ny) * 0.2 + 1, 1), W.Seed(nx * 0.6, ny * 0.4, 0, 3.0, 2 if ids else 1)]
    aniso = [W.Aniso("iso"), entry, W.Aniso("sectoral", eps=0.04, q=4, phi0=0.0)] if ids else [entry]
    return W.SimConfig(lattice="D2Q9_D2Q5", nx=nx, ny=ny, nz=1, boundary="mirror_low", gradient=grad,
                       storage=storage, delta=0.55, kappa=W.KAPPA_C0, aniso=aniso, seeds=seeds,
                       use_ids=ids, tip_dir=(1, 0, 0))


def _mirror_3d(shape, lattice="D3Q19_D3Q7", grad="dd", entry=None, storage="fp64"):
    nx, ny, nz = shape
    return W.small_3d(nx=nx, ny=ny, nz=nz, aniso=entry or W.Aniso("cubic", eps=0.05), boundary="mirror_low",
                      radius=min(shape) * 0.3 + 1, storage=storage).replace(
        lattice=lattice, gradient=grad,
        seeds=[W.Seed(0, 0, 0, min(shape) * 0.3 + 1, 1), W.Seed(nx * 0.55, ny * 0.5, nz * 0.45, 2.5, 1)])


def _compare(lb, O, cfg, steps, tol=FP64_TOL, tile=None):
    _say(f"{cfg.lattice} {cfg.nx}x{cfg.ny}x{cfg.nz} mirror_low {cfg.gradient} {cfg.storage} "
         f"ids={cfg.use_ids} steps={steps} tile={tile}")
    sim = lb.Simulation(cfg)
    if tile:
        sim.set_tile(*tile)
    sim.step(steps)
    phi, u, ids = _fields(sim)
    orc = O.OracleSim(cfg.replace(storage="fp64"))
    orc.step(steps)
    dphi = np.abs(phi - orc.phi())
    ephi, eu = dphi.max(), np.abs(u - orc.u()).max()
    _say(f"  max|dphi| = {ephi:.3e} at {np.unravel_index(dphi.argmax(), phi.shape)}  max|du| = {eu:.3e}")
    assert ephi <= tol and eu <= tol, (ephi, eu)
    if cfg.use_ids:
        assert np.array_equal(ids, orc.ids())
    # the crystal on the corner has grown: the planes carry an interface
    assert phi.reshape(-1)[0] > 0.5
    return sim, orc


@pytest.mark.parametrize("nx,ny,grad,ids", [(70, 45, "dd", False), (130, 67, "cd", True), (64, 64, "dd", True),
                                            (3, 3, "dd", False)])
def test_mirror_2d_fp64_parity(gpu, oracle_mod, nx, ny, grad, ids):
    _compare(gpu, oracle_mod, _mirror_2d(nx, ny, grad, ids), 300 if nx > 3 else 20)


@pytest.mark.parametrize("lattice,grad,shape,entry,steps", [
    ("D3Q19_D3Q7", "dd", (66, 20, 18), W.Aniso("cubic", eps=0.05), 60),
    ("D3Q19_D3Q7", "cd", (40, 36, 33), W.Aniso("cubic_hak", eps=0.0, gamma=-0.02), 60),
    ("D3Q15_D3Q7", "dd", (40, 36, 33), W.Aniso("cubic_hak", eps=0.0, gamma=-0.02), 60),
    ("D3Q15_D3Q7", "dd", (70, 22, 20), W.Aniso("cubic_s", gamma=0.02), 50),
    ("D3Q19_D3Q7", "dd", (3, 3, 3), W.Aniso("cubic", eps=0.05), 10),
])
def test_mirror_3d_fp64_parity(gpu, oracle_mod, lattice, grad, shape, entry, steps):
    _compare(gpu, oracle_mod, _mirror_3d(shape, lattice, grad, entry), steps)


@pytest.mark.parametrize("shape", [(48, 44, 40), (70, 30, 26)])
def test_mirror_3d_crystal_index_parity(gpu, oracle_mod, shape):
    # every entry symmetric about the planes (the library refuses others); the
    # second box has tiles beyond the planes' reach (run by the plain instance)
    cfg = W.multi_3d(boundary="mirror_low", y66_phi0=0.0, shape=shape)
    cfg = cfg.replace(seeds=[W.Seed(0, 0, 0, 5.0, 1)] + cfg.seeds[1:])
    _compare(gpu, oracle_mod, cfg, 60)


@pytest.mark.parametrize("lattice", ["D2Q9_D2Q5", "D3Q19_D3Q7", "D3Q15_D3Q7"])
def test_mirror_distributions_parity(gpu, oracle_mod, lattice):
    cfg = _mirror_2d(72, 40) if lattice == "D2Q9_D2Q5" else _mirror_3d((40, 20, 18), lattice)
    _say(f"distributions {lattice} mirror_low, 30 steps")
    sim = gpu.Simulation(cfg)
    sim.step(30)
    g, f = sim.dists()
    orc = oracle_mod.OracleSim(cfg)
    orc.step(30)
    dg = np.abs(g.cpu().numpy() - orc.g())
    df = np.abs(f.cpu().numpy() - orc.f())
    _say(f"  max|dg| = {dg.max():.3e} at {np.unravel_index(dg.argmax(), dg.shape)}  max|df| = {df.max():.3e}")
    assert dg.max() < 1e-12 and df.max() < 1e-12


@pytest.mark.parametrize("storage,tol", [("fp32", 1e-4), ("fp16", 1e-3)])
def test_mirror_offset_storage_accuracy(gpu, oracle_mod, storage, tol):
    _compare(gpu, oracle_mod, _mirror_3d((66, 36, 33), storage=storage), 80, tol=tol)
    _compare(gpu, oracle_mod, _mirror_2d(130, 67, storage=storage), 300, tol=tol)


# (4, 3) and (8, 3): chunks too short to leave chunk 1 beyond the planes' reach,
# so every tile runs with the mirror instance; the others split the tiles
# between the two instances
@pytest.mark.parametrize("storage,tiles", [("fp64", [(4, 8), (4, 64), (4, 3)]),
                                           ("fp16", [(12, 32), (4, 7), (8, 64), (12, 5), (8, 3)])])
def test_mirror_tile_shapes_bitwise_equal(gpu, storage, tiles):
    cfg = _mirror_3d((70, 50, 45), storage=storage)
    _say(f"mirror tiles {storage} {tiles}")
    ref = gpu.Simulation(cfg)
    ref.step(40)
    p0, u0, _ = _fields(ref)
    for t in tiles:
        s = gpu.Simulation(cfg)
        s.set_tile(*t)
        s.step(40)
        p, u, _ = _fields(s)
        assert np.array_equal(p, p0) and np.array_equal(u, u0), t


@pytest.mark.parametrize("lattice,n,storage,tol", [("D3Q19_D3Q7", 65, "fp64", 1e-11),
                                                   ("D3Q15_D3Q7", 65, "fp64", 1e-11),
                                                   ("D2Q9_D2Q5", 257, "fp64", 1e-11),
                                                   ("D3Q19_D3Q7", 97, "fp16", 1e-3)])
def test_mirror_octant_equals_whole_domain(gpu, lattice, n, storage, tol):
    """The mirror box of n nodes per axis against the whole mirror-symmetric
    zero-flux domain of 2n - 1 nodes centred on node n - 1, both on the GPU."""
    dim = 2 if lattice == "D2Q9_D2Q5" else 3
    N, c = 2 * n - 1, n - 1
    entry = W.Aniso("cubic", eps=0.05) if dim == 3 else W.Aniso("sectoral", eps=0.05, q=4, phi0=0.0)
    full = W.SimConfig(lattice=lattice, nx=N, ny=N, nz=N if dim == 3 else 1, boundary="zero_flux",
                       gradient="dd", storage=storage, delta=0.55, kappa=W.KAPPA_C0, aniso=[entry],
                       seeds=[W.Seed(c, c, c if dim == 3 else 0, 8.0, 1)], tip_dir=(1, 0, 0))
    octant = full.replace(nx=n, ny=n, nz=n if dim == 3 else 1, boundary="mirror_low",
                          seeds=[W.Seed(0, 0, 0, 8.0, 1)])
    steps = 400
    _say(f"octant {lattice} {storage} n={n} vs whole {N}, {steps} steps")
    a = gpu.Simulation(full)
    b = gpu.Simulation(octant)
    a.step(steps)
    b.step(steps)
    pa, ua, _ = _fields(a)
    pb, ub, _ = _fields(b)
    part = (slice(c, None),) * dim
    ep, eu = np.abs(pb - pa[part]).max(), np.abs(ub - ua[part]).max()
    _say(f"  max|dphi| = {ep:.3e}  max|du| = {eu:.3e}")
    assert ep <= tol and eu <= tol
    # the tip is measured from seed 0's centre in both boxes
    da, db = a.diagnostics()[0], b.diagnostics()[0]
    _say(f"  tip {da['tip_position']:.6f} / {db['tip_position']:.6f}")
    assert abs(da["tip_position"] - db["tip_position"]) < (1e-8 if storage == "fp64" else 1e-3)
    del a, b


def test_mirror_batched_matches_oracle(gpu, oracle_mod):
    """A batched ensemble mixing mirror, zero-flux and periodic boxes."""
    cfgs = [_mirror_2d(96, 64), W.c0(n=64).replace(boundary="zero_flux"), _mirror_2d(130, 72, grad="cd"),
            W.c0(n=80)]
    steps = 40
    _say(f"batched fp64 ensemble with mirror boxes vs oracle, {steps} steps")
    sim = gpu.Simulation(cfgs)
    sim.step(steps)
    for k, cfg in enumerate(cfgs):
        phi, u, _ = _fields(sim, k)
        orc = oracle_mod.OracleSim(cfg)
        orc.step(steps)
        ep = np.abs(phi - orc.phi()).max()
        eu = np.abs(u - orc.u()).max()
        _say(f"  sim {k} {cfg.boundary}: max|dphi| = {ep:.3e} max|du| = {eu:.3e}")
        assert ep <= FP64_TOL and eu <= FP64_TOL

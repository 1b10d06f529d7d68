"""Benchmark of the coupled LB phase-field step on one MI355X.

Workload: D3Q19 (phi) + D3Q7 (u), 512^3 nodes, zero-flux walls, one central
seed of radius 8, the Hoyt-Asta-Karma anisotropy (Eq. As_MatSci) with
(eps1, eps2) = (0.1, 0), undercooling 0.6.  A step is one pass of the whole
hot path (gradient, a_s / N, the nonlocal phase-field LBE, bounce-back, the
heat LBE) over the full grid, one fused kernel launch.

The JSON line reports the FP16-offset storage form (FP32 arithmetic) as the
headline `value` and the plain FP64 form beside it, both in MLUPS (million
node updates per second), each with its HBM roofline; plus the CPU FP64
oracle timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import sqlite3
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "coupled φ+u MLUPS & %HBM roofline, D3Q19 512³, FP64 vs FP16-offset storage"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per node-step: every distribution read once and written
# once; offset forms also read and write the FP32 phi and u* fields.
B_ALG = {("D3Q19_D3Q7", "fp64"): 416, ("D3Q19_D3Q7", "fp32"): 224, ("D3Q19_D3Q7", "fp16"): 120,
         ("D3Q15_D3Q7", "fp64"): 352, ("D3Q15_D3Q7", "fp32"): 192, ("D3Q15_D3Q7", "fp16"): 104,
         ("D2Q9_D2Q5", "fp64"): 224, ("D2Q9_D2Q5", "fp32"): 128, ("D2Q9_D2Q5", "fp16"): 72}
KERNEL_SOURCES = ["paper_1606_09432_amd/csrc/lbpf_step_kernel.hpp", "paper_1606_09432_amd/csrc/lbpf_common.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def kernel_sha() -> str:
    """Hash of the kernel sources without comments and blank lines, so that a
    change of wording leaves the recorded counters valid."""
    import re

    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        text = open(os.path.join(ROOT, p)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update("\n".join(l.rstrip() for l in text.splitlines() if l.strip()).encode())
    return h.hexdigest()[:16]


def traffic_key(lattice: str, storage: str) -> str:
    return storage if lattice == "D3Q19_D3Q7" else f"{lattice.split('_')[0].lower()}_{storage}"


BATCHED_KEY = "c4_ensemble_fp32"


def measured_traffic(lattice: str, storage: str, key: str = None):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    ent = d.get("kernels", {}).get(key or traffic_key(lattice, storage))
    if not ent or ent.get("kernel_sha") != kernel_sha():
        return None
    return ent.get("bytes_per_launch")


def time_stream_copy(sim, reps: int = 5):
    """The plain streaming copy of the simulation's current state block into
    its other block (the step's own buffers): every state byte read once and
    written once, as the step must.  Returns (ms per copy, bytes moved)."""
    import torch

    import paper_1606_09432_amd as lb

    src, nbytes = sim.state_block()
    other = src + nbytes if src + nbytes + nbytes <= sim.workspace.data_ptr() + sim.workspace.numel() else None
    if other is None:
        return None, 0
    stream = torch.cuda.current_stream()
    # one work-group of 256 threads per compute unit: the fastest of 1..32 per
    # CU in a sweep on an 8 GiB copy (5.44 TB/s; 4.87 at 8 per CU)
    lb.stream_copy(src, other, nbytes, 1)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        lb.stream_copy(src, other, nbytes, 1)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, 2 * nbytes


def run_gpu(cfg, steps: int, warmup: int, autotune: bool, copy_ceiling: bool = False, pre_steps: int = 0):
    import torch

    import paper_1606_09432_amd as lb

    print(f"[bench] {cfg.storage}: init {cfg.nx}x{cfg.ny}x{cfg.nz} ({len(cfg.seeds)} seeds)", file=sys.stderr,
          flush=True)
    sim = lb.Simulation(cfg)
    if pre_steps:
        sim.step(pre_steps)
    if autotune:
        sim.autotune(2)
    stream = torch.cuda.current_stream()
    sim.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    diag = sim.diagnostics()[0]
    tile = sim.get_tile()
    aniso_frac = anisotropic_fraction(sim) if cfg.nodes <= 512 ** 3 else None
    copy = None
    if copy_ceiling:
        # the step's parity is even after an even number of steps: the state
        # block read next is the first, and the copy writes the second
        if sim.step_count % 2:
            sim.step(1)
        cms, cbytes = time_stream_copy(sim)
        if cms:
            copy = {"ms": cms, "bytes": cbytes, "GBps": cbytes / (cms * 1e-3) / 1e9,
                    "kind": "lb_pf_stream_copy of the state block into the other block (one work-group of 256 per CU, 16-byte nontemporal "
                            "vectors), read + written bytes"}
            print(f"[bench] {cfg.storage}: state-block copy {cbytes / 1e9:.2f} GB in {cms:.3f} ms, "
                  f"{copy['GBps']:.0f} GB/s", file=sys.stderr, flush=True)
    del sim
    torch.cuda.empty_cache()
    nodes = cfg.nodes
    mlups = nodes * steps / (ms * 1e-3) / 1e6
    b_alg = B_ALG[(cfg.lattice, cfg.storage)]
    achieved = b_alg * nodes / (ms / steps * 1e-3) / 1e9
    traffic = measured_traffic(cfg.lattice, cfg.storage)
    print(f"[bench] {cfg.storage}: {ms / steps:.3f} ms/step  {mlups:.1f} MLUPS  {achieved:.0f} GB/s "
          f"tile={tile} tip={diag['tip_position']:.3f}", file=sys.stderr, flush=True)
    return {
        "value": mlups, "ms_per_step": ms / steps, "tile": list(tile),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_node_step": b_alg},
        "diag": {"tip_position": diag["tip_position"], "solid_fraction": diag["solid_fraction"],
                 "nonfinite": diag["nonfinite"]},
        "copy": copy, "anisotropic_fraction": aniso_frac,
    }


def anisotropic_fraction(sim) -> float:
    """Share of nodes whose phi gradient exceeds the isotropic cutoff
    |p| > 1e-8 (lattice units), i.e. that evaluate a_s and N in the step.  The
    gradient is taken here by central differences of the exported phi (a
    measurement of the state, not the step's own gradient)."""
    import torch

    phi = sim.fields()[0]
    if phi.dim() == 2:
        phi = phi.unsqueeze(0)
    p2 = torch.zeros(phi.shape[1:], dtype=torch.float64, device=phi.device)
    count = 0
    for k in range(phi.shape[0]):  # one plane at a time keeps the memory small
        zl, zh = max(k - 1, 0), min(k + 1, phi.shape[0] - 1)
        p2.zero_()
        if phi.shape[0] > 1:
            p2 += ((phi[zh] - phi[zl]) / max(zh - zl, 1)) ** 2
        gy, gx = torch.gradient(phi[k])
        p2 += gx * gx + gy * gy
        count += int((p2 > 1e-16).sum())
    del phi
    return count / sim.nodes()


def run_batched(steps: int, warmup: int):
    """The batched ensemble of 256 uneven 2D FP32-offset simulations, one
    persistent graph-replayed launch per step."""
    import torch

    import paper_1606_09432_amd as lb
    from paper_1606_09432_amd import workloads as W

    cfgs = W.c4()
    nodes = sum(c.nodes for c in cfgs)
    print(f"[bench] batched: init {len(cfgs)} sims, {nodes} nodes", file=sys.stderr, flush=True)
    sim = lb.Simulation(cfgs)
    stream = torch.cuda.current_stream()
    # the ensemble's rows per work item come from the autotuner (8 to 64 rows,
    # 4 timed steps each), outside the timed region
    sim.autotune(4)
    sim.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    tile = sim.get_tile()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    b_alg = B_ALG[("D2Q9_D2Q5", "fp32")]
    achieved = b_alg * nodes / (ms / steps * 1e-3) / 1e9
    print(f"[bench] batched: {ms / steps:.3f} ms/step  {nodes * steps / (ms * 1e-3) / 1e6:.1f} MLUPS "
          f"chunk={tile[1]}",
          file=sys.stderr, flush=True)
    return {"workload": f"{len(cfgs)} independent 2D D2Q9/D2Q5 simulations, sides 32*U{{2..16}}, "
                        "FP32-offset storage, one persistent launch per step",
            "nodes": nodes, "value": nodes * steps / (ms * 1e-3) / 1e6, "unit": "MLUPS",
            "ms_per_step": ms / steps, "dtype": "f32", "chunk": tile[1], "chunk_from": "lb_pf_autotune",
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS,
                         "traffic": measured_traffic("D2Q9_D2Q5", "fp32", BATCHED_KEY),
                         "bytes_per_node_step": b_alg}}


def run_c1_throughput(steps: int, grow: int = 1000):
    """The twenty-crystal 2048^2 workload (its own four-fold orientation per
    crystal in the index field), directional derivatives and central
    differences advancing together as one batched pair, in FP64 and in
    FP32-offset storage: MLUPS over `steps` steps after `grow` steps of growth
    (rows per work item from the autotuner)."""
    import torch

    import paper_1606_09432_amd as lb
    from paper_1606_09432_amd import workloads as W

    out = {"workload": "2048^2 D2Q9/D2Q5, 20 crystals with their own orientation (index field, 21 entries), "
                       "DD and CD as one batched pair", "steps": steps, "after_steps": grow}
    for st in ("fp64", "fp32"):
        cfgs = [W.c1(st, g) for g in ("dd", "cd")]
        nodes = sum(c.nodes for c in cfgs)
        sim = lb.Simulation(cfgs)
        sim.autotune(4)
        sim.step(grow)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        stream = torch.cuda.current_stream()
        e0.record(stream)
        sim.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        tile = sim.get_tile()
        sim.close()
        del sim
        torch.cuda.empty_cache()
        out[st] = {"value": nodes / (ms * 1e-3) / 1e6, "unit": "MLUPS", "ms_per_step": ms, "chunk": tile[1]}
        print(f"[bench] c1 {st}: {ms:.3f} ms/step  {out[st]['value']:.1f} MLUPS chunk={tile[1]}", file=sys.stderr,
              flush=True)
    return out


def run_accuracy(workload: str, n: int, steps: int, every: int, variant: str):
    """Error of the FP32- and FP16-offset forms against the FP64 form (itself
    checked against the FP64 oracle) over a run: max |d phi|, max |d u|,
    |d solid fraction| and |d tip| every `every` steps, one JSON line each."""
    import torch

    import paper_1606_09432_amd as lb
    from paper_1606_09432_amd import workloads as W

    make = (lambda st: W.c2(st, n=n)) if workload == "c2" else (lambda st: W.c3(st, variant, n=n))
    sims = {st: lb.Simulation(make(st)) for st in ("fp64", "fp32", "fp16")}
    done = 0
    while True:
        ref_phi, ref_u, _ = sims["fp64"].fields()
        ref_d = sims["fp64"].diagnostics()[0]
        row = {"workload": workload, "n": n, "step": done, "tip_fp64": ref_d["tip_position"],
               "solid_fraction_fp64": ref_d["solid_fraction"]}
        for st in ("fp32", "fp16"):
            phi, u, _ = sims[st].fields()
            d = sims[st].diagnostics()[0]
            row[st] = {"max_dphi": float((phi - ref_phi).abs().max()), "max_du": float((u - ref_u).abs().max()),
                       "d_solid_fraction": abs(d["solid_fraction"] - ref_d["solid_fraction"]),
                       "d_tip": abs(d["tip_position"] - ref_d["tip_position"])}
            del phi, u
        del ref_phi, ref_u
        print(json.dumps(row), flush=True)
        if done >= steps:
            break
        k = min(every, steps - done)
        for sim in sims.values():
            sim.step(k)
        torch.cuda.synchronize()
        done += k


def profile_l2_error(phi, centre, n_a=(1.0, 0.0), n_b=(0.5, -math.sqrt(3.0) / 2.0), length=None) -> float:
    """Relative l2 difference of two phi profiles sampled from `centre` along
    the unit directions n_a and n_b at unit spacing (Eq. Error_L2), phi_a the
    reference.  Off-lattice points use cubic convolution (Keys, a = -1/2),
    whose error on a resolved tanh front is far below the bilinear one.
    phi is [y][x]."""
    import numpy as np

    ny, nx = phi.shape
    cx, cy = centre
    if length is None:
        length = int(min(nx - 3 - cx, cx - 2, ny - 3 - cy, cy - 2))

    def w(t):  # Keys cubic convolution weights for offsets -1, 0, 1, 2
        t2, t3 = t * t, t * t * t
        return [(-t3 + 2 * t2 - t) / 2, (3 * t3 - 5 * t2 + 2) / 2, (-3 * t3 + 4 * t2 + t) / 2, (t3 - t2) / 2]

    def sample(d):
        j = np.arange(length + 1, dtype=np.float64)
        x = cx + j * d[0]
        y = cy + j * d[1]
        x0 = np.floor(x).astype(int)
        y0 = np.floor(y).astype(int)
        wx, wy = w(x - x0), w(y - y0)
        out = np.zeros_like(x)
        for a in range(4):
            for b in range(4):
                out += wy[a] * wx[b] * phi[y0 + a - 1, x0 + b - 1]
        return out

    pa, pb = sample(n_a), sample(n_b)
    return float(np.sqrt(np.sum((pa - pb) ** 2) / np.sum(pa ** 2)))


def _cubic_sample(phi, x, y):
    """phi (indexed [y][x]) at the points (x, y) by cubic convolution (Keys, a = -1/2)."""
    import numpy as np

    x0 = np.floor(x).astype(int)
    y0 = np.floor(y).astype(int)

    def w(t):
        t2, t3 = t * t, t * t * t
        return [(-t3 + 2 * t2 - t) / 2, (3 * t3 - 5 * t2 + 2) / 2, (-3 * t3 + 4 * t2 + t) / 2, (t3 - t2) / 2]

    wx, wy = w(x - x0), w(y - y0)
    out = np.zeros_like(x, dtype=np.float64)
    for a in range(4):
        for b in range(4):
            out += wy[a] * wx[b] * phi[y0 + a - 1, x0 + b - 1]
    return out


def rotation_difference(phi, centre, degrees=60.0, margin=3):
    """phi^rot - phi over the box (Sec. 4.2, Fig. Differences-Fields): phi^rot
    is phi turned by `degrees` about `centre`, phi^rot(x) = phi(c + R(-theta)
    (x - c)), sampled by cubic convolution.  Nodes whose rotated point leaves
    the box (less `margin`) are skipped.  Returns (max, min, x of the max,
    x of the min); phi is [y][x]."""
    import numpy as np

    ny, nx = phi.shape
    cx, cy = centre
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    t = math.radians(degrees)
    xs = cx + math.cos(t) * (x - cx) + math.sin(t) * (y - cy)
    ys = cy - math.sin(t) * (x - cx) + math.cos(t) * (y - cy)
    ok = (xs >= margin) & (xs <= nx - 1 - margin) & (ys >= margin) & (ys <= ny - 1 - margin)
    d = np.full(phi.shape, np.nan)
    d[ok] = _cubic_sample(phi, xs[ok], ys[ok]) - phi[ok]
    imax, imin = np.nanargmax(d), np.nanargmin(d)
    at = lambda i: (int(i % nx), int(i // nx))
    return float(np.nanmax(d)), float(np.nanmin(d)), at(imax), at(imin)


def tip_radius(phi, cx, cy, theta, rmax=40.0, dr=0.125):
    """Distance from (cx, cy) to the phi = 0 crossing along the ray of angle
    theta (the first sign change from solid to liquid, linearly interpolated)."""
    import numpy as np

    r = np.arange(0.0, rmax, dr)
    v = _cubic_sample(phi, cx + r * math.cos(theta), cy + r * math.sin(theta))
    k = np.nonzero((v[:-1] > 0) & (v[1:] <= 0))[0]
    if len(k) == 0:
        return float("nan")
    i = int(k[0])
    return float(r[i] + dr * v[i] / (v[i] - v[i + 1]))


def run_orientation_spread(storage: str, n_orient: int = 10, side: int = 400, stop_radius: float = 80.0,
                           max_steps: int = 40000):
    """Orientation dependence of the growth with directional derivatives and with
    central differences.  One batched ensemble holds, for each gradient method,
    n_orient independent simulations of the twenty-crystal workload's physics
    (four-fold a_s, eps = 0.05, Delta = 0.5, zero-flux side^2 boxes with a
    centred seed of radius 5) whose crystal orientation theta0 runs over
    [0, pi/4].  When the largest tip is stop_radius from the centre, the tip
    radius along theta0 is compared across orientations: with an isotropic
    discretisation it would not depend on theta0."""
    import numpy as np

    import paper_1606_09432_amd as lb
    from paper_1606_09432_amd import workloads as W

    thetas = [k * (math.pi / 4) / (n_orient - 1) for k in range(n_orient)]
    c = side / 2.0
    cfgs = []
    for grad in ("dd", "cd"):
        for t in thetas:
            cfgs.append(W.SimConfig(lattice="D2Q9_D2Q5", nx=side, ny=side, nz=1, boundary="zero_flux",
                                    gradient=grad, storage=storage, delta=0.5, kappa=W.KAPPA_C0,
                                    aniso=[W.Aniso("sectoral", eps=0.05, q=4, phi0=t)],
                                    seeds=[W.Seed(c, c, 0.0, 5.0, 1)], tip_dir=(1, 0, 0)))
    sim = lb.Simulation(cfgs)
    done = 0
    radii = None
    while done < max_steps:
        sim.step(500)
        done += 500
        radii = [tip_radius(sim.fields(k)[0].cpu().numpy(), c, c, thetas[k % n_orient], rmax=side / 2 - 4)
                 for k in range(len(cfgs))]
        print(f"[orientation] step {done}: largest tip radius {max(radii):.2f}", file=sys.stderr, flush=True)
        if max(radii) >= stop_radius:
            break
    sim.close()
    out = {"workload": f"{n_orient} orientations x (DD, CD), {side}^2 each, four-fold a_s eps 0.05, Delta 0.5",
           "steps": done, "storage": storage, "theta0": [round(t, 4) for t in thetas]}
    for j, name in enumerate(("dd", "cd")):
        r = np.array(radii[j * n_orient:(j + 1) * n_orient])
        out[f"tip_radius_{name}"] = [round(float(v), 3) for v in r]
        out[f"cv_{name}"] = float(r.std() / r.mean())
        out[f"spread_{name}"] = float(r.max() - r.min())
    out["cv_cd_over_dd"] = out["cv_cd"] / out["cv_dd"]
    return out


def run_c1(steps: int, every: int):
    """The twenty-crystal 2048^2 workload as stated: each crystal has its own
    four-fold orientation theta0_k in the index field (Sec. 4.3), run with
    directional derivatives and with central differences, in FP64 and in FP32
    offset storage.  Every `every` steps: the mean tip radius R_k of each
    crystal along theta0_k + m pi/2 (m = 0..3), the coefficient of variation
    of R_k across the crystals that touch no other yet (Sec. 4.2: an isotropic
    discretisation grows every orientation alike), and the FP32-vs-FP64
    differences.  One JSON line per report."""
    import numpy as np
    import torch

    import paper_1606_09432_amd as lb
    from paper_1606_09432_amd import workloads as W

    grads = ("dd", "cd")
    sims = {st: lb.Simulation([W.c1(st, g) for g in grads]) for st in ("fp64", "fp32")}
    cfg = W.c1("fp64", "dd")
    centres = np.array([(s.x, s.y) for s in cfg.seeds])
    theta = np.array([cfg.aniso[s.id].phi0 for s in cfg.seeds])
    width = math.sqrt(2.0) * cfg.W0 / cfg.dx
    dist = np.linalg.norm(centres[:, None, :] - centres[None, :, :], axis=-1) + np.eye(len(centres)) * 1e9
    done = 0
    while True:
        row = {"workload": "C1 2048^2, 20 crystals", "step": done}
        if done == 0:
            row["theta0"] = [round(float(t), 4) for t in theta]
            row["nearest"] = [round(float(d), 1) for d in dist.min(axis=1)]
        phis = {}
        for st, sim in sims.items():
            for k, g in enumerate(grads):
                phis[(st, g)] = sim.fields(k)[0].cpu().numpy()
        torch.cuda.synchronize()
        radii = {}
        for (st, g), phi in phis.items():
            ny_, nx_ = phi.shape
            # distance to the box edge, less the reach of the cubic ray stencil
            edge = np.array([min(c[0], c[1], nx_ - 1 - c[0], ny_ - 1 - c[1]) - 3.0 for c in centres])
            rmax = np.minimum(np.minimum(200.0, dist.min(axis=1)), edge)
            rays = np.array([[tip_radius(phi, c[0], c[1], t + m * math.pi / 2, rmax=rmax[j])
                              for m in range(4)] for j, (c, t) in enumerate(zip(centres, theta))])
            whole = np.all(np.isfinite(rays), axis=1)
            R = np.where(whole, np.nanmean(np.where(whole[:, None], rays, 0.0), axis=1), np.nan)
            # a crystal with a ray beyond its search radius has reached at least that
            Rmax = np.where(whole, np.max(np.where(whole[:, None], rays, 0.0), axis=1), rmax)
            # free: all four tips found, and the interfaces (4 widths apart) meet
            # neither another crystal's nor the box wall
            free = np.array([whole[j] and Rmax[j] + 2 * width < edge[j] and
                             np.all((Rmax[j] + Rmax + 4 * width < dist[j]) | (np.arange(len(R)) == j))
                             for j in range(len(R))])
            key = f"{st}_{g}"
            row[key] = {"mean_R_free": float(R[free].mean()) if free.any() else None,
                        "free_crystals": int(free.sum()),
                        "cv_free": float(R[free].std() / R[free].mean()) if free.sum() > 1 else None,
                        "R": [None if not np.isfinite(r) else round(float(r), 4) for r in R],
                        "free": [int(f) for f in free]}
            radii[(st, g)] = R
        for g in grads:
            row[f"fp32_vs_fp64_{g}"] = {
                "max_dphi": float(np.abs(phis[("fp32", g)] - phis[("fp64", g)]).max()),
                "max_dR": float(np.nanmax(np.abs(radii[("fp32", g)] - radii[("fp64", g)])))
                if np.isfinite(radii[("fp32", g)] - radii[("fp64", g)]).any() else None}
        print(json.dumps(row), flush=True)
        if done >= steps:
            break
        k = min(every, steps - done)
        for sim in sims.values():
            sim.step(k)
        done += k
    for sim in sims.values():
        sim.close()


def run_isotropy(steps: int, storage: str, with_up2: bool = True):
    """The isotropy comparison of Sec. 4.2 (six-fold a_s, 800^2): the DD and CD
    runs advance together as one batched ensemble; prints Err_l2 of each and
    the throughput."""
    import numpy as np
    import torch

    import paper_1606_09432_amd as lb
    from paper_1606_09432_amd import workloads as W

    cfgs = [W.e2("dd", storage=storage), W.e2("cd", storage=storage)]
    sim = lb.Simulation(cfgs)
    done, every = 0, max(1, steps // 10)
    t_ms = 0.0
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    while done < steps:
        k = min(every, steps - done)
        e0.record()
        sim.step(k)
        e1.record()
        torch.cuda.synchronize()
        t_ms += e0.elapsed_time(e1)
        done += k
        print(f"[e2] step {done}", file=sys.stderr, flush=True)
    out = {"workload": "isotropy comparison, six-fold a_s, 800^2, DD and CD in one batch", "steps": steps,
           "storage": storage, "MLUPS": 2 * cfgs[0].nodes * steps / (t_ms * 1e-3) / 1e6}
    for k, name in enumerate(("dd", "cd")):
        phi = sim.fields(k)[0].cpu().numpy()
        c = cfgs[k].seeds[0]
        out[f"err_l2_{name}"] = profile_l2_error(phi, (c.x, c.y))
        out[f"tip_{name}"] = sim.diagnostics()[k]["tip_position"]
        dmax, dmin, xmax, xmin = rotation_difference(phi, (c.x, c.y))
        out[f"rot60_{name}"] = {"max": dmax, "min": dmin, "at_max": xmax, "at_min": xmin}
    out["cd_over_dd"] = out["err_l2_cd"] / out["err_l2_dd"]
    sim.close()
    del sim
    if with_up2:
        # the second-order upwind directional derivatives (Sec. 4.2) through the
        # same moment: a single simulation (not batched)
        cfg = W.e2("up2", storage=storage)
        one = lb.Simulation(cfg)
        one.step(steps)
        phi = one.fields()[0].cpu().numpy()
        c = cfg.seeds[0]
        out["err_l2_up2"] = profile_l2_error(phi, (c.x, c.y))
        out["tip_up2"] = one.diagnostics()[0]["tip_position"]
        dmax, dmin, xmax, xmin = rotation_difference(phi, (c.x, c.y))
        out["rot60_up2"] = {"max": dmax, "min": dmin, "at_max": xmax, "at_min": xmin}
        one.close()
    return out


def run_paper3d(steps: int, warmup: int):
    """The paper's own 3D runs (D3Q15, 351^3, dendrites A, B, C) timed here, next
    to the wall-clock times the paper gives for them on 100 CPU cores."""
    from paper_1606_09432_amd import workloads as W

    out = []
    for d, (_entry, paper_steps, paper_seconds) in W.PAPER3D.items():
        for st in ("fp64", "fp16"):
            cfg = W.paper3d(d, st)
            r = run_gpu(cfg, steps, warmup, False)
            out.append({"dendrite": d, "storage": st, "MLUPS": r["value"], "ms_per_step": r["ms_per_step"],
                        "paper_steps": paper_steps, "time_for_paper_steps_s": r["ms_per_step"] * paper_steps / 1e3,
                        "paper_wall_clock_s": paper_seconds, "paper_hardware": "100 CPU cores (unnamed cluster)",
                        "paper_MLUPS": cfg.nodes * paper_steps / paper_seconds / 1e6})
    # dendrite B grown from the origin of a box with mirror planes (one octant)
    entry, paper_steps, paper_seconds, cores = W.PAPER3D_OCTANT
    for st in ("fp64", "fp16"):
        cfg = W.paper3d_octant(st)
        r = run_gpu(cfg, steps, warmup, False)
        out.append({"dendrite": "B, octant", "storage": st, "MLUPS": r["value"], "ms_per_step": r["ms_per_step"],
                    "paper_steps": paper_steps, "time_for_paper_steps_s": r["ms_per_step"] * paper_steps / 1e3,
                    "paper_wall_clock_s": paper_seconds, "paper_hardware": f"{cores} CPU cores (unnamed cluster)",
                    "paper_MLUPS": cfg.nodes * paper_steps / paper_seconds / 1e6})
    return out


def measure_copy(mib: int = 2048, reps: int = 10):
    """Device-to-device copy bandwidth on the same GPU (the STREAM-copy
    reference for the step's HBM roofline): bytes read + written per second."""
    import torch

    n = mib * (1 << 20)
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    gbs = 2 * n / (ms * 1e-3) / 1e9
    print(f"[bench] copy: {mib} MiB in {ms:.3f} ms, {gbs:.0f} GB/s", file=sys.stderr, flush=True)
    return {"value": gbs, "unit": "GB/s", "bytes_per_copy": 2 * n, "ms_per_copy": ms,
            "kind": f"device-to-device copy of {mib} MiB (torch copy_), read + written bytes"}


def cpu_baseline(cfg_full, sample_n: int, sample_steps: int):
    """The CPU FP64 oracle on a bounded sample: the same parameters on a
    sample_n^3 box around the seed, sample_steps steps."""
    from oracle import oracle as O

    c = sample_n // 2
    cfg = cfg_full.replace(nx=sample_n, ny=sample_n, nz=sample_n, storage="fp64")
    cfg.seeds = [type(cfg_full.seeds[0])(c, c, c, cfg_full.seeds[0].radius, 1)]
    sim = O.OracleSim(cfg)
    sim.step(1)
    t0 = time.perf_counter()
    sim.step(sample_steps)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": cfg.nodes * sample_steps / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{sample_n}^3 box of the same workload (seed centred), {sample_steps} FP64 steps, "
                      f"{dt:.1f} s",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def cpu_model() -> str:
    """The host CPU's model name (what lscpu prints as 'Model name'), with the
    family / model / stepping numbers, which identify it where a virtualised
    host reports only a generic name."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" in line:
                k, v = line.split(":", 1)
                info.setdefault(k.strip().lower(), v.strip())
            if not line.strip() and info:
                break
    except OSError:
        pass
    name = info.get("model name")
    if not name:
        import platform
        name = platform.processor() or "unknown"
    ids = [f"{k} {info[k]}" for k in ("cpu family", "model", "stepping") if k in info]
    return f"{name} ({', '.join(ids)})" if ids else name


# -- rocprofv3 summaries ---------------------------------------------------------
# The profiler writes one SQLite database (*_results.db) per process; these
# helpers turn them into the short text summaries kept next to the numbers.
STORAGE_OF_KERNEL = {"StF64": "fp64", "StF32": "fp32", "StF16": "fp16"}


def _dbs(d):
    return sorted(glob.glob(os.path.join(d, "**", "*_results.db"), recursive=True))


def _short(name):
    return name.split("(")[0].replace("void ", "").replace("lbpf::", "")


def summarize_trace(d, command, bench_json=None):
    """Per-kernel dispatch statistics (--kernel-trace) as markdown."""
    rows, spans = {}, {}
    for db in _dbs(d):
        con = sqlite3.connect(db)
        q = ("SELECT S.display_name, K.start, K.end FROM rocpd_kernel_dispatch K "
             "JOIN rocpd_info_kernel_symbol S ON S.id = K.kernel_id AND S.guid = K.guid")
        for name, t0, t1 in con.execute(q):
            rows.setdefault(_short(name), []).append(t1 - t0)
            spans.setdefault(_short(name), []).append((t0, t1))
    out = ["# Kernel trace: " + ", ".join(sorted(k for k in rows if "step_kernel" in k)), "",
           "Command (from the repository root):", "", "```", command, "```", "",
           "| kernel | calls | avg ms | min ms | max ms | total ms |", "|---|---|---|---|---|---|"]
    for k, v in sorted(rows.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"| `{k}` | {len(v)} | {sum(v) / len(v) / 1e6:.4f} | {min(v) / 1e6:.4f} | "
                   f"{max(v) / 1e6:.4f} | {sum(v) / 1e6:.3f} |")
    # one step kernel serves several runs of bench.py (the headline workload,
    # the dense-interface leg): dispatches more than 50 ms apart start a new run
    runs = ["", "Runs of each step kernel (dispatches more than 50 ms apart start a new run; the "
                "first dispatches of a run are its warm-up):", "",
            "| kernel | run | calls | avg ms |", "|---|---|---|---|"]
    for k in sorted(spans):
        if "step_kernel" not in k:
            continue
        sp = sorted(spans[k])
        cur = [sp[0]]
        parts = []
        for a, b in zip(sp, sp[1:]):
            if b[0] - a[1] > 50e6:
                parts.append(cur)
                cur = []
            cur.append(b)
        parts.append(cur)
        if len(parts) > 1:
            for j, p in enumerate(parts):
                runs.append(f"| `{k}` | {j + 1} | {len(p)} | "
                            f"{sum(t1 - t0 for t0, t1 in p) / len(p) / 1e6:.4f} |")
    if len(runs) > 5:
        out += runs
    if bench_json:
        b = json.loads(open(bench_json).read().strip().splitlines()[-1])
        out += ["", "bench.py's own HIP-event figures in the same run (ms per step = per launch):", ""]
        out.append(f"- {b['config']['storage']}: {b['ms_per_step']:.4f} ms, {b['value']:.1f} {b['unit']}, "
                   f"{b['roofline']['achieved']:.0f} GB/s algorithmic")
        for st in ("fp64", "fp32", "fp16", "batched"):
            if st in b:
                out.append(f"- {st}: {b[st]['ms_per_step']:.4f} ms, {b[st]['value']:.1f} {b[st]['unit']}, "
                           f"{b[st]['roofline']['achieved']:.0f} GB/s algorithmic")
        for st, r in b.get("d3q15", {}).items():
            out.append(f"- D3Q15 {st}: {r['ms_per_step']:.4f} ms, {r['value']:.1f} {r['unit']}, "
                       f"{r['roofline']['achieved']:.0f} GB/s algorithmic")
        for st in ("fp64", "fp32"):
            r = b.get("c1", {}).get(st)
            if r:
                out.append(f"- C1 pair (2048^2, index field) {st}: {r['ms_per_step']:.4f} ms, {r['value']:.1f} MLUPS")
        for st in ("fp16", "fp64"):
            r = b.get("dense", {}).get(st)
            if r:
                out.append(f"- dense interfaces {st}: {r['ms_per_step']:.4f} ms, {r['value']:.1f} {r['unit']}, "
                           f"anisotropic fraction {r['anisotropic_fraction']:.3f}")
        for st, c in [(b["config"]["storage"], b.get("stream_copy"))] + [
                (st, b[st].get("stream_copy")) for st in ("fp64", "fp32", "fp16") if st in b]:
            if c:
                out.append(f"- state-block copy ({st}): {c['ms']:.4f} ms, {c['bytes'] / 1e9:.2f} GB read + written, "
                           f"{c['GBps']:.0f} GB/s (`lb_pf_stream_copy`)")
        if b.get("hbm_copy"):
            out.append(f"- torch copy_: {json.dumps(b['hbm_copy'])}")
    return "\n".join(out) + "\n"


def _pmc(d):
    """{kernel: {counter: mean over dispatches of the per-dispatch sum}}."""
    acc = {}
    for db in _dbs(d):
        con = sqlite3.connect(db)
        q = ("SELECT name, dispatch_id, counter_name, SUM(counter_value) FROM pmc_events "
             "GROUP BY dispatch_id, counter_name")
        for name, _disp, cn, v in con.execute(q):
            acc.setdefault(_short(name), {}).setdefault(cn, []).append(v)
    return {k: {cn: sum(v) / len(v) for cn, v in c.items()} for k, c in acc.items()}


def summarize_traffic(fetch_dir, write_dir, cfetch_dir, cwrite_dir, copy_bytes, command):
    """HBM bytes per launch of the step kernel from FETCH_SIZE / WRITE_SIZE,
    each scaled by what the counter reads for a plain copy of copy_bytes."""
    fe, wr, cf, cw = _pmc(fetch_dir), _pmc(write_dir), _pmc(cfetch_dir), _pmc(cwrite_dir)
    copy_f = max(v.get("FETCH_SIZE", 0.0) for v in cf.values())
    copy_w = max(v.get("WRITE_SIZE", 0.0) for v in cw.values())
    ff, fw = copy_bytes / copy_f, copy_bytes / copy_w
    sha = kernel_sha()
    res = {"kernel_sha": sha, "copy_bytes": copy_bytes, "copy_fetch_counter": copy_f,
           "copy_write_counter": copy_w, "factor_fetch": ff, "factor_write": fw, "command": command,
           "kernels": {}}
    md = ["# HBM traffic of the step kernel (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)", "",
          "Commands (from the repository root):", "", "```", command, "```", "",
          f"Calibration: a plain copy of {copy_bytes} bytes reads FETCH_SIZE = {copy_f:.0f} and "
          f"WRITE_SIZE = {copy_w:.0f}, so bytes = FETCH_SIZE x {ff:.1f} + WRITE_SIZE x {fw:.1f}.", "",
          "| kernel | FETCH_SIZE | WRITE_SIZE | read bytes | written bytes | bytes/launch | bytes/node |",
          "|---|---|---|---|---|---|---|"]
    from paper_1606_09432_amd import workloads as W

    ens_nodes = sum(c.nodes for c in W.c4())
    for k in sorted(set(fe) | set(wr)):
        # the 3D workload's kernels: lattice pair 1 (D3Q19) or 2 (D3Q15); the
        # batched 2D ensemble's kernel (lattice pair 0, BATCH = true)
        targs = [a.strip() for a in k[k.find("<") + 1:k.rfind(">")].split(",")] if "<" in k else []
        lat = {"step_kernel<1,": "D3Q19_D3Q7", "step_kernel<2,": "D3Q15_D3Q7",
               "step_kernel<0,": "D2Q9_D2Q5"}.get(k[:14])
        st = next((v for kk, v in STORAGE_OF_KERNEL.items() if kk in k), None)
        f, w = fe.get(k, {}).get("FETCH_SIZE"), wr.get(k, {}).get("WRITE_SIZE")
        if lat is None or st is None or f is None or w is None:
            continue
        if lat == "D2Q9_D2Q5":
            # batched instances: without the index field the C4 ensemble (FP32),
            # with it the twenty-crystal pair (FP64 and FP32)
            if len(targs) < 5 or targs[4] != "true":
                continue
            if targs[3] == "false" and st == "fp32":
                st, nodes = BATCHED_KEY, ens_nodes
            elif targs[3] == "true" and st in ("fp32", "fp64"):
                st, nodes = f"c1_pair_{st}", 2 * 2048 * 2048
            else:
                continue
        else:
            st, nodes = traffic_key(lat, st), 512 ** 3
        rb, wb = f * ff, w * fw
        res["kernels"][st] = {"kernel": k, "kernel_sha": sha, "fetch_counter": f, "write_counter": w,
                              "read_bytes": rb, "write_bytes": wb, "bytes_per_launch": rb + wb,
                              "nodes": nodes, "bytes_per_node": (rb + wb) / nodes}
        md.append(f"| `{k}` | {f:.0f} | {w:.0f} | {rb:.4g} | {wb:.4g} | {rb + wb:.4g} | "
                  f"{(rb + wb) / nodes:.1f} |")
    md += ["", f"Kernel source hash: {sha} (comments and blank lines excluded; bench.py reports this traffic only "
               "while it matches)."]
    return res, "\n".join(md) + "\n"


SQ_PASSES = (("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR", "SQ_INSTS_SALU",
              "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES"),
             ("SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_WAIT_ANY",
              "SQ_ACTIVE_INST_ANY", "SQ_INSTS_SMEM", "SQ_ACTIVE_INST_SCA"))


def summarize_sq(d1, d2, command):
    """Instruction mix and wave-time split of the 512^3 step kernels from two
    --pmc passes of SQ counters (the counts are whole-chip sums per dispatch)."""
    a, b = _pmc(d1), _pmc(d2)
    nodes = 512 ** 3
    md = ["# Instruction mix of the step kernel (rocprofv3 --pmc, SQ counters)", "",
          "Commands (from the repository root):", "", "```", command, "```", "",
          "Instructions are wave instructions x 64 lanes / 512^3 nodes, i.e. per node and step, halo work "
          "included. The time split divides each wave's active or waiting time by its lifetime "
          "(SQ_ACTIVE_INST_* and SQ_WAIT_ANY over SQ_WAVE_CYCLES).", "",
          "| kernel | waves | VALU/node | SALU/node | LDS/node | VMEM rd/node | VMEM wr/node | VALU active | "
          "SALU active | LDS active | waiting | LDS bank conflicts/LDS instr |",
          "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for k in sorted(a):
        if not k.startswith("step_kernel<1,") and not k.startswith("step_kernel<2,"):
            continue
        v = dict(a[k])
        v.update(b.get(k, {}))
        if any(c not in v for c in SQ_PASSES[0] + SQ_PASSES[1]):
            continue
        per = lambda c: v[c] * 64 / nodes  # noqa: E731
        cyc = v["SQ_WAVE_CYCLES"]
        md.append(f"| `{k}` | {v['SQ_WAVES']:.0f} | {per('SQ_INSTS_VALU'):.0f} | {per('SQ_INSTS_SALU'):.0f} | "
                  f"{per('SQ_INSTS_LDS'):.0f} | {per('SQ_INSTS_VMEM_RD'):.1f} | {per('SQ_INSTS_VMEM_WR'):.1f} | "
                  f"{v['SQ_ACTIVE_INST_VALU'] / cyc:.2f} | {v['SQ_ACTIVE_INST_SCA'] / cyc:.2f} | "
                  f"{v['SQ_ACTIVE_INST_LDS'] / cyc:.2f} | {v['SQ_WAIT_ANY'] / cyc:.2f} | "
                  f"{v['SQ_LDS_BANK_CONFLICT'] / max(v['SQ_INSTS_LDS'], 1):.3f} |")
    md += ["", f"Kernel source hash: {kernel_sha()} (comments and blank lines excluded)."]
    return "\n".join(md) + "\n"


def summarize_counters(dirs, command, title):
    """Per-dispatch values and per-node figures of every counter in the given
    --pmc runs, for the 512^3 step kernels of the 3D workload."""
    vals = {}
    for d in dirs:
        for k, c in _pmc(d).items():
            if k.startswith("step_kernel<1,") or k.startswith("step_kernel<2,"):
                vals.setdefault(k, {}).update(c)
    names = sorted({c for v in vals.values() for c in v})
    nodes = 512 ** 3
    md = [f"# {title}", "", "Commands (from the repository root):", "", "```", command, "```", "",
          "Each cell: counter value per dispatch (whole chip) / the same per node of the 512^3 grid.", "",
          "| kernel | " + " | ".join(names) + " |", "|---|" + "---|" * len(names)]
    for k in sorted(vals):
        md.append(f"| `{k}` | " + " | ".join(
            f"{vals[k][c]:.4g} / {vals[k][c] / nodes:.3f}" if c in vals[k] else "—" for c in names) + " |")
    md += ["", f"Kernel source hash: {kernel_sha()} (comments and blank lines excluded)."]
    return "\n".join(md) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=512, help="grid side (the workload is 512)")
    ap.add_argument("--variant", default="100", choices=["100", "111", "110"])
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=128)
    ap.add_argument("--cpu-steps", type=int, default=300)
    ap.add_argument("--only", choices=["fp16", "fp64", "fp32"], default=None)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched 2D ensemble")
    ap.add_argument("--no-d3q15", action="store_true", help="skip the D3Q15 runs")
    ap.add_argument("--no-dense", action="store_true", help="skip the dense-interface 512^3 runs")
    ap.add_argument("--accuracy", choices=["c2", "c3"], default=None,
                    help="only report the FP32/FP16-offset error against FP64 over a run")
    ap.add_argument("--paper3d", action="store_true",
                    help="only time the paper's 351^3 D3Q15 runs (context for its wall-clock times)")
    ap.add_argument("--orientation", action="store_true",
                    help="only run the DD/CD orientation-dependence measurement (four-fold crystals)")
    ap.add_argument("--c1", type=int, default=0, metavar="STEPS",
                    help="only run the twenty-crystal 2048^2 workload (DD/CD x FP64/FP32) for STEPS steps")
    ap.add_argument("--isotropy", type=int, default=0, metavar="STEPS",
                    help="only run the six-fold DD/CD isotropy comparison for STEPS steps")
    ap.add_argument("--acc-steps", type=int, default=2000)
    ap.add_argument("--acc-every", type=int, default=500)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (for HBM counter calibration)")
    ap.add_argument("--summarize-trace", metavar="DIR", help="write a markdown summary of a --kernel-trace run")
    ap.add_argument("--summarize-traffic", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="write profiles/hbm_traffic.json from four --pmc runs")
    ap.add_argument("--summarize-sq", nargs=2, metavar=("PASS1", "PASS2"),
                    help="write a markdown summary of the two SQ counter --pmc runs")
    ap.add_argument("--summarize-counters", nargs="+", metavar="DIR",
                    help="write a markdown table of the counters of one or more --pmc runs")
    ap.add_argument("--title", default="Counters of the step kernel (rocprofv3 --pmc)")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--command", default="", help="the profiling command recorded in the summary "
                    "(default: the commands these summaries are made with)")
    ap.add_argument("--bench-json", default=None)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    if args.summarize_trace:
        cmd = args.command or "\n".join([
            f"rocprofv3 --kernel-trace --stats -d {args.summarize_trace} -o bench -- python bench.py"
            + (f" > {args.bench_json}" if args.bench_json else ""),
            f"python bench.py --summarize-trace {args.summarize_trace}"
            + (f" --bench-json {args.bench_json}" if args.bench_json else "")
            + (f" --out {args.out}" if args.out else "")])
        text = summarize_trace(args.summarize_trace, cmd, args.bench_json)
        open(args.out, "w").write(text) if args.out else print(text)
        return
    if args.summarize_counters:
        if not args.command:
            raise SystemExit("--summarize-counters needs --command (the rocprofv3 runs that made the directories)")
        text = summarize_counters(args.summarize_counters, args.command, args.title)
        open(args.out, "w").write(text) if args.out else print(text)
        return
    if args.summarize_sq:
        run = "python bench.py --steps 3 --warmup 1 --no-cpu-baseline --no-batched --no-dense"
        cmd = args.command or "\n".join(
            [f"rocprofv3 --pmc {' '.join(p)} -d {d} -o bench -- {run}" for p, d in zip(SQ_PASSES, args.summarize_sq)]
            + [f"python bench.py --summarize-sq {' '.join(args.summarize_sq)}" + (f" --out {args.out}" if args.out else "")])
        text = summarize_sq(*args.summarize_sq, cmd)
        open(args.out, "w").write(text) if args.out else print(text)
        return
    if args.summarize_traffic:
        fd, wd, cfd, cwd = args.summarize_traffic
        run = "python bench.py --steps 3 --warmup 1 --no-cpu-baseline --no-dense"
        cal = f"python bench.py --calibrate-copy {args.copy_mib}"
        cmd = args.command or "\n".join([
            f"rocprofv3 --pmc FETCH_SIZE -d {fd} -o bench -- {run}",
            f"rocprofv3 --pmc WRITE_SIZE -d {wd} -o bench -- {run}",
            f"rocprofv3 --pmc FETCH_SIZE -d {cfd} -o copy -- {cal}",
            f"rocprofv3 --pmc WRITE_SIZE -d {cwd} -o copy -- {cal}",
            f"python bench.py --summarize-traffic {fd} {wd} {cfd} {cwd} --copy-mib {args.copy_mib}"
            + (f" --out {args.out}" if args.out else "")])
        res, md = summarize_traffic(*args.summarize_traffic, args.copy_mib * (1 << 20), cmd)
        json.dump(res, open(TRAFFIC_FILE, "w"), indent=1)
        open(args.out, "w").write(md) if args.out else print(md)
        return
    if args.paper3d:
        for row in run_paper3d(args.steps, args.warmup):
            print(json.dumps(row), flush=True)
        return
    if args.orientation:
        print(json.dumps(run_orientation_spread(args.only or "fp64")), flush=True)
        return
    if args.c1:
        run_c1(args.c1, args.acc_every)
        return
    if args.isotropy:
        print(json.dumps(run_isotropy(args.isotropy, args.only or "fp64")), flush=True)
        return
    if args.accuracy:
        run_accuracy(args.accuracy, args.n if args.accuracy == "c3" else min(args.n, 256), args.acc_steps,
                     args.acc_every, args.variant)
        return
    if args.calibrate_copy:
        # a plain elementwise copy kernel (read n bytes, write n bytes)
        import torch
        n = args.calibrate_copy * (1 << 20)
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (the z-slab sharding is a "
              "design note only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    from paper_1606_09432_amd import workloads as W

    results = {}
    storages = [args.only] if args.only else ["fp16", "fp64"]
    for st in storages:
        results[st] = run_gpu(W.c3(st, args.variant, n=args.n), args.steps, args.warmup, args.autotune,
                              copy_ceiling=True)
    head = "fp16" if "fp16" in results else storages[0]
    r = results[head]
    out = {
        "metric": METRIC, "value": r["value"], "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if head != "fp64" else "f64", "data": "synthetic",
        "config": {"workload": f"D3Q19 phi + D3Q7 u, {args.n}^3, zero-flux, one central seed R=8, "
                               f"Eq. As_MatSci variant <{args.variant}>, Delta=0.6, "
                               f"{'FP16-offset storage' if head == 'fp16' else head} (headline)",
                   "grid": [args.n] * 3, "storage": head, "tile_y_chunk": r["tile"]},
        "roofline": r["roofline"],
        "stream_copy": r["copy"], "anisotropic_fraction": r["anisotropic_fraction"],
    }
    for st, rr in results.items():
        if st != head:
            out[st] = {"value": rr["value"], "unit": "MLUPS", "ms_per_step": rr["ms_per_step"],
                       "dtype": "f64" if st == "fp64" else "f32", "roofline": rr["roofline"], "tile_y_chunk": rr["tile"],
                       "stream_copy": rr["copy"]}
    if "fp64" in results and "fp16" in results:
        out["fp16_over_fp64"] = results["fp16"]["value"] / results["fp64"]["value"]
    if not args.no_dense and not args.only:
        # a state where nearly every node is at an interface (512 crystals)
        dsteps = min(args.steps, 200)
        out["dense"] = {"workload": f"{args.n}^3, a crystal every 64 nodes (512 seeds R=20, jittered), "
                                    f"Eq. As_MatSci <100>, Delta=0.6", "steps": dsteps}
        for st in ("fp16", "fp64"):
            rr = run_gpu(W.dense_3d(st, n=args.n), dsteps, min(args.warmup, 20), args.autotune)
            out["dense"][st] = {"value": rr["value"], "unit": "MLUPS", "ms_per_step": rr["ms_per_step"],
                                "roofline": rr["roofline"], "tile_y_chunk": rr["tile"],
                                "anisotropic_fraction": rr["anisotropic_fraction"]}
    if not args.no_batched and not args.only:
        out["batched"] = run_batched(args.steps, args.warmup)
        out["c1"] = run_c1_throughput(min(args.steps, 500))
    if not args.no_d3q15 and not args.only:
        # the paper's own 3D phase-field lattice on the same workload
        out["d3q15"] = {}
        for st in ("fp16", "fp64"):
            rr = run_gpu(W.c3(st, args.variant, n=args.n, lattice="D3Q15_D3Q7"), args.steps, args.warmup,
                         args.autotune)
            out["d3q15"][st] = {"value": rr["value"], "unit": "MLUPS", "ms_per_step": rr["ms_per_step"],
                                "roofline": rr["roofline"], "tile_y_chunk": rr["tile"]}
    if not args.only:
        out["hbm_copy"] = measure_copy()
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(W.c3("fp64", args.variant, n=args.n), args.cpu_sample, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

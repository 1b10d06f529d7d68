"""The C-ABI library loads and exports every entry point include/lb_pf.h declares.

Runs without a GPU: only host-side entry points are called (workspace
planning, configuration checks and the sharp-interface helper); no kernel is
launched.
"""
import ctypes as C
import json
import os
import re
import subprocess

import pytest

import paper_1606_09432_amd as lb
from paper_1606_09432_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lb_pf.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(lb_pf_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    return lb.load_library()


def test_header_declares_what_binding_uses():
    assert _declared() == sorted(lb.EXPORTED_SYMBOLS)


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", lb.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (lb_pf_\w+)", out))
    missing = set(_declared()) - exported
    assert not missing, missing
    for name in _declared():
        assert hasattr(lib, name)


def test_library_is_gfx950(lib):
    blob = open(lb.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


def test_workspace_bytes_layout(lib):
    cfg = W.c3("fp16")
    b = lb.workspace_bytes(cfg)
    n = 512**3
    # two copies of 26 FP16 distributions + FP32 phi and u* fields
    assert 2 * n * (26 * 2 + 8) <= b < 2 * n * (26 * 2 + 8) * 1.001 + (1 << 20)
    b64 = lb.workspace_bytes(W.c3("fp64"))
    assert 2 * n * (26 * 8 + 8) <= b64 < 2 * n * (26 * 8 + 8) * 1.001 + (1 << 20)
    assert b64 < 288e9 * 0.25


def test_workspace_pads_rows_to_64(lib):
    a = lb.workspace_bytes(W.c0(n=100))
    b = lb.workspace_bytes(W.c0(n=128).replace(ny=100))
    assert a == b  # 100 -> pitch 128


@pytest.mark.parametrize("mutate,code", [
    (dict(nx=2), -1), (dict(lattice="D3Q19_D3Q7", nz=1), -1), (dict(dt=0.0), -2), (dict(W0=-1.0), -1),
    (dict(aniso=[]), -1), (dict(use_ids=True), -1),
    # one FP32 field of 4 GiB or more cannot be addressed with 32-bit byte offsets
    (dict(lattice="D3Q19_D3Q7", nx=1024, ny=1024, nz=1024, storage="fp16"), -1),
    (dict(lattice="D3Q19_D3Q7", nx=1024, ny=1024, nz=512, storage="fp64"), -1),
])
def test_invalid_configs_rejected(lib, mutate, code):
    cfg = W.c0(n=32).replace(**mutate)
    keep = []
    try:
        s = lb._to_struct(cfg, keep)
    except AssertionError:
        pytest.skip("rejected by the Python-side check already")
    b = C.c_size_t()
    rc = lib.lb_pf_workspace_bytes(C.byref(s), 1, C.byref(b))
    assert rc == code, lib.lb_pf_last_error()
    assert lib.lb_pf_last_error()


def test_boundary_values(lib):
    """LBPF_MIRROR_LOW (2) is a valid boundary; 3 is not."""
    keep = []
    b = C.c_size_t()
    s = lb._to_struct(W.c0(n=32).replace(boundary="mirror_low"), keep)
    assert s.boundary == 2
    assert lib.lb_pf_workspace_bytes(C.byref(s), 1, C.byref(b)) == 0
    s.boundary = 3
    assert lib.lb_pf_workspace_bytes(C.byref(s), 1, C.byref(b)) == -1
    assert "boundary" in lib.lb_pf_last_error().decode()


def test_upwind_gradient_rules(lib):
    """LBPF_GRAD_UP2 (2) is valid for single simulations without mirror planes,
    with or without the index field, with every extent >= 4; 3 is no
    gradient."""
    keep = []
    b = C.c_size_t()

    def rc(cfg, n=1):
        arr = (lb.LbpfConfig * n)(*[lb._to_struct(cfg, keep) for _ in range(n)])
        return lib.lb_pf_workspace_bytes(arr, n, C.byref(b))

    base = W.c0(n=32).replace(gradient="up2")
    assert rc(base) == 0
    assert rc(W.small_3d(n=8).replace(gradient="up2")) == 0
    assert rc(base.replace(nx=3)) == -1
    assert rc(base.replace(boundary="mirror_low")) == -6
    assert rc(base, n=2) == -6
    assert rc(W.c1(n=64, count=3, gradient="up2")) == 0
    assert rc(W.oriented_3d(gradient="up2")) == 0
    s = lb._to_struct(base, keep)
    s.gradient = 3
    assert lib.lb_pf_workspace_bytes(C.byref(s), 1, C.byref(b)) == -1


def test_init_rejects_missing_workspace(lib):
    keep = []
    s = lb._to_struct(W.c0(n=32), keep)
    h = C.c_void_p()
    rc = lib.lb_pf_init(C.byref(s), 1, None, 0, None, C.byref(h))
    assert rc == -3 and not h.value
    rc = lib.lb_pf_init(C.byref(s), 1, C.c_void_p(0x1001), 1 << 40, None, C.byref(h))
    assert rc == -3  # misaligned


def test_batched_requires_2d(lib):
    keep = []
    arr = (lb.LbpfConfig * 2)(lb._to_struct(W.c0(n=32), keep), lb._to_struct(W.small_3d(n=8), keep))
    b = C.c_size_t()
    assert lib.lb_pf_workspace_bytes(arr, 2, C.byref(b)) == -6


def test_sharp_interface_printed_values(lib):
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_values.json")))["sharp_interface"]
    _, _, ls = lb.sharp_interface(1.0, 1.0, 1.0, g["kappa"])
    assert abs(ls - g["lambda_star"]) < g["printed_digits_tolerance"]
    d0, beta, _ = lb.sharp_interface(1.0, 1.0, ls, g["kappa"])
    assert abs(d0 - g["d0"]) < g["printed_digits_tolerance"] and abs(beta) < 1e-12


def test_product_never_imports_oracle():
    pkg = os.path.join(ROOT, "paper_1606_09432_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"(import\s+oracle|from\s+oracle|lbpf_oracle|orc_\w+\()", txt), f


def _ws_rc(lib, cfg):
    keep = []
    s = lb._to_struct(cfg, keep)
    b = C.c_size_t()
    return lib.lb_pf_workspace_bytes(C.byref(s), 1, C.byref(b))


ROT_GENERIC = W.rotation((1.0, 2.0, 3.0), 0.7)
ROT_Z45 = W.rotation((0.0, 0.0, 1.0), 0.7853981633974483)


@pytest.mark.parametrize("entry,dim,code", [
    (W.Aniso("sectoral", eps=1.2, q=4), 2, -2),        # a_s = 1 - 1.2 on the diagonals
    (W.Aniso("sectoral", eps=0.9, q=4), 2, 0),
    (W.Aniso("cubic", eps=0.7), 3, -2),                # 1 - 5 eps / 3 < 0 on <111>
    (W.Aniso("cubic", eps=0.55), 3, 0),
    (W.Aniso("cubic_s", gamma=-0.5), 3, -2),           # 1 + 66 gamma / 27 < 0 on <111>
    (W.Aniso("cubic_hak", eps=0.0, gamma=1.2), 3, -2),  # 1 + gamma (3/2 - 17/7) < 0 on <110>
    (W.Aniso("cubic", eps=0.05, R=ROT_GENERIC), 3, 0),
    (W.Aniso("cubic", eps=0.05, R=(1.0, 0.1, 0, 0, 1, 0, 0, 0, 1)), 3, -1),  # not orthogonal
    (W.Aniso("cubic", eps=0.05, R=(2.0, 0, 0, 0, 2, 0, 0, 0, 2)), 3, -1),
])
def test_entries_checked_on_the_sphere(lib, entry, dim, code):
    """Entries must keep a_s > 0 (LBPF_ERR_UNSTABLE otherwise) and a given R
    must be orthogonal (LBPF_ERR_ARG)."""
    cfg = W.c0(n=32) if dim == 2 else W.small_3d(n=8)
    assert _ws_rc(lib, cfg.replace(aniso=[entry])) == code, lib.lb_pf_last_error()


@pytest.mark.parametrize("entry,ok", [
    (W.Aniso("cubic", eps=0.05), True), (W.Aniso("cubic_hak", eps=0.1, gamma=-0.02), True),
    (W.Aniso("cubic_s", gamma=0.02), True), (W.Aniso("sectoral", eps=0.05, q=6), True),
    (W.Aniso("cubic", eps=0.05, R=ROT_Z45), True),
    (W.Aniso("sectoral", eps=0.05, q=6, phi0=0.3), False), (W.Aniso("sectoral", eps=0.05, q=3), False),
    (W.Aniso("cubic", eps=0.05, R=ROT_GENERIC), False),
])
def test_mirror_boxes_need_symmetric_entries(lib, oracle_mod, entry, ok):
    """LBPF_MIRROR_LOW refuses entries that are not symmetric about the planes
    (LBPF_ERR_UNSUPPORTED); zero-flux boxes accept them.  The oracle takes the
    same decisions."""
    cfg = W.small_3d(n=10, aniso=entry).replace(seeds=[W.Seed(0, 0, 0, 3.0, 1)])
    assert _ws_rc(lib, cfg) == 0
    rc = _ws_rc(lib, cfg.replace(boundary="mirror_low"))
    assert rc == (0 if ok else -6), lib.lb_pf_last_error()
    assert oracle_mod.aniso_mirror_symmetric(entry, 3) == ok
    if not ok:
        assert "symmetric" in lib.lb_pf_last_error().decode()
    # 2D: the sectoral four-fold function turned by 0.2 is asymmetric about the axes
    c2 = W.c0(n=16).replace(boundary="mirror_low", seeds=[W.Seed(0, 0, 0, 3.0, 1)])
    assert _ws_rc(lib, c2) == 0
    assert _ws_rc(lib, c2.replace(aniso=[W.Aniso("sectoral", eps=0.05, q=4, phi0=0.2)])) == -6


"""MI355X-native coupled lattice Boltzmann phase-field step (arXiv:1606.09432).

Thin Python binding of the C ABI in ``include/lb_pf.h``: it marshals
arguments and hands the library a torch-allocated device workspace and the
current torch stream.  Every step of the method runs in the HIP kernels of
``liblbpf.so``; there is no Python or CPU fallback, and every entry point
raises if the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Sequence, Union

from . import workloads
from .workloads import Aniso, Seed, SimConfig

HERE = os.path.dirname(os.path.abspath(__file__))
# LBPF_LIBRARY selects another build of the same library (e.g. to compare two
# kernel versions); the default is the in-tree build.
LIB_PATH = os.environ.get("LBPF_LIBRARY", os.path.join(HERE, "liblbpf.so"))

__all__ = ["Simulation", "SimConfig", "Aniso", "Seed", "workloads", "load_library", "sharp_interface",
           "LbpfError", "EXPORTED_SYMBOLS"]

# C ABI mirrors (include/lb_pf.h).
LATTICE = {"D2Q9_D2Q5": 0, "D3Q19_D3Q7": 1, "D3Q15_D3Q7": 2}
BOUNDARY = {"periodic": 0, "zero_flux": 1, "mirror_low": 2}
GRADIENT = {"dd": 0, "cd": 1, "up2": 2}
STORAGE = {"fp64": 0, "fp32": 1, "fp16": 2}
ANISO = {"iso": 0, "sectoral": 1, "cubic": 2, "cubic_hak": 3, "cubic_s": 4}
ERR_NONFINITE = -5

EXPORTED_SYMBOLS = (
    "lb_pf_workspace_bytes", "lb_pf_init", "lb_pf_step", "lb_pf_diagnostics", "lb_pf_export_fields",
    "lb_pf_export_dists", "lb_pf_import_fields", "lb_pf_state_bytes", "lb_pf_save_state",
    "lb_pf_load_state", "lb_pf_set_tile", "lb_pf_get_tile", "lb_pf_autotune", "lb_pf_info",
    "lb_pf_destroy", "lb_pf_last_error", "lb_pf_sharp_interface", "lb_pf_diagnostics_noalloc",
    "lb_pf_stream_copy", "lb_pf_state_ptr",
)


class LbpfAniso(C.Structure):
    _fields_ = [("kind", C.c_int32), ("q", C.c_int32), ("eps", C.c_double), ("gamma", C.c_double),
                ("phi0", C.c_double), ("R", C.c_double * 9)]


class LbpfSeed(C.Structure):
    _fields_ = [("x", C.c_double), ("y", C.c_double), ("z", C.c_double), ("radius", C.c_double),
                ("crystal_id", C.c_int32)]


class LbpfConfig(C.Structure):
    _fields_ = [("lattice", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("boundary", C.c_int32), ("gradient", C.c_int32), ("storage", C.c_int32),
                ("use_ids", C.c_int32),
                ("W0", C.c_double), ("tau0", C.c_double), ("lam", C.c_double), ("kappa", C.c_double),
                ("delta", C.c_double), ("dx", C.c_double), ("dt", C.c_double), ("xi", C.c_double),
                ("n_aniso", C.c_int32), ("aniso", C.POINTER(LbpfAniso)),
                ("n_seeds", C.c_int32), ("seeds", C.POINTER(LbpfSeed)),
                ("tip_dir", C.c_int32 * 3)]


class LbpfDiag(C.Structure):
    _fields_ = [("step", C.c_int64), ("sum_phi", C.c_double), ("sum_u", C.c_double),
                ("sum_u_minus_half_phi", C.c_double), ("solid_fraction", C.c_double),
                ("n_solid", C.c_double), ("tip_position", C.c_double), ("nonfinite", C.c_int32)]


class LbpfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lb_pf error {code}: {msg}")
        self.code = code


_lib = None


def load_library():
    """Loads the in-tree HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(or python paper_1606_09432_amd/build.py)")
    lib = C.CDLL(LIB_PATH)
    vp, sz = C.c_void_p, C.c_size_t
    cfgp = C.POINTER(LbpfConfig)
    sig = {
        "lb_pf_workspace_bytes": [cfgp, C.c_int, C.POINTER(sz)],
        "lb_pf_init": [cfgp, C.c_int, vp, sz, vp, C.POINTER(vp)],
        "lb_pf_step": [vp, C.c_int, vp],
        "lb_pf_diagnostics": [vp, C.POINTER(LbpfDiag), vp],
        "lb_pf_diagnostics_noalloc": [vp, C.POINTER(LbpfDiag), vp],
        "lb_pf_export_fields": [vp, C.c_int, vp, vp, vp, vp],
        "lb_pf_export_dists": [vp, C.c_int, vp, vp, vp],
        "lb_pf_import_fields": [vp, C.c_int, vp, vp, vp, vp],
        "lb_pf_state_bytes": [vp, C.POINTER(sz)],
        "lb_pf_save_state": [vp, vp, sz, vp],
        "lb_pf_load_state": [vp, vp, sz, vp],
        "lb_pf_set_tile": [vp, C.c_int, C.c_int],
        "lb_pf_get_tile": [vp, C.POINTER(C.c_int), C.POINTER(C.c_int)],
        "lb_pf_autotune": [vp, C.c_int, vp],
        "lb_pf_info": [vp, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int),
                       C.POINTER(C.c_int)],
        "lb_pf_destroy": [vp],
        "lb_pf_stream_copy": [vp, vp, sz, C.c_int, vp],
        "lb_pf_state_ptr": [vp, C.c_int, C.POINTER(vp), C.POINTER(sz)],
        "lb_pf_sharp_interface": [C.c_double] * 4 + [C.POINTER(C.c_double)] * 3,
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.lb_pf_last_error.argtypes = []
    lib.lb_pf_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        raise LbpfError(rc, load_library().lb_pf_last_error().decode())


def sharp_interface(W0: float, tau0: float, lam: float, kappa: float):
    """(d0, beta, lambda_star) of Eqs. Capillary-Length / Kinetic-Coeff."""
    lib = load_library()
    d0, beta, ls = C.c_double(), C.c_double(), C.c_double()
    _check(lib.lb_pf_sharp_interface(W0, tau0, lam, kappa, C.byref(d0), C.byref(beta), C.byref(ls)))
    return d0.value, beta.value, ls.value


def _to_struct(cfg: SimConfig, keep: list) -> LbpfConfig:
    cfg.validate()
    an = (LbpfAniso * len(cfg.aniso))(*[LbpfAniso(ANISO[a.kind], int(a.q), float(a.eps), float(a.gamma),
                                                  float(a.phi0), (C.c_double * 9)(*a.rotation_row_major()))
                                        for a in cfg.aniso])
    sd = (LbpfSeed * max(1, len(cfg.seeds)))(*[LbpfSeed(float(s.x), float(s.y), float(s.z), float(s.radius),
                                                        int(s.id)) for s in cfg.seeds])
    keep.extend([an, sd])
    c = LbpfConfig()
    c.lattice = LATTICE[cfg.lattice]
    c.nx, c.ny, c.nz = cfg.nx, cfg.ny, cfg.nz
    c.boundary = BOUNDARY[cfg.boundary]
    c.gradient = GRADIENT[cfg.gradient]
    c.storage = STORAGE[cfg.storage]
    c.use_ids = 1 if cfg.use_ids else 0
    c.W0, c.tau0, c.lam, c.kappa = cfg.W0, cfg.tau0, cfg.lam, cfg.kappa
    c.delta, c.dx, c.dt, c.xi = cfg.delta, cfg.dx, cfg.dt, cfg.xi
    c.n_aniso = len(cfg.aniso)
    c.aniso = an
    c.n_seeds = len(cfg.seeds)
    c.seeds = sd
    c.tip_dir[:] = list(cfg.tip_dir)
    return c


def stream_copy(src, dst, nbytes: int, blocks_per_cu: int = 8) -> None:
    """Plain streaming copy of nbytes between two device buffers (torch
    tensors or raw device addresses) on the current torch stream."""
    import torch

    sp = src if isinstance(src, int) else src.data_ptr()
    dp = dst if isinstance(dst, int) else dst.data_ptr()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    _check(load_library().lb_pf_stream_copy(C.c_void_p(sp), C.c_void_p(dp), int(nbytes), int(blocks_per_cu), st))


def workspace_bytes(cfgs: Union[SimConfig, Sequence[SimConfig]]) -> int:
    cfgs = [cfgs] if isinstance(cfgs, SimConfig) else list(cfgs)
    keep: list = []
    arr = (LbpfConfig * len(cfgs))(*[_to_struct(c, keep) for c in cfgs])
    b = C.c_size_t()
    _check(load_library().lb_pf_workspace_bytes(arr, len(cfgs), C.byref(b)))
    return b.value


class Simulation:
    """One simulation (or a batched 2D ensemble) living in a torch-owned workspace."""

    def __init__(self, cfgs: Union[SimConfig, Sequence[SimConfig]], device: str = "cuda"):
        import torch

        self.torch = torch
        self.lib = load_library()
        self.cfgs: List[SimConfig] = [cfgs] if isinstance(cfgs, SimConfig) else list(cfgs)
        self.device = torch.device(device)
        self._keep: list = []
        arr = (LbpfConfig * len(self.cfgs))(*[_to_struct(c, self._keep) for c in self.cfgs])
        self._arr = arr
        b = C.c_size_t()
        _check(self.lib.lb_pf_workspace_bytes(arr, len(self.cfgs), C.byref(b)))
        self.workspace = torch.empty(b.value, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        _check(self.lib.lb_pf_init(arr, len(self.cfgs), C.c_void_p(self.workspace.data_ptr()), b.value,
                                   self._stream(), C.byref(h)))
        self.h = h

    def _stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def close(self) -> None:
        """Waits for the enqueued work and frees the handle (the workspace
        tensor goes with the object)."""
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.torch.cuda.current_stream(self.device).synchronize()
            self.lib.lb_pf_destroy(h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: torch may already be torn down
            pass

    # -- stepping ----------------------------------------------------------------
    def step(self, n: int = 1) -> None:
        _check(self.lib.lb_pf_step(self.h, int(n), self._stream()))

    def diagnostics(self, allow_nonfinite: bool = False) -> List[dict]:
        out = (LbpfDiag * len(self.cfgs))()
        rc = self.lib.lb_pf_diagnostics(self.h, out, self._stream())
        if rc != 0 and not (allow_nonfinite and rc == ERR_NONFINITE):
            _check(rc)
        return [{k: getattr(d, k) for k, _ in LbpfDiag._fields_} for d in out]

    def diagnostics_noalloc(self, allow_nonfinite: bool = False) -> List[dict]:
        """The same records through the entry point that allocates nothing
        (reduction scratch in the library's static device array)."""
        out = (LbpfDiag * len(self.cfgs))()
        rc = self.lib.lb_pf_diagnostics_noalloc(self.h, out, self._stream())
        if rc != 0 and not (allow_nonfinite and rc == ERR_NONFINITE):
            _check(rc)
        return [{k: getattr(d, k) for k, _ in LbpfDiag._fields_} for d in out]

    # -- fields --------------------------------------------------------------------
    def nodes(self, sim: int = 0) -> int:
        n = C.c_int64()
        _check(self.lib.lb_pf_info(self.h, sim, C.byref(n), None, None, None))
        return n.value

    def fields(self, sim: int = 0):
        """(phi, u, ids) of simulation `sim` as device tensors shaped like the config."""
        t = self.torch
        cfg = self.cfgs[sim]
        phi = t.empty(cfg.shape, dtype=t.float64, device=self.device)
        u = t.empty_like(phi)
        ids = t.empty(cfg.shape, dtype=t.int16, device=self.device)
        _check(self.lib.lb_pf_export_fields(self.h, sim, C.c_void_p(phi.data_ptr()), C.c_void_p(u.data_ptr()),
                                            C.c_void_p(ids.data_ptr()), self._stream()))
        return phi, u, ids

    def dists(self, sim: int = 0):
        """Post-streaming (g, f) of simulation `sim`, FP64, shaped [q, *shape]."""
        t = self.torch
        cfg = self.cfgs[sim]
        qp, qu = (9, 5) if cfg.dim == 2 else ((15, 7) if cfg.lattice == "D3Q15_D3Q7" else (19, 7))
        g = t.empty((qp,) + cfg.shape, dtype=t.float64, device=self.device)
        f = t.empty((qu,) + cfg.shape, dtype=t.float64, device=self.device)
        _check(self.lib.lb_pf_export_dists(self.h, sim, C.c_void_p(g.data_ptr()), C.c_void_p(f.data_ptr()),
                                           self._stream()))
        return g, f

    def import_fields(self, phi, u, ids=None, sim: int = 0) -> None:
        t = self.torch
        phi = t.as_tensor(phi, dtype=t.float64, device=self.device).contiguous()
        u = t.as_tensor(u, dtype=t.float64, device=self.device).contiguous()
        idp = None
        if ids is not None:
            ids = t.as_tensor(ids, dtype=t.int16, device=self.device).contiguous()
            idp = C.c_void_p(ids.data_ptr())
        self._import_keep = (phi, u, ids)
        _check(self.lib.lb_pf_import_fields(self.h, sim, C.c_void_p(phi.data_ptr()), C.c_void_p(u.data_ptr()),
                                            idp, self._stream()))

    # -- checkpoint --------------------------------------------------------------
    def save_state(self):
        b = C.c_size_t()
        _check(self.lib.lb_pf_state_bytes(self.h, C.byref(b)))
        buf = self.torch.empty(b.value, dtype=self.torch.uint8, device=self.device)
        _check(self.lib.lb_pf_save_state(self.h, C.c_void_p(buf.data_ptr()), b.value, self._stream()))
        return buf

    def load_state(self, buf) -> None:
        _check(self.lib.lb_pf_load_state(self.h, C.c_void_p(buf.data_ptr()), buf.numel(), self._stream()))

    # -- tiling ------------------------------------------------------------------
    def set_tile(self, tile_y: int = 0, chunk: int = 0) -> None:
        _check(self.lib.lb_pf_set_tile(self.h, int(tile_y), int(chunk)))

    def get_tile(self):
        ty, ch = C.c_int(), C.c_int()
        _check(self.lib.lb_pf_get_tile(self.h, C.byref(ty), C.byref(ch)))
        return ty.value, ch.value

    def autotune(self, steps_per_trial: int = 3):
        _check(self.lib.lb_pf_autotune(self.h, int(steps_per_trial), self._stream()))
        return self.get_tile()

    def state_block(self, sim: int = 0):
        """(device address, bytes) of simulation `sim`'s current state block."""
        p, b = C.c_void_p(), C.c_size_t()
        _check(self.lib.lb_pf_state_ptr(self.h, sim, C.byref(p), C.byref(b)))
        return p.value, b.value

    @property
    def step_count(self) -> int:
        s = C.c_int64()
        _check(self.lib.lb_pf_info(self.h, 0, None, C.byref(s), None, None))
        return s.value

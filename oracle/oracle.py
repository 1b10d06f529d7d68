"""ctypes wrapper of the CPU FP64 oracle (test infrastructure only).

The oracle shares no code with the GPU path: it has its own C structs, its own
lattice tables and formulas (lbpf_oracle.c), and this wrapper converts a
workload description (any object with the ``SimConfig`` attributes) into the
oracle's own config struct.  It imports nothing from the product package.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LBPF_ORACLE_LIB", os.path.join(HERE, "liblbpf_oracle.so"))

_KIND = {"iso": 0, "sectoral": 1, "cubic": 2, "cubic_hak": 3, "cubic_s": 4}


class OrcAniso(C.Structure):
    _fields_ = [("kind", C.c_int32), ("q", C.c_int32), ("eps", C.c_double),
                ("gamma", C.c_double), ("phi0", C.c_double), ("R", C.c_double * 9)]


class OrcSeed(C.Structure):
    _fields_ = [("x", C.c_double), ("y", C.c_double), ("z", C.c_double),
                ("radius", C.c_double), ("id", C.c_int32)]


class OrcConfig(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("periodic", C.c_int32), ("grad_cd", C.c_int32), ("use_ids", C.c_int32),
                ("W0", C.c_double), ("tau0", C.c_double), ("lam", C.c_double),
                ("kappa", C.c_double), ("delta", C.c_double), ("dx", C.c_double),
                ("dt", C.c_double), ("xi", C.c_double),
                ("n_aniso", C.c_int32), ("aniso", C.POINTER(OrcAniso)),
                ("n_seeds", C.c_int32), ("seeds", C.POINTER(OrcSeed)),
                ("tip_dir", C.c_int32 * 3), ("q_phi", C.c_int32), ("mirror_low", C.c_int32)]


class OrcDiag(C.Structure):
    _fields_ = [("sum_phi", C.c_double), ("sum_u", C.c_double),
                ("sum_u_minus_half_phi", C.c_double), ("solid_fraction", C.c_double),
                ("n_solid", C.c_double), ("tip_position", C.c_double),
                ("nonfinite", C.c_double)]


_lib = None


def load(build_if_missing: bool = True):
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        if not build_if_missing:
            raise RuntimeError(f"oracle library not built: {LIB_PATH}")
        from . import build as _b
        _b.build()
    lib = C.CDLL(LIB_PATH)
    dp = C.POINTER(C.c_double)
    lib.orc_create.argtypes = [C.POINTER(OrcConfig), C.POINTER(C.c_void_p)]
    lib.orc_create.restype = C.c_int
    lib.orc_destroy.argtypes = [C.c_void_p]
    lib.orc_step.argtypes = [C.c_void_p, C.c_int]
    lib.orc_step.restype = C.c_int
    lib.orc_nodes.argtypes = [C.c_void_p]
    lib.orc_nodes.restype = C.c_longlong
    lib.orc_q_phi.argtypes = [C.c_void_p]
    lib.orc_q_u.argtypes = [C.c_void_p]
    for name in ("orc_get_phi", "orc_get_u", "orc_get_g", "orc_get_f"):
        getattr(lib, name).argtypes = [C.c_void_p, dp]
    lib.orc_get_ids.argtypes = [C.c_void_p, C.POINTER(C.c_int16)]
    lib.orc_set_fields.argtypes = [C.c_void_p, dp, dp, C.POINTER(C.c_int16)]
    lib.orc_set_fields.restype = C.c_int
    lib.orc_params.argtypes = [C.c_void_p, dp, dp, dp, dp, dp]
    lib.orc_diagnostics.argtypes = [C.c_void_p, C.POINTER(OrcDiag)]
    lib.orc_lattice.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), dp,
                                C.POINTER(C.c_int), dp]
    lib.orc_lattice.restype = C.c_int
    lib.orc_aniso_eval.argtypes = [C.POINTER(OrcAniso), dp, dp, dp]
    lib.orc_flux.argtypes = [C.POINTER(OrcAniso), dp, dp, dp]
    lib.orc_aniso_min.argtypes = [C.POINTER(OrcAniso), C.c_int]
    lib.orc_aniso_min.restype = C.c_double
    lib.orc_aniso_mirror_symmetric.argtypes = [C.POINTER(OrcAniso), C.c_int]
    lib.orc_aniso_mirror_symmetric.restype = C.c_int
    lib.orc_sharp_interface.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, dp]
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _aniso_struct(a) -> OrcAniso:
    R = getattr(a, "R", None)
    R = [0.0] * 9 if R is None else [float(v) for v in R]
    return OrcAniso(_KIND[a.kind], int(a.q), float(a.eps), float(a.gamma), float(a.phi0),
                    (C.c_double * 9)(*R))


class OracleSim:
    """One simulation advanced by the oracle."""

    def __init__(self, cfg):
        self.cfg = cfg
        self.lib = load()
        an = (OrcAniso * len(cfg.aniso))(*[_aniso_struct(a) for a in cfg.aniso])
        sd = (OrcSeed * max(1, len(cfg.seeds)))(
            *[OrcSeed(float(s.x), float(s.y), float(s.z), float(s.radius), int(s.id))
              for s in cfg.seeds])
        self._keep = (an, sd)
        c = OrcConfig()
        c.dim = 2 if cfg.lattice == "D2Q9_D2Q5" else 3
        c.q_phi = 15 if cfg.lattice == "D3Q15_D3Q7" else 0
        c.nx, c.ny, c.nz = cfg.nx, cfg.ny, cfg.nz
        c.periodic = 1 if cfg.boundary == "periodic" else 0
        c.mirror_low = 1 if cfg.boundary == "mirror_low" else 0
        c.grad_cd = {"dd": 0, "cd": 1, "up2": 2}[cfg.gradient]
        c.use_ids = 1 if cfg.use_ids else 0
        c.W0, c.tau0, c.lam, c.kappa = cfg.W0, cfg.tau0, cfg.lam, cfg.kappa
        c.delta, c.dx, c.dt, c.xi = cfg.delta, cfg.dx, cfg.dt, cfg.xi
        c.n_aniso = len(cfg.aniso)
        c.aniso = an
        c.n_seeds = len(cfg.seeds)
        c.seeds = sd
        c.tip_dir[:] = list(cfg.tip_dir)
        h = C.c_void_p()
        rc = self.lib.orc_create(C.byref(c), C.byref(h))
        if rc != 0:
            err = ValueError(f"orc_create failed: {rc}")
            err.code = rc
            raise err
        self.h = h
        self.N = int(self.lib.orc_nodes(h))
        self.q_phi = int(self.lib.orc_q_phi(h))
        self.q_u = int(self.lib.orc_q_u(h))
        self.shape = tuple(cfg.shape)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.orc_destroy(h)
            self.h = None

    def step(self, n: int = 1) -> None:
        self.lib.orc_step(self.h, int(n))

    def phi(self) -> np.ndarray:
        o = np.empty(self.N)
        self.lib.orc_get_phi(self.h, _dptr(o))
        return o.reshape(self.shape)

    def u(self) -> np.ndarray:
        o = np.empty(self.N)
        self.lib.orc_get_u(self.h, _dptr(o))
        return o.reshape(self.shape)

    def ids(self) -> np.ndarray:
        o = np.empty(self.N, dtype=np.int16)
        self.lib.orc_get_ids(self.h, o.ctypes.data_as(C.POINTER(C.c_int16)))
        return o.reshape(self.shape)

    def g(self) -> np.ndarray:
        o = np.empty(self.N * self.q_phi)
        self.lib.orc_get_g(self.h, _dptr(o))
        return o.reshape((self.q_phi,) + self.shape)

    def f(self) -> np.ndarray:
        o = np.empty(self.N * self.q_u)
        self.lib.orc_get_f(self.h, _dptr(o))
        return o.reshape((self.q_u,) + self.shape)

    def set_fields(self, phi, u, ids=None) -> None:
        phi = np.ascontiguousarray(phi, dtype=np.float64).ravel()
        u = np.ascontiguousarray(u, dtype=np.float64).ravel()
        idp = None
        if ids is not None:
            ids = np.ascontiguousarray(ids, dtype=np.int16).ravel()
            idp = ids.ctypes.data_as(C.POINTER(C.c_int16))
        rc = self.lib.orc_set_fields(self.h, _dptr(phi), _dptr(u), idp)
        if rc != 0:
            raise ValueError("orc_set_fields rejected the fields")

    def params(self) -> dict:
        N = self.N
        p = np.empty(3 * N)
        a = np.empty(N)
        fl = np.empty(3 * N)
        eta = np.empty(N)
        q = np.empty(N)
        self.lib.orc_params(self.h, _dptr(p), _dptr(a), _dptr(fl), _dptr(eta), _dptr(q))
        sh = self.shape
        return {"p": p.reshape(sh + (3,)), "a": a.reshape(sh), "N": fl.reshape(sh + (3,)),
                "eta": eta.reshape(sh), "Q": q.reshape(sh)}

    def diagnostics(self) -> dict:
        d = OrcDiag()
        self.lib.orc_diagnostics(self.h, C.byref(d))
        return {k: getattr(d, k) for k, _ in OrcDiag._fields_}


def lattice(which: str):
    """Lattice tables: which in {'D2Q5', 'D2Q9', 'D3Q7', 'D3Q19', 'D3Q15'}."""
    lib = load()
    idx = {"D2Q5": 0, "D2Q9": 1, "D3Q7": 2, "D3Q19": 3, "D3Q15": 4}[which]
    q = C.c_int()
    e = (C.c_int * 57)()
    w = np.zeros(19)
    opp = (C.c_int * 19)()
    e2 = C.c_double()
    rc = lib.orc_lattice(idx, C.byref(q), e, _dptr(w), opp, C.byref(e2))
    assert rc == 0
    Q = q.value
    return (np.array(e[: 3 * Q]).reshape(Q, 3), w[:Q].copy(), np.array(opp[:Q]), e2.value)


def aniso_eval(entry, n):
    lib = load()
    a = C.c_double()
    G = np.zeros(3)
    nn = np.ascontiguousarray(n, dtype=np.float64)
    s = _aniso_struct(entry)
    lib.orc_aniso_eval(C.byref(s), _dptr(nn), C.byref(a), _dptr(G))
    return a.value, G


def flux(entry, p):
    lib = load()
    a = C.c_double()
    N = np.zeros(3)
    pp = np.ascontiguousarray(p, dtype=np.float64)
    s = _aniso_struct(entry)
    lib.orc_flux(C.byref(s), _dptr(pp), C.byref(a), _dptr(N))
    return a.value, N


def sharp_interface(W0, tau0, lam, kappa):
    """(d0, beta, lambda_star, a1) of Eqs. Capillary-Length / Kinetic-Coeff."""
    lib = load()
    out = np.zeros(4)
    lib.orc_sharp_interface(float(W0), float(tau0), float(lam), float(kappa), _dptr(out))
    return tuple(float(v) for v in out)


def aniso_min(entry, dim: int = 3) -> float:
    """Smallest a_s of the entry over the oracle's fixed direction set."""
    s = _aniso_struct(entry)
    return float(load().orc_aniso_min(C.byref(s), int(dim)))


def aniso_mirror_symmetric(entry, dim: int = 3) -> bool:
    """Whether a_s is unchanged by n_k -> -n_k for every axis of the box."""
    s = _aniso_struct(entry)
    return bool(load().orc_aniso_mirror_symmetric(C.byref(s), int(dim)))

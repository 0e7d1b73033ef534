"""CPU oracle for the SMAME step of arXiv 2012.03525 (TEST INFRASTRUCTURE ONLY).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The GPU library never loads it and
shares no code with it.

`smame_oracle.c` is a plain single-thread FP64 C implementation of the
simplified continuity and momentum updates (Eqs. 2.10-2.13), the body
force, and the two-phase extension in 2D and 3D (surface-tension force,
chemical potential, the Cahn-Hilliard equation 2.14 with Heun's RK2 and the
wetting condition on walls).  This module
compiles it with gcc and exposes it through ctypes with numpy arrays.
`cnn.py` holds the FP64 reference of the learned-closure network.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "smame_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

PERIODIC, WALL, SYMMETRY = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, single thread)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-shared", "-fPIC",
            "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("dx", ctypes.c_double), ("dt", ctypes.c_double), ("nu", ctypes.c_double),
        ("cs", ctypes.c_double), ("rho0", ctypes.c_double),
        ("sat_rho", ctypes.c_double), ("sat_mom", ctypes.c_double),
        ("g", ctypes.c_double * 3),
        ("bc", ctypes.c_int * 6),
        ("wall_u", (ctypes.c_double * 3) * 6),
        ("two_phase", ctypes.c_int),
        ("sigma", ctypes.c_double), ("width", ctypes.c_double), ("mobility", ctypes.c_double),
        ("wet_cos", ctypes.c_double * 6),
        ("axisym", ctypes.c_int),
    ]


@dataclass
class Params:
    """Problem statement of one run (Sec. 2 and Sec. 3 opening paragraph).

    Lattice units by default: dx = dt = 1, cs = 1/sqrt(3) (c = dx/dt, cs = c/sqrt 3).
    bc: six faces (-x,+x,-y,+y,-z,+z), each PERIODIC, WALL or SYMMETRY.
    """
    dim: int
    nx: int
    ny: int
    nz: int = 1
    dx: float = 1.0
    dt: float = 1.0
    nu: float = 0.0
    cs: float = 1.0 / np.sqrt(3.0)
    rho0: float = 1.0
    sat_rho: float = 1.0
    sat_mom: float = 1.0
    g: Sequence[float] = (0.0, 0.0, 0.0)
    bc: Sequence[int] = (0, 0, 0, 0, 0, 0)
    wall_u: Sequence[Sequence[float]] = field(default_factory=lambda: [[0.0] * 3 for _ in range(6)])
    two_phase: bool = False
    sigma: float = 0.0
    width: float = 4.0
    mobility: float = 0.0
    wet_cos: Sequence[float] = (0.0, 0.0, 0.0, 0.0, 0.0, 0.0)  # cos(contact angle) per wall face
    axisym: bool = False  # 2D: x axial, y radial with the axis on the -y face (a symmetry plane)

    def c(self) -> _Params:
        p = _Params()
        p.dim, p.nx, p.ny, p.nz = self.dim, self.nx, self.ny, (self.nz if self.dim == 3 else 1)
        p.dx, p.dt, p.nu, p.cs, p.rho0 = self.dx, self.dt, self.nu, self.cs, self.rho0
        p.sat_rho, p.sat_mom = self.sat_rho, self.sat_mom
        for a in range(3):
            p.g[a] = float(self.g[a])
        for f in range(6):
            p.bc[f] = int(self.bc[f])
            for a in range(3):
                p.wall_u[f][a] = float(self.wall_u[f][a])
        p.two_phase = 1 if self.two_phase else 0
        p.sigma, p.width, p.mobility = self.sigma, self.width, self.mobility
        for f in range(6):
            p.wet_cos[f] = float(self.wet_cos[f])
        p.axisym = 1 if self.axisym else 0
        return p

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx) if self.dim == 3 else (self.ny, self.nx)


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_step.argtypes = [ctypes.POINTER(_Params), dp] + [dp] * 10
        L.orc_step.restype = ctypes.c_int
        L.orc_run.argtypes = [ctypes.POINTER(_Params), dp, ctypes.c_long] + [dp] * 5
        L.orc_run.restype = ctypes.c_int
        L.orc_diag.argtypes = [ctypes.POINTER(_Params)] + [dp] * 9
        L.orc_diag.restype = ctypes.c_int
        L.orc_chemical_potential.argtypes = [ctypes.POINTER(_Params), dp, dp]
        L.orc_chemical_potential.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


FIELDS = ("drho", "u", "v", "w", "phi")


def _state(p: Params, st: dict) -> dict:
    out = {}
    for k in FIELDS:
        if k == "w" and p.dim != 3:
            continue
        if k == "phi" and not p.two_phase:
            continue
        a = np.ascontiguousarray(st[k], dtype=np.float64).reshape(p.shape)
        out[k] = a.copy()
    return out


def step(p: Params, st: dict, force_x_row: Optional[np.ndarray] = None) -> dict:
    """One SMAME step; returns a new state dict."""
    s = _state(p, st)
    o = {k: np.empty_like(v) for k, v in s.items()}
    fx = None if force_x_row is None else np.ascontiguousarray(force_x_row, dtype=np.float64)
    pc = p.c()
    rc = lib().orc_step(ctypes.byref(pc), _ptr(fx),
                        _ptr(s["drho"]), _ptr(s["u"]), _ptr(s["v"]), _ptr(s.get("w")), _ptr(s.get("phi")),
                        _ptr(o["drho"]), _ptr(o["u"]), _ptr(o["v"]), _ptr(o.get("w")), _ptr(o.get("phi")))
    if rc != 0:
        raise ValueError(f"orc_step failed ({rc})")
    return o


def run(p: Params, st: dict, nsteps: int, force_x_row: Optional[np.ndarray] = None) -> dict:
    """nsteps SMAME steps; returns a new state dict."""
    s = _state(p, st)
    fx = None if force_x_row is None else np.ascontiguousarray(force_x_row, dtype=np.float64)
    pc = p.c()
    rc = lib().orc_run(ctypes.byref(pc), _ptr(fx), int(nsteps),
                       _ptr(s["drho"]), _ptr(s["u"]), _ptr(s["v"]), _ptr(s.get("w")), _ptr(s.get("phi")))
    if rc != 0:
        raise ValueError(f"orc_run failed ({rc})")
    return s


DIAG_KEYS = ("mass", "mom_x", "mom_y", "mom_z", "ke", "dumax", "umax", "enstrophy",
             "energy", "div_rms", "div_max", "phi_sum", "nonfinite")


def diag(p: Params, st: dict, prev: Optional[dict] = None) -> dict:
    s = _state(p, st)
    out = np.zeros(13)
    pv = _state(p, prev) if prev is not None else {}
    pc = p.c()
    rc = lib().orc_diag(ctypes.byref(pc), _ptr(s["drho"]), _ptr(s["u"]), _ptr(s["v"]), _ptr(s.get("w")),
                        _ptr(s.get("phi")), _ptr(pv.get("u")), _ptr(pv.get("v")), _ptr(pv.get("w")),
                        _ptr(out))
    if rc != 0:
        raise ValueError(f"orc_diag failed ({rc})")
    return dict(zip(DIAG_KEYS, out.tolist()))


def chemical_potential(p: Params, phi: np.ndarray) -> np.ndarray:
    ph = np.ascontiguousarray(phi, dtype=np.float64).reshape(p.shape).copy()
    mu = np.empty_like(ph)
    pc = p.c()
    rc = lib().orc_chemical_potential(ctypes.byref(pc), _ptr(ph), _ptr(mu))
    if rc != 0:
        raise ValueError(f"orc_chemical_potential failed ({rc})")
    return mu

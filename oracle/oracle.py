"""Python access to the C oracle (vdwlb_oracle.c).

TEST INFRASTRUCTURE ONLY: only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this module.  It shares no code
with the GPU library.

Arrays are numpy float64 (or complex128 for the complex-step build) in the
layout f[c][i][y][x]; parameters follow the paper's notation (Sec. II):
kT, a^{cc'}, b^c, kappa^{cc'}, plus the LB parameters tau, gamma_mu and the
friction coefficients lambda^{cc'} (Eq. forceFriction).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vdwlb_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

ORC_OK, ORC_INVALID, ORC_UNPHYSICAL = 0, 1, 4


def build(force: bool = False) -> str:
    """Compile the oracle (real and complex builds into one shared library)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    objs = []
    for tag, extra in (("re", []), ("cx", ["-DORC_COMPLEX"])):
        obj = os.path.join(_HERE, f"_orc_{tag}.o")
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-Wall", "-fopenmp", "-c", _SRC, "-o", obj] + extra)
        objs.append(obj)
    subprocess.check_call(["gcc", "-shared", "-fopenmp", "-o", tmp] + objs + ["-lm"])
    os.replace(tmp, _LIB)
    for o in objs:
        os.remove(o)
    return _LIB


class _Config(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("nx", ctypes.c_int),
        ("ny", ctypes.c_int),
        ("C", ctypes.c_int),
        ("force", ctypes.c_int),
        ("tau", ctypes.c_double),
        ("gamma_mu", ctypes.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_LIB)
        for sfx in ("", "_cx"):
            for name in ("orc_step", "orc_run", "orc_equilibrium_state", "orc_moments"):
                getattr(_lib, name + sfx).restype = ctypes.c_int
    return _lib


def set_threads(n: int = 0) -> int:
    """Threads for the oracle's per-site loops on lattices of at least 16,384
    sites (n <= 0: the OpenMP default, all host cores); returns the count in
    effect.  Results do not depend on it."""
    L = _load()
    L.orc_set_threads.restype = ctypes.c_int
    return int(L.orc_set_threads(ctypes.c_int(n)))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


@dataclass
class Params:
    """Physical and LB parameters of one lattice (paper notation)."""

    kT: float
    a: np.ndarray
    b: np.ndarray
    kappa: np.ndarray
    tau: float = 1.0
    gamma_mu: float = 1.0
    lam: np.ndarray | None = None
    force: int = 0  # 0 log (Eq. forceMuLog), 1 nid (Eq. forceMuId)

    def __post_init__(self):
        self.a = np.asarray(self.a)
        self.b = np.asarray(self.b)
        self.kappa = np.asarray(self.kappa)
        C = self.b.shape[0]
        if self.lam is None:
            self.lam = np.ones((C, C))
        self.lam = np.asarray(self.lam, dtype=np.float64)

    @property
    def C(self) -> int:
        return int(self.b.shape[0])

    def vector(self, dtype=np.float64) -> np.ndarray:
        C = self.C
        v = np.empty(1 + 2 * C * C + C, dtype=dtype)
        v[0] = self.kT
        v[1 : 1 + C * C] = np.asarray(self.a).reshape(-1)
        v[1 + C * C : 1 + C * C + C] = self.b
        v[1 + C * C + C :] = np.asarray(self.kappa).reshape(-1)
        return v


def _cfg(p: Params, dim: int, nx: int, ny: int) -> _Config:
    return _Config(dim, nx, ny, p.C, p.force, p.tau, p.gamma_mu)


def nq(dim: int) -> int:
    return 3 if dim == 1 else 9


class Lattice:
    """An oracle lattice: state f[c][i][y][x] and the parameters that evolve it."""

    def __init__(self, p: Params, dim: int, nx: int, ny: int, complex_step: bool = False):
        self.p, self.dim, self.nx, self.ny = p, dim, nx, ny
        self.cx = complex_step
        self.dtype = np.complex128 if complex_step else np.float64
        self.sfx = "_cx" if complex_step else ""
        self.cfg = _cfg(p, dim, nx, ny)
        self.shape = (p.C, nq(dim), ny, nx)
        self.f = np.zeros(self.shape, dtype=self.dtype)
        self.prm = p.vector(self.dtype)
        self.status = ORC_OK

    def _fn(self, name):
        return getattr(_load(), name + self.sfx)

    def init(self, rho: np.ndarray, mom: np.ndarray | None = None) -> None:
        rho = np.ascontiguousarray(rho, dtype=self.dtype).reshape(self.p.C, self.ny, self.nx)
        m = None if mom is None else np.ascontiguousarray(mom, dtype=self.dtype).reshape(self.p.C, 2, self.ny, self.nx)
        st = self._fn("orc_equilibrium_state")(ctypes.byref(self.cfg), _ptr(rho), _ptr(m), _ptr(self.f))
        if st != ORC_OK:
            raise ValueError(f"oracle init failed ({st})")

    def run(self, nsteps: int) -> int:
        work = np.empty_like(self.f)
        st = self._fn("orc_run")(
            ctypes.byref(self.cfg), _ptr(self.prm), _ptr(self.p.lam), _ptr(self.f), _ptr(work), ctypes.c_long(nsteps)
        )
        if st == ORC_INVALID:
            raise ValueError("oracle rejected the configuration")
        if st != ORC_OK:
            self.status = st
        return st

    def step_from(self, fin: np.ndarray) -> tuple[np.ndarray, int]:
        fin = np.ascontiguousarray(fin, dtype=self.dtype)
        out = np.empty_like(fin)
        st = self._fn("orc_step")(ctypes.byref(self.cfg), _ptr(self.prm), _ptr(self.p.lam), _ptr(fin), _ptr(out))
        return out, st

    def moments(self):
        """rho [C,ny,nx], mom [C,2,ny,nx], mu [C,ny,nx], p [ny,nx] of the current state."""
        C, ny, nx = self.p.C, self.ny, self.nx
        rho = np.empty((C, ny, nx), self.dtype)
        mom = np.empty((C, 2, ny, nx), self.dtype)
        mu = np.empty((C, ny, nx), self.dtype)
        pr = np.empty((ny, nx), self.dtype)
        st = self._fn("orc_moments")(
            ctypes.byref(self.cfg), _ptr(self.prm), _ptr(self.f), _ptr(rho), _ptr(mom), _ptr(mu), _ptr(pr)
        )
        return rho, mom, mu, pr, st

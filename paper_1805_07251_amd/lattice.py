"""Python front end of the plain sweep: one periodic D2Q9 (or D1Q3) lattice on
the GPU.

torch supplies device memory and the stream; every lattice operation is a
call into libvdwlb.so.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import vdwlb as V

_TORCH_DT = {V.F64: torch.float64, V.F32: torch.float32}


def _dtype_code(dtype) -> int:
    if dtype in ("f64", "float64", torch.float64, np.float64, V.F64):
        return V.F64
    if dtype in ("f32", "float32", torch.float32, np.float32, V.F32):
        return V.F32
    raise ValueError(f"unsupported dtype {dtype!r}")


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Plan:
    """Owns a vdwlb_plan handle."""

    def __init__(self, nx, ny, kT, a, b, kappa, tau=1.0, gamma_mu=1.0, lam=None, dtype="f64", force=V.FORCE_LOG,
                 dim=2):
        self.a = np.ascontiguousarray(a, dtype=np.float64)
        self.b = np.ascontiguousarray(b, dtype=np.float64)
        self.kappa = np.ascontiguousarray(kappa, dtype=np.float64)
        C = self.b.shape[0]
        self.lam = None if lam is None else np.ascontiguousarray(lam, dtype=np.float64)
        self.C, self.nx, self.ny = C, int(nx), int(ny)
        self.dim = int(dim)
        self.Q = 3 if self.dim == 1 else 9
        self.dtype = _dtype_code(dtype)
        self.torch_dtype = _TORCH_DT[self.dtype]
        ptr = lambda arr: arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if arr is not None else None
        d = V.Desc(self.dim, self.nx, self.ny, C, self.dtype, force, float(kT), float(tau), float(gamma_mu),
                   ptr(self.a), ptr(self.b), ptr(self.kappa), ptr(self.lam))
        h = ctypes.c_void_p()
        V.check(V.lib().vdwlb_plan_create(ctypes.byref(d), ctypes.byref(h)), "vdwlb_plan_create")
        self.handle = h
        self.plane = int(V.lib().vdwlb_plane_elems(h))
        self.state_bytes = int(V.lib().vdwlb_state_bytes(h))

    def __del__(self):
        h = getattr(self, "handle", None)
        # at interpreter exit the module globals may already be gone
        lib = getattr(V, "_lib", None) if V is not None else None
        if h is not None and lib is not None:
            lib.vdwlb_plan_destroy(h)
            self.handle = None

    @property
    def state_elems(self) -> int:
        return self.Q * self.C * self.plane


class Lattice:
    """A lattice with its two population buffers on the current CUDA device."""

    def __init__(self, nx, ny, kT, a, b, kappa, tau=1.0, gamma_mu=1.0, lam=None, dtype="f64", force=V.FORCE_LOG,
                 device="cuda", dim=2):
        self.plan = Plan(nx, ny, kT, a, b, kappa, tau, gamma_mu, lam, dtype, force, dim)
        self.device = torch.device(device)
        n = self.plan.state_elems
        self.buf = [torch.empty(n, dtype=self.plan.torch_dtype, device=self.device) for _ in range(2)]
        self.cur = 0
        self.steps_done = 0

    @classmethod
    def from_workload(cls, w, dtype=None, device="cuda"):
        return cls(w.nx, w.ny, w.kT, w.a, w.b, w.kappa, w.tau, w.gamma_mu, w.lam, dtype or w.dtype, w.force, device,
                   getattr(w, "dim", 2))

    @property
    def C(self):
        return self.plan.C

    @property
    def nx(self):
        return self.plan.nx

    @property
    def ny(self):
        return self.plan.ny

    def _field(self, arr, shape):
        t = torch.as_tensor(arr, dtype=self.plan.torch_dtype).to(self.device).contiguous()
        if tuple(t.shape) != shape:
            t = t.reshape(shape)
        return t

    def init(self, rho, mom=None, stream=None):
        r = self._field(rho, (self.C, self.ny, self.nx))
        m = None if mom is None else self._field(mom, (self.C, 2, self.ny, self.nx))
        self.cur = 0
        self.steps_done = 0
        V.check(V.lib().vdwlb_init(self.plan.handle, self.buf[0].data_ptr(), r.data_ptr(),
                                   m.data_ptr() if m is not None else None, _stream_ptr(stream)), "vdwlb_init")
        self._keep = (r, m)  # keep inputs alive until the stream has consumed them

    def run(self, n: int, stream=None) -> None:
        which = ctypes.c_int32()
        a, b = self.buf[self.cur], self.buf[1 - self.cur]
        V.check(V.lib().vdwlb_step(self.plan.handle, a.data_ptr(), b.data_ptr(), int(n), _stream_ptr(stream),
                                   ctypes.byref(which)), "vdwlb_step")
        if which.value == 1:
            self.cur = 1 - self.cur
        self.steps_done += int(n)

    @property
    def Q(self):
        return self.plan.Q

    @property
    def state(self) -> torch.Tensor:
        """The current population buffer in its storage layout [Q, plane, C]
        (velocity planes of sites, the components of a site adjacent)."""
        return self.buf[self.cur].view(self.Q, self.plan.plane, self.C)

    def state_sites(self) -> torch.Tensor:
        """Populations as [C, Q, ny, nx] (a copy without the plane padding)."""
        n = self.nx * self.ny
        return self.state[:, :n, :].permute(2, 0, 1).reshape(self.C, self.Q, self.ny, self.nx).clone()

    def set_state(self, f) -> None:
        """Load populations given as [C, Q, ny, nx] into the current buffer."""
        n = self.nx * self.ny
        t = self._field(f, (self.C, self.Q, self.ny, self.nx)).reshape(self.C, self.Q, n)
        self.state[:, :n, :].copy_(t.permute(1, 2, 0))

    def pressure_tensor(self, rho=None, stream=None):
        """(P_xx, P_yy, P_xy), each [ny, nx], of the density field rho
        [C, ny, nx] (default: the current state's densities)."""
        if rho is None:
            rho = self.moments(want_mu=False, want_p=False, stream=stream)[0]
        r = self._field(rho, (self.C, self.ny, self.nx))
        kw = dict(dtype=self.plan.torch_dtype, device=self.device)
        out = [torch.empty((self.ny, self.nx), **kw) for _ in range(3)]
        V.check(V.lib().vdwlb_pressure_tensor(self.plan.handle, r.data_ptr(), *[t.data_ptr() for t in out],
                                              _stream_ptr(stream)), "vdwlb_pressure_tensor")
        self._keep_p = r  # the input stays alive until the stream has consumed it
        return tuple(out)

    def moments(self, want_mu=True, want_p=True, stream=None):
        """rho [C,ny,nx], mom [C,2,ny,nx], mu [C,ny,nx] or None, p [ny,nx] or None.
        Raises VdwlbError(E_UNPHYSICAL) if the sticky device flag is set."""
        C, ny, nx = self.C, self.ny, self.nx
        kw = dict(dtype=self.plan.torch_dtype, device=self.device)
        rho = torch.empty((C, ny, nx), **kw)
        mom = torch.empty((C, 2, ny, nx), **kw)
        mu = torch.empty((C, ny, nx), **kw) if want_mu else None
        p = torch.empty((ny, nx), **kw) if want_p else None
        st = V.lib().vdwlb_moments(self.plan.handle, self.state.data_ptr(), rho.data_ptr(), mom.data_ptr(),
                                   mu.data_ptr() if mu is not None else None,
                                   p.data_ptr() if p is not None else None, _stream_ptr(stream))
        V.check(st, "vdwlb_moments")
        return rho, mom, mu, p

    def status(self, stream=None) -> int:
        return int(V.lib().vdwlb_sync_status(self.plan.handle, _stream_ptr(stream)))

    def autotune(self, stream=None) -> int:
        """Pick the fastest tile schedule (clobbers the spare buffer only; the
        error flag keeps the state it had before the call)."""
        k = ctypes.c_int32()
        V.check(V.lib().vdwlb_autotune(self.plan.handle, self.buf[self.cur].data_ptr(),
                                       self.buf[1 - self.cur].data_ptr(), _stream_ptr(stream), ctypes.byref(k)),
                "vdwlb_autotune")
        return k.value

    def set_schedule(self, k: int) -> None:
        V.check(V.lib().vdwlb_set_schedule(self.plan.handle, int(k)), "vdwlb_set_schedule")

    def schedule_count(self) -> int:
        return int(V.lib().vdwlb_schedule_count(self.plan.handle))

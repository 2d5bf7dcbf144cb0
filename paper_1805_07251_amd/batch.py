"""Python front end of the batched sweep: many quasi-1-D lattices with their
own sizes and parameters, advanced together by one persistent launch.

torch supplies the two pool buffers and the stream; the instance table,
queue and status words belong to the library.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import vdwlb as V
from .lattice import _dtype_code, _stream_ptr, _TORCH_DT


class Batch:
    def __init__(self, workloads, dtype="f64", device="cuda"):
        self.n = len(workloads)
        if self.n < 1:
            raise ValueError("empty batch")
        self.dtype = _dtype_code(dtype)
        self.torch_dtype = _TORCH_DT[self.dtype]
        self.device = torch.device(device)
        self._keep = []
        descs = (V.Desc * self.n)()
        dptr = lambda arr: arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        for k, w in enumerate(workloads):
            arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (w.a, w.b, w.kappa, w.lam)]
            self._keep.append(arrs)
            descs[k] = V.Desc(getattr(w, "dim", 2), w.nx, w.ny, w.C, self.dtype, w.force, float(w.kT), float(w.tau),
                              float(w.gamma_mu), *[dptr(x) for x in arrs])
        h = ctypes.c_void_p()
        V.check(V.lib().vdwlb_batch_create(self.n, descs, ctypes.byref(h)), "vdwlb_batch_create")
        self.handle = h
        self.shapes = [(w.C, w.ny, w.nx) for w in workloads]
        self.C = workloads[0].C
        self.Q = 3 if getattr(workloads[0], "dim", 2) == 1 else 9
        self.sites = np.array([w.nx * w.ny for w in workloads], dtype=np.int64)
        nbytes = int(V.lib().vdwlb_batch_state_bytes(h))
        elems = nbytes // torch.tensor([], dtype=self.torch_dtype).element_size()
        self.pools = [torch.empty(elems, dtype=self.torch_dtype, device=self.device) for _ in range(2)]
        self.offsets = [int(V.lib().vdwlb_batch_offset(h, k)) for k in range(self.n)]
        self.rho_offsets = [int(V.lib().vdwlb_batch_density_offset(h, k)) for k in range(self.n)]
        self.rho_elems = int(sum(int(np.prod(s)) for s in self.shapes))
        self.cur = 0

    def __del__(self):
        h = getattr(self, "handle", None)
        # at interpreter exit the module globals may already be gone
        lib = getattr(V, "_lib", None) if V is not None else None
        if h is not None and lib is not None:
            lib.vdwlb_batch_destroy(h)
            self.handle = None

    def set_launch(self, threads=256, blocks=0):
        V.check(V.lib().vdwlb_batch_set_launch(self.handle, int(threads), int(blocks)), "vdwlb_batch_set_launch")

    def set_blocking(self, steps_per_block: int):
        """Run in blocks of this many steps held in LDS (2, 4, 8), or step by
        step (0)."""
        V.check(V.lib().vdwlb_batch_set_blocking(self.handle, int(steps_per_block)), "vdwlb_batch_set_blocking")

    def pack(self, arrays) -> torch.Tensor:
        flat = np.concatenate([np.asarray(a, dtype=np.float64).reshape(-1) for a in arrays])
        return torch.as_tensor(flat, dtype=self.torch_dtype).to(self.device)

    def init(self, rho_list, stream=None):
        r = self.pack(rho_list)
        self.cur = 0
        V.check(V.lib().vdwlb_batch_init(self.handle, self.pools[0].data_ptr(), r.data_ptr(), _stream_ptr(stream)),
                "vdwlb_batch_init")
        self._rho_in = r

    def run(self, nsteps: int, stream=None):
        which = ctypes.c_int32()
        a, b = self.pools[self.cur], self.pools[1 - self.cur]
        V.check(V.lib().vdwlb_batch_run(self.handle, a.data_ptr(), b.data_ptr(), int(nsteps), _stream_ptr(stream),
                                        ctypes.byref(which)), "vdwlb_batch_run")
        if which.value == 1:
            self.cur = 1 - self.cur

    def status(self, stream=None) -> np.ndarray:
        st = (ctypes.c_int32 * self.n)()
        V.lib().vdwlb_batch_status(self.handle, st, _stream_ptr(stream))
        return np.array(st[:], dtype=np.int32)

    def densities(self, stream=None):
        out = torch.empty(self.rho_elems, dtype=self.torch_dtype, device=self.device)
        V.check(V.lib().vdwlb_batch_density(self.handle, self.pools[self.cur].data_ptr(), out.data_ptr(),
                                            _stream_ptr(stream)), "vdwlb_batch_density")
        return [out[o:o + int(np.prod(s))].view(*s) for o, s in zip(self.rho_offsets, self.shapes)]

    def state(self, k) -> torch.Tensor:
        """Populations of instance k as [C, Q, ny, nx] (a copy)."""
        C, ny, nx = self.shapes[k]
        Q = self.Q
        plane = (nx * ny + 63) // 64 * 64
        v = self.pools[self.cur][self.offsets[k]:self.offsets[k] + Q * C * plane].view(Q, plane, C)
        return v[:, :nx * ny, :].permute(2, 0, 1).reshape(C, Q, ny, nx).clone()

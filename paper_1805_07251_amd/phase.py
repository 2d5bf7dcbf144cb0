"""Phase diagrams of two-component mixtures on the GPU (Appendix A).

`phase_points` marshals arguments for `vdwlb_phase_points`: every step (the
stability test, the three-phase direct search, the classification and the
Newton polish of the coexistence conditions) runs in the library's kernels.
`composition_grid` lays out the (A, B) points the paper loops over: a regular
grid below the line b . N = 1 that joins the two van der Waals
discontinuities.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import vdwlb as V

STATUS_INVALID, STATUS_FAILED, STATUS_STABLE = -1, 0, 1


def phase_points(kT, a, b, NA, NB, threshold=1e-12, max_iter=200000, stream=None):
    """Run the Appendix A pipeline on the overall compositions (NA[k], NB[k]).

    NA, NB: float64 CUDA tensors (or array-likes, copied to the GPU) of equal
    length.  Returns a dict of CUDA tensors: phases [n, 3, 3] (rho_A, rho_B, V
    of the distinct phases), raw [n, 3, 3] (the search's three phases), F [n],
    status, iterations, n_unstable, polished [n] (int32).  Asynchronous on the
    stream; the caller synchronises before reading on the host."""
    NA = torch.as_tensor(NA, dtype=torch.float64).to("cuda").contiguous().reshape(-1)
    NB = torch.as_tensor(NB, dtype=torch.float64).to("cuda").contiguous().reshape(-1)
    if NA.numel() != NB.numel():
        raise ValueError("NA and NB must have the same length")
    n = NA.numel()
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(4)
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(2)
    phases = torch.empty((n, 3, 3), dtype=torch.float64, device="cuda")
    raw = torch.empty((n, 3, 3), dtype=torch.float64, device="cuda")
    F = torch.empty(n, dtype=torch.float64, device="cuda")
    info = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    s = (stream or torch.cuda.current_stream()).cuda_stream
    dp = ctypes.POINTER(ctypes.c_double)
    V.check(V.lib().vdwlb_phase_points(float(kT), a.ctypes.data_as(dp), b.ctypes.data_as(dp), n, NA.data_ptr(),
                                       NB.data_ptr(), float(threshold), int(max_iter), phases.data_ptr(),
                                       raw.data_ptr(), F.data_ptr(), info.data_ptr(), s), "vdwlb_phase_points")
    return {"phases": phases, "raw": raw, "F": F, "status": info[:, 0], "iterations": info[:, 1],
            "n_unstable": info[:, 2], "polished": info[:, 3], "_keep": (NA, NB)}


def composition_grid(b, n, margin=1e-3):
    """Points (A, B) = ((i + 1/2) / (n b_A), (j + 1/2) / (n b_B)) of an n x n
    grid with b . N <= 1 - margin (below the line joining the excluded-volume
    limits 1/b^c of the pure components).  Returns two float64 numpy arrays."""
    b = np.asarray(b, dtype=np.float64)
    u = (np.arange(n) + 0.5) / n
    A, B = np.meshgrid(u / b[0], u / b[1], indexing="xy")
    keep = b[0] * A + b[1] * B <= 1.0 - margin
    return A[keep].ravel(), B[keep].ravel()

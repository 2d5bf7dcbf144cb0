"""Helpers shared by the GPU tests: run the oracle and the GPU library on the
same seeded workload."""
from __future__ import annotations

import numpy as np

VX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
VY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def oracle_params(orc, w):
    return orc.Params(w.kT, w.a, w.b, w.kappa, tau=w.tau, gamma_mu=w.gamma_mu, lam=w.lam, force=w.force)


def oracle_run(orc, w, nsteps, rho=None, dim=2):
    """Oracle lattice for workload w initialised from rho (default w.rho), run nsteps."""
    lat = orc.Lattice(oracle_params(orc, w), dim, w.nx, w.ny)
    lat.init(w.rho if rho is None else rho)
    st = lat.run(nsteps) if nsteps else 0
    return lat, st


def window_rho(orc, w, x, y, k):
    """rho^c at site (x, y) after k steps of the full periodic lattice of w,
    computed by the oracle on a periodic window of half-width 3k + 2 centred
    on (x, y): one step reaches 3 sites (pull radius 1, potential gradient
    radius 2) and the final moments pull once more, so the wrapped edges of
    the window cannot reach the centre."""
    R = 3 * k + 2
    W = 2 * R + 1
    xs = (x + np.arange(-R, R + 1)) % w.nx
    ys = (y + np.arange(-R, R + 1)) % w.ny
    sub = w.rho[:, ys][:, :, xs]
    lat = orc.Lattice(oracle_params(orc, w), 2, W, W)
    lat.init(sub)
    lat.run(k)
    rho, _, _, _, _ = lat.moments()
    return rho[:, R, R]


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / np.abs(b).max())

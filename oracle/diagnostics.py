"""Pressure tensor of a density field (oracle side).

TEST INFRASTRUCTURE ONLY: used by the test suite to check the GPU diagnostic
kernel.  Shares no code with the GPU library.

The tensor is the one of Sec. II that obeys the Gibbs-Duhem relation
(Eq. GibbsDuehem) for the van der Waals mixture free energy:

    P_ab = sum_c [ rho^c kT / (1 - eta) - sum_c' a^{cc'} rho^c rho^c'
                   - sum_c' kappa^{cc'} (grad rho^c . grad rho^c' + rho^c Lap rho^c') ] delta_ab
           + sum_{cc'} kappa^{cc'} d_a rho^c d_b rho^c'

with the lattice's own stencils for the derivatives: the isotropic
gradient 3 sum_i w_i v_i g(x + v_i) and Laplacian 6 sum_i w_i (g(x + v_i) - g(x))
of the D2Q9 (or D1Q3) velocity set, evaluated here with periodic shifts of the
whole field, one velocity at a time.
"""
from __future__ import annotations

import numpy as np

_D2 = [((0, 0), 4 / 9), ((1, 0), 1 / 9), ((0, 1), 1 / 9), ((-1, 0), 1 / 9), ((0, -1), 1 / 9),
       ((1, 1), 1 / 36), ((-1, 1), 1 / 36), ((-1, -1), 1 / 36), ((1, -1), 1 / 36)]
_D1 = [((0, 0), 2 / 3), ((1, 0), 1 / 6), ((-1, 0), 1 / 6)]


def _shift(g, vx, vy):
    """g(x + v) for a periodic field g[..., y, x]."""
    return np.roll(np.roll(g, -vy, axis=-2), -vx, axis=-1)


def gradient(g, dim=2):
    """(d_x g, d_y g) with the isotropic stencil 3 sum_i w_i v_i g(x + v_i)."""
    vel = _D2 if dim == 2 else _D1
    gx = np.zeros_like(g)
    gy = np.zeros_like(g)
    for (vx, vy), w in vel[1:]:
        s = _shift(g, vx, vy)
        gx = gx + 3 * w * vx * s
        gy = gy + 3 * w * vy * s
    return gx, gy


def laplacian(g, dim=2):
    """6 sum_i w_i (g(x + v_i) - g(x))."""
    vel = _D2 if dim == 2 else _D1
    out = np.zeros_like(g)
    for (vx, vy), w in vel[1:]:
        out = out + 6 * w * (_shift(g, vx, vy) - g)
    return out


def pressure_tensor(rho, kT, a, b, kappa, dim=2):
    """P_xx, P_yy, P_xy of the density field rho[c][y][x] (Sec. II)."""
    rho = np.asarray(rho, dtype=float)
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    kappa = np.asarray(kappa, dtype=float)
    C = rho.shape[0]
    eta = np.tensordot(b, rho, axes=1)
    scalar = rho.sum(0) * kT / (1.0 - eta)
    grads = [gradient(rho[c], dim) for c in range(C)]
    laps = [laplacian(rho[c], dim) for c in range(C)]
    pxx = np.zeros_like(scalar)
    pyy = np.zeros_like(scalar)
    pxy = np.zeros_like(scalar)
    for c in range(C):
        for d in range(C):
            gg = grads[c][0] * grads[d][0] + grads[c][1] * grads[d][1]
            scalar = scalar - a[c, d] * rho[c] * rho[d] - kappa[c, d] * (gg + rho[c] * laps[d])
            pxx = pxx + kappa[c, d] * grads[c][0] * grads[d][0]
            pyy = pyy + kappa[c, d] * grads[c][1] * grads[d][1]
            pxy = pxy + kappa[c, d] * grads[c][0] * grads[d][1]
    return scalar + pxx, scalar + pyy, pxy

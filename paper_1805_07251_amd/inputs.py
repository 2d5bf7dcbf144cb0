"""Seeded synthetic inputs for the lattice sweep (shared by tests and benchmark).

This module only draws random numbers and lays out parameter sets and initial
density fields; it contains none of the lattice Boltzmann arithmetic.  Both the
GPU library and the CPU oracle receive the arrays produced here.

Draw order is fixed: scalar parameters first (in the order listed for each
workload), then fields in [c][y][x] order, all from one
numpy.random.default_rng(seed) stream.

Workloads (sizes follow the paper's own regime of small quasi-1-D lattices and
long runs, Sec. VI, and the 2-D extension it announces in Sec. VII):
  spinodal_small   D2Q9, 2 components, 64x64, FP64, equal split at packing
                   fraction 0.5, a12 = 0.9 a11, +-1 % multiplicative noise
  spinodal_large   2048x2048, a12 drawn in [0.7, 1.1] a11, otherwise as above
  mixture4         1024x1024, 4 components: a_ij in [0.6, 1.0] a_ii,
                   b_i in [0.08, 0.12], Dirichlet(1,1,1,1) composition at
                   total density 0.4 / b_mean
  batch_slabs      many quasi-1-D L x 4 lattices with a tanh liquid slab
                   (bulk densities from a caller-supplied coexistence solver)
  adjoint_case     256x256, spinodal_small parameters plus a smooth target
  binary_mixture   a^{cc'}, b^c of the Sec. VI.A phase-diagram mixtures from
                   their critical temperatures, critical densities and nu
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# One van der Waals component with critical temperature 4/7 and critical
# density 7/2 (a = 9/49, b = 2/21; Eqs. tetcr and rhocr).
A11 = 9.0 / 49.0
B1 = 2.0 / 21.0
KT_CRIT = 4.0 / 7.0
KAPPA = 0.1
# gamma_mu from the paper's stability rule c_s^2 = 1 - 4 kappa rho_l gamma_mu
# (Eq. kappaGammaMuRelation) with c_s^2 = 1/3, kappa = 0.1 and the liquid
# density 6.7645 of the component above at 0.8 kT_cr, rounded to 0.25.
GAMMA_MU = 0.25


@dataclass
class Workload:
    """Parameters and initial densities of one lattice."""

    nx: int
    ny: int
    kT: float
    a: np.ndarray
    b: np.ndarray
    kappa: np.ndarray
    rho: np.ndarray  # [C, ny, nx]
    tau: float = 1.0
    gamma_mu: float = GAMMA_MU
    lam: np.ndarray = field(default=None)
    force: int = 0
    dtype: str = "f64"
    name: str = ""
    dim: int = 2  # 2: D2Q9, 1: D1Q3 (ny = 1)

    def __post_init__(self):
        C = self.b.shape[0]
        if self.lam is None:
            self.lam = np.ones((C, C))

    @property
    def C(self) -> int:
        return int(self.b.shape[0])


def kappa_matrix(a: np.ndarray, kappa: float = KAPPA) -> np.ndarray:
    """kappa^{cc} = kappa, kappa^{cc'} = nu^{cc'} kappa with nu^{cc'} the
    mixing factor a^{cc'} / sqrt(a^{cc} a^{c'c'}) (Sec. VI.A uses the same nu
    for the interface terms)."""
    d = np.sqrt(np.diag(a))
    return kappa * a / np.outer(d, d)


def _noise_field(rng, mean: np.ndarray, ny: int, nx: int, amp: float = 0.01) -> np.ndarray:
    C = mean.shape[0]
    u = rng.uniform(-amp, amp, size=(C, ny, nx))
    return mean[:, None, None] * (1.0 + u)


def spinodal_small(seed: int = 0, n: int = 64, nu: float = 0.9, dtype: str = "f64") -> Workload:
    rng = np.random.default_rng(seed)
    a = np.array([[A11, nu * A11], [nu * A11, A11]])
    b = np.array([B1, B1])
    kT = 0.8 * KT_CRIT
    mean = np.full(2, 0.5 / B1 / 2.0)
    rho = _noise_field(rng, mean, n, n)
    return Workload(n, n, kT, a, b, kappa_matrix(a), rho, dtype=dtype, name=f"spinodal {n}x{n} C=2")


def spinodal_large(seed: int = 0, n: int = 2048, dtype: str = "f64") -> Workload:
    rng = np.random.default_rng(seed)
    nu = float(rng.uniform(0.7, 1.1))
    a = np.array([[A11, nu * A11], [nu * A11, A11]])
    b = np.array([B1, B1])
    kT = 0.8 * KT_CRIT
    mean = np.full(2, 0.5 / B1 / 2.0)
    rho = _noise_field(rng, mean, n, n)
    return Workload(n, n, kT, a, b, kappa_matrix(a), rho, dtype=dtype, name=f"spinodal {n}x{n} C=2 nu={nu:.4f}")


def mixture4(seed: int = 0, n: int = 1024, dtype: str = "f32", C: int = 4) -> Workload:
    rng = np.random.default_rng(seed)
    a = np.full((C, C), A11)
    for i in range(C):
        for j in range(i + 1, C):
            a[i, j] = a[j, i] = A11 * rng.uniform(0.6, 1.0)
    b = rng.uniform(0.08, 0.12, size=C)
    x = rng.dirichlet(np.ones(C))
    b_mean = float(np.dot(x, b))
    rho_tot = 0.4 / b_mean
    # 0.8 of the critical temperature 8 a_ii / (27 b_mean) of the mean fluid
    kT = 0.8 * 8.0 * A11 / (27.0 * b_mean)
    rho = _noise_field(rng, rho_tot * x, n, n)
    # gamma_mu by the same rule as above, liquid density scaled by 1/b_mean
    gamma = GAMMA_MU * B1 / b_mean
    return Workload(n, n, kT, a, b, kappa_matrix(a), rho, gamma_mu=gamma, dtype=dtype,
                    name=f"mixture {n}x{n} C={C}")


@dataclass
class SlabDraw:
    """Per-instance draws of the batched quasi-1-D workload."""

    L: np.ndarray  # x extents
    t: np.ndarray  # kT / kT_crit
    xbar: np.ndarray  # mean mole fraction of component 1
    nu: np.ndarray  # a12 / a11


def batch_draws(seed: int = 0, n: int = 1024, lmin: int = 128, lmax: int = 1024) -> SlabDraw:
    rng = np.random.default_rng(seed)
    L = rng.integers(lmin, lmax + 1, size=n)
    t = rng.uniform(0.6, 1.0, size=n)
    xbar = rng.uniform(0.05, 0.95, size=n)
    nu = rng.uniform(0.6, 1.2, size=n)
    return SlabDraw(L, t, xbar, nu)


def one_fluid_a(xbar: float, nu: float) -> float:
    """Attraction of the one-fluid approximation of a binary mixture of mole
    fraction xbar: sum_cd x_c x_d a^{cd} with a^{12} = nu a^{11} = nu a^{22}.
    Callers use it to pick the bulk densities of the initial slab."""
    return A11 * (xbar * xbar + (1.0 - xbar) ** 2 + 2.0 * nu * xbar * (1.0 - xbar))


def slab_instance(L: int, ny: int, t: float, xbar: float, nu: float, rho_gas: float, rho_liq: float,
                  width: float = 2.0, dim: int = 2) -> Workload:
    """One quasi-1-D lattice: a liquid slab between x = L/4 and 3L/4 with tanh
    edges of the given width (Sec. V initialises with tanh profiles), bulk
    total densities rho_liq / rho_gas supplied by the caller, uniform mole
    fraction xbar, y-uniform (dim = 1: a D1Q3 line, ny = 1).  gamma_mu is
    half the value of the rule
    c_s^2 = 1 - 4 kappa rho_l gamma_mu (Eq. kappaGammaMuRelation): Sec. VI.A
    lowers gamma_mu by factors of 2 to 10 for runs that are unstable at the
    rule's value."""
    a = np.array([[A11, nu * A11], [nu * A11, A11]])
    b = np.array([B1, B1])
    x = np.arange(L) + 0.5
    tot = rho_gas + (rho_liq - rho_gas) * 0.5 * (np.tanh((x - L / 4) / width) - np.tanh((x - 3 * L / 4) / width))
    rho = np.empty((2, ny, L))
    rho[0] = (xbar * tot)[None, :]
    rho[1] = ((1.0 - xbar) * tot)[None, :]
    gamma = 0.5 * (1.0 - 1.0 / 3.0) / (4.0 * KAPPA * rho_liq)
    return Workload(L, ny, t * KT_CRIT, a, b, kappa_matrix(a), rho, gamma_mu=gamma, name=f"slab L={L}", dim=dim)


def batch_slabs(maxwell, seed: int = 0, n: int = 1024, ny: int = 4, idx=None, lmax=None, dim: int = 2):
    """The batched phase-diagram workload: n quasi-1-D L x ny lattices with L
    uniform in [128, 1024], kT in [0.6, 1.0] kT_crit, mole fraction in
    [0.05, 0.95] and a12/a11 in [0.6, 1.2], each initialised with a liquid
    slab.  maxwell(a, b, kT) -> (rho_gas, rho_liquid) or None supplies the
    bulk densities of the one-fluid approximation of each mixture (uniform
    density 0.5 / b when it is above its critical temperature).  dim = 1
    gives the same draws as D1Q3 lines (ny is then 1)."""
    d = batch_draws(seed, n)
    out = []
    for k in (range(n) if idx is None else idx):
        L = int(d.L[k]) if lmax is None else int(min(d.L[k], lmax))
        m = maxwell(one_fluid_a(d.xbar[k], d.nu[k]), B1, d.t[k] * KT_CRIT)
        rg, rl = m if m else (0.5 / B1, 0.5 / B1)
        out.append(slab_instance(L, 1 if dim == 1 else ny, d.t[k], d.xbar[k], d.nu[k], rg, rl, dim=dim))
    return out


def line_spinodal(seed: int = 0, L: int = 512, C: int = 2, nu: float = 0.9, dtype: str = "f64") -> Workload:
    """The spinodal_small parameters on a D1Q3 line of L sites (Sec. V's own
    lattice): C components split equally at packing fraction 0.5, +-1 %
    multiplicative noise."""
    a = np.full((C, C), nu * A11)
    np.fill_diagonal(a, A11)
    b = np.full(C, B1)
    rng = np.random.default_rng(seed)
    rho = _noise_field(rng, np.full(C, 0.5 / (B1 * C)), 1, L)
    return Workload(L, 1, 0.8 * KT_CRIT, a, b, kappa_matrix(a), rho, dtype=dtype, name=f"line L={L} C={C}", dim=1)


def adjoint_case(seed: int = 0, n: int = 256):
    """spinodal_small parameters at n x n plus the smooth target of the
    density-profile loss: rho1_bar (1 + 0.05 g(x)), g a sum of four seeded
    cosines with |k| <= 4 (2 pi / n), normalised to max |g| = 1."""
    w = spinodal_small(seed, n)
    rng = np.random.default_rng(seed + 1000)
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    g = np.zeros((n, n))
    for _ in range(4):
        kx, ky = rng.integers(-4, 5, size=2)
        ph = rng.uniform(0, 2 * np.pi)
        g += np.cos(2 * np.pi * (kx * xx + ky * yy) / n + ph)
    g /= np.abs(g).max()
    target = w.rho[0].mean() * (1.0 + 0.05 * g)
    return w, target


def binary_mixture(theta_cr_a: float, theta_cr_b: float, rho_cr_a: float, rho_cr_b: float, nu: float):
    """(a [2x2], b [2]) of a two-component mixture specified the way Sec. VI.A
    specifies its phase diagrams: each component's critical temperature and
    density fix b = 1/(3 rho_cr) and a = 9 theta_cr / (8 rho_cr) (Eqs. tetcr,
    rhocr solved for a and b), and a^{AB} = nu sqrt(a^A a^B) (Eq. vdwConstantAB)."""
    aa = 9.0 * theta_cr_a / (8.0 * rho_cr_a)
    ab = 9.0 * theta_cr_b / (8.0 * rho_cr_b)
    cross = nu * np.sqrt(aa * ab)
    return np.array([[aa, cross], [cross, ab]]), np.array([1.0 / (3.0 * rho_cr_a), 1.0 / (3.0 * rho_cr_b)])


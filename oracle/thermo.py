"""Bulk thermodynamics of the van der Waals mixture free energy (oracle side).

TEST INFRASTRUCTURE ONLY: used by the test suite to pin the lattice Boltzmann
oracle and the GPU library against quantities the paper fixes independently of
any lattice update.  Shares no code with the GPU library.

Notation follows Sec. II of the paper: densities rho^c, kT = theta, attraction
a^{cc'}, excluded volume b^c, packing eta = sum_c b^c rho^c.

Contents
  critical_point           Eqs. tetcr, rhocr, pcr
  two_component_params     the (theta_cr^A, theta_cr^B, rho_cr^B, nu) mapping of
                           Sec. VI.A with the geometric mixing rule of Eq.
                           vdwConstantAB (read as a = 9 theta_cr / (8 rho_cr),
                           which is what Eqs. tetcr/rhocr give)
  vks_parameters           van Konynenburg-Scott xi, zeta, Lambda (Sec. VI.A)
  free_energy_density      bulk part of Eq. continuousFreeEnergy
  chemical_potential       d f / d rho^c (including the +kT constant)
  pressure                 bulk pressure of Sec. II
  hessian                  the 2x2 (CxC) Hessian of Sec. VI.A
  maxwell_single           liquid-gas coexistence of one component
  coexistence_two_phase    common tangent between two bulk phases (Newton)
  minimize_three_phase     the quasi-brute-force direct search of Appendix A
                           (direct_search also returns its iteration count)
  phase_point              one (A, B) point of a phase diagram: stability test,
                           direct search, classification, Newton polish
  coexistence_invariant_point  C + 1 coexisting phases of C components (equal
                           mu^c and p in all phases; Newton from a start),
                           coexistence_three_phase the C = 2 case
  gamma_from_width_rule    gamma_mu from Eq. kappaGammaMuRelation
"""
from __future__ import annotations

import numpy as np

THETA_LB = 1.0 / 3.0


def critical_point(a: float, b: float):
    """(kT_cr, rho_cr, p_cr) of one van der Waals component (Eqs. tetcr, rhocr, pcr)."""
    return 8.0 * a / (27.0 * b), 1.0 / (3.0 * b), a / (27.0 * b * b)


def two_component_params(theta_cr_a: float, theta_cr_b: float, rho_cr_b: float, nu: float, rho_cr_a: float = 1.0):
    """a^{cc'} (2x2) and b^c from critical temperatures/densities (Sec. VI.A).

    Inverting Eqs. tetcr and rhocr gives b = 1/(3 rho_cr) and
    a = 27 b theta_cr / 8 = 9 theta_cr / (8 rho_cr).  The cross term follows
    the geometric mixing rule a^{AB} = nu sqrt(a^A a^B) (Eq. vdwConstantAB).
    """
    aA = 9.0 * theta_cr_a / (8.0 * rho_cr_a)
    aB = 9.0 * theta_cr_b / (8.0 * rho_cr_b)
    bA = 1.0 / (3.0 * rho_cr_a)
    bB = 1.0 / (3.0 * rho_cr_b)
    aAB = nu * np.sqrt(aA * aB)
    return np.array([[aA, aAB], [aAB, aB]]), np.array([bA, bB])


def vks_parameters(a: np.ndarray, b: np.ndarray):
    """(xi, zeta, Lambda) of van Konynenburg and Scott for a binary mixture (Sec. VI.A)."""
    pa = a[0, 0] / b[0] ** 2
    pb = a[1, 1] / b[1] ** 2
    xi = (b[1] - b[0]) / (b[0] + b[1])
    zeta = (pb - pa) / (pa + pb)
    lam = (pa - 2.0 * a[0, 1] / (b[0] * b[1]) + pb) / (pa + pb)
    return xi, zeta, lam


def _eta(rho, b):
    return float(np.dot(b, rho))


def free_energy_density(rho, kT, a, b):
    """f(rho) = sum_c rho^c kT ln(rho^c/(1-eta)) - sum_{cc'} a^{cc'} rho^c rho^c'."""
    rho = np.asarray(rho, dtype=float)
    eta = _eta(rho, b)
    return float(np.sum(rho * kT * np.log(rho / (1.0 - eta))) - rho @ a @ rho)


def chemical_potential(rho, kT, a, b):
    """Full bulk chemical potential d f / d rho^c (keeps the +kT constant)."""
    rho = np.asarray(rho, dtype=float)
    eta = _eta(rho, b)
    tot = rho.sum()
    return kT * (np.log(rho / (1.0 - eta)) + 1.0 + b * tot / (1.0 - eta)) - 2.0 * (a @ rho)


def pressure(rho, kT, a, b):
    """Bulk pressure p = sum_c rho^c kT/(1-eta) - sum a rho rho (Sec. II)."""
    rho = np.asarray(rho, dtype=float)
    eta = _eta(rho, b)
    return float(rho.sum() * kT / (1.0 - eta) - rho @ a @ rho)


def hessian(rho, kT, a, b):
    """H_cd = d^2 f / d rho^c d rho^d of the bulk free-energy density."""
    rho = np.asarray(rho, dtype=float)
    b = np.asarray(b, dtype=float)
    eta = _eta(rho, b)
    tot = rho.sum()
    g = 1.0 - eta
    H = kT * (np.diag(1.0 / rho) + (b[:, None] + b[None, :]) / g + np.outer(b, b) * tot / g**2) - 2.0 * np.asarray(a)
    return H


def maxwell_single(a: float, b: float, kT: float, tol: float = 1e-15, maxit: int = 200):
    """Coexisting (rho_gas, rho_liquid) of one component at kT < kT_cr.

    Newton on mu(rho_g) = mu(rho_l), p(rho_g) = p(rho_l), started from the
    spinodal-bracketed guesses; returns None above the critical temperature.
    """
    kTc, rc, _ = critical_point(a, b)
    if kT >= kTc:
        return None

    def mu(r):
        return kT * (np.log(r / (1 - b * r)) + 1 + b * r / (1 - b * r)) - 2 * a * r

    def dmu(r):
        return kT / (r * (1 - b * r) ** 2) - 2 * a

    def p(r):
        return r * kT / (1 - b * r) - a * r * r

    def dp(r):
        return kT / (1 - b * r) ** 2 - 2 * a * r

    def bisect(fn, lo, hi):
        flo = fn(lo)
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            fm = fn(mid)
            if (fm > 0) == (flo > 0):
                lo, flo = mid, fm
            else:
                hi = mid
        return 0.5 * (lo + hi)

    # Start: the spinodals (dp/drho = 0) bracket the van der Waals loop; the
    # guesses are the outer-branch densities at the mid-loop pressure.
    sp_lo = bisect(dp, 1e-12, rc)
    sp_hi = bisect(dp, rc, (1 - 1e-12) / b)
    p_star = 0.5 * (max(p(sp_hi), 0.0) + p(sp_lo))
    rg = bisect(lambda r: p(r) - p_star, 1e-300, sp_lo)
    rl = bisect(lambda r: p(r) - p_star, sp_hi, (1 - 1e-15) / b)
    for _ in range(maxit):
        F = np.array([mu(rg) - mu(rl), p(rg) - p(rl)])
        J = np.array([[dmu(rg), -dmu(rl)], [dp(rg), -dp(rl)]])
        step = np.linalg.solve(J, F)
        # damp to stay inside the physical domain
        lam = 1.0
        while True:
            ng, nl = rg - lam * step[0], rl - lam * step[1]
            if ng > 0 and nl * b < 1 and nl > ng:
                break
            lam *= 0.5
        rg, rl = ng, nl
        if np.max(np.abs(lam * step) / np.array([rg, rl])) < tol:
            break
    return rg, rl


def coexistence_two_phase(rho_bar, rho_alpha, rho_beta, kT, a, b, tol=1e-14, maxit=100):
    """Two coexisting bulk phases of overall composition rho_bar (common tangent).

    Unknowns: the densities of phases alpha and beta and the volume fraction
    phi of alpha.  Equations: equal mu^c, equal p (Sec. II), and the lever rule
    phi rho_alpha + (1 - phi) rho_beta = rho_bar.  Solved by Newton with a
    central-difference Jacobian, from the given starting phases.
    """
    rho_bar = np.asarray(rho_bar, dtype=float)
    C = rho_bar.size
    ra = np.asarray(rho_alpha, dtype=float)
    rb = np.asarray(rho_beta, dtype=float)
    d = ra - rb
    phi0 = float(np.dot(rho_bar - rb, d) / np.dot(d, d))

    def resid(z):
        xa, xb, phi = z[:C], z[C:2 * C], z[2 * C]
        return np.concatenate([chemical_potential(xa, kT, a, b) - chemical_potential(xb, kT, a, b),
                               [pressure(xa, kT, a, b) - pressure(xb, kT, a, b)],
                               phi * xa + (1.0 - phi) * xb - rho_bar])

    z = np.concatenate([ra, rb, [phi0]])
    n = z.size
    for _ in range(maxit):
        F = resid(z)
        J = np.empty((n, n))
        for k in range(n):
            dz = np.zeros(n)
            dz[k] = 1e-7 * max(1.0, abs(z[k]))
            J[:, k] = (resid(z + dz) - resid(z - dz)) / (2 * dz[k])
        step = np.linalg.solve(J, F)
        lam = 1.0
        while True:
            t = z - lam * step
            if np.all(t[:2 * C] > 0) and np.dot(b, t[:C]) < 1 and np.dot(b, t[C:2 * C]) < 1:
                break
            lam *= 0.5
        z = t
        if np.max(np.abs(lam * step)) < tol * max(1.0, np.max(np.abs(z))):
            break
    return z[:C], z[C:2 * C], float(z[2 * C])


def minimize_three_phase(NA: float, NB: float, kT, a, b, threshold=1e-12, max_iter=200000):
    """Quasi-brute-force three-phase free-energy minimisation (Appendix A).

    Total volume 1 with particle numbers (NA, NB).  Phases 1 and 2 carry six
    free variables (A1, B1, V1, A2, B2, V2); phase 3 follows from
    conservation.  Each iteration evaluates the 6 x 3 array of trial moves
    (each variable moved by +step, 0, -step), accepts the lowest total free
    energy if it improves, otherwise halves the step; it stops once the step
    no longer changes the free energy by more than the threshold.  The first
    split follows the unstable eigenvector of the Hessian at (NA, NB).
    Returns a list of (rho_A, rho_B, V) per phase with V > 0.
    """
    phases, F, _ = direct_search(NA, NB, kT, a, b, threshold, max_iter)
    return phases, F


def unstable_direction(H):
    """Unit eigenvector of the lowest eigenvalue of the symmetric 2 x 2 H,
    with its sign fixed (first component >= 0; the second > 0 if the first
    is zero): the paper only says the split follows this eigenvector."""
    w, v = np.linalg.eigh(np.asarray(H, dtype=float))
    d = v[:, 0].copy()
    if d[0] < 0 or (d[0] == 0 and d[1] < 0):
        d = -d
    return d


def _free_energy_ext(rho, kT, a, b):
    """free_energy_density extended to empty components (rho^c ln rho^c -> 0)."""
    rho = np.asarray(rho, dtype=float)
    g = 1.0 - _eta(rho, b)
    ent = sum(rho[c] * kT * np.log(rho[c] / g) for c in range(rho.size) if rho[c] > 0)
    return float(ent - rho @ a @ rho)


def direct_search(NA: float, NB: float, kT, a, b, threshold=1e-12, max_iter=200000):
    """The search of minimize_three_phase; also returns the iteration count.

    Start (step 3 of Appendix A): phase 3 empty; phases 1 and 2 share the
    particles, displaced by +-eps/2 d along the unstable direction d
    (eps = 0.05 min(NA, NB)), phase 2 holding exactly what phase 1 does not.
    The volumes are 1/3 each as printed while the overall packing
    eta_N = b . N is at most 1/3; above that the empty phase gets
    (1 - eta_N)/2 and phases 1 and 2 the rest in equal parts, which keeps
    them below the excluded-volume limit (the printed thirds would pack them
    to 1.5 eta_N) and is continuous at eta_N = 1/3.  An empty component
    contributes nothing to the free energy (rho ln rho -> 0), so phase 3 can
    start empty with a volume; negative amounts are inadmissible.  Initial
    step 0.01.  Trial order: variable k = A1, B1, V1, A2, B2, V2, the + move
    before the - move; the first strict minimum wins.  A phase of zero volume
    is reported with zero densities.
    """
    NA, NB = float(NA), float(NB)
    d = unstable_direction(hessian(np.array([NA, NB]), kT, a, b))
    eps = 0.05 * min(NA, NB)
    V3 = min(1.0 / 3.0, 0.5 * (1.0 - (b[0] * NA + b[1] * NB)))
    V12 = 0.5 * (1.0 - V3)
    A1 = 0.5 * NA + 0.5 * eps * d[0]
    B1 = 0.5 * NB + 0.5 * eps * d[1]
    return search_from(NA, NB, [A1, B1, V12, NA - A1, NB - B1, V12], kT, a, b, threshold, max_iter)


def search_from(NA, NB, z, kT, a, b, threshold=1e-12, max_iter=200000):
    """The direct search of Appendix A from the amounts z = (A1, B1, V1, A2,
    B2, V2), phase 3 holding the rest of (NA, NB) and of the unit volume."""
    NA, NB = float(NA), float(NB)
    z = np.array(z, dtype=float)

    def total(z):
        A1, B1, V1, A2, B2, V2 = z
        A3, B3, V3 = NA - A1 - A2, NB - B1 - B2, 1.0 - V1 - V2
        F = 0.0
        for A, B, V in ((A1, B1, V1), (A2, B2, V2), (A3, B3, V3)):
            if V < 0 or A < 0 or B < 0:
                return np.inf
            if V == 0:
                if A == 0 and B == 0:
                    continue
                return np.inf
            r = np.array([A / V, B / V])
            if np.dot(b, r) >= 1:
                return np.inf
            F += V * _free_energy_ext(r, kT, a, b)
        return F

    F = total(z)
    step = 0.01
    it = 0
    while it < max_iter:
        it += 1
        best, bestz = F, None
        for k in range(6):
            for sgn in (1.0, -1.0):
                t = z.copy()
                t[k] += sgn * step
                Ft = total(t)
                if Ft < best:
                    best, bestz = Ft, t
        if bestz is not None and F - best > 0:
            z, F = bestz, best
        else:
            step *= 0.5
            if step < threshold:
                break
    A1, B1, V1, A2, B2, V2 = z
    phases = []
    for A, B, V in ((A1, B1, V1), (A2, B2, V2), (NA - A1 - A2, NB - B1 - B2, 1.0 - V1 - V2)):
        phases.append((A / V, B / V, V) if V > 0 else (0.0, 0.0, V))
    return phases, F, it


# Classification constants of the phase-diagram pipeline (step 6 of Appendix A)
MERGE_TOL = 1e-3   # phases whose densities differ by less (max norm, relative to max(1, |rho|)) are one phase
VOLUME_MIN = 1e-6  # merged phases with a smaller volume are dropped
F_SLACK = 1e-12    # a polish may not raise the free energy by more than this (relative to max(1, |F|))
RESTARTS = 2       # restarts of step 6(b) when a phase is left unstable


def _stable(r, kT, a, b):
    H = hessian(r, kT, a, b)
    return H[0, 0] > 0 and H[0, 0] * H[1, 1] - H[0, 1] * H[1, 0] > 0


def phase_point(NA: float, NB: float, kT, a, b, threshold=1e-12, max_iter=200000):
    """One (A, B) point of the phase diagram of a two-component mixture
    (Appendix A): stability test, direct search, classification, and a Newton
    polish of the coexistence conditions.

    Step 6(b): while a distinct phase is unstable (at most RESTARTS times),
    the search starts again with the largest unstable phase split along its
    unstable direction into phases 1 and 2 (eps = 0.05 of its smaller
    amount) and phase 3 holding the other phases packed together; the
    iterations of all searches add up.

    status: -1 invalid overall composition (a density <= 0 or eta >= 1);
             1 stable (Hessian positive definite): no search (step 2a);
             otherwise the number of distinct phases the search ends with (2 or
             3), or 0 if it ends with an infinite free energy.
    Distinct phases: the search's three phases merged greedily in their
    order when their densities agree within MERGE_TOL, the merged density
    being total particles over total volume; then phases with volume below
    VOLUME_MIN dropped; sorted by rho_A - rho_B ascending.
    Polish: with 2 phases Newton on equal mu^c, equal p and the lever rule
    through (NA, NB) (coexistence_two_phase); with 3 phases Newton on equal
    mu^c and p in all three (coexistence_three_phase), the volumes then from
    the lever rule.  Accepted when finite, every volume lies in (0, 1), the
    phases stay distinct (the trivial root of these equations has equal
    phases), each is locally stable (positive-definite Hessian), and their
    free energy sum_k V_k f(rho_k) does not exceed the search's by more than
    F_SLACK.  A rejected three-phase polish merges the closest two phases and
    polishes the pair (status 2), and if that is rejected too drops the
    phase of smallest volume and polishes the other two; if every polish is
    rejected the search's distinct phases are kept.  The search supplies the phase count and the
    start; the polish makes the result exact even where the search stopped
    at its iteration cap before converging.
    Returns a dict with phases [(rho_A, rho_B, V)], raw (the search's three
    phases), F, iterations, n_unstable (distinct phases whose Hessian is not
    positive definite) and polished (0 not attempted, 1 accepted, 2 rejected).
    """
    NA, NB = float(NA), float(NB)
    N = np.array([NA, NB])
    out = dict(phases=[], raw=[], F=np.nan, iterations=0, n_unstable=0, polished=0, status=-1)
    if not (NA > 0 and NB > 0 and np.dot(b, N) < 1):
        return out
    out["F"] = free_energy_density(N, kT, a, b)
    if _stable(N, kT, a, b):
        out.update(phases=[(NA, NB, 1.0)], status=1)
        return out
    raw, F, it = direct_search(NA, NB, kT, a, b, threshold, max_iter)
    restarts = 0
    while True:
        out.update(raw=raw, F=F, iterations=out["iterations"] + it)
        if not np.isfinite(F):
            out["status"] = 0
            return out
        ph = _distinct_phases(raw)
        unstable = [p for p in ph if not _stable(np.array(p[:2]), kT, a, b)]
        if unstable and restarts < RESTARTS:
            # step 6(b): split the (largest) unstable phase along its unstable
            # direction into phases 1 and 2; phase 3 holds the others packed
            u = unstable[0]
            for p in unstable[1:]:
                if p[2] > u[2]:
                    u = p
            Au, Bu, Vu = u[0] * u[2], u[1] * u[2], u[2]
            d = unstable_direction(hessian(np.array(u[:2]), kT, a, b))
            eps = 0.05 * min(Au, Bu)
            A1 = 0.5 * Au + 0.5 * eps * d[0]
            B1 = 0.5 * Bu + 0.5 * eps * d[1]
            raw, F, it = search_from(NA, NB, [A1, B1, 0.5 * Vu, Au - A1, Bu - B1, 0.5 * Vu], kT, a, b, threshold,
                                     max_iter)
            restarts += 1
            continue
        break
    out["n_unstable"] = len(unstable)
    out["phases"] = ph
    out["status"] = len(ph)
    if len(ph) not in (2, 3):
        return out
    new = _polish(N, ph, F, kT, a, b)
    if new is None and len(ph) == 3:
        # a search stopped at its iteration cap can leave two nearly equal
        # phases: merge the closest pair and polish as two phases
        pairs = [(0, 1), (0, 2), (1, 2)]
        i, j = min(pairs, key=lambda q: max(abs(ph[q[0]][0] - ph[q[1]][0]), abs(ph[q[0]][1] - ph[q[1]][1])))
        k = 3 - i - j
        V = ph[i][2] + ph[j][2]
        m = ((ph[i][0] * ph[i][2] + ph[j][0] * ph[j][2]) / V, (ph[i][1] * ph[i][2] + ph[j][1] * ph[j][2]) / V, V)
        two = sorted([m, ph[k]], key=lambda p: p[0] - p[1])
        new = _polish(N, two, F, kT, a, b)
        if new is None:
            # or the smallest phase is a seed the search left behind: drop it
            k = min(range(3), key=lambda q: ph[q][2])
            two = [ph[q] for q in range(3) if q != k]
            new = _polish(N, two, F, kT, a, b)
        if new is not None:
            out["status"] = 2
            out["n_unstable"] = sum(not _stable(np.array(p[:2]), kT, a, b) for p in two)
    if new is not None:
        out["phases"] = new
        out["polished"] = 1
    else:
        out["polished"] = 2
    return out


def _distinct_phases(raw):
    """Step 6 classification: the search's phases merged greedily in their
    order when their densities agree within MERGE_TOL (the merged density
    being total particles over total volume), phases below VOLUME_MIN
    dropped, the rest sorted by rho_A - rho_B."""
    groups = []  # [particles A, particles B, volume]
    for ra, rb, V in raw:
        if not V > 0:
            continue
        r = np.array([ra, rb])
        for g in groups:
            rg = np.array([g[0] / g[2], g[1] / g[2]])
            if np.max(np.abs(r - rg)) <= MERGE_TOL * max(1.0, np.max(np.abs(rg))):
                g[0] += ra * V
                g[1] += rb * V
                g[2] += V
                break
        else:
            groups.append([ra * V, rb * V, V])
    ph = [(g[0] / g[2], g[1] / g[2], g[2]) for g in groups if g[2] >= VOLUME_MIN]
    ph.sort(key=lambda p: p[0] - p[1])
    return ph


def _distinct(p, q):
    scale = max(1.0, abs(p[0]), abs(p[1]), abs(q[0]), abs(q[1]))
    return max(abs(p[0] - q[0]), abs(p[1] - q[1])) > MERGE_TOL * scale


def _polish(N, ph, F_search, kT, a, b):
    """Newton polish of 2 or 3 phases (see phase_point); None if rejected."""
    if len(ph) == 2:
        xa, xb, phi = coexistence_two_phase(N, ph[0][:2], ph[1][:2], kT, a, b)
        new = [(xa[0], xa[1], phi), (xb[0], xb[1], 1.0 - phi)]
    else:
        rs, _ = coexistence_three_phase([np.array(p[:2]) for p in ph], kT, a, b)
        M = np.vstack([np.column_stack(rs), np.ones(3)])
        vol = np.linalg.solve(M, np.array([N[0], N[1], 1.0]))
        new = [(r[0], r[1], v) for r, v in zip(rs, vol)]
    if not (all(np.isfinite(x) for p in new for x in p) and all(0 < p[2] < 1 for p in new)):
        return None
    if not all(_distinct(new[i], new[j]) for i in range(len(new)) for j in range(i + 1, len(new))):
        return None
    if not all(_stable(np.array(p[:2]), kT, a, b) for p in new):
        return None
    F_new = sum(p[2] * free_energy_density(np.array(p[:2]), kT, a, b) for p in new)
    if not F_new <= F_search + F_SLACK * max(1.0, abs(F_search)):
        return None
    return new


def coexistence_invariant_point(phases, kT, a, b, tol=1e-15, maxit=50):
    """C + 1 coexisting bulk phases of a C-component mixture.

    At fixed temperature the state with the maximal number of phases has no
    free variable (Gibbs phase rule): its (C + 1) C densities satisfy as many
    equations, mu^c equal in all phases for every c and equal pressure
    (Sec. II).  Newton with the analytic Jacobian (d mu / d rho is the
    Hessian, d p / d rho = rho^T H by Gibbs-Duhem), started from `phases`
    (C + 1 density vectors).  Returns the phases and the residual norm.
    """
    P = len(phases)
    C = len(phases[0])
    assert P == C + 1
    z = np.concatenate([np.asarray(ph, dtype=float) for ph in phases])
    split = lambda z: [z[k * C:(k + 1) * C] for k in range(P)]

    def resid(z):
        rs = split(z)
        m0, p0 = chemical_potential(rs[0], kT, a, b), pressure(rs[0], kT, a, b)
        out = [m0 - chemical_potential(r, kT, a, b) for r in rs[1:]]
        out.append(np.array([p0 - pressure(r, kT, a, b) for r in rs[1:]]))
        return np.concatenate(out)

    for _ in range(maxit):
        F = resid(z)
        rs = split(z)
        Hs = [hessian(r, kT, a, b) for r in rs]
        gs = [r @ H for r, H in zip(rs, Hs)]
        n = P * C
        J = np.zeros((n, n))
        for k in range(1, P):  # mu rows: (k - 1) C .. k C
            J[(k - 1) * C:k * C, 0:C] = Hs[0]
            J[(k - 1) * C:k * C, k * C:(k + 1) * C] = -Hs[k]
        for k in range(1, P):  # pressure rows
            J[(P - 1) * C + k - 1, 0:C] = gs[0]
            J[(P - 1) * C + k - 1, k * C:(k + 1) * C] = -gs[k]
        step = np.linalg.solve(J, F)
        lam = 1.0
        while True:
            t = z - lam * step
            if all(np.all(r > 0) and np.dot(b, r) < 1 for r in split(t)):
                break
            lam *= 0.5
        z = t
        if np.max(np.abs(lam * step)) < tol * max(1.0, np.max(np.abs(z))):
            break
    return [r.copy() for r in split(z)], float(np.linalg.norm(resid(z)))


def coexistence_three_phase(phases, kT, a, b, tol=1e-15, maxit=50):
    """The three-phase point of a two-component mixture (see
    coexistence_invariant_point), e.g. from the Appendix A direct search."""
    return coexistence_invariant_point(phases, kT, a, b, tol, maxit)


def gamma_from_width_rule(kappa: float, rho_liquid: float, cs2: float = THETA_LB):
    """gamma_mu from Eq. kappaGammaMuRelation: c_s^2 = 1 - 4 kappa rho_l gamma_mu."""
    return (1.0 - cs2) / (4.0 * kappa * rho_liquid)


def linear_growth_matrix(rho, kT, a, b, kappa, lap_symbol):
    """H + K * (-lap_symbol): the quadratic form of the discrete free energy for a
    Fourier mode whose discrete-Laplacian eigenvalue is lap_symbol (<= 0)."""
    return hessian(rho, kT, a, b) - np.asarray(kappa) * lap_symbol

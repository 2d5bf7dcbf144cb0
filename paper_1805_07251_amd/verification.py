"""The paper's verification workload (Sec. VI.A with Appendix A): points of a
phase diagram computed on the GPU seed batched D1Q3 lattice Boltzmann runs
that start from tanh profiles at the computed phases (Sec. V: bulk values
from the minimiser, interfaces of about the equilibrium width), and the
lattice's bulk densities after the run are measured against the binodal.

Measures (all densities absolute):
  shift      distance of the lattice's bulk states from the tie-line ends the
             minimiser predicted for the point's overall composition (the
             interfaces hold excess mass, so a finite lattice ends on a
             slightly different tie line);
  deviation  distance from the binodal line itself (the paper's measure):
             vdwlb_phase_points solves the tie lines through the midpoint of
             the two measured bulk states displaced by +-DELTA across the tie
             line, which gives two nearby points on each branch of the
             binodal; the deviation is the larger distance of a measured
             state from its branch's chord between them;
  end_deviation  distance of the measured states from the ends of the tie
             line through their midpoint (an upper bound of the deviation;
             zero exactly when the lattice phases coexist in the bulk
             thermodynamics of Sec. II).
Distances take the better assignment of measured to computed phases.

Every arithmetic step of the method runs in the library's kernels; this
module lays out the initial profiles and reads bulk values off the results.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import inputs as I
from . import phase as P
from .batch import Batch

CS2 = 1.0 / 3.0  # lattice speed of sound squared (theta)
DELTA = 1e-5  # displacement across the tie line that brackets the local binodal (small: the chord's offset
# from the curved binodal grows with the square of its length)


@dataclass
class SlabSetup:
    L: int = 256
    kappa: float = 0.4
    width: float = 2.0
    tau: float = 1.0
    gamma_scale: float = 1.0  # fraction of the width rule's gamma_mu (Eq. kappaGammaMuRelation)
    window: int = 2  # bulk values are means over 2 window + 1 sites (period-2 ripple of the central difference)
    lam: float = 0.01  # friction lambda^{cc'} between the components (Eq. forceFriction): it sets how fast they interdiffuse


def two_phase_profile(L, rho_in, rho_out, n_in, width):
    """[2, L] densities: phase `rho_in` on n_in sites centred on L/2 inside
    phase `rho_out`, tanh edges of the given width (periodic)."""
    x = np.arange(L, dtype=np.float64)
    x0 = 0.5 * (L - n_in)
    x1 = x0 + n_in
    s = 0.5 * (np.tanh((x - x0) / width) - np.tanh((x - x1) / width))
    rin, rout = np.asarray(rho_in, float), np.asarray(rho_out, float)
    return rout[:, None] + (rin - rout)[:, None] * s[None, :]


def slab_workloads(kT, a, b, phases, setup: SlabSetup = SlabSetup(), dim=1):
    """One Workload per two-phase point: phases[k] = ((rA, rB, V), (rA, rB,
    V)) of the point's distinct phases; the denser phase is the slab, sized
    by its volume fraction (lever rule).  dim = 1: a D1Q3 line of L sites;
    dim = 2: a D2Q9 lattice of L x 4 sites uniform in y."""
    kap = I.kappa_matrix(np.asarray(a, float), setup.kappa)
    ws = []
    for (p0, p1) in phases:
        dense, light = (p0, p1) if p0[0] + p0[1] >= p1[0] + p1[1] else (p1, p0)
        n_in = int(np.clip(round(dense[2] * setup.L), 8, setup.L - 8))
        prof = two_phase_profile(setup.L, dense[:2], light[:2], n_in, setup.width)
        rho_l = dense[0] + dense[1]
        gam = setup.gamma_scale * (1.0 - CS2) / (4.0 * setup.kappa * rho_l)
        ny = 1 if dim == 1 else 4
        ws.append(I.Workload(setup.L, ny, kT, np.asarray(a, float), np.asarray(b, float), kap,
                             np.repeat(prof[:, None, :], ny, axis=1), tau=setup.tau, gamma_mu=gam, dim=dim,
                             lam=np.full((2, 2), setup.lam)))
    return ws


def interface_width(rho, window):
    """Equilibrium half-width of the two interfaces of a slab rho [C, L]: for
    the component with the largest bulk contrast D, D / (2 max |d rho / dx|)
    with the central difference (the w of a profile m + D/2 tanh(x / w))."""
    inner, outer = bulk_states(rho, window)
    c = int(np.argmax(np.abs(inner - outer)))
    d = 0.5 * np.abs(np.roll(rho[c], -1) - np.roll(rho[c], 1))
    return float(abs(inner[c] - outer[c]) / (2.0 * d.max()))


def bulk_states(rho, window):
    """(slab centre, far edge) window means of rho [C, L]."""
    L = rho.shape[1]
    idx = lambda c: (c + np.arange(-window, window + 1)) % L
    return rho[:, idx(L // 2)].mean(1), rho[:, idx(0)].mean(1)


@dataclass
class VerificationResult:
    points: np.ndarray      # [m, 2] overall compositions run
    predicted: np.ndarray   # [m, 2, 2] minimiser phases (dense, light) x (A, B)
    measured: np.ndarray    # [m, 2, 2] lattice bulk states (dense, light)
    binodal: np.ndarray     # [m, 2, 2] tie-line ends through the measured midpoint
    shift: np.ndarray       # [m] max |measured - predicted|
    deviation: np.ndarray   # [m] distance from the binodal line (nan where a re-solve failed)
    end_deviation: np.ndarray  # [m] max |measured - binodal| (tie line through the measured midpoint)
    status: np.ndarray      # [m] batch status (0 = ran to the end)
    steps: int
    gamma_mu: np.ndarray    # [m] gamma_mu of each instance's last run
    halvings: np.ndarray    # [m] times the stability search halved gamma_mu
    widths: np.ndarray      # [m] interface width of each instance's last start


def _matched(meas, ends):
    """Distance of the measured pair from a tie line's ends, taking the
    better of the two assignments (liquid-liquid pairs have nearly equal
    total densities, so a dense/light label does not identify a phase)."""
    d0 = np.abs(meas - ends).max()
    d1 = np.abs(meas - ends[::-1]).max()
    return min(d0, d1)


def run(kT, a, b, NA, NB, steps=50000, setup: SlabSetup = SlabSetup(), max_iter=200000, gamma_halvings=4,
        width_iterations=0, dim=1):
    """Phase-diagram points (NA, NB) -> minimiser on the GPU -> one D1Q3 slab
    per polished two-phase point -> `steps` lattice Boltzmann steps in one
    batched launch -> bulk states against the binodal.

    gamma_mu stability search (Sec. VI.A lowers gamma_mu for runs that go
    unstable): instances that end unphysical are run again from their
    initial profile with gamma_mu halved, up to `gamma_halvings` times, each
    round one batched launch over the instances still failing.

    Interface-width iteration (Sec. VI.A): `width_iterations` times, the
    equilibrium width of each run's interfaces is measured and the run is
    started again from tanh profiles at the minimiser's bulk values with
    that width (and the gamma_mu it ended with).

    dim = 2 runs the same slabs as L x 4 D2Q9 lattices (the 2-D extension)."""
    res = P.phase_points(kT, a, b, NA, NB, max_iter=max_iter)
    torch.cuda.synchronize()
    st = res["status"].cpu().numpy()
    pol = res["polished"].cpu().numpy()
    ph = res["phases"].cpu().numpy()
    keep = np.flatnonzero((st == 2) & (pol == 1))
    if keep.size == 0:
        raise ValueError("no polished two-phase point among the compositions")
    pairs = [(tuple(ph[k, 0]), tuple(ph[k, 1])) for k in keep]
    ws = slab_workloads(kT, a, b, pairs, setup, dim)
    m = len(ws)
    status = np.full(m, -1, dtype=np.int32)
    dens = [None] * m
    halvings = np.zeros(m, dtype=np.int32)
    widths = np.full(m, setup.width)
    for it in range(width_iterations + 1):
        if it > 0:
            # restart from the minimiser's bulk values with the measured widths
            for j in range(m):
                if status[j] != 0:
                    continue
                widths[j] = interface_width(dens[j], setup.window)
                p0, p1 = pairs[j]
                dense, light = (p0, p1) if p0[0] + p0[1] >= p1[0] + p1[1] else (p1, p0)
                n_in = int(np.clip(round(dense[2] * setup.L), 8, setup.L - 8))
                prof = two_phase_profile(setup.L, dense[:2], light[:2], n_in, widths[j])
                ws[j].rho = np.repeat(prof[:, None, :], ws[j].ny, axis=1)
        todo = np.arange(m)
        for round_ in range(gamma_halvings + 1):
            sub = [ws[j] for j in todo]
            batch = Batch(sub, dtype="f64")
            batch.init([w.rho for w in sub])
            batch.run(steps)
            st_b = batch.status()
            rho_b = batch.densities()
            for i, j in enumerate(todo):
                status[j] = st_b[i]
                dens[j] = rho_b[i].cpu().numpy()[:, 0]
            todo = todo[st_b != 0]
            if todo.size == 0 or round_ == gamma_halvings:
                break
            for j in todo:
                ws[j].gamma_mu *= 0.5
                halvings[j] += 1
    gamma = np.array([w.gamma_mu for w in ws])
    pred = np.empty((m, 2, 2))
    meas = np.empty((m, 2, 2))
    for j, (p0, p1) in enumerate(pairs):
        dense, light = (p0, p1) if p0[0] + p0[1] >= p1[0] + p1[1] else (p1, p0)
        pred[j] = [dense[:2], light[:2]]
        meas[j] = bulk_states(dens[j], setup.window)
    # the binodal near the measured states: tie lines through the measured
    # midpoint and through two points beside it, displaced across the tie line
    mid = 0.5 * (meas[:, 0] + meas[:, 1])
    along = meas[:, 0] - meas[:, 1]
    along /= np.maximum(np.linalg.norm(along, axis=1, keepdims=True), 1e-300)
    normal = np.stack([-along[:, 1], along[:, 0]], 1)
    probes = np.concatenate([mid, mid + DELTA * normal, mid - DELTA * normal])
    again = P.phase_points(kT, a, b, probes[:, 0], probes[:, 1], max_iter=max_iter)
    torch.cuda.synchronize()
    st2 = again["status"].cpu().numpy()
    pol2 = again["polished"].cpu().numpy()
    ph2 = again["phases"].cpu().numpy()
    ends = np.full((3, m, 2, 2), np.nan)
    for q in range(3):
        for j in range(m):
            i = q * m + j
            if st2[i] == 2 and pol2[i] == 1:
                e = ph2[i, :2, :2]
                # order the ends like the measured pair (nearest assignment)
                if np.abs(meas[j] - e).max() > np.abs(meas[j] - e[::-1]).max():
                    e = e[::-1]
                ends[q, j] = e
    bino = ends[0]
    shift = np.array([_matched(meas[j], pred[j]) for j in range(m)])
    end_dev = np.array([_matched(meas[j], bino[j]) for j in range(m)])
    dev = np.full(m, np.nan)
    for j in range(m):
        d = 0.0
        for s in range(2):  # each measured state against its branch's local chord
            p0, p1 = ends[1, j, s], ends[2, j, s]
            chord = p1 - p0
            nrm = np.linalg.norm(chord)
            if not np.isfinite(nrm) or nrm == 0:
                d = np.nan
                break
            x = meas[j, s] - p0
            d = max(d, abs(chord[0] * x[1] - chord[1] * x[0]) / nrm)
        dev[j] = d
    return VerificationResult(np.stack([np.asarray(NA, float)[keep], np.asarray(NB, float)[keep]], 1), pred, meas,
                              bino, shift, dev, end_dev, status, steps, gamma, halvings, widths)


def three_phase_profile(L, gas, lq_a, lq_b, na, nb, width):
    """[2, L] densities: gas | A-rich liquid | gas | B-rich liquid | gas, the
    liquids on na and nb sites, the gas split into two domains of equal size
    (the first and last pieces are one domain across the periodic boundary),
    tanh edges of the given width."""
    ng = L - na - nb
    e0 = ng // 4
    e1 = e0 + na
    e2 = e1 + ng // 2
    e3 = e2 + nb
    x = np.arange(L, dtype=np.float64) + 0.5
    box = lambda lo, hi: 0.5 * (np.tanh((x - lo) / width) - np.tanh((x - hi) / width))
    g, la, lb = (np.asarray(v, float) for v in (gas, lq_a, lq_b))
    prof = g[:, None] + (la - g)[:, None] * box(e0, e1)[None, :] + (lb - g)[:, None] * box(e2, e3)[None, :]
    centres = [((e3 + L + e0) // 2) % L, (e0 + e1) // 2, (e1 + e2) // 2, (e2 + e3) // 2]
    return prof, centres


@dataclass
class ThreePhaseResult:
    points: np.ndarray      # [m, 2] overall compositions run
    predicted: np.ndarray   # [m, 3, 2] gas, A-rich, B-rich phases of the minimiser
    measured: np.ndarray    # [m, 4, 2] bulk states at the centres of gas, A-rich, gas, B-rich
    deviation: np.ndarray   # [m] max |measured - predicted| over the four domains
    status: np.ndarray      # [m] batch status
    steps: int
    gamma_mu: np.ndarray
    halvings: np.ndarray


def run_three_phase(kT, a, b, NA, NB, steps=50000, setup: SlabSetup = SlabSetup(), max_iter=200000,
                    gamma_halvings=4, min_domain=24):
    """The verification of the three-phase regions: every polished
    three-phase point of (NA, NB) is run as a D1Q3 line with tanh domains of
    the minimiser's three phases (gas | A-rich | gas | B-rich, the gas being
    the phase of lowest total density), sized by the lever rule; points whose
    smallest domain would have fewer than `min_domain` sites are skipped
    (domains of 12-23 sites leave the bulk windows inside the interfaces' tails:
    on the baseline mixture they made every run more than 1e-3 off).
    The three-phase state of a binary mixture is unique at fixed temperature
    (Gibbs phase rule), so every run should end at the same densities: the
    deviation is the largest distance of a domain's bulk state from them.
    gamma_mu is halved for runs that go unphysical, as in `run`."""
    res = P.phase_points(kT, a, b, NA, NB, max_iter=max_iter)
    torch.cuda.synchronize()
    st = res["status"].cpu().numpy()
    pol = res["polished"].cpu().numpy()
    ph = res["phases"].cpu().numpy()
    kap = I.kappa_matrix(np.asarray(a, float), setup.kappa)
    ws, preds, cents, pts = [], [], [], []
    for k in np.flatnonzero((st == 3) & (pol == 1)):
        phases = ph[k]
        g = int(np.argmin(phases[:, 0] + phases[:, 1]))
        rest = [q for q in range(3) if q != g]
        ia = max(rest, key=lambda q: phases[q, 0] - phases[q, 1])
        ib = min(rest, key=lambda q: phases[q, 0] - phases[q, 1])
        na, nb = int(round(phases[ia, 2] * setup.L)), int(round(phases[ib, 2] * setup.L))
        ng = setup.L - na - nb
        if min(na, nb, ng // 2) < min_domain:
            continue
        prof, centres = three_phase_profile(setup.L, phases[g, :2], phases[ia, :2], phases[ib, :2], na, nb,
                                            setup.width)
        rho_l = max(phases[ia, :2].sum(), phases[ib, :2].sum())
        gam = setup.gamma_scale * (1.0 - CS2) / (4.0 * setup.kappa * rho_l)
        ws.append(I.Workload(setup.L, 1, kT, np.asarray(a, float), np.asarray(b, float), kap, prof[:, None, :],
                             tau=setup.tau, gamma_mu=gam, dim=1,
                             lam=np.full((2, 2), setup.lam)))
        preds.append(np.stack([phases[g, :2], phases[ia, :2], phases[ib, :2]]))
        cents.append(centres)
        pts.append((NA[k], NB[k]))
    m = len(ws)
    if m == 0:
        raise ValueError("no three-phase point with domains of at least min_domain sites")
    status = np.full(m, -1, dtype=np.int32)
    dens = [None] * m
    halvings = np.zeros(m, dtype=np.int32)
    todo = np.arange(m)
    for round_ in range(gamma_halvings + 1):
        sub = [ws[j] for j in todo]
        batch = Batch(sub, dtype="f64")
        batch.init([w.rho for w in sub])
        batch.run(steps)
        st_b = batch.status()
        rho_b = batch.densities()
        for i, j in enumerate(todo):
            status[j] = st_b[i]
            dens[j] = rho_b[i].cpu().numpy()[:, 0]
        todo = todo[st_b != 0]
        if todo.size == 0 or round_ == gamma_halvings:
            break
        for j in todo:
            ws[j].gamma_mu *= 0.5
            halvings[j] += 1
    pred = np.array(preds)
    meas = np.empty((m, 4, 2))
    dev = np.empty(m)
    win = np.arange(-setup.window, setup.window + 1)
    for j in range(m):
        L = dens[j].shape[1]
        for q, c in enumerate(cents[j]):
            meas[j, q] = dens[j][:, (c + win) % L].mean(1)
        want = np.stack([pred[j, 0], pred[j, 1], pred[j, 0], pred[j, 2]])
        dev[j] = np.abs(meas[j] - want).max()
    return ThreePhaseResult(np.array(pts), pred, meas, dev, status, steps, np.array([w.gamma_mu for w in ws]),
                            halvings)

"""Benchmark of the fused D2Q9 sweep on one MI355X.

Workload: the 2048x2048 two-component spinodal-decomposition lattice in FP64
(D2Q9, a12 drawn in [0.7, 1.1] a11, +-1 % seeded noise), one step = one fused
sweep over the whole lattice (stream, moments, chemical potential, force,
friction, collision).  Prints one JSON line.

value      MLUPS x components (million site updates per second times C), inputs
           resident in HBM, timed with HIP events over exactly --steps steps.
roofline   the sweep kernel against the 8 TB/s HBM peak, with algorithmic bytes
           2 * 9 * C * sizeof(real) per site update.
cpu_baseline  the CPU oracle on the host, a bounded sample of the same workload;
           with the extras also oracle samples beside the batched, adjoint and
           phase-diagram legs (cpu_baseline.legs).
extra      the headline's median over 5 separate runs, with init, readback and
           host copies timed on their own; FP32 and 4-component sweeps; the
           batched phase-diagram workload in D2Q9 (strips through L2/MALL) and
           D1Q3 (instances resident in LDS); a 2^24-site D1Q3 line; the
           adjoint against the plain forward; the Appendix A phase diagram on
           a 256 x 256 composition grid; and the verification workload
           (phase-diagram points run as D1Q3 slabs, bulk states against the
           binodal).
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS×components & % HBM roofline; batched sweep and adjoint vs plain step"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="only the headline workload")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--profile", action="store_true",
                    help="profiling run: the headline sweep for --steps steps and the 1 GiB copy kernel only")
    ap.add_argument("--schedule", type=int, default=-1,
                    help="with --profile or --legs adjoint: use this sweep schedule instead of autotuning")
    ap.add_argument("--phase", action="store_true",
                    help="profiling run: the 256 x 256 Appendix A phase-diagram leg only")
    ap.add_argument("--legs", default="",
                    help="profiling run: only these comma-separated legs (" + ", ".join(LEGS) + ")")
    return ap.parse_args()


def time_steps(lat, steps, warmup):
    import torch

    lat.run(warmup)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    lat.run(steps)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3


def sweep_line(w, dtype, steps, warmup, schedule=-1):
    import torch

    from paper_1805_07251_amd.lattice import Lattice

    lat = Lattice.from_workload(w, dtype=dtype)
    # the densities go to HBM once, before anything is timed: re-initialising
    # from the resident copy leaves no host transfer (and no idle device)
    # between the autotuner and the warm-up steps
    rho = torch.as_tensor(w.rho, dtype=lat.plan.torch_dtype, device="cuda")
    lat.init(rho)
    if schedule >= 0:
        lat.set_schedule(schedule)
        sched = schedule
    else:
        sched = lat.autotune()
    lat.init(rho)
    secs = time_steps(lat, steps, warmup)
    st = lat.status()
    sites = w.nx * w.ny
    real = 8 if dtype == "f64" else 4
    bytes_per_site = 2 * (3 if getattr(w, "dim", 2) == 1 else 9) * w.C * real
    us = secs / steps * 1e6
    return {
        "workload": w.name,
        "dtype": dtype,
        "steps": steps,
        "seconds": secs,
        "us_per_step": us,
        "mlups": sites * steps / secs / 1e6,
        "mlups_x_c": sites * w.C * steps / secs / 1e6,
        "gbs": bytes_per_site * sites / (us * 1e-6) / 1e9,
        "bytes_per_site": bytes_per_site,
        "schedule": sched,
        "status": st,
    }


def protocol_leg(w, dtype, schedule, repeats=5, steps=1000):
    """Timings kept out of the headline: the spread of `repeats` separate runs of
    `steps` steps (median reported), the init kernel from a density field already
    in HBM, the moments readback (rho, j, mu, p; the call ends with the error-flag
    poll, so it is a wall-clock figure), and the host <-> device copies of rho."""
    import statistics

    import torch

    from paper_1805_07251_amd.lattice import Lattice

    lat = Lattice.from_workload(w, dtype=dtype)
    lat.set_schedule(schedule)
    tdt = lat.plan.torch_dtype
    host = torch.as_tensor(w.rho, dtype=tdt).pin_memory()
    dev = torch.empty(host.shape, dtype=tdt, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev.copy_(host, non_blocking=True)
    torch.cuda.synchronize()
    h2d = time.perf_counter() - t0
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    lat.init(dev)
    torch.cuda.synchronize()
    e0.record(s)
    lat.init(dev)
    e1.record(s)
    torch.cuda.synchronize()
    init_us = e0.elapsed_time(e1) * 1e3
    runs = [time_steps(lat, steps, 2) / steps * 1e6 for _ in range(repeats)]
    lat.moments()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rho, _, _, _ = lat.moments()
    moments_us = (time.perf_counter() - t0) * 1e6
    back = torch.empty(rho.shape, dtype=tdt).pin_memory()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    back.copy_(rho, non_blocking=True)
    torch.cuda.synchronize()
    d2h = time.perf_counter() - t0
    nbytes = host.numel() * host.element_size()
    return {
        "repeats_us_per_step": runs,
        "median_us_per_step": statistics.median(runs),
        "steps_per_repeat": steps,
        "init_us": init_us,
        "moments_readback_us": moments_us,
        "rho_h2d_ms": h2d * 1e3,
        "rho_d2h_ms": d2h * 1e3,
        "rho_bytes": nbytes,
        "status": lat.status(),
    }


def copy_gbs(nbytes=1 << 30, reps=20):
    import torch

    from paper_1805_07251_amd import vdwlb as V

    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    s = torch.cuda.current_stream()
    V.check(V.lib().vdwlb_copy(b.data_ptr(), a.data_ptr(), nbytes, s.cuda_stream))
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        V.check(V.lib().vdwlb_copy(b.data_ptr(), a.data_ptr(), nbytes, s.cuda_stream))
    e1.record(s)
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1e3 / reps
    return 2 * nbytes / secs / 1e9


def traffic_from_profiles(schedule: int):
    """HBM bytes per launch of the sweep kernel under `schedule`, measured
    with rocprofv3 FETCH_SIZE / WRITE_SIZE and recorded in profiles/ together
    with the hash of the sweep source and of the plan code that lays out the
    state they were taken on; None when either has changed since or the
    schedule was not profiled."""
    path = os.path.join(ROOT, "profiles", "k_sweep_spinodal2048_f64_traffic.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"source_sha256:\s*([0-9a-f]{64})", txt)
    if not m or m.group(1) != sweep_source_hash():
        return None
    m = re.search(rf"traffic_bytes_per_launch:\s*schedule {schedule}\s*=\s*([0-9.eE+]+)", txt)
    return float(m.group(1)) if m else None


def sweep_source_hash():
    import hashlib

    h = hashlib.sha256()
    for fn in ("sweep.hpp", "schedules.hpp", "api.cpp"):
        h.update(open(os.path.join(ROOT, "paper_1805_07251_amd", "csrc", fn), "rb").read())
    return h.hexdigest()


def batch_leg(seed, steps, warmup):
    """The batched phase-diagram workload: 1024 quasi-1-D lattices L x 4,
    L in [128, 1024], own kT / composition / a12, one persistent launch."""
    import numpy as np
    import torch

    from paper_1805_07251_amd import inputs as I
    from paper_1805_07251_amd import vdwlb as V
    from paper_1805_07251_amd.batch import Batch
    from paper_1805_07251_amd.lattice import Lattice

    def maxwell(a, b, kT):
        try:
            return V.maxwell(a, b, kT)
        except V.VdwlbError:
            return None

    ws = I.batch_slabs(maxwell, seed)
    sites = np.array([w.nx * w.ny for w in ws], dtype=np.float64)
    C = ws[0].C
    b = Batch(ws)
    # temporal blocking (steps per block held in LDS) or step by step, and the
    # launch shape: short timed runs of each candidate, reported; the timed run
    # uses the library's default (3 steps per block), which is within a few
    # per cent of the fastest on every box measured and keeps the profiled
    # kernel the same from run to run
    cand = []
    for blocking, threads, blocks in ((3, 256, 0), (4, 256, 0), (0, 1024, 0), (0, 256, 0)):
        b.set_blocking(blocking)
        b.set_launch(threads, blocks)
        b.init([w.rho for w in ws])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.run(1000)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1)
        cand.append({"blocking": blocking, "threads": threads,
                     "mlups_x_c": float(sites.sum()) * C * 1000 / (t / 1e3) / 1e6})
    blocking, threads, blocks = 3, 256, 0
    b.set_blocking(blocking)
    b.set_launch(threads, blocks)
    b.init([w.rho for w in ws])
    b.run(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.run(steps)
    e1.record()
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1e3
    st = b.status()
    done = np.where(st == 0, steps, np.maximum(st - warmup, 0))
    mlups_c = float((sites * done).sum() * C / secs / 1e6)
    # the plain per-instance path on a subset spanning the size range
    order = np.argsort(sites)
    subset = [int(order[i]) for i in np.linspace(0, len(ws) - 1, 16).astype(int)]
    nplain = 200
    lats = []
    for k in subset:
        lat = Lattice.from_workload(ws[k])
        lat.init(ws[k].rho)
        lat.run(2)
        lats.append(lat)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for lat in lats:
        lat.run(nplain)
    torch.cuda.synchronize()
    psecs = time.perf_counter() - t0
    plain_mlups_c = float(sites[subset].sum() * nplain * C / psecs / 1e6)
    return {
        "workload": f"{len(ws)} lattices Lx4, L in [128,1024], C={C}, FP64, slab init",
        "steps": steps,
        "seconds": secs,
        "launch": {"blocking_steps": blocking, "threads": threads, "blocks": blocks},
        "candidates_1000_steps": cand,
        "step_by_step_mlups_x_c": max(c["mlups_x_c"] for c in cand if c["blocking"] == 0),
        "mlups_x_c": mlups_c,
        "instances_stopped_unphysical": int((st != 0).sum()),
        "plain_per_instance_mlups_x_c": plain_mlups_c,
        "plain_sample": f"16 instances across the size range, {nplain} steps each, one plan per instance",
        "speedup_vs_plain_per_instance": mlups_c / plain_mlups_c,
        "equivalent_streamed_gbs": mlups_c / C * 1e6 * 288 / 1e9,
        "note": "blocked runs move about (64/(64-6K) + 1)/K of the algorithmic bytes through HBM; "
                "equivalent_streamed_gbs is the algorithmic rate, not measured traffic",
    }


def batch_d1q3_leg(seed, steps):
    """The same phase-diagram draws as D1Q3 lines (the paper's own lattice):
    1024 lines, L in [128, 1024], every instance resident in LDS for the
    whole run, against the plain D1Q3 path per instance."""
    import numpy as np
    import torch

    from paper_1805_07251_amd import inputs as I
    from paper_1805_07251_amd import vdwlb as V
    from paper_1805_07251_amd.batch import Batch
    from paper_1805_07251_amd.lattice import Lattice

    def maxwell(a, b, kT):
        try:
            return V.maxwell(a, b, kT)
        except V.VdwlbError:
            return None

    ws = I.batch_slabs(maxwell, seed, dim=1)
    sites = np.array([w.nx for w in ws], dtype=np.float64)
    C = ws[0].C
    b = Batch(ws)
    b.init([w.rho for w in ws])
    b.run(1000)
    torch.cuda.synchronize()
    b.init([w.rho for w in ws])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.run(steps)
    e1.record()
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1e3
    st = b.status()
    done = np.where(st == 0, steps, np.maximum(st - 1, 0))
    mlups_c = float((sites * done).sum() * C / secs / 1e6)
    order = np.argsort(sites)
    subset = [int(order[i]) for i in np.linspace(0, len(ws) - 1, 16).astype(int)]
    nplain = 2000
    lats = []
    for k in subset:
        lat = Lattice.from_workload(ws[k])
        lat.init(ws[k].rho)
        lat.run(64)
        lats.append(lat)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for lat in lats:
        lat.run(nplain)
    torch.cuda.synchronize()
    psecs = time.perf_counter() - t0
    plain_mlups_c = float(sites[subset].sum() * nplain * C / psecs / 1e6)
    return {
        "workload": f"{len(ws)} D1Q3 lines, L in [128,1024], C={C}, FP64, slab init, LDS-resident",
        "steps": steps,
        "seconds": secs,
        "mlups_x_c": mlups_c,
        "instances_stopped_unphysical": int((st != 0).sum()),
        "plain_per_instance_mlups_x_c": plain_mlups_c,
        "plain_sample": f"16 instances across the size range, {nplain} steps each, one plan per instance",
        "speedup_vs_plain_per_instance": mlups_c / plain_mlups_c,
    }


def adjoint_leg(seed, schedule=-1):
    """Gradient of a density-profile loss after 2000 steps of the 256 x 256
    lattice w.r.t. (kT, a11, a12, a22, b1, b2, kappa), checkpoints every 100."""
    import numpy as np
    import torch

    from paper_1805_07251_amd import adjoint as A
    from paper_1805_07251_amd import inputs as I
    from paper_1805_07251_amd.lattice import Lattice

    w, tgt = I.adjoint_case(seed)
    # the plain forward on the autotuner's schedule (or the one asked for); the
    # adjoint's forward and recompute run the same schedule
    lat = Lattice.from_workload(w)
    lat.init(w.rho)
    if schedule >= 0:
        lat.set_schedule(schedule)
        sched = schedule
    else:
        sched = lat.autotune()
    theta = A.theta_from_params(w.kT, w.a, w.b, I.KAPPA)
    spec = A.Spec(w.nx, w.ny, 2, w.kappa / I.KAPPA, 2000, ckpt=100, tau=w.tau, gamma_mu=w.gamma_mu, lam=w.lam,
                  schedule=sched)
    rho0 = torch.as_tensor(w.rho, device="cuda")
    tg = torch.as_tensor(tgt, device="cuda")
    # warm-up (allocator, code objects); each call below builds its own plan,
    # as a caller of the autograd function does
    A.run_and_grad(theta, rho0, spec, lambda r: ((r[0] - tg) ** 2).sum())
    torch.cuda.synchronize()
    fwd, bwd = [], []
    for _ in range(3):
        t = torch.as_tensor(theta).clone().requires_grad_(True)
        t0 = time.perf_counter()
        rho = A.VdwLBFunction.apply(t, rho0, spec)
        loss = ((rho[0] - tg) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fwd.append(t1 - t0)
        bwd.append(t2 - t1)
    grad = t.grad.cpu().numpy()
    # the same gradient with every segment's moments kept by the forward
    # (Spec.keep_moments: no recompute; about 7 GB here)
    kspec = A.Spec(w.nx, w.ny, 2, w.kappa / I.KAPPA, 2000, ckpt=100, tau=w.tau, gamma_mu=w.gamma_mu, lam=w.lam,
                   schedule=sched, keep_moments=True)
    A.run_and_grad(theta, rho0, kspec, lambda r: ((r[0] - tg) ** 2).sum())
    kf, kb = [], []
    for _ in range(3):
        tk = torch.as_tensor(theta).clone().requires_grad_(True)
        t0 = time.perf_counter()
        rho = A.VdwLBFunction.apply(tk, rho0, kspec)
        kloss = ((rho[0] - tg) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kloss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        kf.append(t1 - t0)
        kb.append(t2 - t1)
    kgrad = tk.grad.cpu().numpy()
    # the plain forward for the same 2000 steps (its step graph captured beforehand)
    lat.init(w.rho)
    lat.run(64)
    torch.cuda.synchronize()
    plain = []
    for _ in range(3):
        lat.init(w.rho)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        lat.run(2000)
        torch.cuda.synchronize()
        plain.append(time.perf_counter() - t3)
    f, b, pf = min(fwd), min(bwd), min(plain)
    sites = w.nx * w.ny
    return {
        "workload": "256x256 D2Q9, C=2, FP64, 2000 steps, checkpoints every 100",
        "timing": "best of 3 of each",
        "schedule": sched,
        "forward_ms": f * 1e3,
        "backward_ms": b * 1e3,
        "plain_forward_ms": pf * 1e3,
        "fwd_plus_bwd_over_plain_forward": (f + b) / pf,
        "adjoint_mlups": sites * 2000 / b / 1e6,
        "loss": float(loss.detach().cpu()),
        "grad": [float(v) for v in grad],
        "theta_names": ["kT", "a11", "a12", "a22", "b1", "b2", "kappa"],
        "keep_moments": {
            "forward_ms": min(kf) * 1e3,
            "backward_ms": min(kb) * 1e3,
            "fwd_plus_bwd_over_plain_forward": (min(kf) + min(kb)) / pf,
            "same_gradient_bits": bool(np.array_equal(kgrad, grad)),
        },
    }


def phase_diagram_leg(n=256, max_iter=200000):
    """Appendix A phase diagram of the baseline mixture on the GPU: the
    n x n composition grid below the excluded-volume line, one thread per
    point (stability test, direct search, step-6(b) restarts, Newton polish)."""
    import numpy as np
    import torch

    from paper_1805_07251_amd import inputs as I
    from paper_1805_07251_amd import phase

    a, b = I.binary_mixture(0.4, 0.4, 1.0, 1.0, 0.5)
    NA, NB = phase.composition_grid(b, n)
    phase.phase_points(1 / 3, a, b, NA[:64], NB[:64])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = phase.phase_points(1 / 3, a, b, NA, NB, max_iter=max_iter)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    st = r["status"].cpu().numpy()
    pol = r["polished"].cpu().numpy()
    it = r["iterations"].cpu().numpy()
    return {"mixture": "theta_cr 0.4/0.4, rho_cr 1/1, nu 0.5, kT 1/3", "grid": n, "points": int(len(NA)),
            "seconds": secs, "points_per_s": len(NA) / secs, "max_iter": max_iter,
            "status_counts": {int(s): int((st == s).sum()) for s in np.unique(st)},
            "polish_rejected": int((pol == 2).sum()), "mean_iterations_searched": float(it[it > 0].mean()),
            "searched_at_cap": int((it >= max_iter).sum())}


def verification_leg(n=16, steps=50000):
    """The paper's verification workload: the two-phase points of an n x n
    grid, minimiser on the GPU, one D1Q3 slab each at the computed phases,
    `steps` steps in one batched launch (gamma_mu halved for runs that go
    unphysical), bulk states against the binodal."""
    import numpy as np

    from paper_1805_07251_amd import inputs as I
    from paper_1805_07251_amd import phase
    from paper_1805_07251_amd import verification as VV

    out = {}
    a, b = I.binary_mixture(0.4, 0.4, 1.0, 1.0, 0.5)
    NA, NB = phase.composition_grid(b, 64)
    t0 = time.perf_counter()
    r = VV.run_three_phase(1 / 3, a, b, NA, NB, steps=steps, setup=VV.SlabSetup(kappa=0.1, L=512))
    secs = time.perf_counter() - t0
    ok = r.status == 0
    out["baseline_three_phase"] = {"grid": 64, "kappa": 0.1, "line": 512, "min_domain": 24,
                                   "runs": int(len(r.status)),
                                   "unphysical": int((~ok).sum()), "steps": steps, "seconds": secs,
                                   "deviation_median": float(np.median(r.deviation[ok])),
                                   "deviation_p90": float(np.percentile(r.deviation[ok], 90)),
                                   "deviation_max": float(r.deviation[ok].max())}
    import csv

    with open(os.path.join(ROOT, "tests", "golden", "vks_captions.csv")) as fh:
        rows = list(csv.DictReader(line for line in fh if not line.startswith("#")))
    caps = {}
    t0 = time.perf_counter()
    for row in rows:  # the mixtures printed in the figure captions of Sec. VI.A
        a, b = I.binary_mixture(float(row["theta_cr_a"]), float(row["theta_cr_b"]), 1.0, float(row["rho_cr_b"]),
                                float(row["nu"]))
        NA, NB = phase.composition_grid(b, n)
        r = VV.run(1 / 3, a, b, NA, NB, steps=steps)
        ok = r.status == 0
        d = r.deviation[ok]
        d = d[np.isfinite(d)]
        caps[row["label"]] = {"runs": int(len(r.status)), "unphysical": int((~ok).sum()),
                              "deviation_median": float(np.median(d)) if d.size else None,
                              "deviation_p90": float(np.percentile(d, 90)) if d.size else None}
    out["captions"] = {"grid": n, "steps": steps, "seconds": time.perf_counter() - t0, "mixtures": caps}
    for name, nu, wi in (("baseline", 0.5, 0), ("identical", 1.0, 0), ("baseline_width_iterated", 0.5, 1)):
        a, b = I.binary_mixture(0.4, 0.4, 1.0, 1.0, nu)
        NA, NB = phase.composition_grid(b, n)
        t0 = time.perf_counter()
        r = VV.run(1 / 3, a, b, NA, NB, steps=steps, width_iterations=wi)
        secs = time.perf_counter() - t0
        ok = r.status == 0
        d = r.deviation[ok]
        out[name] = {"runs": int(len(r.status)), "unphysical": int((~ok).sum()), "steps": steps, "seconds": secs,
                     "deviation_median": float(np.nanmedian(d)), "deviation_p90": float(np.nanpercentile(d, 90)),
                     "deviation_max": float(np.nanmax(d)), "frac_le_1e-4": float(np.mean(d <= 1e-4)),
                     "frac_le_1e-3": float(np.mean(d <= 1e-3)),
                     "gamma_halvings_histogram": np.bincount(r.halvings, minlength=5).tolist(),
                     "width_iterations": wi, "width_median": float(np.median(r.widths))}
    return out


def host_cpu():
    """CPU model (from /proc/cpuinfo) and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "nproc": usable, "cpu_count": os.cpu_count()}


def _oracle_sweep(O, w, steps, threads):
    used = O.set_threads(threads)
    lat = O.Lattice(O.Params(w.kT, w.a, w.b, w.kappa, tau=w.tau, gamma_mu=w.gamma_mu, lam=w.lam), 2, w.nx, w.ny)
    lat.init(w.rho)
    t0 = time.perf_counter()
    lat.run(steps)
    secs = time.perf_counter() - t0
    return {"value": w.nx * w.ny * w.C * steps / secs / 1e6, "unit": "MLUPS×C", "cores": used, "steps": steps,
            "seconds": secs}


def cpu_baseline(w, seed=0, legs=True, steps_all=16, steps_one=4):
    """The CPU oracle on the same workload for a few steps, on all host cores
    (OpenMP over sites; the value reported) and on one thread, with the host's
    CPU model and core count; with `legs` bounded single-thread samples beside
    the other GPU legs: the first 32 lattices of the batched workload,
    complex-step gradient directions of the adjoint case, and Appendix A
    points of the phase-diagram leg."""
    from oracle import oracle as O

    allc = _oracle_sweep(O, w, steps_all, 0)
    one = _oracle_sweep(O, w, steps_one, 1)
    out = {
        "value": allc["value"],
        "unit": "MLUPS×C",
        "cores": allc["cores"],
        "kind": "oracle",
        "sample": f"{steps_all} steps of the same {w.nx}x{w.ny} C={w.C} FP64 workload, C oracle with its per-site "
                  f"loops on {allc['cores']} OpenMP threads",
        "seconds": allc["seconds"],
        "single_thread": one,
        "host": host_cpu(),
    }
    if legs:
        O.set_threads(1)
        out["legs"] = cpu_legs(O, seed)
        O.set_threads(0)
    return out


def cpu_legs(O, seed):
    """Single-threaded oracle samples beside the batched, adjoint and
    phase-diagram legs (each a few seconds)."""
    import numpy as np

    from oracle import thermo as T
    from paper_1805_07251_amd import inputs as I
    from paper_1805_07251_amd import vdwlb as V

    legs = {}

    def maxwell(a, b, kT):
        try:
            return V.maxwell(a, b, kT)
        except V.VdwlbError:
            return None

    ws = I.batch_slabs(maxwell, seed)[:32]
    nsteps = 200
    t0 = time.perf_counter()
    site_steps = 0
    for w in ws:
        lat = O.Lattice(O.Params(w.kT, w.a, w.b, w.kappa, tau=w.tau, gamma_mu=w.gamma_mu, lam=w.lam), 2, w.nx, w.ny)
        lat.init(w.rho)
        lat.run(nsteps)
        site_steps += w.nx * w.ny * nsteps
    secs = time.perf_counter() - t0
    legs["batched"] = {"value": site_steps * ws[0].C / secs / 1e6, "unit": "MLUPS×C", "seconds": secs,
                       "sample": f"the first 32 lattices of the batched workload, {nsteps} steps each, one after "
                                 "another"}

    w, _ = I.adjoint_case(seed)
    p = O.Params(w.kT, w.a, w.b, w.kappa, tau=w.tau, gamma_mu=w.gamma_mu, lam=w.lam)
    nsteps, ndir, h = 10, 7, 1e-20
    t0 = time.perf_counter()
    for q in range(ndir):
        lc = O.Lattice(p, 2, w.nx, w.ny, complex_step=True)
        d = np.zeros(lc.prm.shape)
        d[q] = 1.0
        lc.prm = lc.prm.astype(np.complex128) + 1j * h * d
        lc.init(w.rho)
        lc.run(nsteps)
    secs = time.perf_counter() - t0
    full = secs / nsteps * 2000
    legs["adjoint"] = {"seconds": secs, "extrapolated_gradient_seconds": full,
                       "sample": f"complex-step forward of the 256x256 adjoint case in {ndir} parameter directions, "
                                 f"{nsteps} steps each; the 2000-step gradient extrapolated linearly"}

    a, b = T.two_component_params(0.4, 0.4, 1.0, 0.5)
    pts = [(2.0, 0.5), (1.2, 0.3), (0.8, 0.8)]
    t0 = time.perf_counter()
    its = [T.phase_point(NA, NB, 1 / 3, a, b)["iterations"] for NA, NB in pts]
    secs = time.perf_counter() - t0
    legs["phase_points"] = {"seconds": secs, "seconds_per_point": secs / len(pts), "iterations": its,
                            "sample": f"Appendix A pipeline at {pts} of the baseline mixture (Python oracle)"}
    return legs


def _inputs():
    from paper_1805_07251_amd import inputs as I

    return I


# The legs besides the headline, by name (each takes the parsed arguments).
LEGS = {
    # the 64^2 correctness case: L2-resident, so a latency figure, not a roofline one
    "spinodal_64_f64": lambda a: sweep_line(_inputs().spinodal_small(a.seed), "f64", 1000, a.warmup),
    # at least 1,000 steps: the first ~200 steps of a run are a few per cent slower
    "spinodal_2048_f32": lambda a: sweep_line(_inputs().spinodal_large(a.seed, dtype="f32"), "f32",
                                              max(a.steps, 1000), a.warmup),
    "mixture4_1024_f32": lambda a: sweep_line(_inputs().mixture4(a.seed), "f32", 5000, a.warmup),
    "batched": lambda a: batch_leg(a.seed, 20000, 10),
    "d1q3_line_16M_f64": lambda a: sweep_line(_inputs().line_spinodal(a.seed, L=1 << 24), "f64", 2000, a.warmup),
    "batched_d1q3": lambda a: batch_d1q3_leg(a.seed, 50000),
    "adjoint": lambda a: adjoint_leg(a.seed, a.schedule if a.legs else -1),
    "copy": lambda a: {"gbs": copy_gbs(reps=5), "bytes": 1 << 30},
}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the sweep is not sharded.", file=sys.stderr)
        sys.exit(2)
    names = [n for n in args.legs.split(",") if n]
    unknown = [n for n in names if n not in LEGS]
    if unknown:
        print(f"unknown legs {unknown}; choose from {list(LEGS)}", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1805_07251_amd import inputs as I

    torch.cuda.set_device(0)
    if args.phase:
        print(json.dumps({"profile": True, "phase_diagram_256": phase_diagram_leg()}))
        return
    if args.legs:
        out = {"profile": True}
        for n in names:
            out[n] = LEGS[n](args)
            print(f"leg {n} done", file=sys.stderr, flush=True)
        print(json.dumps(out))
        return
    w = I.spinodal_large(args.seed)
    head = sweep_line(w, "f64", args.steps, args.warmup, args.schedule if args.profile else -1)
    if args.profile:
        gbs = copy_gbs(reps=5)
        print(json.dumps({"profile": True, "sweep": head, "copy_kernel_gbs": gbs, "copy_bytes": 1 << 30}))
        return
    sites = w.nx * w.ny
    achieved = head["gbs"]
    traffic = traffic_from_profiles(head["schedule"])
    out = {
        "metric": METRIC,
        "value": head["mlups_x_c"],
        "unit": "MLUPS×C",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["us_per_step"] / 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "spinodal decomposition 2048x2048 D2Q9, 2 components, FP64",
                   "lattice": [w.nx, w.ny], "components": w.C, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic},
        "mlups": head["mlups"],
        "status": head["status"],
        "schedule": head["schedule"],
    }
    extra = {}
    if not args.no_extra:
        extra["headline_protocol"] = protocol_leg(w, "f64", head["schedule"])
        for n in ("spinodal_64_f64", "spinodal_2048_f32", "mixture4_1024_f32"):
            extra[n] = LEGS[n](args)
        extra["copy_kernel_gbs"] = copy_gbs()
        for n in ("batched", "d1q3_line_16M_f64", "batched_d1q3", "adjoint"):
            extra[n] = LEGS[n](args)
        extra["phase_diagram_256"] = phase_diagram_leg()
        extra["verification"] = verification_leg()
    out["extra"] = extra
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, seed=args.seed, legs=not args.no_extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

"""Benchmark of the fused D2Q9 sweep on one MI355X.

Workload: the 2048x2048 two-component spinodal-decomposition lattice in FP64
(D2Q9, a12 drawn in [0.7, 1.1] a11, +-1 % seeded noise), one step = one fused
sweep over the whole lattice (stream, moments, chemical potential, force,
friction, collision).  Prints one JSON line.

value      MLUPS x components (million site updates per second times C), inputs
           resident in HBM, timed with HIP events over exactly --steps steps.
roofline   the sweep kernel against the 8 TB/s HBM peak, with algorithmic bytes
           2 * 9 * C * sizeof(real) per site update.
cpu_baseline  the CPU oracle on the host, a bounded sample of the same workload.
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


def sweep_line(w, dtype, steps, warmup):
    from paper_1805_07251_amd.lattice import Lattice

    lat = Lattice.from_workload(w, dtype=dtype)
    lat.init(w.rho)
    sched = lat.autotune()
    lat.init(w.rho)
    secs = time_steps(lat, steps, warmup)
    st = lat.status()
    sites = w.nx * w.ny
    real = 8 if dtype == "f64" else 4
    bytes_per_site = 2 * 9 * w.C * real
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


def traffic_from_profiles(kernel_key: str):
    """HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE,
    recorded in profiles/traffic.md together with the hash of the sweep
    source they were taken on; None when the source has changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"source_sha256:\s*([0-9a-f]{64})", txt)
    if not m or m.group(1) != sweep_source_hash():
        return None
    m = re.search(rf"{re.escape(kernel_key)}\s*\|\s*([0-9.eE+]+)\s*\|", txt)
    return float(m.group(1)) if m else None


def sweep_source_hash():
    import hashlib

    h = hashlib.sha256()
    for fn in ("sweep.hpp", "launch.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1805_07251_amd", "csrc", fn), "rb").read())
    return h.hexdigest()


def cpu_baseline(w, steps=5):
    """The CPU oracle on the same workload for a few steps (single thread)."""
    from oracle import oracle as O

    lat = O.Lattice(O.Params(w.kT, w.a, w.b, w.kappa, tau=w.tau, gamma_mu=w.gamma_mu, lam=w.lam), 2, w.nx, w.ny)
    lat.init(w.rho)
    t0 = time.perf_counter()
    lat.run(steps)
    secs = time.perf_counter() - t0
    return {
        "value": w.nx * w.ny * w.C * steps / secs / 1e6,
        "unit": "MLUPS×C",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{steps} steps of the same {w.nx}x{w.ny} C={w.C} FP64 workload, single-threaded C oracle",
        "seconds": secs,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the sweep is not sharded.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1805_07251_amd import inputs as I

    torch.cuda.set_device(0)
    w = I.spinodal_large(args.seed)
    head = sweep_line(w, "f64", args.steps, args.warmup)
    if args.profile:
        gbs = copy_gbs(reps=5)
        print(json.dumps({"profile": True, "sweep": head, "copy_kernel_gbs": gbs, "copy_bytes": 1 << 30}))
        return
    sites = w.nx * w.ny
    achieved = head["gbs"]
    traffic = traffic_from_profiles("k_sweep<double, 2")
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
        extra["spinodal_2048_f32"] = sweep_line(I.spinodal_large(args.seed, dtype="f32"), "f32", args.steps,
                                                args.warmup)
        w2 = I.mixture4(args.seed)
        extra["mixture4_1024_f32"] = sweep_line(w2, "f32", 5000, args.warmup)
        extra["copy_kernel_gbs"] = copy_gbs()
    out["extra"] = extra
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

"""Write tests/golden/sweep_*.json: densities of the full-size workloads at
the parity horizons, computed by the CPU oracle alone from the seeded inputs.

  sweep_spinodal2048_f64.json  2048 x 2048, 2 components, FP64 input; rho^c at
                               512 seeded sites (and the four corners) after
                               100 and 1000 steps.
  sweep_spinodal2048_f32.json  the same lattice from its FP32-rounded input;
                               rho^c at the same sites after 100 steps.
  sweep_mixture4_1024.json     1024 x 1024, 4 components, FP32-rounded input;
                               rho^c at 512 seeded sites after 100 steps.
  sweep_adjoint256.json        256 x 256, 2 components (the adjoint case);
                               rho^c on the stride-4 sub-grid (x, y = 1, 5, ...,
                               253) after 2000 steps.

The oracle runs in FP64 on all host cores (its results do not depend on the
thread count).  Run: python tests/golden/make_sweep_goldens.py [name ...]
(about 12 minutes on eight cores).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1805_07251_amd import inputs as I  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def lattice(w):
    p = O.Params(w.kT, w.a, w.b, w.kappa, tau=w.tau, gamma_mu=w.gamma_mu, lam=w.lam, force=w.force)
    lat = O.Lattice(p, 2, w.nx, w.ny)
    rho = np.asarray(w.rho, dtype=np.float64)
    if w.dtype == "f32":  # the densities an FP32 plan starts from
        rho = rho.astype(np.float32).astype(np.float64)
    lat.init(rho)
    return lat


def sample_sites(nx, ny, n, seed):
    rng = np.random.default_rng(seed)
    pts = [(0, 0), (nx - 1, ny - 1), (0, ny - 1), (nx - 1, 0)]
    pts += [(int(x), int(y)) for x, y in zip(rng.integers(0, nx, n), rng.integers(0, ny, n))]
    return pts


def sampled(lat, pts):
    rho = lat.moments()[0]
    return [[float(rho[c, y, x]) for c in range(rho.shape[0])] for x, y in pts]


def run_sampled(w, horizons, pts):
    lat = lattice(w)
    out, done = {}, 0
    for h in horizons:
        st = lat.run(h - done)
        assert st == 0, (w.name, h, st)
        done = h
        out[str(h)] = sampled(lat, pts)
        print(f"{w.name}: {h} steps", flush=True)
    return out


def write(name, payload):
    payload["script"] = "tests/golden/make_sweep_goldens.py"
    payload["method"] = "CPU oracle (FP64) from the seeded inputs of paper_1805_07251_amd.inputs"
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(payload, f, indent=0)


def spinodal_f64():
    w = I.spinodal_large(0)
    pts = sample_sites(w.nx, w.ny, 512, 2048)
    write("sweep_spinodal2048_f64.json", {"case": "spinodal_large(seed=0), FP64 input", "sites_xy": pts,
                                          "rho": run_sampled(w, [100, 1000], pts)})


def spinodal_f32():
    w = I.spinodal_large(0, dtype="f32")
    pts = sample_sites(w.nx, w.ny, 512, 2048)
    write("sweep_spinodal2048_f32.json", {"case": "spinodal_large(seed=0, dtype='f32'), FP32-rounded input",
                                          "sites_xy": pts, "rho": run_sampled(w, [100], pts)})


def mixture4():
    w = I.mixture4(0)
    pts = sample_sites(w.nx, w.ny, 512, 1024)
    write("sweep_mixture4_1024.json", {"case": "mixture4(seed=0), FP32-rounded input", "sites_xy": pts,
                                       "rho": run_sampled(w, [100], pts)})


def adjoint256():
    w, _ = I.adjoint_case(0)
    lat = lattice(w)
    assert lat.run(2000) == 0
    rho = lat.moments()[0]
    sub = rho[:, 1::4, 1::4]
    write("sweep_adjoint256.json", {"case": "adjoint_case(seed=0), 2000 steps", "stride": 4, "offset": 1,
                                    "rho": sub.tolist()})
    print("adjoint256: 2000 steps", flush=True)


JOBS = {"spinodal_f64": spinodal_f64, "spinodal_f32": spinodal_f32, "mixture4": mixture4, "adjoint256": adjoint256}

if __name__ == "__main__":
    O.set_threads(0)
    for name in sys.argv[1:] or list(JOBS):
        t0 = time.time()
        JOBS[name]()
        print(f"{name} done in {time.time() - t0:.0f} s", flush=True)

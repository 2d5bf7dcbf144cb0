"""GPU tests of the batched sweep (persistent kernel over many quasi-1-D
lattices) through the C-ABI.

The batch walks each lattice in full-height strips whose rows wrap inside
LDS, with the same per-site arithmetic as the plain sweep, so every instance
must match a plain per-instance run bit for bit; small instances are also
compared with the oracle.
"""
import numpy as np
import pytest

from oracle import thermo as T
from paper_1805_07251_amd import inputs as I

from ._util import oracle_run, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_07251_amd import batch, lattice

    return batch, lattice


def slabs(seed, idx, ny=4, lmax=None):
    return I.batch_slabs(T.maxwell_single, seed, ny=ny, idx=list(idx), lmax=lmax)


def plain_state(lattice, w, nsteps, dtype="f64"):
    lat = lattice.Lattice.from_workload(w, dtype=dtype)
    lat.init(w.rho)
    lat.run(nsteps)
    return lat.state_sites().cpu().numpy()


def batch_run(batch, ws, nsteps, dtype="f64", threads=256, chunks=None, blocking=0):
    b = batch.Batch(ws, dtype=dtype)
    b.set_launch(threads, 0)
    b.set_blocking(blocking)
    b.init([w.rho for w in ws])
    for n in chunks or [nsteps]:
        b.run(n)
    return b


@pytest.mark.parametrize("threads", [256, 1024])
def test_batch_matches_plain_bitwise(gpu, threads):
    batch, lattice = gpu
    ws = slabs(0, range(10))
    b = batch_run(batch, ws, 60, threads=threads)
    st = b.status()
    for k, w in enumerate(ws):
        got = b.state(k).cpu().numpy()
        ref = plain_state(lattice, w, 60)
        if st[k] == 0:
            assert np.array_equal(got, ref), k


@pytest.mark.parametrize("taus", ["mixed", "none"])
def test_batch_tau_mix_matches_plain(gpu, taus):
    """Instances with tau != 1 (all of them, or every other one) take the
    general collision; each must still equal its plain run bit for bit."""
    batch, lattice = gpu
    ws = slabs(6, range(6), lmax=300)
    for k, w in enumerate(ws):
        if taus == "none" or k % 2 == 1:
            w.tau = 0.8 + 0.05 * k
    b = batch_run(batch, ws, 30)
    st = b.status()
    for k, w in enumerate(ws):
        assert st[k] == 0, k
        assert np.array_equal(b.state(k).cpu().numpy(), plain_state(lattice, w, 30)), k


def test_batch_against_oracle(gpu, orc):
    batch, _ = gpu
    ws = slabs(1, range(3), lmax=40)
    b = batch_run(batch, ws, 30)
    assert np.all(b.status() == 0)
    rho = [r.cpu().numpy() for r in b.densities()]
    for k, w in enumerate(ws):
        ref, st = oracle_run(orc, w, 30)
        assert st == 0
        assert rel_err(rho[k], ref.moments()[0]) <= 1e-13


@pytest.mark.parametrize("ny", [1, 2, 8])
def test_batch_heights(gpu, ny):
    batch, lattice = gpu
    ws = slabs(2, range(5), ny=ny, lmax=300)
    for w in ws:  # break the y-uniformity so the y stencils matter
        w.rho = w.rho * (1 + 0.005 * np.random.default_rng(ny).uniform(-1, 1, w.rho.shape))
    b = batch_run(batch, ws, 40)
    for k, w in enumerate(ws):
        assert np.array_equal(b.state(k).cpu().numpy(), plain_state(lattice, w, 40)), k


def test_batch_f32(gpu):
    batch, lattice = gpu
    ws = slabs(3, range(6), lmax=256)
    b = batch_run(batch, ws, 40, dtype="f32")
    for k, w in enumerate(ws):
        assert np.array_equal(b.state(k).cpu().numpy(), plain_state(lattice, w, 40, dtype="f32")), k


def test_unphysical_instance_is_isolated(gpu):
    batch, lattice = gpu
    ws = slabs(4, range(4), lmax=200)
    ws[1].rho = ws[1].rho.copy()
    ws[1].rho[:, :, 10:20] = 12.0  # eta > 1 in a block of instance 1
    b = batch_run(batch, ws, 25)
    st = b.status()
    assert st[1] == 1
    for k in (0, 2, 3):
        assert st[k] == 0
        assert np.array_equal(b.state(k).cpu().numpy(), plain_state(lattice, ws[k], 25)), k


def test_split_runs_replay_graph(gpu):
    """Runs are replayed from a captured graph (queue counter reset by a
    kernel inside it); 3 x 20 steps equal 60 steps."""
    batch, _ = gpu
    ws = slabs(5, range(6), lmax=300)
    a = batch_run(batch, ws, 0, chunks=[20, 20, 20])
    b = batch_run(batch, ws, 60)
    for k in range(len(ws)):
        assert np.array_equal(a.state(k).cpu().numpy(), b.state(k).cpu().numpy()), k


def test_full_batch_sampled(gpu):
    """The 1024-lattice workload in the benchmark's launch shape: 100 steps,
    six sampled instances (largest, smallest, random) against plain runs."""
    batch, lattice = gpu
    d = I.batch_draws(0)
    ws = slabs(0, range(len(d.L)))
    b = batch_run(batch, ws, 100, threads=1024)
    st = b.status()
    order = np.argsort(d.L)
    for k in [int(order[0]), int(order[-1]), 3, 77, 500, 1000]:
        if st[k] == 0:
            assert np.array_equal(b.state(k).cpu().numpy(), plain_state(lattice, ws[k], 100)), k
    assert (st == 0).mean() > 0.9


def test_full_size_instances_against_oracle(gpu, orc):
    """The 1024-lattice workload in the benchmark's launch shape (1024-thread
    workgroups), 200 steps: the smallest, a middle-sized and the largest
    instance (L = 128 .. 1024, several strips each, the single-wrap path of
    every production instance) against the oracle, element by element on the
    densities within 1e-12 of the largest density, the FP64 bound used for
    runs of hundreds of steps (round-off grows with the step count: measured
    1.3e-13 at L = 128 after 200 steps, against 1e-13 after 30)."""
    batch, _ = gpu
    d = I.batch_draws(0)
    ws = slabs(0, range(len(d.L)))
    b = batch_run(batch, ws, 200, threads=1024)
    st = b.status()
    order = np.argsort(d.L, kind="stable")
    mid = int(np.argmin(np.abs(np.asarray(d.L) - 577)))
    picks = [int(order[0]), mid, int(order[-1])]
    assert d.L[picks[0]] <= 140 and d.L[picks[2]] >= 1000
    rho = b.densities()
    for k in picks:
        assert st[k] == 0, k
        ref, ost = oracle_run(orc, ws[k], 200)
        assert ost == 0
        err = rel_err(rho[k].cpu().numpy(), ref.moments()[0])
        print(f"batch instance {k}: L = {d.L[k]}, max rel density error {err:.2e}", flush=True)
        assert err <= 1e-12, k


@pytest.mark.parametrize("K", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("nsteps", [1, 7, 30])
def test_blocked_batch_matches_plain_bitwise(gpu, K, nsteps):
    """Temporal blocking (K steps per block in LDS, strips of 64 - 6K columns
    with 3K halo columns each side) against plain per-instance runs, bit for
    bit, for step counts below, between and above multiples of K (the block
    count keeps the parity of the step count, so the result is in the same
    pool), on instances from 30 columns (narrower than a strip and its halo:
    the halo wraps onto the instance itself) to several strips."""
    batch, lattice = gpu
    ws = slabs(7, range(6), lmax=300)
    ws[0] = slabs(8, [0], lmax=30)[0]
    ws[1] = slabs(9, [0], lmax=45)[0]
    for w in ws:  # break the y-uniformity so the y stencils matter
        w.rho = w.rho * (1 + 0.005 * np.random.default_rng(K).uniform(-1, 1, w.rho.shape))
    b = batch_run(batch, ws, nsteps, blocking=K)
    st = b.status()
    for k, w in enumerate(ws):
        assert st[k] == 0, k
        assert np.array_equal(b.state(k).cpu().numpy(), plain_state(lattice, w, nsteps)), (k, w.nx)


@pytest.mark.parametrize("taus", ["mixed", "none"])
def test_blocked_batch_tau_mix_and_f32(gpu, taus):
    """The blocked kernel with instances of tau != 1 (all, or every other one)
    and in FP32: each equals its plain run bit for bit."""
    batch, lattice = gpu
    ws = slabs(10, range(5), lmax=260)
    for k, w in enumerate(ws):
        if taus == "none" or k % 2 == 1:
            w.tau = 0.8 + 0.05 * k
    b = batch_run(batch, ws, 21, blocking=4)
    for k, w in enumerate(ws):
        assert np.array_equal(b.state(k).cpu().numpy(), plain_state(lattice, w, 21)), k
    if taus == "mixed":
        b = batch_run(batch, ws, 21, dtype="f32", blocking=4)
        for k, w in enumerate(ws):
            assert np.array_equal(b.state(k).cpu().numpy(), plain_state(lattice, w, 21, dtype="f32")), k


def test_blocked_unphysical_instance_is_isolated(gpu):
    """An instance with eta > 1 in a block of sites stops at the end of the
    first block with the first unphysical step in its status word (step 1);
    the others run on and equal their plain runs."""
    batch, lattice = gpu
    ws = slabs(4, range(4), lmax=200)
    ws[1].rho = ws[1].rho.copy()
    ws[1].rho[:, :, 10:20] = 12.0
    b = batch_run(batch, ws, 25, blocking=4)
    st = b.status()
    assert st[1] == 1
    for k in (0, 2, 3):
        assert st[k] == 0
        assert np.array_equal(b.state(k).cpu().numpy(), plain_state(lattice, ws[k], 25)), k


def test_blocked_full_batch_sampled(gpu):
    """The 1024-lattice workload with temporal blocking (4 steps per block):
    100 steps, six sampled instances against plain runs bit for bit."""
    batch, lattice = gpu
    d = I.batch_draws(0)
    ws = slabs(0, range(len(d.L)))
    b = batch_run(batch, ws, 100, blocking=4)
    st = b.status()
    order = np.argsort(d.L)
    for k in [int(order[0]), int(order[-1]), 3, 77, 500, 1000]:
        if st[k] == 0:
            assert np.array_equal(b.state(k).cpu().numpy(), plain_state(lattice, ws[k], 100)), k
    assert (st == 0).mean() > 0.9


def test_blocking_rejects_unsupported(gpu):
    """Blocking is built for D2Q9 batches of height 4 with C <= 2."""
    batch, _ = gpu
    from paper_1805_07251_amd import vdwlb as V

    b = batch.Batch(slabs(2, range(2), ny=2, lmax=100))
    with pytest.raises(V.VdwlbError) as ei:
        b.set_blocking(4)
    assert ei.value.status == V.E_UNSUPPORTED
    b = batch.Batch(slabs(2, range(2), lmax=100))
    for bad in (1, 7, -1):
        with pytest.raises(V.VdwlbError) as ei:
            b.set_blocking(bad)
        assert ei.value.status == V.E_INVALID_ARG

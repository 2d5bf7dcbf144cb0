"""The no-allocation adjoint segment (vdwlb_adjoint_segment_noalloc) against
vdwlb_adjoint_segment with a caller-owned workspace, through the C-ABI.

Both run the same kernels in the same order on the same inputs, so the
cotangent state and the parameter cotangents must agree bit for bit.  Two
calls in a row: the second on a smaller lattice with fewer (and an odd number
of) steps, so it runs on the array the first call left behind.  A request
whose workspace would exceed the fixed array is refused before anything is
enqueued.
"""
import numpy as np
import pytest

from paper_1805_07251_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_07251_amd import lattice
    from paper_1805_07251_amd import vdwlb as V

    return lattice, V


def _case(lattice, nx, ny, seed, fwd_steps=5):
    """A plan-bound lattice advanced a few steps from seeded densities, and a
    seeded cotangent state of the same shape."""
    w = I.spinodal_small(seed, n=max(nx, ny))
    rng = np.random.default_rng(seed)
    rho = 2.625 * (1 + 0.02 * rng.uniform(-1, 1, (2, ny, nx)))
    lat = lattice.Lattice(nx, ny, w.kT, w.a, w.b, w.kappa, w.tau, w.gamma_mu, w.lam)
    lat.init(rho)
    lat.run(fwd_steps)
    n = lat.plan.state_elems
    fbar = torch.as_tensor(rng.standard_normal(n), device="cuda")
    return lat, fbar


def _segment(lattice, V, lat, fbar0, nsteps, noalloc):
    lib = V.lib()
    plan = lat.plan.handle
    f_ckpt = lat.state
    fbar = fbar0.clone()
    pbar = torch.zeros(int(lib.vdwlb_adjoint_param_count(plan)), dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    if noalloc:
        st = lib.vdwlb_adjoint_segment_noalloc(plan, f_ckpt.data_ptr(), nsteps, fbar.data_ptr(), pbar.data_ptr(), s)
    else:
        ws = torch.empty(int(lib.vdwlb_adjoint_workspace_bytes(plan, nsteps)) // 8 + 1, dtype=torch.float64,
                         device="cuda")
        st = lib.vdwlb_adjoint_segment(plan, f_ckpt.data_ptr(), nsteps, fbar.data_ptr(), ws.data_ptr(),
                                       pbar.data_ptr(), s)
    V.check(st, "adjoint segment")
    torch.cuda.synchronize()
    # lattice sites only: the plane padding of an odd-length segment's result
    # is copied from the workspace and carries whatever that held
    sites = fbar.view(9, lat.plan.plane, 2)[:, :lat.nx * lat.ny, :]
    return sites.cpu().numpy(), pbar.cpu().numpy()


def test_noalloc_segment_equals_workspace_segment(gpu):
    lattice, V = gpu
    for (nx, ny, nsteps, seed) in [(64, 64, 12, 1), (40, 28, 7, 2)]:
        print(f"noalloc adjoint segment: {nx}x{ny} C=2 FP64, {nsteps} steps, seed {seed}", flush=True)
        lat, fbar0 = _case(lattice, nx, ny, seed)
        want_f, want_p = _segment(lattice, V, lat, fbar0, nsteps, noalloc=False)
        got_f, got_p = _segment(lattice, V, lat, fbar0, nsteps, noalloc=True)
        assert np.abs(want_f).max() > 0 and np.abs(want_p).max() > 0
        assert np.array_equal(got_f, want_f), (nx, ny, np.abs(got_f - want_f).max())
        assert np.array_equal(got_p, want_p), (nx, ny, got_p, want_p)


def test_noalloc_segment_refuses_oversized_requests(gpu):
    """A 256 x 256 lattice needs about 3 MB of workspace per step, so 100
    steps exceed the fixed 64 MiB array: refused with E_CAPACITY, the
    cotangent left untouched; 5 steps fit."""
    lattice, V = gpu
    lib = V.lib()
    lat, fbar0 = _case(lattice, 256, 256, 3, fwd_steps=1)
    plan = lat.plan.handle
    assert lib.vdwlb_adjoint_workspace_bytes(plan, 100) > 64 << 20
    fbar = fbar0.clone()
    pbar = torch.zeros(int(lib.vdwlb_adjoint_param_count(plan)), dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    st = lib.vdwlb_adjoint_segment_noalloc(plan, lat.state.data_ptr(), 100, fbar.data_ptr(), pbar.data_ptr(), s)
    assert st == V.E_CAPACITY
    torch.cuda.synchronize()
    assert torch.equal(fbar, fbar0) and float(pbar.abs().max()) == 0.0
    assert lib.vdwlb_adjoint_workspace_bytes(plan, 5) <= 64 << 20
    want_f, want_p = _segment(lattice, V, lat, fbar0, 5, noalloc=False)
    got_f, got_p = _segment(lattice, V, lat, fbar0, 5, noalloc=True)
    assert np.array_equal(got_f, want_f) and np.array_equal(got_p, want_p)

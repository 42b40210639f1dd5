"""Host-side checks of facts the kernels rely on (no GPU needed)."""
import numpy as np


def test_bitwise_max_of_wavespeeds():
    """The final sweep folds |u_d| + c into the time-step slots with a 64-bit
    unsigned max on the bit patterns.  For values that are +0 or above, or
    NaN, that is the floating-point maximum, and any NaN wins (so dt turns
    NaN as the NaN-propagating maximum of the separate pass makes it)."""
    rng = np.random.default_rng(7)
    for _ in range(200):
        v = np.abs(rng.standard_normal(64)) * 10.0 ** rng.uniform(-300, 300, 64)
        v[rng.integers(0, 64, 3)] = rng.choice([0.0, np.inf, 5e-324])
        bits = v.view(np.uint64)
        assert bits.max().view(np.float64) == v.max()
        w = v.copy()
        w[rng.integers(0, 64)] = rng.choice([np.nan, -np.nan])
        assert np.isnan(w.view(np.uint64).max().view(np.float64))
    # |u| + c is never -0: +0 + -0 is +0 under round-to-nearest
    assert np.signbit(np.float64(0.0) + np.float64(-0.0)) == False  # noqa: E712


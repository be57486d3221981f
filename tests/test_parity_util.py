"""CPU checks of the test-side helpers that other tests trust."""
import numpy as np

from parity_util import chebyshev_capped


def test_chebyshev_capped_is_brute_force_distance():
    # brute force on small random grids: min over occupied cells of max |dc|
    rng = np.random.default_rng(11)
    for shape, p, cap in (((7, 9, 8), 0.05, 32), ((12, 5, 6), 0.01, 3), ((4, 4, 4), 0.0, 5)):
        occ = rng.random(shape) < p
        got = chebyshev_capped(occ, cap)
        idx = np.argwhere(occ)
        for c in np.ndindex(*shape):
            d = cap if len(idx) == 0 else min(cap, int(np.abs(idx - np.array(c)).max(axis=1).min()))
            assert got[c] == d, (shape, c, got[c], d)

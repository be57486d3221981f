"""The octant fields of the FP32 walk's empty-cell records (the test helper
that the GPU walk view is compared with), pinned on the CPU against brute
force: for every empty cell and octant, blocks grown one step at a time and
checked cell by cell; and the property the walk relies on, that the block
of max(d, 2M + 1) cells per axis ahead of a cell in its octant is empty."""
import numpy as np
import pytest

from parity_util import chebyshev_capped, octant_blocks


def _brute(occ, cap):
    nz, ny, nx = occ.shape
    mcap = min(7, (cap - 1) // 2)
    out = np.zeros(occ.shape, dtype=np.uint32)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if occ[z, y, x]:
                    continue
                for o in range(8):
                    sx, sy, sz = [(-1 if (o >> a) & 1 else 1) for a in range(3)]
                    M = 0
                    for m in range(1, mcap + 1):
                        cz, cy, cx = z + m * sz, y + m * sy, x + m * sx
                        if not (0 <= cz < nz and 0 <= cy < ny and 0 <= cx < nx):
                            break
                        zs = range(min(z, z + 2 * m * sz), max(z, z + 2 * m * sz) + 1)
                        ys = range(min(y, y + 2 * m * sy), max(y, y + 2 * m * sy) + 1)
                        xs = range(min(x, x + 2 * m * sx), max(x, x + 2 * m * sx) + 1)
                        if any(occ[a, b, c] for a in zs if 0 <= a < nz
                               for b in ys if 0 <= b < ny for c in xs if 0 <= c < nx):
                            break
                        M = m
                    out[z, y, x] |= np.uint32(M << (3 * o))
    return out


@pytest.mark.parametrize("seed,shape,frac,cap", [(1, (7, 8, 9), 0.08, 32), (2, (6, 11, 5), 0.02, 32),
                                                  (3, (9, 9, 9), 0.01, 4), (4, (5, 6, 7), 0.3, 32),
                                                  (5, (8, 7, 6), 0.05, 1), (6, (20, 20, 20), 0.0, 32)])
def test_blocks_match_brute_force(seed, shape, frac, cap):
    rng = np.random.default_rng(seed)
    occ = rng.random(shape) < frac
    if seed == 6:  # open space but for the far corner
        occ[-1, -1, -1] = True
    got = octant_blocks(occ, cap)
    assert np.array_equal(got, _brute(occ, cap))
    if cap <= 2:  # no block beyond a single cell fits the cap
        assert not got.any()
    if seed == 6:  # the near corner's block ahead reaches the 7 the field holds
        assert got[0, 0, 0] & 7 == 7


def test_jump_block_is_empty():
    rng = np.random.default_rng(9)
    occ = rng.random((12, 10, 11)) < 0.03
    dist = chebyshev_capped(occ)
    blocks = octant_blocks(occ)
    n_longer = 0
    for z, y, x in zip(*np.nonzero(~occ)):
        d = max(int(dist[z, y, x]), 1)
        for o in range(8):
            M = int(blocks[z, y, x] >> np.uint32(3 * o)) & 7
            k = max(d, 2 * M + 1)
            n_longer += k > d
            sx, sy, sz = [(-1 if (o >> a) & 1 else 1) for a in range(3)]
            zs = sorted((z, z + (k - 1) * sz)); ys = sorted((y, y + (k - 1) * sy)); xs = sorted((x, x + (k - 1) * sx))
            blk = occ[max(zs[0], 0):zs[1] + 1, max(ys[0], 0):ys[1] + 1, max(xs[0], 0):xs[1] + 1]
            assert not blk.any(), (z, y, x, o, d, M)
    assert n_longer > 0  # the case is not vacuous

"""GPU grid build (count / scan / scatter / sort) and device Philox against the
oracle: cell lists and Philox words bit for bit."""
import math

import numpy as np
import pytest

import scenegen
from parity_util import chebyshev_capped, octant_blocks

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tr():
    import paper_0801_1500_amd as tr
    tr.lib()
    return tr


def _bare_cylinders():
    pos, _ = scenegen.random_walk(400, 12.0, 9)
    return scenegen.Scene(np.zeros((0, 3)), np.zeros(0), np.zeros((0, 3), np.float32),
                          pos[:-1].copy(), pos[1:].copy(), np.full(399, 0.4),
                          np.full((399, 3), 0.7, np.float32),
                          np.array([scenegen.LIGHT0]), np.ones((1, 3)))


@pytest.mark.parametrize("which,lam", [("tiny", 0.5), ("tiny", 4.0), ("tiny", 30.0),
                                       ("protein", 4.0), ("protein", 1.5), ("cyl", 3.0)])
def test_grid_equals_oracle(tr, oracle_mod, which, lam):
    scene = {"tiny": lambda: scenegen.tiny_scene(1), "protein": scenegen.protein_scene,
             "cyl": _bare_cylinders}[which]()
    print("grid case", which, lam, flush=True)
    gs = tr.Scene(scene, cells_per_prim=lam)
    og = oracle_mod.Grid(scene, lam)
    lo, hi, res, n_refs = gs.grid_info()
    olo, ohi, ores, on = og.info()
    assert np.array_equal(res, ores) and np.array_equal(lo, olo) and np.array_equal(hi, ohi)
    assert n_refs == on
    cb, refs = gs.grid_arrays()
    ocb, orefs = og.arrays()
    assert np.array_equal(cb, ocb)
    assert np.array_equal(refs, orefs)


@pytest.mark.parametrize("which,lam", [("tiny", 4.0), ("protein", 4.0), ("protein", 24.0),
                                       ("cyl", 3.0)])
def test_walk_view_matches_grid(tr, which, lam):
    # The FP32 walk's cell records and per-cell lists (with end markers),
    # rebuilt here from the canonical grid and the empty-space distance.
    scene = {"tiny": lambda: scenegen.tiny_scene(1), "protein": scenegen.protein_scene,
             "cyl": _bare_cylinders}[which]()
    print("walk view case", which, lam, flush=True)
    gs = tr.Scene(scene, cells_per_prim=lam)
    lo, hi, res, n_refs = gs.grid_info()
    cb, refs = gs.grid_arrays()
    ci, wr = gs.walk_arrays()
    cnt = np.diff(cb.astype(np.int64))
    occ = cnt > 0
    dist = chebyshev_capped(occ.reshape(res[2], res[1], res[0])).ravel()
    assert len(wr) == n_refs + int(occ.sum())
    # empty cells: (-distance, bit 31 and the empty block ahead per octant)
    assert np.array_equal(ci[~occ, 0], -np.maximum(dist[~occ], 1))
    ext = octant_blocks(occ.reshape(res[2], res[1], res[0])).ravel()
    want_c = (ext[~occ] | np.uint32(0x80000000)).view(np.int32)
    assert np.array_equal(ci[~occ, 1], want_c)
    print("empty cells", int((~occ).sum()), "with a block ahead", int((ext[~occ] != 0).sum()), flush=True)
    # occupied cells: byte offset of the list (4 x the exclusive prefix of
    # list lengths + 1) and its first entry, 16 x the first id, bit 0 set
    # when that entry is the list's only one
    size = np.where(occ, cnt + 1, 0)
    start = np.cumsum(size) - size
    assert np.array_equal(ci[occ, 0], 4 * start[occ])
    assert np.array_equal(ci[occ, 1], 16 * refs[cb[:-1][occ]].astype(np.int64) + (cnt[occ] == 1))
    # lists: the canonical references in cell order as 16 x id, the last of
    # each with bit 0 set, each list closed by ~0
    want = np.empty(len(wr), dtype=np.uint32)
    end = np.zeros(len(wr), dtype=bool)
    end[(start + cnt)[occ]] = True
    last = np.zeros(len(wr), dtype=bool)
    last[(start + cnt - 1)[occ]] = True
    want[end] = 0xFFFFFFFF
    want[~end] = refs * 16
    want[last] |= 1
    assert np.array_equal(wr, want)


def test_grid_rebuild_changes_density(tr, oracle_mod):
    scene = scenegen.protein_scene()
    gs = tr.Scene(scene, cells_per_prim=4.0)
    gs.rebuild(8.0)
    cb, refs = gs.grid_arrays()
    ocb, orefs = oracle_mod.Grid(scene, 8.0).arrays()
    assert np.array_equal(cb, ocb) and np.array_equal(refs, orefs)
    gs.rebuild(0.0)  # keeps 8.0
    assert np.array_equal(gs.grid_arrays()[1], orefs)


def test_philox_bit_identical(tr, oracle_mod):
    import torch
    rng = np.random.default_rng(4)
    n = 1 << 16
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:1024, :] = 0
    ctr[:1024, 0] = np.arange(1024)
    key = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    key[:512] = 0
    want = oracle_mod.philox(ctr, key)
    got = tr.debug_philox(torch.from_numpy(ctr.view(np.int32)).cuda(),
                          torch.from_numpy(key.view(np.int32)).cuda())
    assert np.array_equal(got.cpu().numpy().view(np.uint32), want)


def test_ao_directions_match_fp64(tr, oracle_mod):
    import torch
    rng = np.random.default_rng(5)
    n = 4096
    nrm = rng.standard_normal((n, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    nrm[:4] = [[0, 0, 1], [0, 0, -1], [1, 0, 0], [0, -1, 0]]
    pix = rng.integers(0, 1 << 24, n).astype(np.uint32)
    smp = rng.integers(0, 64, n).astype(np.uint32)
    seed = (7 << 32) + 11
    w = tr.debug_ao_dirs(torch.from_numpy(nrm.astype(np.float32)).cuda(),
                         torch.from_numpy(pix.view(np.int32)).cuda(),
                         torch.from_numpy(smp.view(np.int32)).cuda(), 3, seed).cpu().numpy()
    err = 0.0
    for i in range(n):
        u1, u2 = oracle_mod.ao_uniforms(int(pix[i]), int(smp[i]), 3, seed)
        n32 = nrm[i].astype(np.float32).astype(np.float64)
        ref = oracle_mod.ao_direction(n32 / np.linalg.norm(n32), u1, u2)
        err = max(err, float(np.abs(w[i] - ref).max()))
        assert w[i] @ nrm[i] > -1e-6
    assert err < 2e-6, err

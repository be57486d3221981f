"""Statistical pins of the oracle's Philox4x32-10 stream and invariants of the
seeded scene generators.  The published known-answer vectors are not
available, so Philox is pinned by bijectivity, avalanche and uniformity;
against those vectors it is parity unpinned.  CPU only."""
import math

import numpy as np

import scenegen


def test_philox_bijective_per_word(oracle_mod):
    # a bijection of the counter for a fixed key: varying any single word
    # over 2^16 values never collides
    rng = np.random.default_rng(0)
    key = rng.integers(0, 2 ** 32, size=(1, 2), dtype=np.uint64).astype(np.uint32)
    for word in range(4):
        ctr = np.tile(rng.integers(0, 2 ** 32, size=4, dtype=np.uint64).astype(np.uint32), (65536, 1))
        ctr[:, word] = np.arange(65536, dtype=np.uint32)
        out = oracle_mod.philox(ctr, np.repeat(key, 65536, axis=0))
        packed = out.view(np.dtype((np.void, 16))).ravel()
        assert len(np.unique(packed)) == 65536, word
        # and every output word depends on the varied word
        for w in range(4):
            assert len(np.unique(out[:, w])) > 65000, (word, w)


def test_philox_avalanche(oracle_mod):
    rng = np.random.default_rng(1)
    n = 4096
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    base = oracle_mod.philox(ctr, key)
    for word in range(6):  # 4 counter words, 2 key words
        c2, k2 = ctr.copy(), key.copy()
        bit = np.uint32(1) << np.uint32(rng.integers(32))
        if word < 4:
            c2[:, word] ^= bit
        else:
            k2[:, word - 4] ^= bit
        flip = oracle_mod.philox(c2, k2) ^ base
        frac = np.unpackbits(flip.view(np.uint8)).mean()
        assert abs(frac - 0.5) < 0.01, (word, frac)


def test_philox_uniformity(oracle_mod):
    n = 1 << 20
    pix = np.arange(n, dtype=np.uint32)
    ctr = np.stack([pix, np.zeros(n, np.uint32) + 3, np.zeros(n, np.uint32), np.zeros(n, np.uint32)], 1)
    key = np.tile(np.array([[12345, 0]], dtype=np.uint32), (n, 1))
    out = oracle_mod.philox(ctr, key)
    for w in range(4):
        u24 = out[:, w] >> 8
        counts = np.bincount((u24 >> 8).astype(np.int64), minlength=65536)
        exp = n / 65536
        chi2 = ((counts - exp) ** 2 / exp).sum()
        # chi^2 with 65535 dof: mean 65535, sd ~362; allow 6 sd
        assert abs(chi2 - 65535) < 6 * math.sqrt(2 * 65535), (w, chi2)
    # words uncorrelated
    u = (out >> 8).astype(np.float64) / 2 ** 24
    cc = np.corrcoef(u.T)
    assert np.all(np.abs(cc - np.eye(4)) < 5 / math.sqrt(n))


def test_ao_uniforms_exact_in_float32(oracle_mod):
    for pix in (0, 1, 1000, 17555279):
        for s in (0, 5, 31):
            u1, u2 = oracle_mod.ao_uniforms(pix, s, 7, (1 << 40) + 3)
            assert 0.0 <= u1 < 1.0 and 0.0 <= u2 < 1.0
            assert float(np.float32(u1)) == u1 and float(np.float32(u2)) == u2
            assert (u1 * 2 ** 24) == int(u1 * 2 ** 24)


def test_ao_uniforms_key_and_view_matter(oracle_mod):
    a = oracle_mod.ao_uniforms(10, 2, 0, 5)
    assert a != oracle_mod.ao_uniforms(10, 2, 1, 5)
    assert a != oracle_mod.ao_uniforms(10, 2, 0, 5 + (1 << 32))
    assert a != oracle_mod.ao_uniforms(10, 3, 0, 5)
    assert a == oracle_mod.ao_uniforms(10, 2, 0, 5)


def test_tiny_scene_invariants():
    s = scenegen.tiny_scene(seed=1)
    assert s.n_spheres == 64 and s.n_cylinders == 0 and s.n_lights == 1
    assert np.all(np.linalg.norm(s.sph_center, axis=1) <= 10.0)
    assert np.all((s.sph_radius >= 0.5) & (s.sph_radius <= 1.5))
    s2 = scenegen.tiny_scene(seed=1)
    assert np.array_equal(s.sph_center, s2.sph_center)


def test_random_walk_scene_invariants():
    s = scenegen.protein_scene(seed=2)
    assert s.n_spheres == 13159 and s.n_cylinders == 13159 and s.n_prims == 26318
    assert np.all(np.linalg.norm(s.sph_center, axis=1) <= 40.0 + 1e-9)
    assert np.all((s.sph_radius >= 1.2) & (s.sph_radius <= 1.9))
    assert np.all(s.cyl_radius == 0.3)
    # bonds join consecutive atoms; the last one dangles from atom 13158
    assert np.array_equal(s.cyl_a[:-1], s.sph_center[:-1])
    assert np.array_equal(s.cyl_b[:-1], s.sph_center[1:])
    assert np.array_equal(s.cyl_a[-1], s.sph_center[-1])
    # unfolded steps have length exactly 1.5 (up to rounding); folds never lengthen
    step = np.linalg.norm(s.cyl_b - s.cyl_a, axis=1)
    assert np.all(step <= 1.5 + 1e-12)
    assert np.mean(np.abs(step - 1.5) < 1e-12) > 0.8
    s2 = scenegen.protein_scene(seed=2)
    assert np.array_equal(s.sph_center, s2.sph_center) and np.array_equal(s.sph_radius, s2.sph_radius)
    assert not np.array_equal(s.sph_center, scenegen.protein_scene(seed=3).sph_center)


def test_serving_pool_sizes():
    pool = scenegen.serving_pool(n_scenes=16)
    n = [s.n_prims for s in pool]
    assert min(n) >= 2000 - 2 and max(n) <= 200000
    jobs = scenegen.serving_requests([40.0] * 16, 200)
    assert all(4 <= j[3].ao_samples <= 32 for j in jobs)
    gaps = np.diff([0.0] + [j[0] for j in jobs])
    assert 0.01 < gaps.mean() < 0.03  # mean 1/50 s

"""Binary scene files: save -> load builds the same scene (grid arrays and
frames bit for bit), and re-saving gives the same bytes."""
import numpy as np
import pytest

import scenegen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tr():
    import paper_0801_1500_amd as tr
    tr.lib()
    return tr


def _cyl_only():
    pos, _ = scenegen.random_walk(200, 10.0, 3)
    return scenegen.Scene(np.zeros((0, 3)), np.zeros(0), np.zeros((0, 3), np.float32),
                          pos[:-1].copy(), pos[1:].copy(), np.full(199, 0.4),
                          np.full((199, 3), 0.6, np.float32),
                          np.array([[0.3, 1.0, 2.0]]), np.ones((1, 3)))


def _empty():
    z3, z = np.zeros((0, 3)), np.zeros(0)
    return scenegen.Scene(z3, z, np.zeros((0, 3), np.float32), z3, z3, z,
                          np.zeros((0, 3), np.float32), np.array([[0.0, 0.0, 1.0]]), np.ones((1, 3)))


@pytest.mark.parametrize("which", ["tiny", "protein", "cyl", "empty"])
def test_scene_file_round_trip(tr, tmp_path, which):
    import torch
    scene = {"tiny": lambda: scenegen.tiny_scene(1), "protein": scenegen.protein_scene,
             "cyl": _cyl_only, "empty": _empty}[which]()
    print("scene file case", which, flush=True)
    a = tr.Scene(scene, cells_per_prim=7.0)
    path = str(tmp_path / "s.trs")
    a.save(path)
    b = tr.Scene.load(path)
    assert (b.n_spheres, b.n_cylinders, b.n_lights) == (a.n_spheres, a.n_cylinders, a.n_lights)
    ia, ib = a.grid_info(), b.grid_info()
    assert all(np.array_equal(x, y) for x, y in zip(ia, ib))
    for x, y in zip(a.grid_arrays(), b.grid_arrays()):
        assert np.array_equal(x, y)
    c = scenegen.Camera((0.0, 0.0, 60.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 50.0, 96, 80)
    p = scenegen.Params(ao_samples=8, seed=9)
    fa = tr.render(a, c, p, precision="fp32_resolve", outputs=("rgb", "hit_id"))
    fb = tr.render(b, c, p, precision="fp32_resolve", outputs=("rgb", "hit_id"))
    torch.cuda.synchronize()
    for k in ("rgb", "hit_id"):
        assert torch.equal(fa[k], fb[k]), k
    path2 = str(tmp_path / "s2.trs")
    b.save(path2)
    assert open(path, "rb").read() == open(path2, "rb").read()

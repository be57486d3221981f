"""Host-side check of the grid's reference-count limit.

The walk addresses its per-cell lists with signed 32-bit byte offsets, so
the library refuses a grid whose references and cells together pass 2^29
(TR_EUNSUPPORTED).  The total has to be summed in 64 bits: overlapping large
primitives can list more than 2^32 references, and a 32-bit sum wraps to a
value that passes the limit.  This test computes, from the grid's definition
(resolution rule and box membership), the total of a scene built for that
case -- 14,000 identical cylinders whose boxes span the whole scene, each
listed in every cell -- and shows that its 32-bit wrap would pass the limit.
The GPU test of the same scene (tests/test_gpu_limits.py) checks that the
library refuses it.
"""
import math

import scenegen


def _resolution(scene, lam):
    # grid definition: the union of the primitive boxes widened by
    # 1e-4 m + 1e-6 (m = largest extent), res_a = clamp(ceil(ext_a (lam N / V)^(1/3)), 1, 512)
    lo = (scene.cyl_a.min(axis=0) - scene.cyl_radius.max()).tolist()
    hi = (scene.cyl_b.max(axis=0) + scene.cyl_radius.max()).tolist()
    m = max(h - l for l, h in zip(lo, hi))
    pad = 1e-4 * m + 1e-6
    ext = [(h + pad) - (l - pad) for l, h in zip(lo, hi)]
    V = ext[0] * ext[1] * ext[2]
    kk = ((lam * scene.n_prims) / V) ** (1.0 / 3.0)
    return [min(max(math.ceil(e * kk), 1), 512) for e in ext]


def test_stacked_cylinders_wrap_a_32_bit_total():
    s = scenegen.stacked_cylinders()
    assert s.n_prims == 14000
    res = _resolution(s, 24.0)
    assert res == [70, 70, 70]
    n_cells = res[0] * res[1] * res[2]
    # each box is the scene box, so every cylinder is listed in every cell
    total = s.n_prims * n_cells
    assert total > 2 ** 32
    wrapped = total % 2 ** 32
    # a 32-bit total would pass the 2^29 limit on references + cells
    assert wrapped + n_cells + 1 <= 2 ** 29
    # the true total does not
    assert total + n_cells + 1 > 2 ** 29

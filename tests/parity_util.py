"""Parity metrics between a GPU frame and the oracle's frame.

Tolerance reading for the FP32 path (render precision differs from the
oracle's double precision): a flipped visibility decision moves a pixel by a
whole AO step (albedo * skylight / S ~ 0.05), so colour error is bounded only
on pixels whose hit id and every secondary-ray decision agree; the decisions
themselves are bounded by agreement rates.
"""
import numpy as np

# FP32 path bounds (hit-index agreement, decision agreement, colour on agreeing pixels)
HIT_AGREE_MIN = 0.9999
DECISION_AGREE_MIN = 0.9999
MAX_ABS = 1e-3
RMS = 1e-4


def popcount32(x: np.ndarray) -> np.ndarray:
    x = x.astype(np.uint64) & np.uint64(0xFFFFFFFF)
    if hasattr(np, "bitwise_count"):
        return np.bitwise_count(x).astype(np.int64)
    c = np.zeros(x.shape, dtype=np.int64)
    for b in range(32):
        c += ((x >> np.uint64(b)) & np.uint64(1)).astype(np.int64)
    return c


def compare(gpu: dict, ref: dict, ao_samples: int, n_lights: int) -> dict:
    """gpu/ref: flat arrays (same pixel order) rgb [n,3], hit_id [n],
    ao_mask [n] (uint32 bits), light_mask [n]."""
    g_hit = np.asarray(gpu["hit_id"]).reshape(-1).astype(np.int64)
    r_hit = np.asarray(ref["hit_id"]).reshape(-1).astype(np.int64)
    n = r_hit.size
    hit_eq = g_hit == r_hit
    g_ao = np.asarray(gpu["ao_mask"]).reshape(-1).astype(np.int64) & 0xFFFFFFFF
    r_ao = np.asarray(ref["ao_mask"]).reshape(-1).astype(np.int64) & 0xFFFFFFFF
    g_l = np.asarray(gpu["light_mask"]).reshape(-1).astype(np.int64)
    r_l = np.asarray(ref["light_mask"]).reshape(-1).astype(np.int64)
    both_hit = hit_eq & (r_hit >= 0)
    s_bits = min(ao_samples, 32)
    ao_diff = popcount32(np.where(both_hit, g_ao ^ r_ao, 0))
    l_diff = popcount32(np.where(both_hit, g_l ^ r_l, 0))
    n_sec = int(both_hit.sum()) * (s_bits + n_lights)
    flips = int(ao_diff.sum() + l_diff.sum())
    agree = hit_eq & (g_ao == r_ao) & (g_l == r_l)
    g_rgb = np.asarray(gpu["rgb"], dtype=np.float64).reshape(-1, 3)
    r_rgb = np.asarray(ref["rgb"], dtype=np.float64).reshape(-1, 3)
    err = np.abs(g_rgb - r_rgb)
    ea = err[agree]
    return dict(
        n=n, hit_agree=float(hit_eq.mean()) if n else 1.0,
        hit_mismatch=int((~hit_eq).sum()),
        decisions=n_sec, decision_flips=flips,
        decision_agree=1.0 - flips / n_sec if n_sec else 1.0,
        agree_pixels=int(agree.sum()),
        max_abs_agree=float(ea.max()) if ea.size else 0.0,
        rms_agree=float(np.sqrt((ea ** 2).mean())) if ea.size else 0.0,
        max_abs_all=float(err.max()) if err.size else 0.0,
        rms_all=float(np.sqrt((err ** 2).mean())) if err.size else 0.0,
        # share of all pixels with some channel off by more than 1e-3 (what
        # the flipped decisions cost the whole frame; reported, not bound)
        frac_over_1e3_all=float((err.max(axis=1) > MAX_ABS).mean()) if err.size else 0.0)


def assert_fp32_parity(m: dict):
    assert m["hit_agree"] >= HIT_AGREE_MIN, m
    assert m["decision_agree"] >= DECISION_AGREE_MIN, m
    assert m["max_abs_agree"] <= MAX_ABS, m
    assert m["rms_agree"] <= RMS, m


def frame_to_numpy(fr: dict) -> dict:
    out = {}
    for k, v in fr.items():
        a = v.cpu().numpy()
        if k == "ao_mask":
            a = a.view(np.uint32)
        out[k] = a
    return out


def flat_at(fr: dict, pix: np.ndarray) -> dict:
    """Pick pixels (j*W+i) out of full GPU frames."""
    out = {}
    for k in ("rgb", "hit_id", "ao_mask", "light_mask"):
        if k in fr:
            a = fr[k]
            out[k] = a.reshape(-1, 3)[pix] if k == "rgb" else a.reshape(-1)[pix]
    return out


def chebyshev_capped(occ, cap=32):
    """Chebyshev distance (in cells) from each cell to the nearest occupied
    one, capped at cap: grow the occupied set one 26-neighbourhood shell at a
    time (plain definition, no separable passes)."""
    dist = np.where(occ, 0, cap).astype(np.int32)
    cur = occ.copy()
    for k in range(1, cap):
        if cur.all():
            break
        grown = cur.copy()
        p = np.pad(cur, 1)
        nz, ny, nx = cur.shape
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    grown |= p[1 + dz:1 + dz + nz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]
        dist[grown & ~cur] = k
        cur = grown
    return dist


def octant_blocks(occ, cap=32):
    """Per empty cell, the octant fields of the FP32 walk's empty-cell
    record, packed by octant o (bit a of o: direction negative on axis a),
    from the plain definition: M is the largest m <= min(7, (cap - 1) // 2)
    for which the cell m steps along the octant's diagonal lies in the grid
    and the block of 2m + 1 cells per axis ahead of the cell in that octant
    (clipped to the grid) holds no occupied cell.  Block sums come from a
    summed-volume table of the occupancy, not from a distance field.
    occ: [z][y][x]; returns uint32 [z][y][x] (0 on occupied cells)."""
    nz, ny, nx = occ.shape
    sv = np.zeros((nz + 1, ny + 1, nx + 1), dtype=np.int64)
    sv[1:, 1:, 1:] = occ.astype(np.int64).cumsum(0).cumsum(1).cumsum(2)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    mcap = min(7, (cap - 1) // 2)
    out = np.zeros(occ.shape, dtype=np.uint32)
    for o in range(8):
        s = [(-1 if (o >> a) & 1 else 1) for a in range(3)]  # x, y, z
        M = np.zeros(occ.shape, dtype=np.int64)
        alive = ~occ
        for m in range(1, mcap + 1):
            ends = []
            inside = np.ones(occ.shape, dtype=bool)
            for c, sa, n in ((x, s[0], nx), (y, s[1], ny), (z, s[2], nz)):
                inside &= (c + m * sa >= 0) & (c + m * sa < n)
                far = c + 2 * m * sa
                lo_ = np.clip(np.minimum(c, far), 0, n - 1)
                hi_ = np.clip(np.maximum(c, far), 0, n - 1)
                ends.append((lo_, hi_ + 1))
            (x0, x1), (y0, y1), (z0, z1) = ends
            tot = (sv[z1, y1, x1] - sv[z0, y1, x1] - sv[z1, y0, x1] - sv[z1, y1, x0]
                   + sv[z0, y0, x1] + sv[z0, y1, x0] + sv[z1, y0, x0] - sv[z0, y0, x0])
            alive = alive & inside & (tot == 0)
            M[alive] = m
        out |= np.where(occ, 0, M).astype(np.uint32) << np.uint32(3 * o)
    return out


def explain_flips(oracle_mod, scene, cam, got: dict, ref: dict, limit: int = 12) -> list:
    """Describe pixels (full frames) whose hit agrees but some decision
    differs: the primitive, the oracle's viewer-facing normal, its N.z and
    N.L per light, and both masks.  For printing in the GPU tests."""
    gh, rh = got["hit_id"].reshape(-1), ref["hit_id"].reshape(-1)
    ga, ra = got["ao_mask"].reshape(-1), ref["ao_mask"].reshape(-1)
    gl, rl = got["light_mask"].reshape(-1), ref["light_mask"].reshape(-1)
    bad = np.nonzero((gh == rh) & (gh >= 0) & ((ga != ra) | (gl != rl)))[0]
    miss = np.nonzero(gh != rh)[0]
    ld = np.asarray(scene.light_dir, dtype=np.float64)
    ld = ld / np.linalg.norm(ld, axis=1)[:, None]
    out = ["%d pixels with flipped decisions, %d with another hit" % (bad.size, miss.size)]
    for q in list(bad[:limit]) + list(miss[:4]):
        i, j = int(q % cam.width), int(q // cam.width)
        o, d = oracle_mod.camera_ray(cam, i, j)
        k = int(rh[q])
        line = "pix (%d, %d) k gpu %d ref %d" % (i, j, int(gh[q]), k)
        if k >= 0:
            t = float(ref["t"].reshape(-1)[q])
            n = oracle_mod.normal(scene, k, o, d, t)
            inside = float(n @ d) >= 0.0
            if inside:
                n = -n
            line += " t %.6f %s N.z %.3e N.L %s ao %08x/%08x light %d/%d" % (
                t, "inside" if inside else "outside", n[2],
                " ".join("%.3e" % float(n @ l) for l in ld), int(ga[q]), int(ra[q]),
                int(gl[q]), int(rl[q]))
        out.append(line)
    return out

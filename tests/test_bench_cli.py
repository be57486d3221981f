"""bench.py's command-line contract on the host: more than one GPU is
refused with a message, before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_help_lists_the_contract_flags():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for flag in ("--gpus", "--steps", "--warmup"):
        assert flag in r.stdout


def test_flop_count_is_the_cost_table():
    # roofline.frac is the cost table over the kernel's counters: each op's
    # flops times its count, an empty-space jump priced only in the variant
    sys.path.insert(0, ROOT)
    import bench
    st = dict(rays_traced=10, cells=100, jumps=7, sph_tests=50, sph_hits=5, cyl_tests=4,
              cyl_hits=1, pixels=20, hit_pixels=8, ao_rays=128)
    table = (40 * 10 + 4 * 100 + 22 * 50 + 4 * 5 + 45 * 4 + 12 * 1 + 20 * 20 + 10 * 8
             + 8 * 8 * 2 + 12 * 8 + 23 * 128 + 10 * 20)
    assert bench.algorithmic_flops(st, 2, True) == table
    assert bench.algorithmic_flops(st, 2, False) == table - 12 * 8  # no AO basis without AO
    assert bench.algorithmic_flops(st, 2, True, bench.JUMP_COST) == table + 16 * 7

"""Host-side logic of bench.py (no GPU): the transform-flop count behind the
ALU roofline and the one-GPU guard."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def box_sides(n, s, overlap):
    """Per-axis box sides: owned blocks of s cells grown by the overlap,
    clipped at the walls."""
    return [min(n, a + s + overlap) - max(0, a - overlap) for a in range(0, n, s)]


@pytest.mark.parametrize("n,sub,overlap", [(256, 32, 1), (128, 32, 1), (96, 32, 3), (48, 16, 2)])
def test_transform_flops_closed_form(n, sub, overlap):
    # A box of sides (a, b, c): along x each of the b c pencils of each of the
    # 3 components is contracted forward and back with the even/odd butterfly,
    # a^2 / 2 FMAs each way, i.e. 2 a^2 flops: 6 a^2 b c flops; over the three
    # axes 6 abc (a + b + c).  The same side list serves every axis, so the
    # sum over boxes is 6 * 3 (sum a^2) (sum a)^2 = 18 (sum a^2) (sum a)^2.
    s = box_sides(n, sub, overlap)
    s1 = sum(s)
    s2 = sum(a * a for a in s)
    assert bench.transform_flops_per_apply(n, (sub, sub, sub), overlap) == pytest.approx(
        18.0 * s2 * s1 * s1, rel=1e-15)


def test_transform_flops_at_256_cube():
    # boxes of 33 cells at the walls and 34 inside: sum a = 270, sum a^2 = 9114
    assert bench.transform_flops_per_apply(256, (32, 32, 32)) == 18 * 9114 * 270 ** 2


def test_multi_gpu_request_exits_with_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""

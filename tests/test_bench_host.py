"""Host-side parts of bench.py (no GPU): the count of rfft frequencies each
kernel-spectrum matrix serves, which weights the banded adjoint's
algorithmic bytes, against a brute-force enumeration of the symmetry; and
the refusal of more than one GPU."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("p", [16, 32, 64, 256])
def test_matrix_frequency_counts_tile_the_half_spectrum(p):
    # matrix s = (a, b), a <= b <= p/2, in the order b (b + 1)/2 + a, stands
    # for the spectrum at (a, b), (p - a, b), (b, a), (p - b, a) (first
    # index modulo p over the full axis, second over the half axis 0..p/2);
    # together the matrices must cover every (full, half) pair once
    h = p // 2
    seen = {}
    counts = []
    for b in range(h + 1):
        for a in range(b + 1):
            freqs = {(a, b), ((p - a) % p, b), (b, a), ((p - b) % p, a)}
            counts.append(len(freqs))
            for f in freqs:
                seen[f] = seen.get(f, 0) + 1
    assert sorted(seen) == [(x, y) for x in range(p) for y in range(h + 1)]
    assert set(seen.values()) == {1}
    got = bench.matrix_frequency_counts(p)
    assert list(got) == counts
    assert int(got.sum()) == p * (h + 1)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout == ""

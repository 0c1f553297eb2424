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


def test_bin_run_driver_equals_the_oracle_operator():
    # the bin-run evaluation that the full-size parity test and the CPU
    # baseline drive is the oracle's operator: per-bin forward identical,
    # adjoint equal up to the order of the bin sum, and the adjoint
    # identity holds
    import numpy as np

    from oracle import operator as oop
    from tests.gpu_common import BinRunOperator
    rng = np.random.default_rng(5)
    Kq = rng.random((4, 11, 7, 37))
    A = oop.FFTOperator(Kq)
    B = BinRunOperator(Kq, run=8, threads=3)
    mu = rng.random((4, 11, 7))
    r = rng.standard_normal((37, 11, 7))
    np.testing.assert_array_equal(B.forward(mu), A.forward(mu))
    ga, gb = A.adjoint(r), B.adjoint(r)
    assert np.linalg.norm(ga - gb) <= 1e-14 * np.linalg.norm(ga)
    lhs, rhs = float(np.vdot(B.forward(mu), r)), float(np.vdot(mu, gb))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    B.close()


def test_layer_parallel_tabulation_equals_the_oracle():
    import numpy as np

    from oracle import kernel as okernel
    from synth.workloads import Geometry, even_layers
    from tests.gpu_common import tabulate_layers_parallel
    z, dz = even_layers(1.0, 9.0, 5)
    g = Geometry(nx=7, ny=5, pitch_mm=0.5, z_mm=z, dz_mm=dz, nt=20, dt_ps=40.0)
    np.testing.assert_array_equal(tabulate_layers_parallel(g, threads=3), okernel.tabulate(g))

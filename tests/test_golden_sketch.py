"""Pins of the sketched full-vector reference of the 10^4 benchmark
(tests/golden/point12_10x4_sketch.npz, make_sketch_10x4.py): the sketch
generator estimates norms as its definition says, the stored sketches are
those of the complete reference vectors where those are stored too, the
references are converged, and the oracle's own error at the benchmark's
outer sizes is below the benchmark's 1e-8."""
import os
import sys

import numpy as np

import nks_inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")


def _sk():
    return dict(np.load(os.path.join(GOLD, "point12_10x4_sketch.npz")))


def test_sketch_estimates_norms():
    """|S e| / sqrt(rows) is within 15 % of |e| (five spreads of the
    chi-square with 2 * 256 degrees of freedom) for vectors of very different
    shapes: dense Gaussian, one spike, a few large entries on a small floor."""
    n, rows = 3000, 256
    S = I.sketch_rows(n, range(rows), 99)
    assert S.shape == (rows, n)
    assert abs(np.mean(np.abs(S) ** 2) - 1.0) < 0.01
    rng = np.random.default_rng(5)
    spike = np.zeros(n, complex)
    spike[17] = 3.0
    few = 1e-6 * rng.standard_normal(n) + 0j
    few[[3, 900, 2999]] = [1.0, -2.0, 0.5j]
    for e in (rng.standard_normal(n) + 1j * rng.standard_normal(n), spike, few):
        est = np.linalg.norm(S @ e) / np.sqrt(rows)
        assert abs(est / np.linalg.norm(e) - 1.0) < 0.15


def test_sketch_rows_are_reproducible_one_by_one():
    a = I.sketch_rows(500, range(8), 3)
    b = I.sketch_rows(500, [5, 2], 3)
    assert np.array_equal(a[5], b[0]) and np.array_equal(a[2], b[1])


def test_stored_sketches_match_the_complete_references():
    sk = _sk()
    full = dict(np.load(os.path.join(GOLD, "point4_full_10x4.npz")))
    n = full["y"].shape[1]
    S = I.sketch_rows(n, range(int(sk["rows"])), int(sk["seed"]))
    for i in range(len(full["mu"])):
        t = [c for c in range(len(sk["mu"])) if sk["mu"][c] == full["mu"][i] and sk["spin"][c] == full["spin"][i]
             and sk["colour"][c] == full["colour"][i]]
        assert len(t) == 1
        y = full["y"][i]
        assert abs(np.linalg.norm(y) - sk["norm"][t[0]]) <= 1e-12 * sk["norm"][t[0]]
        assert np.linalg.norm(S @ y - sk["sy"][t[0]]) <= 1e-9 * np.linalg.norm(sk["sy"][t[0]])


def test_references_are_converged_and_the_benchmark_k_reaches_1e8():
    sys.path.insert(0, os.path.dirname(HERE))
    import bench
    sk = _sk()
    assert len(sk["mu"]) == 24 and np.all(sk["change_from_k_check"] <= 1e-9)
    ks = list(sk["ks"])
    assert int(sk["ell"]) == bench.ELL
    for c in range(24):
        j = ks.index(bench.K_MU[float(sk["mu"][c])])
        # the method itself (oracle, nested at ell = 64, exact full-vector error)
        # is below the target with room for the GPU's rounding
        assert sk["oracle_err_nested"][c, j] <= 5e-9, (c, sk["oracle_err_nested"][c, j])

"""Host logic of the learned policy: training targets from label rows, the
normalisation and the network file (no GPU)."""
import math

import numpy as np
import pytest

from paper_0912_4457_amd import policy as P


def _row(errs, trace=None, feats=None):
    r = np.full(P.LABEL_WORDS, np.nan)
    r[:P.NFEAT] = np.arange(P.NFEAT) if feats is None else feats
    r[P.NFEAT:P.NFEAT + len(errs)] = errs
    if trace is not None:
        r[P.NFEAT + P.LABEL_NK:] = np.asarray(trace, float).ravel()
    return r


def test_layout_constants_match_the_header():
    import re
    from pathlib import Path
    h = (Path(__file__).resolve().parents[1] / "include" / "nks.h").read_text()
    assert int(re.search(r"#define NKS_MLP_NPARAMS (\d+)", h).group(1)) == P.NPARAMS
    assert int(re.search(r"#define NKS_LABEL_NK (\d+)", h).group(1)) == P.LABEL_NK
    assert int(re.search(r"#define NKS_LABEL_NELL (\d+)", h).group(1)) == P.LABEL_NELL
    assert int(re.search(r"#define NKS_LABEL_DK (\d+)", h).group(1)) == P.LABEL_DK
    assert P.LABEL_WORDS == 316 and P.NFLOATS == 5414


def test_k_target_is_first_stable_crossing_plus_verification_margin():
    # geometric decay 10^(-k/100): e(k) <= 2.5e-9 from k = 860.2, the first k_i is 880
    ks = 20 * (np.arange(60) + 1)
    errs = 10.0 ** (-ks / 100.0)
    trace = np.tile([1e-3, 1e-6, 1e-10, 1e-14], (60, 1))
    f, (lk, le) = P.targets(_row(errs, trace), 1e-8, 1200)
    assert 10 ** lk == pytest.approx(880 + 40)
    assert f[6] == pytest.approx(-8.0)
    # ell: 64 -> 128 change 1e-10 <= tol/10 = 1e-9, so 64 is enough
    assert 10 ** le == pytest.approx(64)


def test_non_monotone_errors_take_the_last_crossing():
    errs = np.full(60, 1e-3)
    errs[10] = 1e-12          # an accidental dip at k = 220
    errs[30:] = 1e-12         # stays below from k = 620
    f, (lk, _) = P.targets(_row(errs, np.full((60, 4), 1e-14)), 1e-8, 1200)
    assert 10 ** lk == pytest.approx(620 + 40)


def test_rows_that_do_not_resolve_the_tolerance_are_dropped():
    ks = 20 * (np.arange(60) + 1)
    errs = 10.0 ** (-ks / 300.0)        # reaches 2.5e-11 only beyond k = 3000
    assert P.targets(_row(errs), 1e-10, 1200) is None
    # crossing too close to the reference length
    errs = np.where(ks >= 1100, 0.0, 1.0)
    assert P.targets(_row(errs), 1e-8, 1200) is None


def test_ell_target_defaults_to_the_largest_traced_size():
    errs = np.where(20 * (np.arange(60) + 1) >= 400, 1e-12, 1.0)
    _, (_, le) = P.targets(_row(errs, np.full((60, 4), 1e-3)), 1e-8, 1200)
    assert 10 ** le == pytest.approx(256)


def test_dataset_expands_tolerances_and_normalisation_passes_constants():
    ks = 20 * (np.arange(60) + 1)
    rows = [_row(10.0 ** (-ks / 80.0), np.full((60, 4), 1e-14)) for _ in range(3)]
    X, T, G = P.dataset(rows, [1200] * 3, [0, 1, 2])
    assert X.shape == (15, 16) and T.shape == (15, 2)
    # tighter tolerances need larger k
    assert np.all(np.diff(T[:5, 0]) > 0)
    fm, fs, tm, ts = P.normalisation(X, T)
    assert fs[0] == 1.0 and fm[0] == 0.0          # constant feature passes through
    assert fs[6] > 0


def test_network_file_round_trip(tmp_path):
    params = P.init_params(3)
    blob = P.pack(params, np.zeros(16), np.ones(16), np.array([2.5, 1.8]), np.array([0.2, 0.3]))
    path = tmp_path / "net.json"
    P.save(path, blob, {"note": "x"})
    b2, meta = P.load(path)
    assert np.array_equal(b2, blob) and meta["note"] == "x"


def test_init_params_layout():
    p = P.init_params(0)
    assert p.size == P.NPARAMS and p.dtype == np.float32
    # biases are zero: b1 after W1, b3 at the end
    assert np.all(p[16 * 64:16 * 64 + 64] == 0) and np.all(p[-2:] == 0)
    assert math.isclose(float(np.std(p[:16 * 64])), math.sqrt(2 / 80), rel_tol=0.1)

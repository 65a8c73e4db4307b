"""Input generators: shapes and structure of the seeded synthetic streams (CPU only)."""
import numpy as np

import synth


def _simple(e, n):
    assert e.dtype == np.uint32 and e.ndim == 2 and e.shape[1] == 2
    assert (e[:, 0] != e[:, 1]).all()
    assert e.max() < n
    lo = np.minimum(e[:, 0], e[:, 1]).astype(np.uint64)
    hi = np.maximum(e[:, 0], e[:, 1]).astype(np.uint64)
    key = (lo << np.uint64(32)) | hi
    assert len(np.unique(key)) == len(key)


def test_config1_shape_and_determinism():
    e = synth.config1_stream()
    assert e.shape == (20000, 2)
    _simple(e, 2000)
    assert np.array_equal(e, synth.er(2000, 20000, 1, 1001))
    d = np.bincount(e.ravel(), minlength=2000)
    assert abs(d.mean() - 20.0) < 1e-9 and d.max() < 50  # Bin(1999, 0.01): mean 20


def test_chung_lu_power_law():
    e, n = synth.scaled_chung_lu(200_000, 5)
    _simple(e, n)
    d = np.bincount(e.ravel(), minlength=n)
    assert d.max() > 20 * d.mean()  # heavy tail
    w = synth.chung_lu_weights(n, 200_000, 2.1, n / 2)
    assert abs(w.sum() - 400_000) < 1e-3 and abs(w[0] - n / 2) / (n / 2) < 1e-6


def test_rmat_small_dedup_generation_order():
    e = synth.rmat(10, 8, 0.57, 0.19, 0.19, 3)
    _simple(e, 1 << 10)
    assert 0.5 * 8192 < len(e) < 8192
    assert np.array_equal(e, synth.rmat(10, 8, 0.57, 0.19, 0.19, 3))


def test_shuffled_is_a_permutation():
    e = synth.complete(9)
    s = synth.shuffled(e, 4, 5)
    key = lambda a: sorted(map(tuple, np.sort(a, axis=1).tolist()))
    assert key(s) == key(e)


def test_serving_trace_ranges():
    tr = synth.serving_trace(seed=5, n_requests=200, rate_per_s=10.0)
    sizes = np.array([r["E"] for r in tr])
    assert sizes.min() >= 1000 and sizes.max() <= 2e7
    assert 1e5 < np.median(sizes) < 4e5  # lognormal, median 2e5
    assert all(r["m"] in (10, 50, 100) and r["c"] in (r["m"], 4 * r["m"]) for r in tr)
    arr = np.array([r["arrival_s"] for r in tr])
    assert (np.diff(arr) > 0).all() and 7.0 < len(arr) / arr[-1] < 13.0  # Poisson rate 10/s

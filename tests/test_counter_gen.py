"""Host counter-based generator: Philox4x32-10 known answers and the moments
of the entry model (the device generator is compared with it bit for bit in
the GPU tests)."""
import json
import pathlib

import numpy as np

from workloads import counter

GOLD = pathlib.Path(__file__).parent / "golden" / "philox_kat.json"


def _hex(words):
    return np.array([int(w, 16) for w in words], dtype=np.uint32)


def test_philox_known_answers():
    for v in json.loads(GOLD.read_text())["vectors"]:
        out = counter.philox4x32_10(_hex(v["ctr"])[None, :], _hex(v["key"]))
        assert out[0].tolist() == _hex(v["out"]).tolist()


def test_entries_are_functions_of_seed_and_index():
    a = counter.gaussian_entries(7, np.arange(50), np.arange(40))
    b = counter.gaussian_entries(7, np.arange(10, 30), np.arange(5, 25))
    np.testing.assert_array_equal(a[10:30, 5:25], b)
    c = counter.gaussian_entries(8, np.arange(50), np.arange(40))
    assert np.mean(a == c) < 0.01
    # the two key words both matter
    d = counter.gaussian_entries(7 + (1 << 32), np.arange(50), np.arange(40))
    assert np.mean(a == d) < 0.01


def test_entry_model_moments_and_range():
    g = counter.gaussian_entries(12345, np.arange(400), np.arange(500)).astype(np.float64)
    # Irwin-Hall(4) scaled: mean 0, variance 1, support [-2 sqrt3, 2 sqrt3],
    # kurtosis 3 - 6/(5*4) = 2.7
    assert abs(g.mean()) < 0.01
    assert abs(g.var() - 1.0) < 0.01
    assert np.max(np.abs(g)) <= 2 * np.sqrt(3)
    kurt = np.mean(g ** 4) / np.mean(g ** 2) ** 2
    assert abs(kurt - 2.7) < 0.03
    # distinct entries are uncorrelated (row and column neighbours)
    assert abs(np.mean(g[1:] * g[:-1])) < 0.01
    assert abs(np.mean(g[:, 1:] * g[:, :-1])) < 0.01


def test_spiked_columns_structure():
    f = counter.spike_factors(3, 200, 1000, [30.0, 20.0], 10)
    A = counter.spiked_matrix(3, 200, 1000, f)
    G = counter.gaussian_entries(3, np.arange(200), np.arange(1000)).astype(np.float64)
    spike = A.astype(np.float64) - G
    # the difference is the rank-2 spike, up to one FP32 rounding of A
    ref = (f.U * f.thetas) @ f.V.T
    assert np.max(np.abs(spike - ref)) <= 4 * 2.0 ** -24 * (np.max(np.abs(A)) + 1)
    assert set(np.flatnonzero(np.any(np.abs(ref) > 0, axis=0))) == \
        set(np.concatenate(f.supports).tolist())
    np.testing.assert_array_equal(counter.spiked_columns(3, 200, [5, 999, 0], f),
                                  A[:, [5, 999, 0]])

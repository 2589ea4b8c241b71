"""The seeded synthetic workloads: shapes, normalisation, reproducibility."""
import numpy as np
import pytest

import w1data


@pytest.mark.parametrize("fn,n", [(w1data.pair_gauss3, 64), (w1data.pair_shapes, 256)])
def test_pairs_are_normalised_and_seeded(fn, n):
    a, b = fn(0)
    assert a.shape == (n + 1, n + 1) and b.shape == (n + 1, n + 1)
    assert a.sum() == pytest.approx(1.0, rel=1e-14) and b.sum() == pytest.approx(1.0, rel=1e-14)
    assert a.min() > 0 and b.min() > 0
    a2, b2 = fn(0)
    np.testing.assert_array_equal(a, a2)
    np.testing.assert_array_equal(b, b2)
    a3, _ = fn(1)
    assert not np.array_equal(a, a3)


def test_shift8_pair():
    a, b, s = w1data.pair_shift8(0, n=64)
    assert 0.0 <= np.linalg.norm(s) <= 0.1
    assert a.sum() == pytest.approx(1.0) and b.sum() == pytest.approx(1.0)


def test_uneven_and_served():
    sizes = [w1data.pair_uneven(i)[0] for i in range(200)]
    assert set(sizes) <= {64, 128, 256, 512}
    assert [w1data.pair_uneven(i)[1] for i in range(4)] == [1, 2, 1, 2]
    reqs = w1data.served_requests(500)
    t = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(t) > 0)
    assert 150 < len(reqs) / t[-1] < 260
    a, b = w1data.served_pair(w1data.Request(0, 0.0, 128, "shapes"))
    assert a.shape == (129, 129)


def test_translated_bump_is_a_translate():
    a, b, mass = w1data.translated_bump_pair(16, (3, -2), floor_mass=0.1, seed=4)
    fl = 0.1 / a.size
    ba, bb = a - fl, b - fl
    np.testing.assert_allclose(np.roll(np.roll(ba, 3, 0), -2, 1), bb, atol=1e-15)
    assert ba.sum() == pytest.approx(mass)

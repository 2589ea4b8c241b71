"""Pins of the cross-level maps (Sec. 3.3): the printed worked examples of
Figures fig:iterphi / fig:iterm, exactness on affine potentials, Lemma 1,
and the restriction's defining identities."""
import json
import os

import numpy as np
import pytest

import oracle.w1_oracle as o

GOLD = os.path.join(os.path.dirname(__file__), "golden", "interp_worked_examples.json")


def _fixture():
    with open(GOLD) as f:
        return json.load(f)


def _apply_examples(rows, coarse, fine, hc, hf):
    for row in rows:
        I, J = (int(round(x / hf)) for x in row["fine"])
        want = np.mean([coarse[int(round(a / hc)), int(round(b / hc))] for a, b in row["coarse"]])
        assert fine[I, J] == pytest.approx(want, rel=0, abs=1e-15), row


def test_worked_example_potential():
    g = _fixture()
    c = np.array([[1.25, -2.0], [3.5, 0.75]])
    f = o.prolong_potential(c)
    _apply_examples(g["potential"], c, f, g["h_coarse"], g["h_fine"])


def test_worked_example_flux():
    g = _fixture()
    c1 = np.array([[1.25, -2.0], [0.0, 0.0]])      # m1 on the last row is zero
    c2 = np.array([[0.5, 0.0], [-3.0, 0.0]])       # m2 on the last column is zero
    f1, f2 = o.prolong_flux(c1, c2)
    _apply_examples(g["flux1"], c1, f1, g["h_coarse"], g["h_fine"])
    _apply_examples(g["flux2"], c2, f2, g["h_coarse"], g["h_fine"])
    assert np.all(f1[-1, :] == 0) and np.all(f2[:, -1] == 0)


@pytest.mark.parametrize("nc", [1, 3, 8])
def test_potential_interpolation_is_exact_on_affine(nc):
    hc = 1.0 / nc
    t = np.arange(nc + 1) * hc
    c = 0.3 + 1.7 * t[:, None] - 0.9 * t[None, :] + 0.0 * t[None, :]
    f = o.prolong_potential(c)
    tf = np.arange(2 * nc + 1) * hc / 2
    want = 0.3 + 1.7 * tf[:, None] - 0.9 * tf[None, :]
    np.testing.assert_allclose(f, want, atol=1e-14)


def test_2d_case_formulas_of_inter_m():
    # the 2-D case list printed after eq. (inter_m) for m_{h_l,1}, written per
    # parity class of (I, J) with coarse index arithmetic of the printed
    # coordinates x_1 - h_l, x_2 -+ h_l
    rng = np.random.default_rng(0)
    nc = 5
    c1 = rng.standard_normal((nc + 1, nc + 1)); c1[nc, :] = 0
    c2 = rng.standard_normal((nc + 1, nc + 1)); c2[:, nc] = 0
    f1, f2 = o.prolong_flux(c1, c2)
    for I in range(2 * nc + 1):
        for J in range(2 * nc + 1):
            ev_i, ev_j = I % 2 == 0, J % 2 == 0
            if ev_i and ev_j:
                w1 = c1[I // 2, J // 2]; w2 = c2[I // 2, J // 2]
            elif not ev_i and ev_j:     # X3: x1 off the coarse grid
                w1 = c1[(I - 1) // 2, J // 2]
                w2 = 0.5 * (c2[(I - 1) // 2, J // 2] + c2[(I + 1) // 2, J // 2])
            elif ev_i and not ev_j:     # X2: x2 off the coarse grid
                w1 = 0.5 * (c1[I // 2, (J - 1) // 2] + c1[I // 2, (J + 1) // 2])
                w2 = c2[I // 2, (J - 1) // 2]
            else:
                w1 = 0.5 * (c1[(I - 1) // 2, (J - 1) // 2] + c1[(I - 1) // 2, (J + 1) // 2])
                w2 = 0.5 * (c2[(I - 1) // 2, (J - 1) // 2] + c2[(I + 1) // 2, (J - 1) // 2])
            assert f1[I, J] == pytest.approx(w1, abs=1e-15)
            assert f2[I, J] == pytest.approx(w2, abs=1e-15)


def _l2h(a, h):
    if isinstance(a, tuple):
        return sum(_l2h(x, h) for x in a)
    return float(np.sum(a * a) * h * h)


@pytest.mark.parametrize("nc", [2, 4, 16, 31])
def test_lemma1_nonexpansive(nc):
    rng = np.random.default_rng(nc)
    hc, hf = 1.0 / nc, 0.5 / nc
    worst = 0.0
    for _ in range(20):
        c = rng.standard_normal((nc + 1, nc + 1))
        r = _l2h(o.prolong_potential(c), hf) / _l2h(c, hc)
        worst = max(worst, r)
        c1 = rng.standard_normal((nc + 1, nc + 1)); c1[nc, :] = 0
        c2 = rng.standard_normal((nc + 1, nc + 1)); c2[:, nc] = 0
        f = o.prolong_flux(c1, c2)
        worst = max(worst, _l2h(f, hf) / _l2h((c1, c2), hc))
    assert worst <= 1.0


@pytest.mark.parametrize("nc", [1, 4, 9])
def test_restriction_is_normalised_transpose(nc):
    nf = 2 * nc
    # assemble P column by column from the potential interpolation
    P = np.zeros(((nf + 1) ** 2, (nc + 1) ** 2))
    for k in range((nc + 1) ** 2):
        e = np.zeros((nc + 1) ** 2); e[k] = 1.0
        P[:, k] = o.prolong_potential(e.reshape(nc + 1, nc + 1)).ravel()
    rng = np.random.default_rng(nc)
    f = rng.uniform(0, 1, size=(nf + 1, nf + 1))
    D = P.T @ np.ones((nf + 1) ** 2)
    want = (P.T @ f.ravel()) / D
    np.testing.assert_allclose(o.restrict_density(f).ravel(), want, rtol=1e-14)
    np.testing.assert_allclose(o.restrict_density(np.ones((nf + 1, nf + 1))), 1.0, rtol=1e-15)


def test_pyramid_masses_and_zero_sum():
    rng = np.random.default_rng(3)
    n, L = 32, 4
    p0 = rng.uniform(size=(n + 1, n + 1)); p1 = rng.uniform(size=(n + 1, n + 1))
    p1 *= p0.sum() / p1.sum()
    rhos = o.prepare_levels(p0, p1, n, L)
    for l, nl in enumerate(o.level_sides(n, L)):
        assert rhos[l].shape == (nl + 1, nl + 1)
        assert abs(rhos[l].sum()) <= 1e-10 * np.abs(rhos[l]).sum()
    with pytest.raises(ValueError):
        o.prepare_levels(p0, p1 * 1.01, n, L)
    bad = p0.copy(); bad[0, 0] = -1
    with pytest.raises(ValueError):
        o.prepare_levels(bad, p1, n, L)
    with pytest.raises(ValueError):
        o.level_sides(12, 4)

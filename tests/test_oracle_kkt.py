"""Pins of the primal part of the normalised KKT residual: the norm of the
minimum-norm flux correction A*(A A*)^{-1}(A m - rho).

The reference values come from a route that shares nothing with the
oracle's DCT Poisson solve: the divergence of Sec. 2.2 assembled here as an
explicit matrix from the grid graph (each flux variable leaves its node
with +1/h and enters the next node with -1/h), and the least-norm solution
of A c = A m - rho by numpy's SVD-based least squares."""
import itertools
import math

import numpy as np
import pytest

import oracle.w1_oracle as o
import oracle.w1_oracle3d as o3


def _assembled_div(n, d, h):
    """Rows: nodes (row-major over d indices); columns: flux variables, one
    per (axis, node) with the node's index along the axis below n."""
    N = n + 1
    nodes = list(itertools.product(range(N), repeat=d))
    nid = {x: k for k, x in enumerate(nodes)}
    cols = []
    for ax in range(d):
        for x in nodes:
            if x[ax] < n:
                cols.append((ax, x))
    A = np.zeros((len(nodes), len(cols)))
    for c, (ax, x) in enumerate(cols):
        y = list(x); y[ax] += 1
        A[nid[x], c] += 1.0 / h
        A[nid[tuple(y)], c] -= 1.0 / h
    return A, cols, nodes


def _flatten(m, cols):
    return np.array([m[ax][x] for ax, x in cols])


@pytest.mark.parametrize("n,seed", [(2, 0), (3, 1), (5, 2), (6, 3)])
def test_primal_residual_2d_least_norm(n, seed):
    h = 1.0 / n
    rng = np.random.default_rng(seed)
    m1 = rng.standard_normal((n + 1, n + 1)); m1[n, :] = 0
    m2 = rng.standard_normal((n + 1, n + 1)); m2[:, n] = 0
    rho = rng.standard_normal((n + 1, n + 1)); rho -= rho.mean()
    A, cols, nodes = _assembled_div(n, 2, h)
    mv = _flatten((m1, m2), cols)
    r = A @ mv - np.array([rho[x] for x in nodes])
    c, *_ = np.linalg.lstsq(A, r, rcond=None)
    ref = math.sqrt(float(c @ c) * h * h)
    assert o.primal_residual(m1, m2, rho, h) == pytest.approx(ref, rel=1e-11)
    # the correction itself, variable by variable
    c1, c2 = o.min_norm_correction(m1, m2, rho, h)
    np.testing.assert_allclose(_flatten((c1, c2), cols), c, atol=1e-11 * np.abs(c).max())
    # and the normalised KKT takes it over f(m)
    phi = np.zeros((n + 1, n + 1))
    P = o.flux_cost(m1, m2, h, 2)
    k, P_, D_ = o.kkt_plain(m1, m2, phi, rho, h, 2)
    assert P_ == P and D_ == 0.0
    assert k == pytest.approx(max(ref / P, 1.0), rel=1e-11)   # gap term = |P - 0| / P = 1
    # the feasible flux of the certificate is m minus that correction
    ev = o.evaluate(m1, m2, phi, rho, h, 2)
    assert ev["r_pri"] == pytest.approx(ref / P, rel=1e-11)


@pytest.mark.parametrize("n,seed", [(2, 4), (3, 5)])
def test_primal_residual_3d_least_norm(n, seed):
    h = 1.0 / n
    rng = np.random.default_rng(seed)
    m = []
    for ax in range(3):
        a = rng.standard_normal((n + 1,) * 3)
        idx = [slice(None)] * 3; idx[ax] = n
        a[tuple(idx)] = 0
        m.append(a)
    rho = rng.standard_normal((n + 1,) * 3); rho -= rho.mean()
    A, cols, nodes = _assembled_div(n, 3, h)
    r = A @ _flatten(m, cols) - np.array([rho[x] for x in nodes])
    c, *_ = np.linalg.lstsq(A, r, rcond=None)
    ref = math.sqrt(float(c @ c) * h ** 3)
    assert o3.primal_residual(tuple(m), rho, h) == pytest.approx(ref, rel=1e-11)


def test_primal_residual_zero_iff_feasible():
    """A feasible flux (here: the projection of eq. (pdhg)) has residual 0;
    adding a divergence-free circulation keeps it 0, while the same
    perturbation of rho does not."""
    n, h = 6, 1 / 6
    rng = np.random.default_rng(9)
    rho = rng.standard_normal((n + 1, n + 1)); rho -= rho.mean()
    m1 = rng.standard_normal((n + 1, n + 1)); m1[n, :] = 0
    m2 = rng.standard_normal((n + 1, n + 1)); m2[:, n] = 0
    c1, c2 = o.min_norm_correction(m1, m2, rho, h)
    f1, f2 = m1 - c1, m2 - c2
    assert o.primal_residual(f1, f2, rho, h) <= 1e-12 * math.sqrt(o.inner_h((m1, m2), (m1, m2), h))
    # unit circulation around the cell (2, 3)
    g1, g2 = f1.copy(), f2.copy()
    g1[2, 3] += 1; g2[3, 3] += 1; g1[2, 4] -= 1; g2[2, 3] -= 1
    assert o.primal_residual(g1, g2, rho, h) <= 1e-12 * math.sqrt(o.inner_h((g1, g2), (g1, g2), h))
    bump = np.zeros_like(rho); bump[1, 1] = 1.0; bump[4, 5] = -1.0
    assert o.primal_residual(f1, f2, rho + bump, h) > 1e-3

"""Pins of the oracle's discrete model (Sec. 2.2), prox maps and Poisson solve.

Each check ties the oracle to something other than itself: a hand-worked
divergence, adjointness, telescoping, explicit DCT eigenvectors, power
iteration, the Moreau decomposition and direct minimisation.
"""
import math

import numpy as np
import pytest

import oracle.w1_oracle as o


def _rand_flux(n, rng):
    m1 = rng.standard_normal((n + 1, n + 1))
    m2 = rng.standard_normal((n + 1, n + 1))
    m1[n, :] = 0.0
    m2[:, n] = 0.0
    return m1, m2


def test_divergence_hand_example():
    # n = 1 (2 x 2 nodes, h = 1): edges m1[0,0] = a (0,0)->(1,0),
    # m1[0,1] = b (0,1)->(1,1), m2[0,0] = c (0,0)->(0,1), m2[1,0] = e (1,0)->(1,1).
    a, b, c, e = 1.5, -2.0, 0.25, 3.0
    m1 = np.array([[a, b], [0.0, 0.0]])
    m2 = np.array([[c, 0.0], [e, 0.0]])
    h = 0.5
    got = o.div(m1, m2, h)
    want = np.array([[a + c, b - c], [-a + e, -b - e]]) / h
    np.testing.assert_allclose(got, want, rtol=0, atol=0)


@pytest.mark.parametrize("n", [1, 2, 7, 16])
def test_adjoint_and_telescoping(n):
    rng = np.random.default_rng(n)
    h = 1.0 / n
    m1, m2 = _rand_flux(n, rng)
    phi = rng.standard_normal((n + 1, n + 1))
    lhs = o.inner_h(o.div(m1, m2, h), phi, h)
    a1, a2 = o.div_adj(phi, h)
    rhs = o.inner_h((m1, m2), (a1, a2), h)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)
    # sum of the divergence telescopes to zero (zero normal flux)
    assert abs(o.div(m1, m2, h).sum()) <= 1e-10 * np.abs(m1).sum() / h
    # the boundary components never enter A
    m1b = m1.copy(); m1b[n, :] = 7.0
    np.testing.assert_array_equal(o.div(m1b, m2, h), o.div(m1, m2, h))
    # A* has zero last component on its own axis, and is minus the forward difference
    assert np.all(a1[n, :] == 0) and np.all(a2[:, n] == 0)
    g1, g2 = o.grad_fwd(phi, h)
    np.testing.assert_allclose(g1[:-1, :], (phi[1:, :] - phi[:-1, :]) / h, rtol=1e-14, atol=1e-12)


@pytest.mark.parametrize("n", [4, 8, 9])
def test_dct_basis_diagonalises_laplacian(n):
    h = 1.0 / n
    N = n + 1
    lam = o.laplacian_eigenvalues(n, h)
    idx = np.arange(N)
    for k, l in [(0, 0), (1, 0), (0, 3), (2, min(5, n)), (n, n), (n - 1, 1)]:
        v = np.outer(np.cos(np.pi * k * (2 * idx + 1) / (2 * N)), np.cos(np.pi * l * (2 * idx + 1) / (2 * N)))
        Lv = o.div(*o.div_adj(v, h), h)
        np.testing.assert_allclose(Lv, lam[k, l] * v, rtol=0, atol=1e-9 * (1 + lam[k, l]))


@pytest.mark.parametrize("n", [4, 16, 33])
def test_poisson_residual(n):
    rng = np.random.default_rng(10 + n)
    h = 1.0 / n
    b = rng.standard_normal((n + 1, n + 1))
    b -= b.mean()
    u = o.poisson_neumann(b, h)
    res = o.div(*o.div_adj(u, h), h) - b
    assert np.linalg.norm(res) <= 1e-12 * np.linalg.norm(b) * n * n
    assert abs(u.mean()) <= 1e-12 * (np.abs(u).max() + 1)


@pytest.mark.parametrize("n", [4, 12])
def test_operator_norm_closed_form_by_power_iteration(n):
    h = 1.0 / n
    rng = np.random.default_rng(1)
    v = rng.standard_normal((n + 1, n + 1))
    for _ in range(4000):
        v = o.div(*o.div_adj(v, h), h)
        v /= np.linalg.norm(v)
    lam = np.sum(v * o.div(*o.div_adj(v, h), h))
    assert abs(math.sqrt(lam) - o.norm_A_exact(n, h)) <= 1e-6 * o.norm_A_exact(n, h)
    assert o.norm_A_exact(n, h) < o.norm_A_bound(h)
    mu, tau = o.plain_step_sizes(h)
    assert mu * tau * o.norm_A_exact(n, h) ** 2 < 0.25 + 1e-15


@pytest.mark.parametrize("p", [1, 2, math.inf])
def test_moreau_decomposition(p):
    rng = np.random.default_rng(3 if p == math.inf else p)
    v1 = rng.standard_normal(2000) * 2
    v2 = rng.standard_normal(2000) * 2
    mu = 0.7
    s1, s2 = o.shrink(v1, v2, mu, p)
    q1, q2 = o.project_dual_ball(v1 / mu, v2 / mu, p)
    np.testing.assert_allclose(s1 + mu * q1, v1, atol=1e-12)
    np.testing.assert_allclose(s2 + mu * q2, v2, atol=1e-12)
    # projections land in the dual-norm ball
    qn = o.pointwise_norm(q1, q2, {1: math.inf, 2: 2, math.inf: 1}[p])
    assert qn.max() <= 1 + 1e-12


@pytest.mark.parametrize("p", [1, 2, math.inf])
def test_shrink_is_the_prox_minimiser(p):
    rng = np.random.default_rng(8 if p == math.inf else 5 + p)
    mu = 0.3
    for _ in range(50):
        v = rng.standard_normal(2)
        s1, s2 = o.shrink(np.array([v[0]]), np.array([v[1]]), mu, p)
        best = np.array([s1[0], s2[0]])

        def obj(m):
            nm = np.abs(m).sum() if p == 1 else (np.abs(m).max() if p == math.inf else np.linalg.norm(m))
            return nm + np.sum((m - v) ** 2) / (2 * mu)

        f0 = obj(best)
        for _ in range(200):
            trial = best + rng.standard_normal(2) * 10 ** rng.uniform(-6, 0)
            assert obj(trial) >= f0 - 1e-12


def test_l1_ball_projection_variational_inequality():
    # p = inf: the dual ball is the l_1 unit ball, a polytope with vertices
    # +-e1, +-e2.  y = P(w) is the projection iff y lies in the ball and
    # <w - y, z - y> <= 0 for every z of the ball, which for a polytope it
    # suffices to check at the vertices.
    rng = np.random.default_rng(17)
    w1 = rng.standard_normal(4000) * 1.5
    w2 = rng.standard_normal(4000) * 1.5
    w1[:4] = [0.3, 2.0, 0.0, -0.5]
    w2[:4] = [-0.2, 0.0, 0.0, 1.5]       # inside, on an axis, zero, an edge case
    y1, y2 = o.project_dual_ball(w1, w2, math.inf)
    assert (np.abs(y1) + np.abs(y2)).max() <= 1 + 1e-12
    for z1, z2 in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        vi = (w1 - y1) * (z1 - y1) + (w2 - y2) * (z2 - y2)
        assert vi.max() <= 1e-12
    inside = np.abs(w1) + np.abs(w2) <= 1
    np.testing.assert_array_equal(y1[inside], w1[inside])
    np.testing.assert_array_equal(y2[inside], w2[inside])
    np.testing.assert_allclose([y1[1], y2[1]], [1.0, 0.0], atol=1e-15)
    np.testing.assert_allclose([y1[3], y2[3]], [0.0, 1.0], atol=1e-15)


def test_linf_shrink_optimality_condition():
    # x = prox of mu ||.||_inf at v iff g = (v - x)/mu is a subgradient of
    # ||.||_inf at x: ||g||_1 <= 1 and <g, x> = ||x||_inf (Fenchel equality
    # of a norm and its dual)
    rng = np.random.default_rng(23)
    mu = 0.4
    v1 = rng.standard_normal(4000)
    v2 = rng.standard_normal(4000)
    v1[:3] = [0.1, 1.0, 0.5]
    v2[:3] = [0.2, 0.9, -0.05]           # inside the ball, both move, one moves
    x1, x2 = o.shrink(v1, v2, mu, math.inf)
    g1, g2 = (v1 - x1) / mu, (v2 - x2) / mu
    assert (np.abs(g1) + np.abs(g2)).max() <= 1 + 1e-12
    np.testing.assert_allclose(g1 * x1 + g2 * x2, np.maximum(np.abs(x1), np.abs(x2)), atol=1e-12)
    np.testing.assert_allclose([x1[0], x2[0]], [0.0, 0.0], atol=1e-15)
    # equal magnitudes (a + b - mu)/2 when |a - b| < mu; only the larger
    # component moves, by mu, when |a - b| >= mu
    np.testing.assert_allclose([x1[1], x2[1]], [0.75, 0.75], atol=1e-15)
    np.testing.assert_allclose([x1[2], x2[2]], [0.1, -0.05], atol=1e-15)


def test_dual_exponent_and_norms():
    v1 = np.array([3.0, -1.0]); v2 = np.array([-4.0, 0.5])
    np.testing.assert_allclose(o.pointwise_norm(v1, v2, 1), [7.0, 1.5])
    np.testing.assert_allclose(o.pointwise_norm(v1, v2, 2), [5.0, math.hypot(1, 0.5)])
    np.testing.assert_allclose(o.pointwise_norm(v1, v2, math.inf), [4.0, 1.0])
    assert o.dual_exponent(1) == math.inf and o.dual_exponent(2) == 2

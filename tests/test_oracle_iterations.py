"""Pins of the iterations themselves: exact first steps, the projection
property of eq. (pdhg), monotone fixed-point residuals (eq. (pd_stop);
eq. (pdhg_stop) on the pairing (vphi^k, m^{k+1})), and Appendix B."""
import numpy as np
import pytest

import oracle.w1_oracle as o
import w1data


def _problem(n, seed=0):
    p0, p1 = w1data.random_pair(n, seed)
    return o.prepare_levels(p0, p1, n, 1)[0]


@pytest.mark.parametrize("p", [1, 2])
def test_first_plain_step_from_zero(p):
    n, h = 8, 1 / 8
    rho = _problem(n)
    mu, tau = o.plain_step_sizes(h)
    z = np.zeros((n + 1, n + 1))
    m1, m2, phi, R = o.pd_step(z, z, z, rho, h, mu, tau, p)
    assert np.all(m1 == 0) and np.all(m2 == 0)
    np.testing.assert_allclose(phi, -tau * rho, rtol=1e-15)
    assert R == pytest.approx(o.inner_h(phi, phi, h) / tau, rel=1e-12)


@pytest.mark.parametrize("p", [1, 2])
def test_prox_step_projects_onto_constraint(p):
    n, h = 12, 1 / 12
    rho = _problem(n, 1)
    rng = np.random.default_rng(2)
    m1 = rng.standard_normal((n + 1, n + 1)); m1[n, :] = 0
    m2 = rng.standard_normal((n + 1, n + 1)); m2[:, n] = 0
    w1 = rng.uniform(-1, 1, (n + 1, n + 1)); w1[n, :] = 0
    w2 = rng.uniform(-1, 1, (n + 1, n + 1)); w2[:, n] = 0
    out = o.prox_step(m1, m2, w1, w2, w1, w2, rho, h, 0.5, 0.5, p)
    np.testing.assert_allclose(o.div(out[0], out[1], h), rho, atol=1e-10 * np.abs(rho).max())
    # the new dual is in the dual-norm ball and boundary components stay zero
    q = o.pointwise_norm(out[2], out[3], o.dual_exponent(p))
    assert q.max() <= 1 + 1e-12
    assert np.all(out[0][n, :] == 0) and np.all(out[1][:, n] == 0)
    # the projection is the closest feasible flux to v = m - mu vphibar
    v1, v2 = m1 - 0.5 * w1, m2 - 0.5 * w2
    d1, d2 = out[0] - v1, out[1] - v2
    for _ in range(5):
        k1 = rng.standard_normal((n + 1, n + 1)); k1[n, :] = 0
        k2 = rng.standard_normal((n + 1, n + 1)); k2[:, n] = 0
        # a kernel direction: subtract its own projection
        u = o.poisson_neumann(o.div(k1, k2, h), h)
        a1, a2 = o.div_adj(u, h)
        k1, k2 = k1 - a1, k2 - a2
        assert abs(o.inner_h((d1, d2), (k1, k2), h)) <= 1e-9 * (1 + np.abs(k1).sum())


@pytest.mark.parametrize("p,seed", [(1, 3), (2, 3), (1, 7)])
def test_plain_fpr_nonincreasing(p, seed):
    n, h = 8, 1 / 8
    rho = _problem(n, seed)
    mu, tau = o.plain_step_sizes(h)
    m1 = np.zeros((n + 1, n + 1)); m2 = m1.copy(); phi = m1.copy()
    prev = np.inf
    for _ in range(1500):
        m1, m2, phi, R = o.pd_step(m1, m2, phi, rho, h, mu, tau, p)
        assert R <= prev * (1 + 1e-10) + 1e-30
        prev = R


@pytest.mark.parametrize("p,seed", [(1, 3), (2, 3)])
def test_prox_fpr_nonincreasing_shifted_pairing(p, seed):
    n, h = 8, 1 / 8
    rho = _problem(n, seed)
    mu, tau = o.prox_step_sizes()
    z = np.zeros((n + 1, n + 1))
    st = (z, z, z, z, z, z)
    hist = []
    for _ in range(800):
        st = o.prox_step(*st, rho, h, mu, tau, p)[:6]
        hist.append(st)
    prev = np.inf
    for k in range(1, len(hist) - 1):
        dm = (hist[k + 1][0] - hist[k][0], hist[k + 1][1] - hist[k][1])
        dw = (hist[k][2] - hist[k - 1][2], hist[k][3] - hist[k - 1][3])
        G = o.inner_h(dm, dm, h) / mu + o.inner_h(dw, dw, h) / tau + 2 * o.inner_h(dw, dm, h)
        assert G >= -1e-15
        assert G <= prev * (1 + 1e-9) + 1e-30
        prev = G


def test_appendix_b_potential_recovers_gradient():
    n, h = 10, 0.1
    rng = np.random.default_rng(4)
    psi = rng.standard_normal((n + 1, n + 1)); psi -= psi.mean()
    g1, g2 = o.div_adj(psi, h)
    np.testing.assert_allclose(o.potential_from_dual(g1, g2, h), psi, atol=1e-10)

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


# ---------------------------------------------------------------------------
# eq. (pdhg) and its residual eq. (pdhg_stop) worked by hand on the smallest
# grid: n = 1, h = 1, nodes a = (0,0), b = (1,0), c = (1,1), d = (0,1).  The
# flux variables are m1[0,0] (a->b), m1[0,1] (d->c), m2[0,0] (a->d),
# m2[1,0] (b->c); A A* is the Laplacian of the 4-cycle a-b-c-d.
#
# Common data: rho = 0, mu = tau = 1/2, p = 1 (q = inf: clip to [-1, 1]),
# vphibar1[0,0] = 24, every other vphibar component 0.
#   v = m - mu vphibar: the circulation part of m plus v1[0,0] -= 12;
#   r = A v - rho = (-12 at a, +12 at b, 0 at c, 0 at d) (the circulation
#   is divergence-free);
#   L u = r on the 4-cycle: u = (a, b, c, d) = (-9/2, 9/2, 3/2, -3/2)
#   (check at a: 2(-9/2) - 9/2 - (-3/2) = -12; at d: 2(-3/2) - 3/2 + 9/2 = 0);
#   A* u: (A*u)1[0,0] = u_a - u_b = -9, (A*u)1[0,1] = u_d - u_c = -3,
#         (A*u)2[0,0] = u_a - u_d = -3, (A*u)2[1,0] = u_b - u_c = 3;
#   m+ = v - A* u.
# ---------------------------------------------------------------------------
_E = [("1", 0, 0), ("1", 0, 1), ("2", 0, 0), ("2", 1, 0)]   # the four variables


def _hand_state(vals):
    a1 = np.zeros((2, 2)); a2 = np.zeros((2, 2))
    for (comp, i, j), v in zip(_E, vals):
        (a1 if comp == "1" else a2)[i, j] = v
    return a1, a2


def _hand_vals(a1, a2):
    return [(a1 if comp == "1" else a2)[i, j] for comp, i, j in _E]


@pytest.mark.parametrize("case", ["zero_flux", "circulating_flux"])
def test_prox_step_residual_worked_by_hand(case):
    h, mu, tau = 1.0, 0.5, 0.5
    rho = np.zeros((2, 2))
    wb1, wb2 = _hand_state([24, 0, 0, 0])
    if case == "zero_flux":
        # m = 0, vphi1[0,0] = 1:
        # m+ = (-12 + 9, 0 + 3, 0 + 3, 0 - 3) = (-3, 3, 3, -3)
        # vphi + tau m+ = (1 - 3/2, 3/2, 3/2, -3/2) -> clip -> (-1/2, 1, 1, -1)
        # d = m+ - m = (-3, 3, 3, -3), e = vphi+ - vphi = (-3/2, 1, 1, -1)
        # ||d||^2/mu = 36/(1/2) = 72; ||e||^2/tau = (9/4 + 3)/(1/2) = 21/2
        # <e, d> = 9/2 + 3 + 3 + 3 = 27/2
        m = [0, 0, 0, 0]
        w = [1, 0, 0, 0]
        m_new = [-3, 3, 3, -3]
        w_new = [-0.5, 1, 1, -1]
        G = 72 + 21 / 2 + 2 * (27 / 2)          # = 219/2
    else:
        # m = the unit circulation a->b->c->d->a: (1, -1, -1, 1); A m = 0
        # m+ = (1 - 12 + 9, -1 + 3, -1 + 3, 1 - 3) = (-2, 2, 2, -2)
        # vphi + tau m+ = (1 - 1, 1, 1, -1) = (0, 1, 1, -1), inside the ball
        # d = m+ - m = (-3, 3, 3, -3), e = (-1, 1, 1, -1)
        # ||d||^2/mu = 72; ||e||^2/tau = 8; <e, d> = 3 + 3 + 3 + 3 = 12
        m = [1, -1, -1, 1]
        w = [1, 0, 0, 0]
        m_new = [-2, 2, 2, -2]
        w_new = [0, 1, 1, -1]
        G = 72 + 8 + 2 * 12                      # = 104
    m1, m2 = _hand_state(m)
    w1_, w2_ = _hand_state(w)
    out = o.prox_step(m1, m2, w1_, w2_, wb1, wb2, rho, h, mu, tau, 1)
    np.testing.assert_allclose(_hand_vals(out[0], out[1]), m_new, atol=1e-13)
    np.testing.assert_allclose(_hand_vals(out[2], out[3]), w_new, atol=1e-13)
    # extrapolation vphibar+ = 2 vphi+ - vphi
    np.testing.assert_allclose(_hand_vals(out[4], out[5]),
                               [2 * a - b for a, b in zip(w_new, w)], atol=1e-13)
    # the non-variables (m1 on the last row, m2 on the last column) stay 0
    assert out[0][1, 0] == 0 and out[0][1, 1] == 0 and out[1][0, 1] == 0 and out[1][1, 1] == 0
    assert out[6] == pytest.approx(G, rel=1e-13)


def test_plain_step_residual_worked_by_hand():
    """eq. (primaldual) and R^k of eq. (pd_stop) on the same 2 x 2 grid
    (h = 1, mu = tau = 1/4, p = 1).  phi = (a, b, c, d) = (0, 1, 0, 0),
    m = 0, rho = (1, -1, 0, 0).
      grad+ phi: g1[0,0] = phi_b - phi_a = 1, g1[0,1] = phi_c - phi_d = 0,
                 g2[0,0] = phi_d - phi_a = 0, g2[1,0] = phi_c - phi_b = -1;
      m + mu g = (1/4, 0, 0, -1/4) -> shrink by 1/4 -> m+ = 0 everywhere;
      2 m+ - m = 0, so phi+ = phi - tau rho = (-1/4, 5/4, 0, 0);
      R = ||dm||^2/mu + ||dphi||^2/tau - 2 <dphi, A dm> = 0 + (1/16 + 1/16)/(1/4) = 1/2.
    A second state with m = (1, 0, 0, 0) gives a non-zero cross term:
      m + mu g = (5/4, 0, 0, -1/4) -> m+ = (1, 0, 0, 0), dm = 0 again;
      instead take phi = 0: m+ = shrink(m) = (3/4, 0, 0, 0), dm = (-1/4, 0, 0, 0),
      b = 2 m+ - m = (1/2, 0, 0, 0), A b = (1/2 at a, -1/2 at b),
      phi+ = tau (A b - rho) = (1/4)(-1/2, 1/2, 0, 0) = (-1/8, 1/8, 0, 0),
      A dm = (-1/4 at a, 1/4 at b), <dphi, A dm> = 1/32 + 1/32 = 1/16,
      R = (1/16)/(1/4) + (1/64 + 1/64)/(1/4) - 2/16 = 1/4 + 1/8 - 1/8 = 1/4."""
    h, mu, tau = 1.0, 0.25, 0.25
    rho = np.array([[1.0, 0.0], [-1.0, 0.0]])          # rho[i, j]: a = [0,0], b = [1,0]
    phi = np.array([[0.0, 0.0], [1.0, 0.0]])
    z = np.zeros((2, 2))
    m1, m2, phin, R = o.pd_step(z, z, phi, rho, h, mu, tau, 1)
    assert np.all(m1 == 0) and np.all(m2 == 0)
    np.testing.assert_allclose(phin, [[-0.25, 0.0], [1.25, 0.0]], atol=1e-15)
    assert R == pytest.approx(0.5, rel=1e-14)
    m1 = np.array([[1.0, 0.0], [0.0, 0.0]])
    n1, n2, phin, R = o.pd_step(m1, z, z, rho, h, mu, tau, 1)
    np.testing.assert_allclose(n1, [[0.75, 0.0], [0.0, 0.0]], atol=1e-15)
    assert np.all(n2 == 0)
    np.testing.assert_allclose(phin, [[-0.125, 0.0], [0.125, 0.0]], atol=1e-15)
    assert R == pytest.approx(0.25, rel=1e-14)

"""Pins of the d-general oracle (used at d = 3): at d = 2 it reproduces the
pinned d = 2 module function by function and solve by solve; at d = 3 it is
held to adjointness, the DCT eigenvectors of A A*, interpolation identities
and Lemma 1, the prox maps' optimality conditions, the 1-D closed form,
axis-aligned translations, exact transport by LP on tiny grids and the norm
sandwich."""
import math

import numpy as np
import pytest
import scipy.fft
from scipy.optimize import linprog

import oracle.w1_oracle as o2
import oracle.w1_oracle3d as o3
import w1data

P_ALL = [1, 2, math.inf]


# ---------------------------------------------------------------- d = 2 ----

def test_reduces_to_the_2d_module_operators():
    rng = np.random.default_rng(1)
    n, h = 9, 1.0 / 9
    m1, m2, phi = (rng.standard_normal((n + 1, n + 1)) for _ in range(3))
    m1[n, :] = 0
    m2[:, n] = 0
    np.testing.assert_allclose(o3.div((m1, m2), h), o2.div(m1, m2, h), atol=1e-12)
    for a, b in zip(o3.div_adj(phi, h), o2.div_adj(phi, h)):
        np.testing.assert_allclose(a, b, atol=1e-12)
    for p in P_ALL:
        for a, b in zip(o3.shrink((m1, m2), 0.3, p), o2.shrink(m1, m2, 0.3, p)):
            np.testing.assert_allclose(a, b, atol=1e-14)
        for a, b in zip(o3.project_dual_ball((m1, m2), p), o2.project_dual_ball(m1, m2, p)):
            np.testing.assert_allclose(a, b, atol=1e-14)
    np.testing.assert_allclose(o3.poisson_neumann(phi - phi.mean(), h), o2.poisson_neumann(phi - phi.mean(), h),
                               atol=1e-12)
    c = rng.standard_normal((5, 5))
    np.testing.assert_allclose(o3.prolong_potential(c), o2.prolong_potential(c), atol=1e-15)
    c1, c2 = rng.standard_normal((5, 5)), rng.standard_normal((5, 5))
    c1[4, :] = 0
    c2[:, 4] = 0
    for a, b in zip(o3.prolong_flux((c1, c2)), o2.prolong_flux(c1, c2)):
        np.testing.assert_allclose(a, b, atol=1e-15)
    f = rng.uniform(size=(9, 9))
    np.testing.assert_allclose(o3.restrict_density(f), o2.restrict_density(f), atol=1e-15)


@pytest.mark.parametrize("p", [1, 2])
def test_reduces_to_the_2d_module_solve(p):
    n, L = 8, 2
    a, b = w1data.random_pair(n, 4)
    eps = 1e-6
    r3 = o3.solve_plain(a, b, n, L=L, p=p, stop="fpr", tol=eps, check_every=10)
    r2 = o2.solve(a, b, n, L=L, p=p, algo=1, stop="fpr", tol=eps, eps_L=eps, check_every=10)
    assert r3["iters"] == r2["iters"]
    assert r3["w1"] == pytest.approx(r2["w1"], rel=1e-12)
    np.testing.assert_allclose(r3["level_w1"], r2["level_w1"], rtol=1e-12)
    ev = o2.evaluate(r2["m1"], r2["m2"], r2["psi"], r2["rho"], 1.0 / n, p)
    assert r3["lo"] == pytest.approx(ev["lo"], rel=1e-10)
    assert r3["hi"] == pytest.approx(ev["hi"], rel=1e-10)


@pytest.mark.parametrize("p", [1, 2, math.inf])
def test_reduces_to_the_2d_module_prox(p):
    n, L = 8, 2
    a, b = w1data.random_pair(n, 6)
    rng = np.random.default_rng(8)
    m1, m2, w1_, w2_ = (rng.standard_normal((n + 1, n + 1)) for _ in range(4))
    rho = o2.prepare_levels(a, b, n, 1)[0]
    h = 1.0 / n
    got = o3.prox_step((m1, m2), (w1_, w2_), (w1_, w2_), rho, h, 0.5, 0.5, p)
    want = o2.prox_step(m1, m2, w1_, w2_, w1_, w2_, rho, h, 0.5, 0.5, p)
    for x, y in zip((*got[0], *got[1], *got[2]), want[:6]):
        np.testing.assert_allclose(x, y, atol=1e-12)
    assert got[3] == pytest.approx(want[6], rel=1e-12)
    eps = 1e-5
    r3 = o3.solve_prox(a, b, n, L=L, p=p, stop="fpr", tol=eps, check_every=1)
    r2 = o2.solve(a, b, n, L=L, p=p, algo=2, stop="fpr", tol=eps, eps_L=eps, check_every=1)
    assert r3["iters"] == r2["iters"]
    assert r3["w1"] == pytest.approx(r2["w1"], rel=1e-11)
    assert r3["lo"] == pytest.approx(r2["lo"], rel=1e-10) and r3["hi"] == pytest.approx(r2["hi"], rel=1e-10)
    np.testing.assert_allclose(r3["psi"], r2["psi"], atol=1e-11)


# ---------------------------------------------------------------- d = 3 ----

def test_adjoint_and_telescoping_3d():
    rng = np.random.default_rng(2)
    n, h = 5, 0.2
    m = tuple(rng.standard_normal((n + 1,) * 3) for _ in range(3))
    for i, mi in enumerate(m):
        idx = [slice(None)] * 3
        idx[i] = -1
        mi[tuple(idx)] = 0.0
    phi = rng.standard_normal((n + 1,) * 3)
    lhs = o3.inner_h(o3.div(m, h), phi, h)
    rhs = o3.inner_h(m, o3.div_adj(phi, h), h)
    assert lhs == pytest.approx(rhs, rel=1e-12)
    assert abs(o3.div(m, h).sum()) < 1e-10          # zero normal flux: mass conserved
    # hand example: a unit flux on the edge (0,0,0) -> (0,0,1)
    e = tuple(np.zeros((n + 1,) * 3) for _ in range(3))
    e[2][0, 0, 0] = 1.0
    d = o3.div(e, h)
    assert d[0, 0, 0] == pytest.approx(1 / h) and d[0, 0, 1] == pytest.approx(-1 / h)
    assert np.count_nonzero(d) == 2


@pytest.mark.parametrize("k", [(0, 0, 1), (2, 1, 3), (4, 4, 4)])
def test_dct_basis_diagonalises_the_3d_laplacian(k):
    n, h = 4, 0.25
    spike = np.zeros((n + 1,) * 3)
    spike[k] = 1.0
    v = scipy.fft.idctn(spike, type=2, norm="ortho")
    Av = o3.div(o3.div_adj(v, h), h)
    lam = o3.laplacian_eigenvalues(n, h, 3)[k]
    np.testing.assert_allclose(Av, lam * v, atol=1e-9 * max(lam, 1))
    r = np.random.default_rng(3).standard_normal((n + 1,) * 3)
    r -= r.mean()
    u = o3.poisson_neumann(r, h)
    np.testing.assert_allclose(o3.div(o3.div_adj(u, h), h), r, atol=1e-9)


def test_gershgorin_bound_3d():
    n, h = 5, 0.2
    lam = o3.laplacian_eigenvalues(n, h, 3).max()
    assert math.sqrt(lam) < o3.norm_A_bound(h, 3)
    assert math.sqrt(lam) > 0.9 * o3.norm_A_bound(h, 3)


def test_interpolation_exact_on_affine_and_lemma1_3d():
    nc = 3
    t = np.arange(nc + 1) / nc
    X = np.meshgrid(t, t, t, indexing="ij")
    c = 0.3 + 1.1 * X[0] - 0.7 * X[1] + 2.0 * X[2]
    tf = np.arange(2 * nc + 1) / (2 * nc)
    Xf = np.meshgrid(tf, tf, tf, indexing="ij")
    np.testing.assert_allclose(o3.prolong_potential(c), 0.3 + 1.1 * Xf[0] - 0.7 * Xf[1] + 2.0 * Xf[2],
                               atol=1e-14)
    rng = np.random.default_rng(5)
    hc, hf = 1.0 / nc, 0.5 / nc
    for _ in range(5):
        phi = rng.standard_normal((nc + 1,) * 3)
        f = o3.prolong_potential(phi)
        assert o3.inner_h(f, f, hf) <= o3.inner_h(phi, phi, hc) + 1e-12
        m = tuple(rng.standard_normal((nc + 1,) * 3) for _ in range(3))
        for i, mi in enumerate(m):
            idx = [slice(None)] * 3
            idx[i] = -1
            mi[tuple(idx)] = 0.0
        fm = o3.prolong_flux(m)
        assert o3.inner_h(fm, fm, hf) <= o3.inner_h(m, m, hc) + 1e-12
    # a constant flux component along its own axis stays constant away from
    # the last node, and the restriction keeps constants
    m = tuple(np.zeros((nc + 1,) * 3) for _ in range(3))
    m[1][:, :-1, :] = 2.5
    fm = o3.prolong_flux(m)
    assert np.allclose(fm[1][:, :-1, :], 2.5) and np.allclose(fm[1][:, -1, :], 0.0)
    np.testing.assert_allclose(o3.restrict_density(np.full((7, 7, 7), 3.0)), 3.0, atol=1e-14)


def test_prox_maps_optimality_3d():
    rng = np.random.default_rng(7)
    mu = 0.35
    v = tuple(rng.standard_normal(3000) for _ in range(3))
    for p in P_ALL:
        x = o3.shrink(v, mu, p)
        g = tuple((vi - xi) / mu for vi, xi in zip(v, x))
        q = o3.dual_exponent(p)
        assert o3.pointwise_norm(g, q).max() <= 1 + 1e-12
        np.testing.assert_allclose(sum(gi * xi for gi, xi in zip(g, x)), o3.pointwise_norm(x, p), atol=1e-12)
    w = tuple(rng.standard_normal(3000) * 1.5 for _ in range(3))
    y = o3.project_dual_ball(w, math.inf)
    assert o3.pointwise_norm(y, 1).max() <= 1 + 1e-12
    for ax in range(3):
        for s in (1.0, -1.0):
            z = [np.full(3000, s) if a == ax else np.zeros(3000) for a in range(3)]
            vi = sum((wi - yi) * (zi - yi) for wi, yi, zi in zip(w, y, z))
            assert vi.max() <= 1e-12


TIGHT = dict(stop="kkt", tol=1e-8, check_every=20, max_iters=400000)


@pytest.mark.parametrize("p", P_ALL)
def test_1d_closed_form_in_3d(p):
    n = 4
    rng = np.random.default_rng(11)
    a1 = rng.uniform(0.1, 1.0, n + 1)
    b1 = rng.uniform(0.1, 1.0, n + 1)
    a1, b1 = a1 / a1.sum(), b1 / b1.sum()
    a = np.broadcast_to(a1[:, None, None], (n + 1,) * 3) / (n + 1) ** 2
    b = np.broadcast_to(b1[:, None, None], (n + 1,) * 3) / (n + 1) ** 2
    closed = float(np.abs(np.cumsum(a1) - np.cumsum(b1)).sum() / n)
    r = o3.solve_plain(a, b, n, p=p, **TIGHT)
    assert r["w1"] == pytest.approx(closed, rel=2e-6)
    assert r["lo"] <= closed * (1 + 1e-9) and r["hi"] >= closed * (1 - 1e-9)


def _transport_lp_l1_3d(a, b, n):
    N = (n + 1) ** 3
    idx = np.stack(np.unravel_index(np.arange(N), (n + 1,) * 3), 1)
    C = np.abs(idx[:, None, :] - idx[None, :, :]).sum(-1) / n
    A_eq = np.zeros((2 * N, N * N))
    for k in range(N):
        A_eq[k, k * N:(k + 1) * N] = 1.0
        A_eq[N + k, k::N] = 1.0
    res = linprog(C.ravel(), A_eq=A_eq, b_eq=np.concatenate([a.ravel(), b.ravel()]), bounds=(0, None),
                  method="highs")
    assert res.status == 0
    return res.fun


@pytest.mark.parametrize("n,seed", [(2, 0), (3, 1)])
def test_brute_force_transport_p1_3d(n, seed):
    a, b = w1data.random_pair_nd(n, 3, seed=30 + seed)
    exact = _transport_lp_l1_3d(a, b, n)
    r = o3.solve_plain(a, b, n, p=1, **TIGHT)
    assert r["w1"] == pytest.approx(exact, rel=5e-6)
    assert r["lo"] <= exact * (1 + 1e-9) and r["hi"] >= exact * (1 - 1e-9)


@pytest.mark.parametrize("p,shift", [(1, (1, 0, 0)), (2, (0, 1, 0)), (math.inf, (0, 0, -1))])
def test_axis_translation_3d(p, shift):
    n = 4
    rng = np.random.default_rng(13)
    bump = rng.uniform(0.2, 1.0, (2, 2, 2))
    a = np.full((n + 1,) * 3, 0.05)
    b = a.copy()
    a[1:3, 1:3, 1:3] += bump
    s = np.array(shift)
    b[1 + s[0]:3 + s[0], 1 + s[1]:3 + s[1], 1 + s[2]:3 + s[2]] += bump
    mass = bump.sum() / a.sum()
    a, b = a / a.sum(), b / b.sum()
    closed = np.abs(s).sum() / n * mass
    r = o3.solve_plain(a, b, n, p=p, **dict(TIGHT, tol=1e-6))
    assert r["w1"] == pytest.approx(closed, rel=2e-6)
    assert r["lo"] <= closed * (1 + 1e-9) and r["hi"] >= closed * (1 - 1e-9)


def test_sandwich_3d():
    n = 4
    a, b = w1data.random_pair_nd(n, 3, seed=9)
    loose = dict(TIGHT, tol=1e-6)
    w = {p: o3.solve_plain(a, b, n, p=p, **loose)["w1"] for p in P_ALL}
    assert w[math.inf] <= w[2] + 1e-8 and w[2] <= w[1] + 1e-8 and w[1] <= 3 * w[math.inf] + 1e-8
    assert w[math.inf] < w[2] < w[1]


def test_cascade_preserves_the_limit_3d():
    n = 4
    a, b = w1data.random_pair_nd(n, 3, seed=19)
    one = o3.solve_plain(a, b, n, L=1, p=2, **TIGHT)
    two = o3.solve_plain(a, b, n, L=2, p=2, **TIGHT)
    assert two["w1"] == pytest.approx(one["w1"], rel=1e-6)
    assert len(two["iters"]) == 2


def test_prox_step_projects_onto_the_constraint_3d():
    n, h = 5, 0.2
    rng = np.random.default_rng(21)
    rho = _rho3(n, 22)
    m = tuple(rng.standard_normal((n + 1,) * 3) for _ in range(3))
    w = tuple(rng.uniform(-1, 1, (n + 1,) * 3) for _ in range(3))
    for p in P_ALL:
        nm, q, qb, _ = o3.prox_step(m, w, w, rho, h, 0.5, 0.5, p)
        np.testing.assert_allclose(o3.div(nm, h), rho, atol=1e-9)   # A m+ = rho
        assert o3.pointwise_norm(q, o3.dual_exponent(p)).max() <= 1 + 1e-12


def _rho3(n, seed):
    a, b = w1data.random_pair_nd(n, 3, seed=seed)
    return o3.prepare_levels(a, b, n, 1)[0]


@pytest.mark.parametrize("n,seed", [(2, 0), (3, 1)])
def test_prox_reaches_the_transport_lp_3d(n, seed):
    a, b = w1data.random_pair_nd(n, 3, seed=30 + seed)
    exact = _transport_lp_l1_3d(a, b, n)
    r = o3.solve_prox(a, b, n, p=1, stop="kkt", tol=1e-9, check_every=10, max_iters=200000)
    assert r["w1"] == pytest.approx(exact, rel=5e-6)
    assert r["lo"] <= exact * (1 + 1e-9) and r["hi"] >= exact * (1 - 1e-9)


@pytest.mark.parametrize("p", [1, 2])
def test_prox_and_plain_share_the_limit_3d(p):
    n = 4
    a, b = w1data.random_pair_nd(n, 3, seed=23)
    plain = o3.solve_plain(a, b, n, L=2, p=p, **dict(TIGHT, tol=1e-7))
    prox = o3.solve_prox(a, b, n, L=2, p=p, stop="kkt", tol=1e-9, check_every=10, max_iters=200000)
    assert prox["w1"] == pytest.approx(plain["w1"], rel=2e-6)

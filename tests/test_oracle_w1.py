"""Pins of the W1 values the oracle converges to: the 1-D closed form,
translated densities, brute-force exact transport on tiny grids (two
independent LP formulations), p = 2 sandwich bounds and invariants."""
import math

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment, linprog

import oracle.w1_oracle as o
import w1data

TIGHT = dict(stop="kkt", tol=1e-9, check_every=10, max_iters=400000)


def _solve(p0, p1, n, p, algo=1, L=1, **kw):
    args = dict(TIGHT)
    args.update(kw)
    return o.solve(p0, p1, n, L=L, p=p, algo=algo, **args)


def _transport_lp_l1(a, b, n):
    """Exact W1 between node masses with Manhattan ground cost (HiGHS LP)."""
    N = (n + 1) ** 2
    ii, jj = np.divmod(np.arange(N), n + 1)
    C = (np.abs(ii[:, None] - ii[None, :]) + np.abs(jj[:, None] - jj[None, :])) / n
    A_eq = np.zeros((2 * N, N * N))
    for k in range(N):
        A_eq[k, k * N:(k + 1) * N] = 1.0
        A_eq[N + k, k::N] = 1.0
    res = linprog(C.ravel(), A_eq=A_eq, b_eq=np.concatenate([a.ravel(), b.ravel()]), bounds=(0, None),
                  method="highs")
    assert res.status == 0
    return res.fun


def _flux_lp_l1(a, b, n):
    """The paper's discrete problem (opt_flux_dis) for p = 1 as an LP over
    edge fluxes split into positive and negative parts."""
    h = 1.0 / n
    rho = (a - b) / h ** 2
    N = (n + 1) ** 2
    edges = []
    for i in range(n + 1):
        for j in range(n + 1):
            if i < n:
                edges.append(((i, j), (i + 1, j)))
            if j < n:
                edges.append(((i, j), (i, j + 1)))
    E = len(edges)
    A = np.zeros((N, 2 * E))
    for e, (s, t) in enumerate(edges):
        si, ti = s[0] * (n + 1) + s[1], t[0] * (n + 1) + t[1]
        # flux along the edge leaves s (+1/h at s) and enters t (-1/h at t)
        A[si, e] += 1 / h; A[ti, e] -= 1 / h
        A[si, E + e] -= 1 / h; A[ti, E + e] += 1 / h
    res = linprog(np.full(2 * E, h * h), A_eq=A, b_eq=rho.ravel(), bounds=(0, None), method="highs")
    assert res.status == 0
    return res.fun


def _assignment_l1(ia, ib, n):
    """Exact W1 for integer masses by the Hungarian method on unit atoms."""
    ai = np.repeat(np.arange(ia.size), ia.ravel())
    bi = np.repeat(np.arange(ib.size), ib.ravel())
    pa = np.stack(np.divmod(ai, n + 1), 1)
    pb = np.stack(np.divmod(bi, n + 1), 1)
    C = np.abs(pa[:, None, :] - pb[None, :, :]).sum(-1) / n
    r, c = linear_sum_assignment(C)
    return C[r, c].sum() / ia.sum()


def _grid_edges(n):
    """Forward edges of the (n+1)^2 node grid: (node, next node, axis)."""
    out = []
    for i in range(n + 1):
        for j in range(n + 1):
            if i < n:
                out.append((i * (n + 1) + j, (i + 1) * (n + 1) + j, 0))
            if j < n:
                out.append((i * (n + 1) + j, i * (n + 1) + j + 1, 1))
    return out


def _flux_lp_linf(a, b, n):
    """The discrete problem (opt_flux_dis) for p = inf as an LP: each node x
    carries the flux of its two forward edges and a bound t_x >= |m1(x)|,
    |m2(x)|; minimise sum t_x h^2 subject to div m = rho."""
    h = 1.0 / n
    N = (n + 1) ** 2
    edges = _grid_edges(n)
    E = len(edges)
    A_eq = np.zeros((N, E + N))
    A_ub = np.zeros((2 * E, E + N))
    for e, (s, t, _) in enumerate(edges):
        A_eq[s, e] += 1 / h
        A_eq[t, e] -= 1 / h
        A_ub[2 * e, e] = 1.0
        A_ub[2 * e + 1, e] = -1.0
        A_ub[2 * e, E + s] = -1.0        # the edge's flux is bounded by t of its tail node
        A_ub[2 * e + 1, E + s] = -1.0
    c = np.concatenate([np.zeros(E), np.full(N, h * h)])
    bounds = [(None, None)] * E + [(0, None)] * N
    res = linprog(c, A_ub=A_ub, b_ub=np.zeros(2 * E), A_eq=A_eq, b_eq=((a - b) / h ** 2).ravel(),
                  bounds=bounds, method="highs")
    assert res.status == 0
    return res.fun


def _potential_lp_q1(a, b, n):
    """Its dual: maximise sum psi (a - b) over node potentials whose forward
    differences satisfy |g1(x)| + |g2(x)| <= 1 at every node (q = 1), a
    missing edge counting as g = 0."""
    h = 1.0 / n
    N = (n + 1) ** 2
    G = {}
    for s, t, ax in _grid_edges(n):
        G.setdefault(s, {})[ax] = t
    rows = []
    for s, nb in G.items():
        for sg1 in (1, -1):
            for sg2 in (1, -1):
                r = np.zeros(N)
                for ax, sg in ((0, sg1), (1, sg2)):
                    if ax in nb:
                        r[nb[ax]] += sg / h
                        r[s] -= sg / h
                rows.append(r)
    res = linprog(-(a - b).ravel(), A_ub=np.array(rows), b_ub=np.ones(len(rows)), bounds=(None, None),
                  method="highs")
    assert res.status == 0
    return -res.fun


@pytest.mark.parametrize("n,seed", [(4, 3), (6, 4), (8, 5)])
def test_brute_force_lp_pinf(n, seed):
    a, b = w1data.random_pair(n, 40 + seed)
    exact = _flux_lp_linf(a, b, n)
    assert exact == pytest.approx(_potential_lp_q1(a, b, n), rel=1e-9, abs=1e-12)
    for algo in (1, 2):
        r = _solve(a, b, n, math.inf, algo=algo)
        assert r["lo"] <= exact * (1 + 1e-9) + 1e-12
        assert r["hi"] >= exact * (1 - 1e-9) - 1e-12
        assert r["w1"] == pytest.approx(exact, rel=2e-6), algo


@pytest.mark.parametrize("n,seed", [(4, 0), (6, 1), (8, 2)])
def test_brute_force_min_cost_flow_p1(n, seed):
    ia, ib = w1data.integer_mass_pair(n, 24, seed)
    a, b = ia / ia.sum(), ib / ib.sum()
    exact_tp = _transport_lp_l1(a, b, n)
    exact_flux = _flux_lp_l1(a, b, n)
    exact_hu = _assignment_l1(ia, ib, n)
    assert exact_tp == pytest.approx(exact_flux, rel=1e-9, abs=1e-12)
    assert exact_tp == pytest.approx(exact_hu, rel=1e-9, abs=1e-12)
    r = _solve(a, b, n, 1)
    assert r["lo"] <= exact_tp * (1 + 1e-9) + 1e-12
    assert r["hi"] >= exact_tp * (1 - 1e-9) - 1e-12
    assert r["w1"] == pytest.approx(exact_tp, rel=2e-6)


@pytest.mark.parametrize("n,p", [(8, 1), (16, 2), (9, 2), (8, math.inf), (9, math.inf)])
def test_stripes_closed_form(n, p):
    a, b = w1data.stripes_pair(n, seed=n)
    F0 = np.cumsum(a.sum(axis=1))
    F1 = np.cumsum(b.sum(axis=1))
    closed = float(np.sum(np.abs(F0 - F1)) / n)
    r = _solve(a, b, n, p, algo=1 if p == 1 else 2)
    assert r["w1"] == pytest.approx(closed, rel=1e-6)
    assert r["lo"] <= closed * (1 + 1e-9) <= r["hi"] * (1 + 2e-9)


@pytest.mark.parametrize("n,shift,p", [(12, (2, 3), 1), (12, (-3, 1), 1), (8, (2, 0), 2), (8, (0, -3), 2),
                                       (8, (3, 0), math.inf), (8, (0, -2), math.inf)])
def test_translation_closed_form(n, shift, p):
    # axis-aligned shifts for p = 2 and p = inf: the grid's edges carry the
    # continuous optimal flux exactly only along an axis
    a, b, mass = w1data.translated_bump_pair(n, shift, floor_mass=0.2, seed=sum(shift) + 7)
    s = np.array(shift, dtype=float) / n
    closed = np.linalg.norm(s, ord=p) * mass
    r = _solve(a, b, n, p, algo=1 if p == 1 else 2)
    assert r["w1"] == pytest.approx(closed, rel=2e-6)
    assert r["lo"] <= closed * (1 + 1e-9)
    assert r["hi"] >= closed * (1 - 1e-9)


def test_p2_sandwich_and_moment_bound():
    n = 10
    a, b = w1data.random_pair(n, 11)
    r1 = _solve(a, b, n, 1, algo=1)["w1"]
    r2 = _solve(a, b, n, 2, algo=2)
    assert r1 / math.sqrt(2) - 1e-8 <= r2["w1"] <= r1 + 1e-8
    x1, x2 = w1data.nodes(n)
    mom = np.array([np.sum((a - b) * x1), np.sum((a - b) * x2)])
    assert r2["w1"] >= np.linalg.norm(mom) - 1e-9
    assert r2["lo"] <= r2["hi"]


def test_pinf_sandwich():
    # ||x||_inf <= ||x||_2 <= ||x||_1 <= 2 ||x||_inf node by node, so the
    # discrete optima obey W_inf <= W_2 <= W_1 <= 2 W_inf
    n = 10
    a, b = w1data.random_pair(n, 12)
    w_1 = _solve(a, b, n, 1, algo=1)["w1"]
    w_2 = _solve(a, b, n, 2, algo=2)["w1"]
    w_i = _solve(a, b, n, math.inf, algo=2)["w1"]
    assert w_i <= w_2 + 1e-8 and w_2 <= w_1 + 1e-8 and w_1 <= 2 * w_i + 1e-8
    assert w_i < w_2 < w_1        # a generic pair moves mass off the axes


def test_invariants():
    n = 8
    a, b = w1data.random_pair(n, 21)
    c, _ = w1data.random_pair(n, 22)
    w_ab = _solve(a, b, n, 2, algo=2)["w1"]
    assert _solve(a, a, n, 2, algo=2)["w1"] == pytest.approx(0.0, abs=1e-14)
    assert _solve(b, a, n, 2, algo=2)["w1"] == pytest.approx(w_ab, rel=1e-7)
    assert _solve(a.T.copy(), b.T.copy(), n, 2, algo=2)["w1"] == pytest.approx(w_ab, rel=1e-7)
    # a flip of an axis maps the grid graph to itself, so the p = 1 problem is
    # invariant; for p = 2 it is not (the isotropic norm pairs each node's two
    # forward edges, and a flip turns them into backward edges)
    w1_ab = _solve(a, b, n, 1, algo=1)["w1"]
    assert _solve(a[::-1].copy(), b[::-1].copy(), n, 1, algo=1)["w1"] == pytest.approx(w1_ab, rel=1e-7)
    assert _solve(a[:, ::-1].copy(), b[:, ::-1].copy(), n, 1, algo=1)["w1"] == pytest.approx(w1_ab, rel=1e-7)
    w_ac = _solve(a, c, n, 2, algo=2)["w1"]
    w_bc = _solve(b, c, n, 2, algo=2)["w1"]
    assert w_ac <= w_ab + w_bc + 1e-9


def test_plain_and_prox_agree_and_cascade_preserves_limit():
    # Algorithms 1-4 are four different iterations with the same limit W1_h
    n = 8
    a, b = w1data.random_pair(n, 3)
    ref = _solve(a, b, n, 1, algo=1)
    for kw in (dict(algo=2), dict(algo=1, L=3), dict(algo=2, L=3)):
        r = _solve(a, b, n, 1, **kw)
        assert r["w1"] == pytest.approx(ref["w1"], rel=1e-7), kw
    assert len(r["iters"]) == 3


def test_level_costs_are_level_optima():
    # with a tight stop at every level, f(m^{K_l}) recorded at a level's end
    # is the optimum of that level's problem: the restricted density solved
    # alone on its grid (split into its positive and negative parts, which
    # the input preparation scales to unit mass, so W1 scales by that mass)
    n, L = 8, 3
    a, b = w1data.random_pair(n, 5)
    r = _solve(a, b, n, 2, algo=2, L=L)
    assert r["level_w1"][-1] == r["w1"]
    rhos = o.prepare_levels(a, b, n, L)
    for l, nl in enumerate(o.level_sides(n, L)):
        d = rhos[l] / nl ** 2
        pos, neg = np.maximum(d, 0.0), np.maximum(-d, 0.0)
        S = pos.sum()
        alone = _solve(pos, neg, nl, 2, algo=2)["w1"] * S
        assert r["level_w1"][l] == pytest.approx(alone, rel=1e-6), l


def test_certificate_brackets_the_limit():
    n = 8
    a, b = w1data.random_pair(n, 31)
    exact = _solve(a, b, n, 2, algo=2, tol=1e-11)["w1"]
    for k in (5, 50, 500):
        r = o.solve(a, b, n, L=1, p=2, algo=1, stop="kkt", tol=0.0, max_iters=k, check_every=k)
        assert r["status"] == "maxiter"
        assert r["lo"] <= exact * (1 + 1e-12) + 1e-15
        assert r["hi"] >= exact * (1 - 1e-12) - 1e-15

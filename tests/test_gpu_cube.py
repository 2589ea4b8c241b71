"""GPU parity of the d = 3 path (w1_op_plain_steps3d, w1_op_prox_steps3d,
w1_solve3d) against the d-general FP64 oracle on identical seeded inputs:
single steps of both algorithms, both cascades under both stop rules, the
certificate and exported fields, argument errors, and a 65^3 case against
the FP64 GPU path."""
import math

import numpy as np
import pytest

import oracle.w1_oracle3d as o3
import w1data
from tests.gpu_util import P_OF, dev, host, rel_err, require_gpu, tdtype

pytestmark = pytest.mark.gpu

FP32, FP64 = 1, 2


def _state(n, seed):
    rng = np.random.default_rng(seed)
    m = [rng.standard_normal((n + 1,) * 3) for _ in range(3)]
    for a in range(3):
        idx = [slice(None)] * 3
        idx[a] = -1
        m[a][tuple(idx)] = 0.0
    return m, rng.standard_normal((n + 1,) * 3) * 0.1


def _rho(n, seed):
    p0, p1 = w1data.random_pair_nd(n, 3, seed=seed)
    return o3.prepare_levels(p0, p1, n, 1)[0]


@pytest.mark.parametrize("precision", [FP64, FP32])
@pytest.mark.parametrize("n", [5, 17, 40])
@pytest.mark.parametrize("metric", [1, 2, 3])
def test_plain_steps_trajectory_3d(precision, n, metric):
    w1 = require_gpu()
    h = 1.0 / n
    rho = _rho(n, n)
    m, phi = _state(n, n + 1)
    mu, tau = o3.plain_step_sizes(h, 3)
    dt = tdtype(precision)
    g = [dev(x, dt) for x in (*m, phi, rho)]
    k = 12
    R = w1.op_plain_steps3d(n, metric, precision, k, *g, fpr=True)
    mm, pp = tuple(m), phi
    for _ in range(k):
        mm, pp, Rw = o3.pd_step(mm, pp, rho, h, mu, tau, P_OF[metric])
    tol = 1e-12 if precision == FP64 else 2e-5 * math.sqrt(k)
    for got, want in zip(g[:4], (*mm, pp)):
        assert rel_err(host(got), want) <= tol
    assert R == pytest.approx(Rw, rel=1e-9 if precision == FP64 else 1e-3)


def _oracle(p0, p1, n, L, metric, rule, tol, cap, ce):
    return o3.solve_plain(p0, p1, n, L=L, p=P_OF[metric], stop="fpr" if rule == 2 else "kkt", tol=tol,
                          alpha=-1.0, max_iters=cap, check_every=ce)


@pytest.mark.parametrize("metric", [1, 2, 3])
@pytest.mark.parametrize("rule", [2, 1])
def test_cascade_fp64_follows_the_oracle(metric, rule):
    w1 = require_gpu()
    n, L = 16, 2
    p0, p1 = w1data.pair_gauss_3d(0, n=n)
    tol = 2e-6 if rule == 2 else 1e-3
    prm = w1.params(n=n, levels=L, metric=metric, algo=w1.ALGO_PLAIN, precision=FP64, stop_rule=rule, tol=tol,
                    alpha=-1.0, max_iters=20000, check_every=10)
    res, m, psi = w1.solve3d(prm, p0, p1, fields=True)
    ref = _oracle(p0, p1, n, L, metric, rule, tol, 20000, 10)
    assert res["iters"] == ref["iters"]
    assert res["w1"] == pytest.approx(ref["w1"], rel=1e-9)
    np.testing.assert_allclose(res["level_w1"], ref["level_w1"], rtol=1e-9)
    assert res["lo"] == pytest.approx(ref["lo"], rel=1e-9)
    assert res["dual"] == pytest.approx(-o3.inner_h(ref["phi"], ref["rho"], 1.0 / n), rel=1e-9, abs=1e-12)
    assert res["hi"] == pytest.approx(ref["hi"], rel=1e-9)
    for a in range(3):
        assert rel_err(m[a], ref["m"][a]) <= 1e-9
    assert rel_err(psi, -(ref["phi"] - ref["phi"].mean())) <= 1e-9
    kkt, _, _ = o3.kkt_plain(tuple(m), -psi, ref["rho"], 1.0 / n, P_OF[metric])
    assert res["kkt"] == pytest.approx(kkt, rel=1e-6)


@pytest.mark.parametrize("metric", [1, 2, 3])
def test_cascade_fp32_at_equal_iteration_counts(metric):
    """FP32 decides the stop tests on rounded iterates; with the KKT rule at a
    tolerance no level reaches, both sides run every level to the same cap
    and the level values are compared there."""
    w1 = require_gpu()
    n, L = 24, 3
    p0, p1 = w1data.pair_gauss_3d(1, n=n)
    prm = w1.params(n=n, levels=L, metric=metric, algo=w1.ALGO_PLAIN, precision=FP32, stop_rule=w1.STOP_KKT,
                    tol=1e-300, alpha=0.0, max_iters=300, check_every=10)
    res = w1.solve3d(prm, p0, p1)
    ref = _oracle(p0, p1, n, L, metric, 1, 1e-300, 300, 10)
    assert res["iters"] == ref["iters"] == [300] * L
    np.testing.assert_allclose(res["level_w1"], ref["level_w1"], rtol=2e-5)
    assert res["lo"] == pytest.approx(ref["lo"], rel=1e-3)


def test_errors_3d():
    w1 = require_gpu()
    n = 8
    p0, p1 = w1data.random_pair_nd(n, 3, seed=2)
    base = dict(n=n, levels=2, metric=2, algo=w1.ALGO_PLAIN, precision=FP32, stop_rule=w1.STOP_FPR, tol=1e-6,
                max_iters=100, check_every=10)
    for bad in (dict(algo=7), dict(tol=0.0), dict(levels=4), dict(metric=4), dict(step_scale=1.5)):
        prm = w1.params(**dict(base, **bad))
        with pytest.raises(w1.W1Error):
            w1.solve3d(prm, p0, p1)
    neg = p0.copy()
    neg[0, 0, 0] = -1e-3
    with pytest.raises(w1.W1Error):
        w1.solve3d(w1.params(**base), neg, p1)
    with pytest.raises(w1.W1Error):
        w1.solve3d(w1.params(**base), p0, p1 * 1.01)


@pytest.mark.parametrize("precision", [FP64, FP32])
@pytest.mark.parametrize("n", [5, 17, 32])
@pytest.mark.parametrize("metric", [1, 2, 3])
def test_prox_steps_trajectory_3d(precision, n, metric):
    w1 = require_gpu()
    h = 1.0 / n
    rho = _rho(n, 40 + n)
    m, _ = _state(n, 41)
    rng = np.random.default_rng(42)
    w = [rng.uniform(-1, 1, (n + 1,) * 3) for _ in range(3)]
    for a in range(3):
        idx = [slice(None)] * 3
        idx[a] = -1
        w[a][tuple(idx)] = 0.0
    dt = tdtype(precision)
    g = [dev(x, dt) for x in (*m, *w, *w, rho)]
    k = 8
    G = w1.op_prox_steps3d(n, metric, precision, k, *g, fpr=True)
    st = (tuple(m), tuple(w), tuple(x.copy() for x in w))
    for _ in range(k):
        mm, ww, wb, Gw = o3.prox_step(*st, rho, h, 0.5, 0.5, P_OF[metric])
        st = (mm, ww, wb)
    tol = 1e-10 if precision == FP64 else 1e-4 * math.sqrt(k)
    for got, want in zip(g[:9], (*st[0], *st[1], *st[2])):
        assert rel_err(host(got), want) <= tol
    assert G == pytest.approx(Gw, rel=1e-8 if precision == FP64 else 1e-2, abs=1e-12)


@pytest.mark.parametrize("metric", [1, 2, 3])
@pytest.mark.parametrize("rule", [2, 1])
def test_prox_cascade_fp64_follows_the_oracle(metric, rule):
    w1 = require_gpu()
    n, L = 16, 2
    p0, p1 = w1data.pair_gauss_3d(0, n=n)
    tol = 1e-5 if rule == 2 else 1e-3
    prm = w1.params(n=n, levels=L, metric=metric, algo=w1.ALGO_PROX, precision=FP64, stop_rule=rule, tol=tol,
                    alpha=-1.0, max_iters=20000, check_every=10)
    res, m, psi = w1.solve3d(prm, p0, p1, fields=True)
    ref = o3.solve_prox(p0, p1, n, L=L, p=P_OF[metric], stop="fpr" if rule == 2 else "kkt", tol=tol, alpha=-1.0,
                        max_iters=20000, check_every=10)
    assert res["iters"] == ref["iters"]
    assert res["w1"] == pytest.approx(ref["w1"], rel=1e-9)
    np.testing.assert_allclose(res["level_w1"], ref["level_w1"], rtol=1e-9)
    for k in ("lo", "hi", "dual"):
        assert res[k] == pytest.approx(ref[k], rel=1e-8), k
    for a in range(3):
        assert rel_err(m[a], ref["m"][a]) <= 1e-9
    assert rel_err(psi, ref["psi"]) <= 1e-8


@pytest.mark.parametrize("metric", [1, 2, 3])
def test_prox_cascade_fp32_at_equal_iteration_counts(metric):
    w1 = require_gpu()
    n, L = 24, 3
    p0, p1 = w1data.pair_gauss_3d(3, n=n)
    prm = w1.params(n=n, levels=L, metric=metric, algo=w1.ALGO_PROX, precision=FP32, stop_rule=w1.STOP_KKT,
                    tol=1e-300, alpha=0.0, max_iters=60, check_every=10)
    res = w1.solve3d(prm, p0, p1)
    ref = o3.solve_prox(p0, p1, n, L=L, p=P_OF[metric], stop="kkt", tol=1e-300, alpha=0.0, max_iters=60,
                        check_every=10)
    assert res["iters"] == ref["iters"] == [60] * L
    np.testing.assert_allclose(res["level_w1"], ref["level_w1"], rtol=1e-4)
    assert res["lo"] == pytest.approx(ref["lo"], rel=2e-3)
    assert res["hi"] == pytest.approx(ref["hi"], rel=1e-4)


@pytest.mark.parametrize("n,L", [(2, 1), (3, 1), (6, 2)])
@pytest.mark.parametrize("algo", [1, 2])
def test_small_and_odd_grids_3d(n, L, algo):
    """Edge sizes: the smallest grid, an odd side, a 4^3 coarse level; FP64
    takes the oracle's decisions; FP32 repeats itself bit for bit."""
    w1 = require_gpu()
    p0, p1 = w1data.random_pair_nd(n, 3, seed=50 + n)
    tol = 1e-6 if algo == 1 else 1e-5
    prm = w1.params(n=n, levels=L, metric=2, algo=algo, precision=FP64, stop_rule=w1.STOP_FPR, tol=tol,
                    alpha=-1.0, max_iters=20000, check_every=10)
    res = w1.solve3d(prm, p0, p1)
    solve = o3.solve_plain if algo == 1 else o3.solve_prox
    ref = solve(p0, p1, n, L=L, p=2, stop="fpr", tol=tol, alpha=-1.0, max_iters=20000, check_every=10)
    assert res["iters"] == ref["iters"]
    assert res["w1"] == pytest.approx(ref["w1"], rel=1e-9)
    assert res["lo"] == pytest.approx(ref["lo"], rel=1e-8) and res["hi"] == pytest.approx(ref["hi"], rel=1e-8)
    prm.precision = FP32
    a, b = w1.solve3d(prm, p0, p1), w1.solve3d(prm, p0, p1)
    assert a["iters"] == b["iters"] and a["w1"] == b["w1"] and a["lo"] == b["lo"]


@pytest.mark.parametrize("algo", [1, 2])
def test_batch_equals_single_3d(algo):
    """w1_solve3d_batch on concurrent streams returns each pair's w1_solve3d
    result bit for bit (host and device masses); a bad pair fails the call."""
    w1 = require_gpu()
    import torch
    n, L = 16, 2
    pairs = [w1data.pair_gauss_3d(i, n=n) for i in range(6)]
    prm = w1.params(n=n, levels=L, metric=2, algo=algo, precision=FP32, stop_rule=w1.STOP_FPR,
                    tol=2e-6 if algo == 1 else 1e-5, alpha=-1.0, max_iters=20000, check_every=10)
    batch = w1.solve3d_batch(prm, pairs, workers=3)
    dev_pairs = [(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for a, b in pairs]
    batch_dev = w1.solve3d_batch(prm, dev_pairs, workers=4)
    for (a, b), r, rd in zip(pairs, batch, batch_dev):
        one = w1.solve3d(prm, a, b)
        for k in ("iters", "w1", "lo", "hi", "dual"):
            assert r[k] == one[k] and rd[k] == one[k], k
    bad = list(pairs)
    bad[3] = (pairs[3][0], pairs[3][1] * 1.01)
    with pytest.raises(w1.W1Error):
        w1.solve3d_batch(prm, bad, workers=2)


def test_cube65_fp32_against_fp64():
    """65^3 nodes, 3 levels (17^3, 33^3, 65^3), paper-style FPR rule: the
    FP32 result within 1e-4 of the FP64 GPU result, the lower bound below
    both, masses on the device."""
    w1 = require_gpu()
    import torch
    n, L = 64, 3
    p0, p1 = w1data.pair_gauss_3d(2, n=n)
    d0, d1 = torch.from_numpy(p0).cuda(), torch.from_numpy(p1).cuda()
    for algo, tol in ((w1.ALGO_PLAIN, 1e-7), (w1.ALGO_PROX, 1e-5)):
        out = {}
        for prec in (FP32, FP64):
            prm = w1.params(n=n, levels=L, metric=2, algo=algo, precision=prec, stop_rule=w1.STOP_FPR,
                            tol=tol, alpha=-1.0, max_iters=20000, check_every=10)
            out[prec] = w1.solve3d(prm, d0, d1)
        a, b = out[FP32], out[FP64]
        assert a["status"] in (0, 1) and b["status"] in (0, 1)
        assert a["w1"] == pytest.approx(b["w1"], rel=1e-4), algo
        for r in (a, b):
            assert r["lo"] <= r["hi"] * (1 + 1e-6) and all(x > 0 for x in r["iters"])

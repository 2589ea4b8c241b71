"""Edge cases of the method through w1_solve / w1_submit: identical
densities (rho = 0, the KKT normalisations divide by ~0), an iteration cap
of one, the 1-D closed form on stripes and exact grid-aligned translations
at full size (Sec. 2: W1 of densities varying along one axis is the sum of
|F0 - F1| h; a translation by whole grid steps costs ||s||_p times the moved
mass), and the admission queue's limit."""
import math

import numpy as np
import pytest

import oracle.w1_oracle as o
import w1data
from tests.gpu_util import P_OF, require_gpu

pytestmark = pytest.mark.gpu

FP32, FP64 = 1, 2


def _levels(n):
    return int(round(math.log2(n // 32))) + 1


@pytest.mark.parametrize("rule", [1, 2])
@pytest.mark.parametrize("algo", [1, 2])
@pytest.mark.parametrize("precision", [FP64, FP32])
def test_identical_densities(rule, algo, precision):
    """W1(rho, rho) = 0: rho is identically zero, every iterate stays zero,
    and the stop test (FPR or KKT, whose normalisations see P = D = 0)
    fires at the first check of every level with a finite, zero result."""
    w1 = require_gpu()
    n, L = 128, 3
    p0, _ = w1data.pair_gauss3(5, n=n)
    prm = w1.params(n=n, levels=L, metric=2, algo=algo, precision=precision, stop_rule=rule,
                    tol=1e-6 if rule == 1 else 0.0, max_iters=20000, check_every=10)
    with w1.Solver(prm) as s:
        res = s.solve([(p0, p0.copy())])[0]
        m1, m2, psi = s.fields(0)
    assert res["status"] == w1.SOLVE_OK
    assert res["iters"] == [10] * L
    assert res["w1"] == 0.0 and res["dual"] == 0.0
    assert res["lo"] <= 0.0 <= res["hi"] and res["hi"] == 0.0
    assert np.isfinite(res["kkt"]) and res["kkt"] == 0.0
    assert not np.any(m1) and not np.any(m2) and not np.any(psi)


@pytest.mark.parametrize("algo", [1, 2])
@pytest.mark.parametrize("precision", [FP64, FP32])
def test_cap_of_one_iteration(algo, precision):
    """A cap of one iteration per level: every level runs exactly one
    step, the solve ends as MAXITER with a valid certificate, and in FP64
    W1 and the bracket equal the oracle's after the same single steps."""
    w1 = require_gpu()
    n, L = 128, 3
    p0, p1 = w1data.pair_gauss3(6, n=n)
    prm = w1.params(n=n, levels=L, metric=2, algo=algo, precision=precision, stop_rule=w1.STOP_FPR,
                    tol=1e-300, max_iters=1, check_every=1)
    with w1.Solver(prm) as s:
        res = s.solve([(p0, p1)])[0]
    assert res["status"] == w1.SOLVE_MAXITER
    assert res["iters"] == [1] * L
    assert np.isfinite(res["lo"]) and np.isfinite(res["hi"]) and res["lo"] <= res["hi"]
    ref = o.solve(p0, p1, n, L=L, p=2, algo=algo, stop="fpr", eps_L=1e-300, alpha=-1.0, max_iters=1,
                  check_every=1, return_fields=False)
    assert ref["iters"] == [1] * L
    rt = 1e-10 if precision == FP64 else 1e-4
    assert res["w1"] == pytest.approx(ref["w1"], rel=rt)
    assert res["lo"] == pytest.approx(ref["lo"], rel=rt, abs=1e-12)
    assert res["hi"] == pytest.approx(ref["hi"], rel=rt)


def _closed_form_case(w1, p0, p1, n, metric, closed, precisions=(2, 1)):
    """Algorithm 4 with the paper's rule: the closed form lies inside the
    certified brackets of the FP64 and FP32 GPU runs and of the oracle; the
    FP64 run takes the oracle's stops (same iterations, W1 to 1e-10); the
    FP32 run, whose stop iterations FP32 arithmetic decides, matches the
    oracle run to its own per-level iteration counts to 1e-4."""
    L = _levels(n)
    eps = o.paper_stop_tolerance(2, n, True)
    kw = dict(p=P_OF[metric], algo=2, stop="fpr", alpha=-1.0, check_every=10, return_fields=False)
    ref = o.solve(p0, p1, n, L=L, eps_L=eps, max_iters=20000, **kw)
    assert ref["lo"] * (1 - 1e-9) <= closed <= ref["hi"] * (1 + 1e-9)
    for precision in precisions:
        prm = w1.params(n=n, levels=L, metric=metric, algo=w1.ALGO_PROX, precision=precision,
                        stop_rule=w1.STOP_FPR, tol=eps, max_iters=20000, check_every=10)
        with w1.Solver(prm) as s:
            res = s.solve([(p0, p1)])[0]
        assert res["status"] == w1.SOLVE_OK
        assert res["lo"] * (1 - 1e-6) <= closed <= res["hi"] * (1 + 1e-6), (res["lo"], closed, res["hi"])
        if precision == FP64:
            assert res["iters"] == ref["iters"]
            assert res["w1"] == pytest.approx(ref["w1"], rel=1e-10)
        else:
            same = o.solve(p0, p1, n, L=L, eps_L=1e-300, max_iters=res["iters"], **kw)
            assert res["w1"] == pytest.approx(same["w1"], rel=1e-4)


@pytest.mark.parametrize("n", [256, 512])
@pytest.mark.parametrize("metric", [1, 2])
def test_stripes_full_size(n, metric):
    """Densities constant along x2: W1_h = sum_i |F0_i - F1_i| h for any
    ground metric (the 1-D closed form).  Under l_1 only the FP64 path is
    held to the oracle: the exact flux has no x2 component, the FP32
    iterate carries transverse rounding noise (mean |m2| ~ 2e-6 at 513^2),
    and l_1 prices it linearly, which on this small W1 (~0.0115) is ~1e-4
    relative (a CPU emulation of the FP32 iteration: 2.0e-4; measured on
    the GPU: 1.0e-4); l_2 prices it quadratically."""
    w1 = require_gpu()
    p0, p1 = w1data.stripes_pair(n, seed=n + metric)
    F0, F1 = np.cumsum(p0.sum(axis=1)), np.cumsum(p1.sum(axis=1))
    closed = float(np.sum(np.abs(F0 - F1)) / n)
    _closed_form_case(w1, p0, p1, n, metric, closed, (FP64,) if metric == 1 else (FP64, FP32))


@pytest.mark.parametrize("n", [256, 512])
@pytest.mark.parametrize("metric,shift", [(1, (7, -12)), (2, (0, 19))])
def test_translation_full_size(n, metric, shift):
    """A bump moved by whole grid steps, plus a shared floor: W1_h =
    ||s||_p times the moved mass (any shift for l_1, axis-aligned for l_2)."""
    w1 = require_gpu()
    p0, p1, mass = w1data.translated_bump_pair(n, shift, floor_mass=0.2, seed=n + sum(shift))
    closed = float(np.linalg.norm(np.array(shift, dtype=float) / n, ord=P_OF[metric]) * mass)
    _closed_form_case(w1, p0, p1, n, metric, closed)


def test_queue_limit_returns_ebusy():
    """w1_serve_config bounds the requests waiting for admission: with one
    slot busy and one request queued, a third submission is refused with
    W1_EBUSY; the admitted and queued requests still finish."""
    w1 = require_gpu()
    n = 256
    slow = w1.params(n=n, levels=1, metric=2, algo=w1.ALGO_PLAIN, precision=FP64, stop_rule=w1.STOP_FPR,
                     tol=1e-300, max_iters=20000, check_every=10)
    quick = w1.params(n=32, levels=1, metric=2, algo=w1.ALGO_PROX, precision=FP32, stop_rule=w1.STOP_FPR,
                      tol=0.0, max_iters=200, check_every=10)
    a, b = w1data.pair_gauss3(9, n=n)
    c, d = w1data.pair_gauss3(10, n=32)
    with w1.Solver(slow, capacity=1, hbm_budget=w1.bytes_per_solve(slow)) as srv:
        srv.serve_config(1)
        t1 = srv.submit(a, b, slow)
        while srv.stats()["admitted"] < 1:   # the first request holds the slot
            pass
        t2 = srv.submit(c, d, quick)   # waits: the only slot and the budget are taken
        with pytest.raises(w1.W1Error) as e:
            srv.submit(c, d, quick)
        assert e.value.status == w1.W1_EBUSY
        srv.drain()
        for t in (t1, t2):
            r = None
            while r is None:
                r = srv.poll(t)
            assert r[0]["status"] in (w1.SOLVE_OK, w1.SOLVE_MAXITER)
        st = srv.stats()
        assert st["finished"] == 2 and st["running"] == 0 and st["bytes"] == 0

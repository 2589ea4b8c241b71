"""End-to-end GPU parity of the multilevel solver (Algorithms 3 and 4)
through w1_solve / w1_submit against the FP64 oracle: W1 within 1e-4
relative, the normalised KKT of both sides' fields within 1e-5, the oracle's
W1 inside the GPU certificate; batch composition and served mode."""
import numpy as np
import pytest

import oracle.w1_oracle as o
import w1data
from tests.gpu_util import P_OF, require_gpu

pytestmark = pytest.mark.gpu

FP32, FP64 = 1, 2


def _oracle(p0, p1, n, L, metric, algo, rule, tol, cap, ce):
    return o.solve(p0, p1, n, L=L, p=P_OF[metric], algo=algo, stop="fpr" if rule == 2 else "kkt",
                   tol=tol, eps_L=tol if rule == 2 and tol > 0 else None, max_iters=cap, check_every=ce,
                   alpha=-1.0)


def _check_parity(w1, res, fields, ref, n, metric, rho, precision=FP64):
    assert res["status"] in (0, 1)
    assert res["w1"] == pytest.approx(ref["w1"], rel=1e-4)
    m1, m2, psi = fields
    ev_gpu = o.evaluate(m1, m2, psi, rho, 1.0 / n, P_OF[metric])
    ev_ref = o.evaluate(ref["m1"], ref["m2"], ref["psi"], rho, 1.0 / n, P_OF[metric])
    assert abs(ev_gpu["kkt"] - ev_ref["kkt"]) <= 1e-5
    # W1_h lies in both certified brackets, so they overlap; the oracle's own
    # f(m^K) need not lie in the GPU bracket when m^K is not yet feasible
    assert max(res["lo"], ref["lo"]) <= min(res["hi"], ref["hi"]) * (1 + 1e-6)
    # the bounds themselves: FP64 agrees to 1e-4; in FP32 the lower bound's
    # max Lipschitz ratio is a max over differences of rounded potentials
    ct = 1e-4 if precision == FP64 else 1e-3
    assert res["lo"] == pytest.approx(ref["lo"], rel=ct)
    assert res["hi"] == pytest.approx(ref["hi"], rel=ct)
    # the library's own FP64 evaluator agrees with the oracle's on its fields
    assert res["w1"] == pytest.approx(ev_gpu["P"], rel=1e-9)
    assert res["hi"] == pytest.approx(ev_gpu["hi"], rel=1e-7)


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_config1_plain_fp64_kkt(precision):
    """64x64, three isotropic Gaussians + floor, L1, plain PDHG, 2 levels,
    KKT 1e-6 or 20k iterations per level."""
    w1 = require_gpu()
    n, L, metric = 64, 2, 1
    p0, p1 = w1data.pair_gauss3(0)
    prm = w1.params(n=n, levels=L, metric=metric, algo=w1.ALGO_PLAIN, precision=precision,
                    stop_rule=w1.STOP_KKT, tol=1e-6, max_iters=20000, check_every=10)
    with w1.Solver(prm) as s:
        res = s.solve([(p0, p1)])[0]
        fields = s.fields(0)
    ref = _oracle(p0, p1, n, L, metric, 1, 1, 1e-6, 20000, 10)
    if precision == FP64:
        assert res["iters"] == ref["iters"]
    rho = o.prepare_levels(p0, p1, n, L)[-1]
    _check_parity(w1, res, fields, ref, n, metric, rho, precision)


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_prox_kkt_rule_resident_levels(precision):
    """Algorithm 4 with the KKT stop rule (tol 1e-4, alpha = -1), 128-grid,
    3 levels: in FP32 the 33^2 and 65^2 levels run in the LDS-resident
    kernel, whose KKT test solves a second Poisson problem for the
    potential."""
    w1 = require_gpu()
    n, L, metric = 128, 3, 2
    p0, p1 = w1data.pair_gauss3(7, n=n)
    prm = w1.params(n=n, levels=L, metric=metric, algo=w1.ALGO_PROX, precision=precision,
                    stop_rule=w1.STOP_KKT, tol=1e-4, max_iters=20000, check_every=10)
    with w1.Solver(prm) as s:
        res = s.solve([(p0, p1)])[0]
        fields = s.fields(0)
    ref = _oracle(p0, p1, n, L, metric, 2, 1, 1e-4, 20000, 10)
    rho = o.prepare_levels(p0, p1, n, L)[-1]
    if precision == FP64:
        assert res["iters"] == ref["iters"]
        _check_parity(w1, res, fields, ref, n, metric, rho, precision)
        return
    # FP32: the primal term is the norm of the minimum-norm flux correction,
    # so the rounding noise of the FP32 Poisson solves enters it once
    # through a gradient (not through the Laplacian of A m - rho): every
    # level stops below the cap, and the FP64 evaluation of the returned
    # fields meets the oracle's to 1e-5
    assert all(k < 20000 for k in res["iters"]), res["iters"]
    _check_parity(w1, res, fields, ref, n, metric, rho, precision)


@pytest.mark.parametrize("algo", [1, 2])
@pytest.mark.parametrize("precision", [FP64, FP32])
@pytest.mark.parametrize("metric", [1, 2, 3])
def test_multilevel_paper_rule(algo, precision, metric):
    """Algorithm 3 / 4 with the paper's tolerance rule eq. (stop_tol),
    alpha = -1, on a 128-grid, 3 levels (tiled plain levels beyond 65)."""
    w1 = require_gpu()
    n, L = 128, 3
    p0, p1 = w1data.pair_gauss3(3, n=n)
    eps = o.paper_stop_tolerance(algo, n, True)
    prm = w1.params(n=n, levels=L, metric=metric, algo=algo, precision=precision, stop_rule=w1.STOP_FPR,
                    tol=eps, max_iters=20000, check_every=10)
    with w1.Solver(prm) as s:
        res = s.solve([(p0, p1)])[0]
        fields = s.fields(0)
    ref = _oracle(p0, p1, n, L, metric, algo, 2, eps, 20000, 10)
    rho = o.prepare_levels(p0, p1, n, L)[-1]
    if precision == FP64:
        assert res["iters"] == ref["iters"]
    _check_parity(w1, res, fields, ref, n, metric, rho, precision)


@pytest.mark.parametrize("algo", [1, 2])
@pytest.mark.parametrize("precision", [FP64, FP32])
def test_level_costs(algo, precision):
    """f(m^{K_l}) at every level's end (W1_FLAG_LEVEL_COST) against the
    oracle's, on a 128-grid, 3 levels (resident and batched levels); the
    flag changes no iterate."""
    w1 = require_gpu()
    n, L, metric = 128, 3, 1
    p0, p1 = w1data.pair_gauss3(5, n=n)
    eps = o.paper_stop_tolerance(algo, n, True)
    out = {}
    for flags in (0, w1.FLAG_LEVEL_COST):
        prm = w1.params(n=n, levels=L, metric=metric, algo=algo, precision=precision, stop_rule=w1.STOP_FPR,
                        tol=eps, max_iters=20000, check_every=10, flags=flags)
        with w1.Solver(prm) as s:
            out[flags] = s.solve([(p0, p1)])[0]
    plain, costs = out[0], out[w1.FLAG_LEVEL_COST]
    assert plain["iters"] == costs["iters"] and plain["w1"] == costs["w1"]
    assert all(np.isnan(x) for x in plain["level_w1"][:-1]) and plain["level_w1"][-1] == plain["w1"]
    assert costs["level_w1"][-1] == costs["w1"]
    assert all(b >= a for a, b in zip(costs["level_seconds"], costs["level_seconds"][1:]))
    if precision == FP64:
        ref = _oracle(p0, p1, n, L, metric, algo, 2, eps, 20000, 10)
        assert costs["iters"] == ref["iters"]
        np.testing.assert_allclose(costs["level_w1"], ref["level_w1"], rtol=1e-9)
        return
    # FP32 decides the paper's stop test on its own rounded iterates and may
    # stop a still-moving level some iterations away from the oracle; with
    # the KKT rule at tolerance 0 every level runs to the same cap on both
    # sides, and the level values are compared at equal iteration counts
    prm = w1.params(n=n, levels=L, metric=metric, algo=algo, precision=FP32, stop_rule=w1.STOP_KKT,
                    tol=0.0, max_iters=400, check_every=10, flags=w1.FLAG_LEVEL_COST)
    with w1.Solver(prm) as s:
        capped = s.solve([(p0, p1)])[0]
    ref = _oracle(p0, p1, n, L, metric, algo, 1, 0.0, 400, 10)
    assert capped["iters"] == ref["iters"] == [400] * L
    np.testing.assert_allclose(capped["level_w1"], ref["level_w1"], rtol=2e-5)


@pytest.mark.parametrize("algo", [1, 2])
def test_practical_steps_follow_the_oracle(algo):
    """step_scale 1 (the footnoted practical steps of Sec. 3.1) through the
    whole cascade: FP64 takes the oracle's stop decisions, W1 and KKT at the
    usual bar."""
    w1 = require_gpu()
    n, L, metric = 128, 3, 2
    p0, p1 = w1data.pair_gauss3(3, n=n)
    eps = o.paper_stop_tolerance(algo, n, True)
    prm = w1.params(n=n, levels=L, metric=metric, algo=algo, precision=FP64, stop_rule=w1.STOP_FPR,
                    tol=eps, max_iters=20000, check_every=10, step_scale=1.0)
    with w1.Solver(prm) as s:
        res = s.solve([(p0, p1)])[0]
        fields = s.fields(0)
    ref = o.solve(p0, p1, n, L=L, p=2, algo=algo, stop="fpr", eps_L=eps, tol=eps, max_iters=20000,
                  check_every=10, alpha=-1.0, step_scale=1.0)
    assert res["iters"] == ref["iters"]
    rho = o.prepare_levels(p0, p1, n, L)[-1]
    _check_parity(w1, res, fields, ref, n, metric, rho, FP64)


def test_batch_equals_alone_bitwise():
    w1 = require_gpu()
    n, L = 64, 2
    pairs = [w1data.pair_gauss3(i) for i in range(5)]
    prm = w1.params(n=n, levels=L, metric=2, algo=w1.ALGO_PLAIN, precision=FP32, stop_rule=w1.STOP_FPR,
                    tol=0.0, max_iters=4000, check_every=10, flags=w1.FLAG_NO_RESIDENT)
    with w1.Solver(prm, capacity=5) as s:
        batch = s.solve(pairs)
        fb = [s.fields(i) for i in range(5)]
    for i, pr in enumerate(pairs):
        with w1.Solver(prm) as s:
            alone = s.solve([pr])[0]
            fa = s.fields(0)
        assert alone["iters"] == batch[i]["iters"]
        assert alone["w1"] == batch[i]["w1"]
        for a, b in zip(fa, fb[i]):
            np.testing.assert_array_equal(a, b)


def test_rejected_pair_does_not_disturb_batch():
    w1 = require_gpu()
    n = 32
    good = w1data.pair_gauss3(0, n=n)
    bad = (good[0], good[1] * 1.5)
    prm = w1.params(n=n, levels=2, metric=1, algo=w1.ALGO_PROX, precision=FP32)
    with w1.Solver(prm, capacity=3) as s:
        out = s.solve([good, bad, good])
    assert out[1]["status"] == w1.SOLVE_REJECTED
    assert out[0]["w1"] == out[2]["w1"]
    assert out[0]["status"] in (0, 1)


def test_served_mix_equals_alone():
    """Continuous batching: requests of different sizes, metrics and
    algorithms arrive while others run; each served result equals the same
    request solved alone."""
    w1 = require_gpu()
    reqs = []
    for i in range(10):
        n = (32, 64, 128)[i % 3]
        p0, p1 = w1data.pair_gauss3(100 + i, n=n)
        algo = 2 if i % 2 == 0 else 1
        L = {32: 1, 64: 2, 128: 3}[n]
        prm = w1.params(n=n, levels=L, metric=1 + (i // 2) % 3, algo=algo, precision=FP32, stop_rule=w1.STOP_FPR,
                        tol=0.0, max_iters=3000, check_every=10, flags=w1.FLAG_NO_RESIDENT)
        reqs.append((prm, p0, p1))
    base = reqs[0][0]
    with w1.Solver(base, capacity=4) as srv:
        tickets = []
        for prm, p0, p1 in reqs:
            tickets.append(srv.submit(p0, p1, prm))
        srv.drain()
        served = []
        for t, (prm, _, _) in zip(tickets, reqs):
            r = None
            while r is None:
                r = srv.poll(t, n=prm.n, fields=True)
            served.append(r)
        st = srv.stats()
        assert st["finished"] == len(reqs) and st["running"] == 0
    for (prm, p0, p1), (res, fields) in zip(reqs, served):
        with w1.Solver(prm) as s:
            alone = s.solve([(p0, p1)])[0]
        assert res["iters"] == alone["iters"]
        assert res["w1"] == pytest.approx(alone["w1"], rel=1e-6)


def test_served_resident_beside_batched():
    """Served mix where LDS-resident levels (sides 33 and 65, on the side
    stream) run while other requests' batched levels (side 129 and up) run
    on the batch's stream, under an HBM budget that admits only part of
    the queue at once: each result equals the request solved alone."""
    w1 = require_gpu()
    reqs = []
    for i in range(8):
        n = (64, 256)[i % 2]
        L = {64: 2, 256: 3}[n]
        p0, p1 = w1data.pair_gauss3(200 + i, n=n)
        algo = 2 if i % 4 < 2 else 1
        prm = w1.params(n=n, levels=L, metric=2, algo=algo, precision=FP32, stop_rule=w1.STOP_FPR,
                        tol=0.0, max_iters=4000, check_every=10)
        reqs.append((prm, p0, p1))
    need = max(w1.bytes_per_solve(prm) for prm, _, _ in reqs)
    small = min(w1.bytes_per_solve(prm) for prm, _, _ in reqs)
    assert 8 * small <= 3 * need   # the plan (capacity x base request) fits the budget
    with w1.Solver(reqs[0][0], capacity=8, hbm_budget=3 * need) as srv:
        tickets = [srv.submit(p0, p1, prm) for prm, p0, p1 in reqs]
        srv.drain()
        served = []
        for t, (prm, _, _) in zip(tickets, reqs):
            r = None
            while r is None:
                r = srv.poll(t)
            served.append(r[0])
        st = srv.stats()
        assert st["finished"] == len(reqs) and st["running"] == 0
        assert st["peak_bytes"] <= 3 * need
    for (prm, p0, p1), res in zip(reqs, served):
        with w1.Solver(prm) as s:
            alone = s.solve([(p0, p1)])[0]
        assert res["iters"] == alone["iters"]
        assert res["w1"] == pytest.approx(alone["w1"], rel=1e-6)


def test_no_certificate_flag():
    """Without the certificate the solve runs the same iterations and gives
    the same dual (and, for Algorithm 1, the same W1); only lo, hi and kkt
    are left as NaN.  With it, Algorithm 2's W1 is the cost of the FP64
    re-projection of m^K onto {A m = rho}, within the FP32 projection noise
    of the unprojected cost."""
    w1 = require_gpu()
    pairs = [w1data.pair_gauss3(60 + i, n=64) for i in range(2)]
    out = []
    for flags in (0, w1.FLAG_NO_CERT):
        for algo in (w1.ALGO_PLAIN, w1.ALGO_PROX):
            prm = w1.params(n=64, levels=2, metric=2, algo=algo, precision=FP32, stop_rule=w1.STOP_FPR,
                            tol=0.0, max_iters=2000, check_every=10, flags=flags)
            with w1.Solver(prm, capacity=2) as s:
                out.append(s.solve(pairs))
    for k, (a, b) in enumerate(zip(out[0] + out[1], out[2] + out[3])):
        assert a["iters"] == b["iters"] and a["dual"] == b["dual"]
        if k < 2:   # Algorithm 1
            assert a["w1"] == b["w1"]
        else:
            assert a["w1"] == pytest.approx(b["w1"], rel=1e-5)
        assert np.isfinite(a["lo"]) and np.isfinite(a["hi"]) and np.isfinite(a["kkt"])
        assert np.isnan(b["lo"]) and np.isnan(b["hi"]) and np.isnan(b["kkt"])


def test_autotuner_exploration_keeps_results():
    """The launch-shape autotuner times candidate shapes on live blocks;
    results while it explores and after it has settled are identical."""
    w1 = require_gpu()
    w1.tuner_reset()
    pairs = [w1data.pair_gauss3(80 + i, n=128) for i in range(4)]
    prm = w1.params(n=128, levels=2, metric=2, algo=w1.ALGO_PLAIN, precision=FP32, stop_rule=w1.STOP_FPR,
                    tol=0.0, max_iters=3000, check_every=10, flags=w1.FLAG_NO_RESIDENT)
    runs = []
    with w1.Solver(prm, capacity=4) as s:
        for _ in range(3):
            runs.append(s.solve(pairs))
    table = w1.tuner_table()
    assert table and all(len(e["arms"]) >= 2 for e in table)
    assert any(a["blocks"] > 0 for e in table for a in e["arms"])
    for other in runs[1:]:
        for a, b in zip(runs[0], other):
            assert a["iters"] == b["iters"] and a["w1"] == b["w1"]


_FAIL_CHILD = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
import paper_1810_00118_amd as w1, w1data
prm = w1.params(n=64, levels=2, metric=2, algo=w1.ALGO_PROX, precision=w1.FP32, stop_rule=w1.STOP_FPR,
                tol=0.0, max_iters=4000, check_every=10, flags=w1.FLAG_NO_RESIDENT)
srv = w1.Solver(prm, capacity=4)
tickets = [srv.submit(*w1data.pair_gauss3(300 + i, n=64), prm) for i in range(4)]
try:
    srv.drain()
    err = 0
except w1.W1Error as e:
    err = e.status
out = []
for t in tickets:
    r = None
    while r is None:
        r = srv.poll(t)
    out.append(r[0]["status"])
st = srv.stats()
srv.close()
print(json.dumps({"err": err, "status": out, "running": st["running"], "finished": st["finished"]}))
"""


def test_served_batch_failure_ends_requests():
    """A batch whose step fails (forced from the host by W1_FAIL_AT_STEP, in
    a child process) ends its unfinished requests as W1_SOLVE_FAILED, and
    w1_drain returns the error instead of waiting for ever."""
    require_gpu()
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, W1_FAIL_AT_STEP="3")
    out = subprocess.run([sys.executable, "-c", _FAIL_CHILD, root], env=env, capture_output=True, text=True,
                         timeout=100)
    assert out.returncode == 0, out.stderr[-2000:]
    res = json.loads(out.stdout.strip().splitlines()[-1])
    import paper_1810_00118_amd as w1lib
    assert res["err"] == w1lib.W1_EDEVICE
    assert res["running"] == 0 and res["finished"] == 4
    assert all(s == w1lib.SOLVE_FAILED for s in res["status"]), res



def test_served_poll_while_running():
    """Requests are polled from a second thread while the worker runs them
    (a request is handed to w1_poll only after the worker's last access):
    every result arrives, equal to the request solved alone, and the
    budget's bytes in use return to 0 after w1_drain."""
    import threading
    w1 = require_gpu()
    reqs = []
    for i in range(12):
        n = (32, 64, 128)[i % 3]
        p0, p1 = w1data.pair_gauss3(400 + i, n=n)
        L = {32: 1, 64: 2, 128: 3}[n]
        prm = w1.params(n=n, levels=L, metric=2, algo=1 + i % 2, precision=FP32, stop_rule=w1.STOP_FPR,
                        tol=0.0, max_iters=2000, check_every=10)
        reqs.append((prm, p0, p1))
    got = {}
    with w1.Solver(reqs[0][0], capacity=3) as srv:
        tickets = [srv.submit(p0, p1, prm) for prm, p0, p1 in reqs]

        def poller():
            pending = list(tickets)
            while pending:
                for t in list(pending):
                    r = srv.poll(t)
                    if r is not None:
                        got[t] = r[0]
                        pending.remove(t)

        th = threading.Thread(target=poller)
        th.start()
        srv.drain()
        th.join(timeout=60)
        assert not th.is_alive()
        st = srv.stats()
        assert st["bytes"] == 0 and st["running"] == 0 and st["finished"] == len(reqs)
    for t, (prm, p0, p1) in zip(tickets, reqs):
        with w1.Solver(prm) as s:
            alone = s.solve([(p0, p1)])[0]
        assert got[t]["iters"] == alone["iters"]
        assert got[t]["w1"] == pytest.approx(alone["w1"], rel=1e-6)


def test_served_without_fields():
    """W1_FLAG_NO_FIELDS: served requests end with the same results as with
    fields kept; asking w1_poll for their fields is refused with W1_EINVAL
    and leaves the result pollable."""
    w1 = require_gpu()
    reqs = []
    for i in range(6):
        n = (64, 128)[i % 2]
        p0, p1 = w1data.pair_gauss3(500 + i, n=n)
        reqs.append((n, p0, p1))

    def prm(n, flags):
        return w1.params(n=n, levels={64: 2, 128: 3}[n], metric=2, algo=1 + (n == 128), precision=FP32,
                         stop_rule=w1.STOP_FPR, tol=0.0, max_iters=2000, check_every=10, flags=flags)

    out = {}
    for flags in (0, w1.FLAG_NO_FIELDS):
        with w1.Solver(prm(128, flags), capacity=4) as srv:
            tickets = [srv.submit(p0, p1, prm(n, flags)) for n, p0, p1 in reqs]
            srv.drain()
            res = []
            for t, (n, _, _) in zip(tickets, reqs):
                if flags:
                    with pytest.raises(w1.W1Error) as e:
                        srv.poll(t, n=n, fields=True)
                    assert e.value.status == w1.W1_EINVAL
                r = srv.poll(t)
                assert r is not None and r[1] is None
                res.append(r[0])
            out[flags] = res
    for a, b in zip(out[0], out[w1.FLAG_NO_FIELDS]):
        assert a["iters"] == b["iters"] and a["w1"] == b["w1"] and a["hi"] == b["hi"]


@pytest.mark.parametrize("algo", [1, 2])
def test_level_caps_match_oracle(algo):
    """Per-level iteration caps (coarsest first): in FP64 the GPU runs every
    level to its own cap exactly as the oracle does (tolerance 0), and a cap
    above a level's natural stop leaves that level's stop unchanged."""
    w1 = require_gpu()
    n, L, metric = 128, 3, 2
    p0, p1 = w1data.pair_gauss3(21, n=n)
    caps = [300, 40, 20] if algo == 1 else [30, 10, 5]
    prm = w1.params(n=n, levels=L, metric=metric, algo=algo, precision=FP64, stop_rule=w1.STOP_FPR,
                    tol=1e-300, max_iters=20000, check_every=5, level_caps=caps)
    with w1.Solver(prm) as s:
        res = s.solve([(p0, p1)])[0]
        fields = s.fields(0)
    ref = o.solve(p0, p1, n, L=L, p=2, algo=algo, stop="fpr", eps_L=1e-300, alpha=-1.0, max_iters=caps,
                  check_every=5)
    assert res["iters"] == caps == ref["iters"]
    assert res["status"] == w1.SOLVE_MAXITER
    assert res["w1"] == pytest.approx(ref["w1"], rel=1e-10)
    np.testing.assert_allclose(fields[0], ref["m1"], rtol=0, atol=1e-9 * np.abs(ref["m1"]).max())
    # caps above the paper rule's stops: the same iterations as without caps
    eps = o.paper_stop_tolerance(algo, n, True)
    free = w1.params(n=n, levels=L, metric=metric, algo=algo, precision=FP64, stop_rule=w1.STOP_FPR, tol=eps,
                     max_iters=20000, check_every=5)
    with w1.Solver(free) as s:
        a = s.solve([(p0, p1)])[0]
    capped = w1.params(n=n, levels=L, metric=metric, algo=algo, precision=FP64, stop_rule=w1.STOP_FPR, tol=eps,
                       max_iters=20000, check_every=5, level_caps=[k + 5 for k in a["iters"]])
    with w1.Solver(capped) as s:
        b = s.solve([(p0, p1)])[0]
    assert a["iters"] == b["iters"] and a["w1"] == b["w1"]


@pytest.mark.parametrize("algo", [1, 2])
def test_step_guard(algo):
    """Steps beyond the convergence condition run only under the FPR rule's
    guard: at the practical steps (scale 1) the guard never fires and the
    FP64 run takes the oracle's stops; at scale 2 (Algorithm 1: the
    metric of R^k turns indefinite, R^k goes negative; Algorithm 2:
    mu tau = 4, G^k climbs to a plateau) the first level ends as diverged
    within a few tests instead of passing the stop test or running to the
    cap."""
    w1 = require_gpu()
    n, L = 64, 2
    p0, p1 = w1data.pair_gauss3(0, n=n)
    eps = o.paper_stop_tolerance(algo, n, True)
    for precision in (FP64, FP32):
        prm = w1.params(n=n, levels=L, metric=2, algo=algo, precision=precision, stop_rule=w1.STOP_FPR, tol=eps,
                        step_scale=1.0, max_iters=20000, check_every=10, diverge_window=3)
        with w1.Solver(prm) as s:
            res = s.solve([(p0, p1)])[0]
        ref = o.solve(p0, p1, n, L=L, p=2, algo=algo, stop="fpr", eps_L=eps, alpha=-1.0, max_iters=20000,
                      check_every=10, step_scale=1.0, return_fields=False)
        assert res["status"] == w1.SOLVE_OK
        if precision == FP64:
            assert res["iters"] == ref["iters"]
        assert res["w1"] == pytest.approx(ref["w1"], rel=1e-4)
        bad = w1.params(n=n, levels=L, metric=2, algo=algo, precision=precision, stop_rule=w1.STOP_FPR, tol=eps,
                        step_scale=2.0, max_iters=20000, check_every=10, diverge_window=3)
        with w1.Solver(bad) as s:
            r2 = s.solve([(p0, p1)])[0]
        assert r2["status"] == w1.SOLVE_DIVERGED
        assert r2["levels_run"] == 1 and r2["iters"][0] <= 200


def test_domain_scale():
    """w1_params.h: the same masses on [0, c]^2 (c = n h) give c times W1,
    dual and bracket, the flux over c and the potential times c."""
    w1 = require_gpu()
    n, L = 64, 2
    p0, p1 = w1data.pair_gauss3(2, n=n)
    base = dict(n=n, levels=L, metric=2, algo=w1.ALGO_PROX, precision=FP64, stop_rule=w1.STOP_FPR, tol=0.0,
                max_iters=20000, check_every=10)
    out = []
    for h in (0.0, 3.0 / n):
        with w1.Solver(w1.params(h=h, **base)) as s:
            out.append((s.solve([(p0, p1)])[0], s.fields(0)))
    (a, fa), (b, fb) = out
    assert a["iters"] == b["iters"]
    for k in ("w1", "dual", "lo", "hi"):
        assert b[k] == pytest.approx(3.0 * a[k], rel=1e-14)
    assert b["kkt"] == a["kkt"]
    np.testing.assert_allclose(fb[0], fa[0] / 3.0, rtol=1e-14)
    np.testing.assert_allclose(fb[2], fa[2] * 3.0, rtol=1e-14)


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_paired_stop_tests_same_bits(precision):
    """Plain levels run their iteration blocks in pairs whose two stop
    tests are taken together after the second block (the second block reads
    the first's output set, which it leaves intact).  The results are
    bit-identical to a stop test after every block (W1_PAIRED_CHECK=0):
    per-level iterations, W1, the bracket, for pairs that stop on either
    block of a pair."""
    import os
    w1 = require_gpu()
    n, L = 128, 3
    pairs = [w1data.pair_gauss3(900 + i, n=n) for i in range(12)]
    prm = w1.params(n=n, levels=L, metric=2, algo=w1.ALGO_PLAIN, precision=precision, stop_rule=w1.STOP_FPR,
                    tol=0.0, alpha=-1.0, max_iters=20000, check_every=10, flags=w1.FLAG_NO_RESIDENT)
    out = {}
    old = os.environ.get("W1_PAIRED_CHECK")
    try:
        for paired in ("1", "0"):
            os.environ["W1_PAIRED_CHECK"] = paired
            with w1.Solver(prm, capacity=len(pairs)) as s:
                out[paired] = s.solve(pairs)
    finally:
        if old is None:
            os.environ.pop("W1_PAIRED_CHECK", None)
        else:
            os.environ["W1_PAIRED_CHECK"] = old
    # both parities of the stop block occur (20 iterations per pair)
    assert {r["iters"][-1] // 10 % 2 for r in out["1"]} == {0, 1}
    for a, b in zip(out["1"], out["0"]):
        assert a["status"] == b["status"] and a["iters"] == b["iters"]
        assert a["w1"] == b["w1"] and a["lo"] == b["lo"] and a["hi"] == b["hi"]


def test_kernel_timing_sample():
    """Per-launch timing (w1_profile) changes no result: the same bits with
    every tiled launch timed, with about one in 8 timed and untimed.  The
    sample times fewer launches than the full count, its average launch
    duration is positive, and a negative setting is rejected."""
    w1 = require_gpu()
    n, L = 128, 2
    pairs = [w1data.pair_gauss3(950 + i, n=n) for i in range(8)]
    prm = w1.params(n=n, levels=L, metric=2, algo=w1.ALGO_PLAIN, precision=FP32, stop_rule=w1.STOP_FPR,
                    tol=0.0, alpha=-1.0, max_iters=4000, check_every=10, flags=w1.FLAG_NO_RESIDENT)
    out, stats = {}, {}
    with w1.Solver(prm, capacity=len(pairs)) as s:
        s.solve(pairs)                      # launch shapes settled by the autotuner
        for every in (0, 1, 8):
            s.profile(every > 0, every=max(every, 1))
            out[every] = s.solve(pairs)
            stats[every] = s.kernel_stats()["plain_tiled"]
        s.profile(False)
        with pytest.raises(RuntimeError):
            s.profile(True, every=-1)
    for k in (1, 8):
        for a, b in zip(out[0], out[k]):
            assert a["iters"] == b["iters"] and a["w1"] == b["w1"] and a["hi"] == b["hi"]
    full, part = stats[1], stats[8]
    assert full["launches"] > 50 and 0 < part["launches"] < full["launches"] / 3
    assert part["ms"] > 0 and part["node_updates"] > 0


def test_device_inputs_read_in_place():
    """w1_solve reads device masses in place: the results equal those of the
    same masses passed from host memory (which are copied), and the caller's
    device buffers are unchanged afterwards, fields fetched included."""
    import torch
    w1 = require_gpu()
    n, L = 96, 2
    pairs = [w1data.pair_gauss3(960 + i, n=n) for i in range(5)]
    dev = [(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for a, b in pairs]
    keep = [(a.clone(), b.clone()) for a, b in dev]
    prm = w1.params(n=n, levels=L, metric=2, algo=w1.ALGO_PLAIN, precision=FP32, stop_rule=w1.STOP_FPR,
                    tol=0.0, alpha=-1.0, max_iters=4000, check_every=10, flags=w1.FLAG_NO_RESIDENT)
    with w1.Solver(prm, capacity=len(pairs)) as s:
        r_host = s.solve(pairs)
    with w1.Solver(prm, capacity=len(pairs)) as s:
        r_dev = s.solve(dev)
        for k in range(len(pairs)):
            s.fields(k)
    torch.cuda.synchronize()
    for a, b in zip(r_host, r_dev):
        assert a["iters"] == b["iters"] and a["w1"] == b["w1"] and a["hi"] == b["hi"]
    for (a, b), (ka, kb) in zip(dev, keep):
        assert torch.equal(a, ka) and torch.equal(b, kb)


def test_graph_replay_same_bits():
    """W1_GRAPH=1: plain-only steps replay their block sequences from
    captured HIP graphs while the slot set is unchanged (each graph is
    replayed over several steps, with the host's own stop handling,
    uploads and synchronisations between replays).  Per-level iterations,
    W1 and the bracket equal those of the eager launches bit for bit, and
    graphs were in fact captured."""
    import os
    w1 = require_gpu()
    n, L = 128, 3
    pairs = [w1data.pair_gauss3(970 + i, n=n) for i in range(10)]
    prm = w1.params(n=n, levels=L, metric=2, algo=w1.ALGO_PLAIN, precision=FP32, stop_rule=w1.STOP_FPR,
                    tol=0.0, alpha=-1.0, max_iters=20000, check_every=10, flags=w1.FLAG_NO_RESIDENT)
    old = os.environ.get("W1_GRAPH")
    out, graphs = {}, {}
    try:
        os.environ["W1_GRAPH"] = "0"
        with w1.Solver(prm, capacity=len(pairs)) as s:
            s.solve(pairs)                       # launch shapes settled by the autotuner
            out["0"] = s.solve(pairs)
        for mode in ("1", "0"):
            os.environ["W1_GRAPH"] = mode
            with w1.Solver(prm, capacity=len(pairs)) as s:
                c0 = s.counters()["graphs_captured"]
                out[mode + "b"] = s.solve(pairs)
                graphs[mode] = s.counters()["graphs_captured"] - c0
    finally:
        if old is None:
            os.environ.pop("W1_GRAPH", None)
        else:
            os.environ["W1_GRAPH"] = old
    assert graphs["1"] > 0 and graphs["0"] == 0
    for a, b, c in zip(out["0"], out["1b"], out["0b"]):
        for x in (b, c):
            assert a["status"] == x["status"] and a["iters"] == x["iters"]
            assert a["w1"] == x["w1"] and a["lo"] == x["lo"] and a["hi"] == x["hi"]


def test_trim_cache_releases_idle_blocks():
    """Finished solves leave their device blocks in the process-wide cache;
    w1_trim_cache returns them to the device (bytes released > 0), a second
    call finds none, and later solves allocate afresh with the same
    results."""
    w1 = require_gpu()
    n, L = 64, 2
    pairs = [w1data.pair_gauss3(990 + i, n=n) for i in range(3)]
    prm = w1.params(n=n, levels=L, metric=2, algo=w1.ALGO_PLAIN, precision=FP32, stop_rule=w1.STOP_FPR,
                    tol=0.0, alpha=-1.0, max_iters=2000, check_every=10)
    with w1.Solver(prm, capacity=len(pairs)) as s:
        a = s.solve(pairs)
    assert w1.trim_cache() > 0
    assert w1.trim_cache() == 0
    with w1.Solver(prm, capacity=len(pairs)) as s:
        b = s.solve(pairs)
    for x, y in zip(a, b):
        assert x["iters"] == y["iters"] and x["w1"] == y["w1"]


def test_closed_batch_budget_same_bits():
    """A closed batch (w1_solve) queues more iteration blocks per host
    synchronisation than served mode once a group holds many slots; the
    blocks past a slot's stop skip it, so every result is the served one bit
    for bit, in fewer host steps."""
    w1 = require_gpu()
    n, L, k = 64, 2, 24
    pairs = [w1data.pair_gauss3(200 + i, n=n) for i in range(k)]
    prm = w1.params(n=n, levels=L, metric=2, algo=w1.ALGO_PLAIN, precision=FP32, stop_rule=w1.STOP_FPR,
                    tol=0.0, max_iters=3000, check_every=10, flags=w1.FLAG_NO_RESIDENT)
    with w1.Solver(prm, capacity=k) as s:
        batch = s.solve(pairs)
        fb = [s.fields(i) for i in range(k)]
        steps_batch = s.counters()["host_steps"]
    with w1.Solver(prm, capacity=k) as srv:
        tickets = [srv.submit(p0, p1, prm) for p0, p1 in pairs]
        srv.drain()
        served = []
        for t in tickets:
            r = None
            while r is None:
                r = srv.poll(t, n=n, fields=True)
            served.append(r)
        steps_served = srv.counters()["host_steps"]
    print(f"host steps: closed batch {steps_batch}, served {steps_served}", flush=True)
    for i in range(k):
        res, fs = served[i]
        assert res["iters"] == batch[i]["iters"]
        assert res["w1"] == batch[i]["w1"]
        for a, b in zip(fs, fb[i]):
            np.testing.assert_array_equal(a, b)
    assert steps_batch < steps_served

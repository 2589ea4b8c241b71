"""GPU parity of each row of the method through the single-step entry
points of the C ABI, against the FP64 oracle on identical seeded inputs.
Sizes span several tiles and ragged tails."""
import math

import numpy as np
import pytest

import oracle.w1_oracle as o
import w1data
from tests.gpu_util import P_OF, dev, host, rel_err, require_gpu, tdtype

pytestmark = pytest.mark.gpu

FP32, FP64 = 1, 2


def _rho(n, seed):
    p0, p1 = w1data.random_pair(n, seed)
    return o.prepare_levels(p0, p1, n, 1)[0]


def _rand_state(n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    m1 = rng.standard_normal((n + 1, n + 1)) * scale; m1[n, :] = 0
    m2 = rng.standard_normal((n + 1, n + 1)) * scale; m2[:, n] = 0
    phi = rng.standard_normal((n + 1, n + 1)) * 0.1
    return m1, m2, phi


@pytest.mark.parametrize("precision", [FP64, FP32])
@pytest.mark.parametrize("n", [33, 100, 200])
@pytest.mark.parametrize("metric", [1, 2, 3])
@pytest.mark.parametrize("block,width", [(1, 0), (4, 0), (-1, 0), (4, 64), (10, 64)])
def test_plain_steps_trajectory(precision, n, metric, block, width):
    w1 = require_gpu()
    if block < 0 and n + 1 > 65:
        pytest.skip("resident kernel holds sides up to 65")
    h = 1.0 / n
    rho = _rho(n, n)
    m1, m2, phi = _rand_state(n, n + 1)
    mu, tau = o.plain_step_sizes(h)
    dt = tdtype(precision)
    g = [dev(x, dt) for x in (m1, m2, phi, rho)]
    for k in (1, 10, 40):
        R = w1.op_plain_steps(n, metric, precision, k, g[0], g[1], g[2], g[3], block_steps=block, fpr=True,
                              width=width)
        a1, a2, ap = m1.copy(), m2.copy(), phi.copy()
        for _ in range(k):
            a1, a2, ap, Rw = o.pd_step(a1, a2, ap, rho, h, mu, tau, P_OF[metric])
        tol = 1e-12 if precision == FP64 else 2e-5 * math.sqrt(k)
        assert rel_err(host(g[0]), a1) <= tol
        assert rel_err(host(g[1]), a2) <= tol
        assert rel_err(host(g[2]), ap) <= tol
        assert R == pytest.approx(Rw, rel=1e-9 if precision == FP64 else 1e-3)
        # restart both sides from the same state for the next k
        m1, m2, phi = a1, a2, ap
        g = [dev(x, dt) for x in (m1, m2, phi, rho)]


@pytest.mark.parametrize("precision", [FP64, FP32])
@pytest.mark.parametrize("block", [4, -1])
def test_practical_step_sizes(precision, block):
    """The footnoted practical steps of Sec. 3.1 (step_scale 1: mu = tau =
    1/||A|| with the Gershgorin bound; mu = tau = 1 for Algorithm 2) follow
    the oracle's iterates like the default steps."""
    w1 = require_gpu()
    n = 64 if block < 0 else 100
    h = 1.0 / n
    rho = _rho(n, 5)
    m1, m2, phi = _rand_state(n, 6)
    mu, tau = o.plain_step_sizes(h, 1.0)
    dt = tdtype(precision)
    g = [dev(x, dt) for x in (m1, m2, phi, rho)]
    k = 30
    R = w1.op_plain_steps(n, 2, precision, k, g[0], g[1], g[2], g[3], step_scale=1.0, block_steps=block, fpr=True)
    a1, a2, ap = m1, m2, phi
    for _ in range(k):
        a1, a2, ap, Rw = o.pd_step(a1, a2, ap, rho, h, mu, tau, 2)
    tol = 1e-12 if precision == FP64 else 2e-5 * math.sqrt(k)
    for got, want in zip(g[:3], (a1, a2, ap)):
        assert rel_err(host(got), want) <= tol
    assert R == pytest.approx(Rw, rel=1e-9 if precision == FP64 else 1e-3)
    rng = np.random.default_rng(7)
    v1 = rng.uniform(-1, 1, (n + 1, n + 1)); v1[n, :] = 0
    v2 = rng.uniform(-1, 1, (n + 1, n + 1)); v2[:, n] = 0
    g = [dev(x, dt) for x in (m1, m2, v1, v2, v1, v2, rho)]
    G = w1.op_prox_steps(n, 2, precision, 10, *g, step_scale=1.0, fpr=True,
                         resident=block < 0 and precision == FP32)
    st = (m1, m2, v1, v2, v1.copy(), v2.copy())
    for _ in range(10):
        out = o.prox_step(*st, rho, h, 1.0, 1.0, 2)
        st, Gw = out[:6], out[6]
    for got, want in zip(g[:6], st):
        assert rel_err(host(got), want) <= (1e-10 if precision == FP64 else 2e-4)
    assert G == pytest.approx(Gw, rel=1e-8 if precision == FP64 else 1e-2, abs=1e-12)


@pytest.mark.parametrize("precision", [FP64, FP32])
@pytest.mark.parametrize("n", [32, 64, 100])
@pytest.mark.parametrize("metric", [2, 3])
def test_resident_and_tiled_agree_bitwise(precision, n, metric):
    w1 = require_gpu()
    if n + 1 > 65:
        pytest.skip("resident kernel holds sides up to 65")
    rho = _rho(n, 3)
    m1, m2, phi = _rand_state(n, 4)
    dt = tdtype(precision)
    outs = []
    for block, waves, width in ((-1, 0, 0), (1, 8, 0), (3, 8, 0), (6, 16, 0), (5, 16, 0), (1, 16, 0),
                                (5, 16, 64), (3, 8, 64), (1, 16, 64)):
        g = [dev(x, dt) for x in (m1, m2, phi, rho)]
        w1.op_plain_steps(n, metric, precision, 25, g[0], g[1], g[2], g[3], block_steps=block, waves=waves,
                          width=width)
        outs.append([host(x) for x in g[:3]])
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("precision", [FP64, FP32])
@pytest.mark.parametrize("n", [100, 200, 300])
@pytest.mark.parametrize("metric", [1, 2, 3])
def test_region_shapes_agree_bitwise(precision, n, metric):
    """The 64 x 128, 64 x 64 and 32 x 64 regions, over 8 or 16 wavefronts and at
    every block depth, give the same iterates bit for bit (grids of several
    tiles in both directions with ragged last tiles).  R^k is a sum of
    per-tile partials, whose grouping follows the tiling: equal up to
    rounding."""
    w1 = require_gpu()
    rho = _rho(n, 11)
    m1, m2, phi = _rand_state(n, 12)
    dt = tdtype(precision)
    outs = []
    for block, waves, width, height in ((10, 16, 0, 0), (1, 8, 0, 0), (7, 8, 0, 0), (10, 16, 64, 0),
                                        (10, 8, 64, 0), (16, 16, 64, 0), (4, 8, 64, 0), (10, 8, 64, 32),
                                        (3, 8, 64, 32)):
        g = [dev(x, dt) for x in (m1, m2, phi, rho)]
        R = w1.op_plain_steps(n, metric, precision, 40, g[0], g[1], g[2], g[3], block_steps=block, waves=waves,
                              width=width, height=height, fpr=True)
        outs.append(([host(x) for x in g[:3]], R))
    for other, R in outs[1:]:
        assert R == pytest.approx(outs[0][1], rel=1e-12 if precision == FP64 else 1e-6)
        for a, b in zip(outs[0][0], other):
            np.testing.assert_array_equal(a, b)


def test_region_width_rejected():
    """Region widths other than 0, 64 and 128, narrow blocks deeper than 16
    steps, and short regions other than 32 x 64 over 8 wavefronts with at
    most 10 steps, are W1_EINVAL."""
    w1 = require_gpu()
    n = 40
    g = [dev(x, tdtype(FP32)) for x in (*_rand_state(n, 1), _rho(n, 1))]
    for width, block in ((32, 4), (96, 4), (64, 17)):
        with pytest.raises(w1.W1Error):
            w1.op_plain_steps(n, 2, FP32, 4, *g, block_steps=block, width=width)
    for width, height, waves, block in ((128, 32, 8, 4), (64, 32, 16, 4), (64, 32, 8, 11), (64, 48, 8, 4)):
        with pytest.raises(w1.W1Error):
            w1.op_plain_steps(n, 2, FP32, 4, *g, block_steps=block, width=width, height=height, waves=waves)


@pytest.mark.parametrize("precision", [FP64, FP32])
@pytest.mark.parametrize("n", [32, 64, 100])
@pytest.mark.parametrize("metric", [1, 2, 3])
def test_prox_steps_trajectory(precision, n, metric):
    w1 = require_gpu()
    h = 1.0 / n
    rho = _rho(n, 7 + n)
    m1, m2, _ = _rand_state(n, 8)
    rng = np.random.default_rng(9)
    v1 = rng.uniform(-1, 1, (n + 1, n + 1)); v1[n, :] = 0
    v2 = rng.uniform(-1, 1, (n + 1, n + 1)); v2[:, n] = 0
    dt = tdtype(precision)
    g = [dev(x, dt) for x in (m1, m2, v1, v2, v1, v2, rho)]
    k = 10
    G = w1.op_prox_steps(n, metric, precision, k, *g, fpr=True)
    st = (m1, m2, v1, v2, v1.copy(), v2.copy())
    for _ in range(k):
        out = o.prox_step(*st, rho, h, 0.5, 0.5, P_OF[metric])
        st, Gw = out[:6], out[6]
    tol = 1e-10 if precision == FP64 else 1e-4
    for got, want in zip(g[:6], st):
        assert rel_err(host(got), want) <= tol
    assert G == pytest.approx(Gw, rel=1e-8 if precision == FP64 else 1e-2, abs=1e-12)


@pytest.mark.parametrize("n", [1024, 2048])
def test_prox_steps_trajectory_fft(n):
    """Algorithm 2 steps on grids whose FP32 Poisson solves take the FFT
    path follow the oracle's iterates and G^k."""
    w1 = require_gpu()
    h = 1.0 / n
    rho = _rho(n, 3 + n)
    m1, m2, _ = _rand_state(n, 4)
    rng = np.random.default_rng(5)
    v1 = rng.uniform(-1, 1, (n + 1, n + 1)); v1[n, :] = 0
    v2 = rng.uniform(-1, 1, (n + 1, n + 1)); v2[:, n] = 0
    g = [dev(x, tdtype(FP32)) for x in (m1, m2, v1, v2, v1, v2, rho)]
    k = 4
    G = w1.op_prox_steps(n, 2, FP32, k, *g, fpr=True)
    st = (m1, m2, v1, v2, v1.copy(), v2.copy())
    for _ in range(k):
        out = o.prox_step(*st, rho, h, 0.5, 0.5, 2)
        st, Gw = out[:6], out[6]
    for got, want in zip(g[:6], st):
        assert rel_err(host(got), want) <= 1e-4
    assert G == pytest.approx(Gw, rel=1e-2, abs=1e-12)


@pytest.mark.parametrize("n", [4, 7, 16, 32, 40, 63, 64])
@pytest.mark.parametrize("metric", [1, 2, 3])
@pytest.mark.parametrize("k", [1, 10, 60])
def test_prox_resident_trajectory(n, metric, k):
    """The whole-level LDS kernel of Algorithm 2 follows the oracle's
    iterates and G^k (FP32) and agrees with the batched kernels."""
    w1 = require_gpu()
    h = 1.0 / n
    rho = _rho(n, 17 + n)
    m1, m2, _ = _rand_state(n, 18)
    rng = np.random.default_rng(19)
    v1 = rng.uniform(-1, 1, (n + 1, n + 1)); v1[n, :] = 0
    v2 = rng.uniform(-1, 1, (n + 1, n + 1)); v2[:, n] = 0
    dt = tdtype(FP32)
    g = [dev(x, dt) for x in (m1, m2, v1, v2, v1, v2, rho)]
    G = w1.op_prox_steps(n, metric, FP32, k, *g, fpr=True, resident=True)
    gb = [dev(x, dt) for x in (m1, m2, v1, v2, v1, v2, rho)]
    Gb = w1.op_prox_steps(n, metric, FP32, k, *gb, fpr=True)
    st = (m1, m2, v1, v2, v1.copy(), v2.copy())
    for _ in range(k):
        out = o.prox_step(*st, rho, h, 0.5, 0.5, P_OF[metric])
        st, Gw = out[:6], out[6]
    tol = 1e-4 * math.sqrt(k)
    for got, other, want in zip(g[:6], gb[:6], st):
        assert rel_err(host(got), want) <= tol
        assert rel_err(host(got), host(other)) <= tol
    assert G == pytest.approx(Gw, rel=1e-2, abs=1e-12)
    assert G == pytest.approx(Gb, rel=1e-2, abs=1e-12)


def test_prox_resident_rejects_unsupported():
    w1 = require_gpu()
    n = 100
    dt = tdtype(FP32)
    z = [dev(np.zeros((n + 1, n + 1)), dt) for _ in range(7)]
    with pytest.raises(w1.W1Error):
        w1.op_prox_steps(n, 2, FP32, 1, *z, resident=True)
    z64 = [dev(np.zeros((33, 33)), tdtype(FP64)) for _ in range(7)]
    with pytest.raises(w1.W1Error):
        w1.op_prox_steps(32, 2, FP64, 1, *z64, resident=True)


@pytest.mark.parametrize("precision", [FP64, FP32])
@pytest.mark.parametrize("n", [4, 16, 63, 64, 99, 128, 129, 200, 512, 1000, 1024, 2048])
def test_poisson(precision, n):
    # FP32 from n = 1024 on: the FFT path (Bluestein DFTs of the DCT lines);
    # below, and in FP64, products with the DCT matrix
    w1 = require_gpu()
    rng = np.random.default_rng(n)
    r = rng.standard_normal((n + 1, n + 1)); r -= r.mean()
    want = o.poisson_neumann(r, 1.0 / n)
    dt = tdtype(precision)
    gr = dev(r, dt)
    gu = dev(np.zeros_like(r), dt)
    w1.op_poisson(n, precision, gr, gu)
    tol = 1e-11 if precision == FP64 else 2e-5
    assert rel_err(host(gu), want) <= tol
    # aliasing input and output is allowed
    w1.op_poisson(n, precision, gr, gr)
    assert rel_err(host(gr), want) <= tol


@pytest.mark.parametrize("precision", [FP64, FP32])
@pytest.mark.parametrize("n", [16, 100])
def test_potential(precision, n):
    w1 = require_gpu()
    rng = np.random.default_rng(n + 5)
    v1 = rng.uniform(-1, 1, (n + 1, n + 1)); v1[n, :] = 0
    v2 = rng.uniform(-1, 1, (n + 1, n + 1)); v2[:, n] = 0
    want = o.potential_from_dual(v1, v2, 1.0 / n)
    dt = tdtype(precision)
    g = [dev(x, dt) for x in (v1, v2, np.zeros_like(v1))]
    w1.op_potential(n, precision, *g)
    assert rel_err(host(g[2]), want) <= (1e-11 if precision == FP64 else 3e-5)


@pytest.mark.parametrize("precision", [FP64, FP32])
@pytest.mark.parametrize("nc", [1, 7, 50])
def test_prolong(precision, nc):
    w1 = require_gpu()
    rng = np.random.default_rng(nc)
    c1 = rng.standard_normal((nc + 1, nc + 1)); c1[nc, :] = 0
    c2 = rng.standard_normal((nc + 1, nc + 1)); c2[:, nc] = 0
    cp = rng.standard_normal((nc + 1, nc + 1))
    f1, f2 = o.prolong_flux(c1, c2)
    fp = o.prolong_potential(cp)
    dt = tdtype(precision)
    g = [dev(x, dt) for x in (c1, c2, cp)]
    out = [dev(np.zeros_like(f1), dt) for _ in range(3)]
    w1.op_prolong(nc, precision, *g, *out)
    tol = 0 if precision == FP64 else 1e-7
    for got, want in zip(out, (f1, f2, fp)):
        assert rel_err(host(got), want) <= tol


@pytest.mark.parametrize("precision", [FP64, FP32])
@pytest.mark.parametrize("n,L", [(64, 3), (100, 1), (256, 4)])
def test_prepare(precision, n, L):
    w1 = require_gpu()
    import torch
    p0, p1 = w1data.pair_shapes(0, n=n) if n % 4 == 0 else w1data.random_pair(n, 1)
    want = o.prepare_levels(p0, p1, n, L)
    dt = tdtype(precision)
    outs = [dev(np.zeros_like(r), dt) for r in want]
    w1.op_prepare(n, L, precision, dev(p0, torch.float64), dev(p1, torch.float64), outs)
    for got, ref in zip(outs, want):
        assert rel_err(host(got), ref) <= (1e-13 if precision == FP64 else 1e-6)


def test_prepare_rejects_bad_masses():
    w1 = require_gpu()
    import torch
    n = 16
    p0, p1 = w1data.random_pair(n, 2)
    bad = p0.copy(); bad[3, 3] = -1e-3
    rho = [dev(np.zeros((n + 1, n + 1)), torch.float64)]
    with pytest.raises(w1.W1Error):
        w1.op_prepare(n, 1, FP64, dev(bad, torch.float64), dev(p1, torch.float64), rho)
    with pytest.raises(w1.W1Error):
        w1.op_prepare(n, 1, FP64, dev(p0, torch.float64), dev(p1 * 1.001, torch.float64), rho)
    nanm = p0.copy(); nanm[0, 0] = np.nan
    with pytest.raises(w1.W1Error):
        w1.op_prepare(n, 1, FP64, dev(nanm, torch.float64), dev(p1, torch.float64), rho)


@pytest.mark.parametrize("precision", [FP64, FP32])
@pytest.mark.parametrize("metric", [1, 2, 3])
@pytest.mark.parametrize("n", [24, 100])
def test_evaluate(precision, metric, n):
    w1 = require_gpu()
    rho = _rho(n, 11)
    r = o.solve(*w1data.random_pair(n, 11), n, L=1, p=P_OF[metric], algo=1, stop="kkt", tol=0.0, max_iters=200,
                check_every=200)
    m1, m2, psi = r["m1"], r["m2"], r["psi"]
    want = o.evaluate(m1, m2, psi, rho, 1.0 / n, P_OF[metric])
    dt = tdtype(precision)
    got = w1.op_evaluate(n, metric, precision, *[dev(x, dt) for x in (m1, m2, psi, rho)])
    rt = 1e-10 if precision == FP64 else 2e-5
    for k in ("P", "D", "lo", "hi"):
        assert got[k] == pytest.approx(want[k], rel=rt, abs=1e-12), k
    assert got["kkt"] == pytest.approx(want["kkt"], rel=1e-6 if precision == FP64 else 2e-3)
    assert got["grad_max"] == pytest.approx(want["grad_max"], rel=rt)

"""The C-ABI library loads and exports every function include/w1.h declares
(no device calls)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "w1.h")
LIB = os.path.join(ROOT, "paper_1810_00118_amd", "libw1.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(w1_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("w1_plan", "w1_solve", "w1_submit", "w1_poll", "w1_destroy", "w1_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libw1.so not built")
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (w1_[a-z_0-9]+)\b", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_library_loads_and_checks_params_without_a_device():
    if not os.path.exists(LIB):
        pytest.skip("libw1.so not built")
    import paper_1810_00118_amd as w1
    assert "gfx950" in w1.version()
    p = w1.params(n=512, levels=4)
    assert w1.check_params(p) == 0
    assert w1.bytes_per_solve(p) > 0
    for m in (1, 2, 3):
        assert w1.check_params(w1.params(n=512, levels=4, metric=m)) == 0
    # the paper's practical step sizes (scale 1) are accepted; larger ones
    # (up to 2) only under the FPR rule with the rise-window guard
    assert w1.check_params(w1.params(n=512, levels=4, step_scale=1.0)) == 0
    assert w1.check_params(w1.params(n=512, levels=4, step_scale=1.5, diverge_window=3)) == 0
    # per-level caps (multiples of check_every, only on existing levels), a domain scale
    assert w1.check_params(w1.params(n=512, levels=4, level_caps=[100, 0, 50, 10])) == 0
    assert w1.check_params(w1.params(n=512, levels=4, h=0.5 / 512)) == 0
    for f in (w1.FLAG_NO_RESIDENT, w1.FLAG_NO_CERT, w1.FLAG_LEVEL_COST, w1.FLAG_NO_FIELDS, 15):
        assert w1.check_params(w1.params(n=512, levels=4, flags=f)) == 0
    for bad in (dict(n=100), dict(levels=0), dict(metric=4), dict(metric=0),
                dict(max_iters=15, check_every=10), dict(step_scale=1.5), dict(algo=7),
                dict(step_scale=1.5, diverge_window=3, stop_rule=w1.STOP_KKT, tol=1e-6),
                dict(step_scale=2.5, diverge_window=3), dict(diverge_window=-1),
                dict(level_caps=[15]), dict(level_caps=[10, 10, 10, 10, 10]), dict(level_caps=[-10]),
                dict(h=float("inf")), dict(reserved=1), dict(flags=16), dict(flags=-1)):
        q = w1.params(**dict(dict(n=512, levels=4), **bad))
        assert w1.check_params(q) == w1.W1_EINVAL, bad
    assert w1.strerror(w1.W1_EINVAL) == "invalid argument"


def test_tuner_table_is_host_only():
    if not os.path.exists(LIB):
        pytest.skip("libw1.so not built")
    import paper_1810_00118_amd as w1
    w1.tuner_reset()
    assert w1.tuner_table() == []


def test_d3_entry_points_check_arguments_without_a_device():
    # the d = 3 entry points validate every argument before touching a device
    if not os.path.exists(LIB):
        pytest.skip("libw1.so not built")
    import ctypes as C

    import numpy as np

    import paper_1810_00118_amd as w1
    L = w1.lib()
    n = 4
    a = np.full((n + 1,) * 3, 1.0 / (n + 1) ** 3)
    out = w1.Result()
    ok = dict(n=n, levels=2, metric=2, algo=w1.ALGO_PLAIN, precision=w1.FP32, stop_rule=w1.STOP_FPR, tol=1e-6,
              max_iters=100, check_every=10)
    for bad in (dict(n=3), dict(levels=3), dict(tol=0.0), dict(metric=0), dict(algo=3), dict(step_scale=2.0),
                dict(max_iters=15), dict(precision=3), dict(level_caps=[15]), dict(level_caps=[10, 10, 10]),
                dict(step_scale=1.5, diverge_window=2, stop_rule=w1.STOP_KKT), dict(diverge_window=-2)):
        prm = w1.params(**dict(ok, **bad))
        st = L.w1_solve3d(C.byref(prm), a.ctypes.data, a.ctypes.data, 0, C.byref(out), None, None, None)
        assert st == w1.W1_EINVAL, bad
    prm = w1.params(**ok)
    assert L.w1_solve3d_batch(C.byref(prm), 0, None, None, 0, None, 4) == w1.W1_OK
    ptrs = (C.c_void_p * 1)(a.ctypes.data)
    res = (w1.Result * 1)()
    assert L.w1_solve3d_batch(C.byref(prm), 1, ptrs, ptrs, 0, res, 17) == w1.W1_EINVAL
    bad = w1.params(**dict(ok, tol=-1.0))
    assert L.w1_solve3d_batch(C.byref(bad), 1, ptrs, ptrs, 0, res, 2) == w1.W1_EINVAL

"""The allocation-free Neumann Poisson solve (w1_op_poisson_noalloc) against
w1_op_poisson, the entry point whose kernels it shares: two calls in a row
on one GPU, the second with a smaller grid (the static working memory keeps
the first call's contents), in both precisions, each also against the FP64
oracle's solve; sizes beyond the stated maximum are rejected before any
device call."""
import ctypes as C

import numpy as np
import pytest

import oracle.w1_oracle as o
from tests.gpu_util import dev, host, rel_err, require_gpu, tdtype

FP32, FP64 = 1, 2


def _rhs(n, seed):
    rng = np.random.default_rng(seed)
    r = rng.standard_normal((n + 1, n + 1))
    return r - r.mean()


def test_noalloc_rejects_beyond_its_maximum():
    import paper_1810_00118_amd as w1
    L = w1.lib()
    assert w1.noalloc_bytes() > 0
    for n in (0, 513, 4096):
        assert L.w1_op_poisson_noalloc(n, FP32, C.c_void_p(16), C.c_void_p(16), None) == w1.W1_EINVAL
    assert L.w1_op_poisson_noalloc(64, 3, C.c_void_p(16), C.c_void_p(16), None) == w1.W1_EINVAL
    assert L.w1_op_poisson_noalloc(64, FP32, None, C.c_void_p(16), None) == w1.W1_EINVAL


@pytest.mark.gpu
@pytest.mark.parametrize("precision", [FP64, FP32])
def test_noalloc_matches_allocating_poisson(precision):
    w1 = require_gpu()
    import torch
    L = w1.lib()
    stream = torch.cuda.current_stream().cuda_stream
    # within the working memory's maximum side (512), two calls in a row,
    # the second smaller than the first
    for n, seed in ((512, 1), (200, 2), (37, 3)):
        r = _rhs(n, seed)
        dt = tdtype(precision)
        gr = dev(r, dt)
        ref = dev(np.zeros_like(r), dt)
        got = dev(np.full_like(r, np.nan), dt)
        w1.op_poisson(n, precision, gr, ref)
        st = L.w1_op_poisson_noalloc(n, precision, C.c_void_p(gr.data_ptr()), C.c_void_p(got.data_ptr()),
                                     C.c_void_p(stream))
        assert st == w1.W1_OK
        a, b = host(got), host(ref)
        assert np.all(np.isfinite(a))
        # same kernels; the DCT tables come from the same closed forms,
        # evaluated on the device instead of the host
        assert rel_err(a, b) <= (1e-13 if precision == FP64 else 1e-6), (n, rel_err(a, b))
        want = o.poisson_neumann(r, 1.0 / n)
        assert rel_err(a, want) <= (1e-11 if precision == FP64 else 2e-5)

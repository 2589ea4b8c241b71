"""Helpers shared by the GPU tests: device buffers through torch."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_1810_00118_amd as w1
    w1.lib()  # raises if the library is missing
    return w1


def dev(a, dtype):
    t = torch.from_numpy(np.ascontiguousarray(a)).to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def tdtype(precision):
    return torch.float32 if precision == 1 else torch.float64


# ground metric code of the C ABI -> the oracle's p
P_OF = {1: 1, 2: 2, 3: math.inf}

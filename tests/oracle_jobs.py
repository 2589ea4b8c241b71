"""Oracle solves run in worker processes by the GPU tests (a spawned pool:
the workers import only the oracle and the input generators, no GPU
state)."""
import oracle.w1_oracle as o
import w1data


def config1(seed):
    """Config 1 of one seed: 64x64, three isotropic Gaussians + floor, l_1,
    plain PDHG (Algorithm 3), 2 levels, KKT 1e-6 or 20k per level."""
    p0, p1 = w1data.pair_gauss3(seed)
    return o.solve(p0, p1, 64, L=2, p=1, algo=1, stop="kkt", tol=1e-6, max_iters=20000, check_every=10,
                   alpha=-1.0)

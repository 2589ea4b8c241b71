"""FP64 CPU oracle of the cascadic multilevel primal-dual W1 solver
(Liu, Yin, Li, Chow, "Multilevel Optimal Transport: a Fast Approximation of
Wasserstein-1 distances", arXiv 1810.00118).

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, links or calls anything here; only the test suite,
the package's smoke check and the benchmark's CPU-baseline leg do.  The
oracle shares no code with the HIP path: the only common dependency is the
seeded input generator module ``w1data``, which holds none of the method's
arithmetic.

Parity status: every public function of ``oracle.w1_oracle`` (d = 2) and of
``oracle.w1_oracle3d`` (the same method written for any d, used at d = 3) is
pinned by the tests under ``tests/test_oracle_*.py`` against closed forms,
exact identities, printed values of the paper, brute force, or (for the
d-general module) the d = 2 module it reduces to.  One quantity is "parity
unpinned": the W1 values the paper prints for its DOTmark / cat experiments,
because those inputs are absent.
"""
from .w1_oracle import *  # noqa: F401,F403

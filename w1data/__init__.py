"""Seeded synthetic density pairs on the vertex grid of [0,1]^2.

This module is shared by the CPU oracle and by the GPU path's tests and
benchmarks.  It holds no part of the solver's arithmetic: it only draws
node masses p0, p1 (float64, shape (n+1, n+1), each summing to 1) from
seeded NumPy generators.

Grid convention (paper Sec. 2.2, "Discretization"): side n means h = 1/n and
vertex nodes x = (i h, j h) for i, j in {0..n}; array index [i, j] has i along
x1 (rows) and j along x2 (contiguous).

The paper measures on the DOTmark "classic images" and on a "cat" pair
(Sec. 5); neither is available here, so the workloads below are synthetic
stand-ins with the shapes and sizes of those experiments (grids 64..2048,
smooth mixtures and piecewise-constant shapes on a small floor).

Every draw uses numpy.random.default_rng(SeedSequence([config_id, index]))
and draws rho0 before rho1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "rng_for", "nodes", "gaussian_mixture", "shapes_density", "normalise",
    "pair_gauss3", "pair_shift8", "pair_shapes", "pair_uneven", "served_requests",
    "stripes_pair", "translated_bump_pair", "integer_mass_pair", "random_pair",
    "Request", "random_pair_nd", "pair_gauss_3d",
]

CONFIG_GAUSS3 = 1      # single pair, n=64, 3 isotropic Gaussians
CONFIG_SHIFT8 = 2      # single pair, n=512, 8 anisotropic Gaussians and a shifted copy
CONFIG_SHAPES = 3      # uniform batch, n=256, unions of rectangles and disks
CONFIG_UNEVEN = 4      # uneven batch, n in {64,128,256,512}
CONFIG_SERVED = 5      # served stream, n in {128..2048}
CONFIG_GAUSS_3D = 6    # d = 3 pairs: isotropic Gaussian mixtures on the unit cube


def rng_for(config_id: int, index: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(config_id), int(index)]))


def nodes(n: int):
    """Coordinates (x1, x2) of the (n+1)^2 vertex nodes, each of shape (n+1, n+1)."""
    t = np.arange(n + 1, dtype=np.float64) / n
    return np.meshgrid(t, t, indexing="ij")


def normalise(g: np.ndarray) -> np.ndarray:
    g = np.asarray(g, dtype=np.float64)
    return g / g.sum()


def gaussian_mixture(n, centres, covs, floor):
    """Node masses of (1/K) sum_k N(x; c_k, S_k) + floor, normalised to sum 1."""
    x1, x2 = nodes(n)
    g = np.zeros_like(x1)
    K = len(centres)
    for c, S in zip(centres, covs):
        S = np.asarray(S, dtype=np.float64)
        Si = np.linalg.inv(S)
        d1 = x1 - c[0]
        d2 = x2 - c[1]
        q = Si[0, 0] * d1 * d1 + 2.0 * Si[0, 1] * d1 * d2 + Si[1, 1] * d2 * d2
        g += np.exp(-0.5 * q) / (2.0 * math.pi * math.sqrt(np.linalg.det(S))) / K
    return normalise(g + floor)


def _iso_mixture_params(rng, K):
    centres = rng.uniform(0.2, 0.8, size=(K, 2))
    sig = rng.uniform(0.05, 0.15, size=K)
    covs = [np.eye(2) * s * s for s in sig]
    return centres, covs


def _aniso_mixture_params(rng, K):
    centres = rng.uniform(0.2, 0.8, size=(K, 2))
    covs = []
    for _ in range(K):
        s1, s2 = rng.uniform(0.05, 0.15, size=2)
        th = rng.uniform(0.0, math.pi)
        R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
        covs.append(R @ np.diag([s1 * s1, s2 * s2]) @ R.T)
    return centres, covs


def shapes_density(n, rng, floor=1e-4):
    """Value 1 on a union of 1..5 axis-aligned rectangles and disks, plus a floor."""
    x1, x2 = nodes(n)
    g = np.zeros_like(x1)
    count = int(rng.integers(1, 6))
    for _ in range(count):
        c = rng.uniform(0.1, 0.9, size=2)
        if rng.uniform() < 0.5:
            a, b = rng.uniform(0.02, 0.2, size=2)
            inside = (np.abs(x1 - c[0]) <= a) & (np.abs(x2 - c[1]) <= b)
        else:
            r = rng.uniform(0.02, 0.2)
            inside = (x1 - c[0]) ** 2 + (x2 - c[1]) ** 2 <= r * r
        g[inside] = 1.0
    return normalise(g + floor)


def pair_gauss3(index: int, n: int = 64, K: int = 3, config_id: int = CONFIG_GAUSS3):
    """Two independent mixtures of K isotropic Gaussians, floor 1e-3."""
    rng = rng_for(config_id, index)
    c0, S0 = _iso_mixture_params(rng, K)
    p0 = gaussian_mixture(n, c0, S0, 1e-3)
    c1, S1 = _iso_mixture_params(rng, K)
    p1 = gaussian_mixture(n, c1, S1, 1e-3)
    return p0, p1


def pair_shift8(index: int, n: int = 512, K: int = 8):
    """Mixture of K anisotropic Gaussians and the same mixture translated by s.

    |s| ~ U[0, 0.1] with a uniform angle; returns (p0, p1, s).
    """
    rng = rng_for(CONFIG_SHIFT8, index)
    c, S = _aniso_mixture_params(rng, K)
    ang = rng.uniform(0.0, 2.0 * math.pi)
    ln = rng.uniform(0.0, 0.1)
    s = np.array([ln * math.cos(ang), ln * math.sin(ang)])
    p0 = gaussian_mixture(n, c, S, 1e-3)
    p1 = gaussian_mixture(n, c + s, S, 1e-3)
    return p0, p1, s


def pair_shapes(index: int, n: int = 256):
    rng = rng_for(CONFIG_SHAPES, index)
    p0 = shapes_density(n, rng)
    p1 = shapes_density(n, rng)
    return p0, p1


UNEVEN_SIZES = (64, 128, 256, 512)
UNEVEN_PROBS = (0.4, 0.3, 0.2, 0.1)


def pair_uneven(index: int):
    """Uneven-batch pair: returns (n, metric, p0, p1); metric 1 for even index, else 2."""
    rng = rng_for(CONFIG_UNEVEN, index)
    n = int(rng.choice(UNEVEN_SIZES, p=UNEVEN_PROBS))
    K = int(rng.integers(2, 11))
    c0, S0 = _iso_mixture_params(rng, K)
    p0 = gaussian_mixture(n, c0, S0, 1e-3)
    c1, S1 = _iso_mixture_params(rng, K)
    p1 = gaussian_mixture(n, c1, S1, 1e-3)
    metric = 1 if index % 2 == 0 else 2
    return n, metric, p0, p1


@dataclass
class Request:
    index: int
    arrival: float      # seconds from stream start
    n: int
    kind: str           # "mixture" or "shapes"


SERVED_SIZES = (128, 256, 512, 1024, 2048)


def served_requests(count: int, rate: float = 200.0, sizes=SERVED_SIZES):
    """Poisson arrival schedule: exponential gaps at `rate` per second."""
    rng = rng_for(CONFIG_SERVED, 0)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps)
    out = []
    for i in range(count):
        n = int(rng.choice(sizes))
        kind = "mixture" if rng.uniform() < 0.5 else "shapes"
        out.append(Request(i, float(t[i]), n, kind))
    return out


def served_pair(req: Request):
    rng = rng_for(CONFIG_SERVED, 1 + req.index)
    if req.kind == "mixture":
        K = int(rng.integers(2, 11))
        c0, S0 = _iso_mixture_params(rng, K)
        c1, S1 = _iso_mixture_params(rng, K)
        return (gaussian_mixture(req.n, c0, S0, 1e-3), gaussian_mixture(req.n, c1, S1, 1e-3))
    return shapes_density(req.n, rng), shapes_density(req.n, rng)


# ---- structured inputs with known answers (used by the oracle's pins) ----

def stripes_pair(n: int, seed: int = 0):
    """Densities constant along x2 (varying along x1 only), each summing to 1."""
    rng = np.random.default_rng(seed)
    a0 = rng.uniform(0.05, 1.0, size=n + 1)
    a1 = rng.uniform(0.05, 1.0, size=n + 1)
    p0 = np.repeat(a0[:, None], n + 1, axis=1)
    p1 = np.repeat(a1[:, None], n + 1, axis=1)
    return normalise(p0), normalise(p1)


def translated_bump_pair(n: int, shift, floor_mass: float = 0.0, seed: int = 0):
    """A random bump and the same bump moved by a whole number of grid steps.

    shift = (k1, k2) in grid steps.  The bump has support at least
    |k| steps away from every wall before and after the move.  A uniform floor
    carrying `floor_mass` of the total mass is shared by both densities.
    Returns (p0, p1, bump_mass).
    """
    rng = np.random.default_rng(seed)
    k1, k2 = int(shift[0]), int(shift[1])
    lo1, hi1 = max(0, -k1) + 1, n - max(0, k1) - 1
    lo2, hi2 = max(0, -k2) + 1, n - max(0, k2) - 1
    if hi1 - lo1 < 2 or hi2 - lo2 < 2:
        raise ValueError("shift too large for grid")
    w1 = int(rng.integers(1, max(2, (hi1 - lo1) // 2)))
    w2 = int(rng.integers(1, max(2, (hi2 - lo2) // 2)))
    a1 = int(rng.integers(lo1, hi1 - w1 + 1))
    a2 = int(rng.integers(lo2, hi2 - w2 + 1))
    bump = np.zeros((n + 1, n + 1))
    bump[a1:a1 + w1 + 1, a2:a2 + w2 + 1] = rng.uniform(0.2, 1.0, size=(w1 + 1, w2 + 1))
    bump /= bump.sum()
    moved = np.zeros_like(bump)
    moved[a1 + k1:a1 + k1 + w1 + 1, a2 + k2:a2 + k2 + w2 + 1] = bump[a1:a1 + w1 + 1, a2:a2 + w2 + 1]
    bump_mass = 1.0 - floor_mass
    flo = np.full_like(bump, floor_mass / bump.size)
    return bump * bump_mass + flo, moved * bump_mass + flo, bump_mass


def integer_mass_pair(n: int, total: int, seed: int = 0):
    """Two integer mass vectors on (n+1)^2 nodes, each summing to `total`."""
    rng = np.random.default_rng(seed)
    N = (n + 1) * (n + 1)
    a = np.bincount(rng.integers(0, N, size=total), minlength=N).reshape(n + 1, n + 1)
    b = np.bincount(rng.integers(0, N, size=total), minlength=N).reshape(n + 1, n + 1)
    return a.astype(np.int64), b.astype(np.int64)


def random_pair(n: int, seed: int = 0, floor: float = 0.05):
    """Smooth-free random positive masses (for small parity cases)."""
    rng = np.random.default_rng(seed)
    p0 = rng.uniform(0.0, 1.0, size=(n + 1, n + 1)) + floor
    p1 = rng.uniform(0.0, 1.0, size=(n + 1, n + 1)) + floor
    return normalise(p0), normalise(p1)


def random_pair_nd(n: int, d: int, seed: int = 0, floor: float = 0.05):
    """Random positive masses on the (n+1)^d vertex grid of [0,1]^d."""
    rng = np.random.default_rng(seed)
    p0 = rng.uniform(0.0, 1.0, size=(n + 1,) * d) + floor
    p1 = rng.uniform(0.0, 1.0, size=(n + 1,) * d) + floor
    return normalise(p0), normalise(p1)


def pair_gauss_3d(index: int, n: int = 64, K: int = 3, floor: float = 1e-3):
    """d = 3 pair: each density a mixture of K isotropic Gaussians on the unit
    cube (centres U[0.2, 0.8]^3, sigma U[0.05, 0.15]) plus a floor, node
    masses of shape (n+1, n+1, n+1), index [i1, i2, i3] with i3 contiguous."""
    rng = rng_for(CONFIG_GAUSS_3D, index)
    t = np.arange(n + 1, dtype=np.float64) / n
    x = np.meshgrid(t, t, t, indexing="ij")
    out = []
    for _ in range(2):
        c = rng.uniform(0.2, 0.8, size=(K, 3))
        sig = rng.uniform(0.05, 0.15, size=K)
        g = np.zeros_like(x[0])
        for k in range(K):
            r2 = sum((x[a] - c[k, a]) ** 2 for a in range(3))
            g += np.exp(-0.5 * r2 / sig[k] ** 2) / ((2 * math.pi) ** 1.5 * sig[k] ** 3) / K
        out.append(normalise(g + floor))
    return out[0], out[1]

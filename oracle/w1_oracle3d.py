"""Plain FP64 implementation of the method in d dimensions (the paper states
it for general d: Sec. 2.2 and Sec. 3.3), used for d = 3.  Test
infrastructure only, like the d = 2 module.

Every function takes node arrays of shape (n+1,)*d (index [i1, ..., id], i1
along x1) and fluxes as tuples of d such arrays; d is read from the arrays,
so the same code run at d = 2 must reproduce the d = 2 module (a pin).
The readings are those of the d = 2 module: R1 (divergence case at x_i = 1),
R2 (A* = minus the forward difference), R3 (Neumann Laplacian by DCT-II),
R4 (Algorithm 1 steps 1/(2||A||) with the Gershgorin bound 2 sqrt(d)/h),
R6 (coarse densities D^-1 P^T, renormalised), R7 (flux interpolation tie
to x_i - h_l), R8 (zero-mean potential), R9 (stop rules).
"""
from __future__ import annotations

import math
import time

import numpy as np
import scipy.fft

__all__ = [
    "div", "div_adj", "grad_fwd", "pointwise_norm", "flux_cost", "inner_h", "shrink", "primal_residual",
    "project_dual_ball", "poisson_neumann", "norm_A_bound", "plain_step_sizes", "pd_step",
    "prolong_potential", "prolong_flux", "restrict_density", "prepare_levels", "kkt_plain",
    "evaluate_plain", "solve_plain", "prox_step", "potential_from_dual", "kkt_prox", "evaluate", "solve_prox",
]


def _shift_down(a, ax):
    """b[..., x_ax, ...] = a[..., x_ax + 1, ...], 0 past the last node."""
    b = np.zeros_like(a)
    src = [slice(None)] * a.ndim
    dst = [slice(None)] * a.ndim
    src[ax] = slice(1, None)
    dst[ax] = slice(None, -1)
    b[tuple(dst)] = a[tuple(src)]
    return b


def _last(a, ax):
    """Index tuple of the last node along axis ax."""
    s = [slice(None)] * a.ndim
    s[ax] = -1
    return tuple(s)


# --------------------------------------------------------------------------
# Sec. 2.2: the divergence D_{h,i} summed over the d axes, its adjoint, and
# the norms and inner products on the grid.
# --------------------------------------------------------------------------

def div(m, h):
    """A_h m = sum_i D_{h,i} m: m_i(x)/h at x_i = 0, (m_i(x) - m_i(x - h e_i))/h
    inside, -m_i(x - h e_i)/h at x_i = 1 (R1); m_i on the last node of axis i
    never enters."""
    out = np.zeros(m[0].shape)
    for ax, mi in enumerate(m):
        mi = mi.copy()
        mi[_last(mi, ax)] = 0.0
        prev = np.zeros_like(mi)
        src = [slice(None)] * mi.ndim
        dst = [slice(None)] * mi.ndim
        src[ax] = slice(None, -1)
        dst[ax] = slice(1, None)
        prev[tuple(dst)] = mi[tuple(src)]
        out += mi - prev
    return out / h


def div_adj(phi, h):
    """A_h^* phi (R2): component i is (phi(x) - phi(x + h e_i))/h, 0 at x_i = 1."""
    out = []
    for ax in range(phi.ndim):
        a = (phi - _shift_down(phi, ax)) / h
        a[_last(a, ax)] = 0.0
        out.append(a)
    return tuple(out)


def grad_fwd(phi, h):
    return tuple(-a for a in div_adj(phi, h))


def pointwise_norm(v, p):
    """||v(x)||_p at every node, p in {1, 2, inf}."""
    A = np.stack([np.abs(x) for x in v])
    if p == 1:
        return A.sum(axis=0)
    if p == 2:
        return np.sqrt((A * A).sum(axis=0))
    if p == math.inf:
        return A.max(axis=0)
    raise ValueError("p must be 1, 2 or inf")


def dual_exponent(p):
    return {1: math.inf, 2: 2, math.inf: 1}[p]


def inner_h(a, b, h):
    """<a, b>_h = sum a b h^d; tuples are summed component by component."""
    if isinstance(a, tuple):
        return sum(inner_h(x, y, h) for x, y in zip(a, b))
    return float(np.sum(a * b) * h ** a.ndim)


def flux_cost(m, h, p):
    """f(m_h) = sum ||m_h(x)||_p h^d (eq. (opt_flux_dis))."""
    return float(np.sum(pointwise_norm(m, p)) * h ** m[0].ndim)


# --------------------------------------------------------------------------
# Proximal maps with d components per node.
# --------------------------------------------------------------------------

def _project_l1_ball(v, r):
    """Projection of each node's d-vector onto {||y||_1 <= r}: the sort and
    threshold method of Duchi et al. (2008) named in Sec. 4.2."""
    V = np.stack(v, axis=-1)
    A = np.abs(V)
    u = -np.sort(-A, axis=-1)
    c = np.cumsum(u, axis=-1)
    j = np.arange(1, V.shape[-1] + 1, dtype=np.float64)
    k = np.maximum(np.sum(u > (c - r) / j, axis=-1), 1)
    theta = (np.take_along_axis(c, (k - 1)[..., None], axis=-1)[..., 0] - r) / k
    Y = np.sign(V) * np.maximum(A - theta[..., None], 0.0)
    Y = np.where((A.sum(axis=-1) <= r)[..., None], V, Y)
    return tuple(Y[..., i] for i in range(V.shape[-1]))


def shrink(v, mu, p):
    """argmin_m ||m||_p + ||m - v||^2/(2 mu) per node (the flux update of eq.
    (primaldual)); p = inf by the Moreau decomposition of Sec. 4.2."""
    if p == 1:
        return tuple(np.sign(x) * np.maximum(np.abs(x) - mu, 0.0) for x in v)
    if p == 2:
        nv = pointwise_norm(v, 2)
        with np.errstate(divide="ignore", invalid="ignore"):
            s = np.where(nv > mu, 1.0 - mu / np.where(nv > 0, nv, 1.0), 0.0)
        return tuple(x * s for x in v)
    if p == math.inf:
        q = _project_l1_ball(v, mu)
        return tuple(x - y for x, y in zip(v, q))
    raise ValueError("p must be 1, 2 or inf")


def project_dual_ball(w, p):
    """Projection onto {||.||_q <= 1}, q dual to p."""
    if p == 1:
        return tuple(np.clip(x, -1.0, 1.0) for x in w)
    if p == 2:
        s = 1.0 / np.maximum(1.0, pointwise_norm(w, 2))
        return tuple(x * s for x in w)
    if p == math.inf:
        return _project_l1_ball(w, 1.0)
    raise ValueError("p must be 1, 2 or inf")


# --------------------------------------------------------------------------
# The node Laplacian A A* (R3) in d dimensions.
# --------------------------------------------------------------------------

def laplacian_eigenvalues(n, h, d):
    """lam_k = (4/h^2) sum_i sin^2(pi k_i / (2N)), N = n + 1."""
    N = n + 1
    s = np.sin(np.pi * np.arange(N) / (2.0 * N)) ** 2 * 4.0 / (h * h)
    lam = np.zeros((N,) * d)
    for ax in range(d):
        shape = [1] * d
        shape[ax] = N
        lam = lam + s.reshape(shape)
    return lam


def poisson_neumann(r, h):
    """u = (A A*)^{-1} r on the zero-mean subspace (constant mode 0)."""
    n = r.shape[0] - 1
    lam = laplacian_eigenvalues(n, h, r.ndim)
    rh = scipy.fft.dctn(r, type=2, norm="ortho")
    z = (0,) * r.ndim
    lam[z] = 1.0
    uh = rh / lam
    uh[z] = 0.0
    return scipy.fft.idctn(uh, type=2, norm="ortho")


def norm_A_bound(h, d):
    """Gershgorin bound ||A_h|| <= 2 sqrt(d) / h."""
    return 2.0 * math.sqrt(d) / h


def plain_step_sizes(h, d, scale=0.5):
    """R4: mu = tau = scale / ||A||, ||A|| by its Gershgorin bound."""
    s = scale / norm_A_bound(h, d)
    return s, s


# --------------------------------------------------------------------------
# Algorithm 1 (eq. (primaldual)) and R^k (eq. (pd_stop)).
# --------------------------------------------------------------------------

def pd_step(m, phi, rho, h, mu, tau, p):
    """One iteration of eq. (primaldual); returns (m', phi', R^k)."""
    g = grad_fwd(phi, h)
    n_ = shrink(tuple(mi + mu * gi for mi, gi in zip(m, g)), mu, p)
    b = tuple(2.0 * ni - mi for ni, mi in zip(n_, m))
    phin = phi + tau * (div(b, h) - rho)
    dm = tuple(ni - mi for ni, mi in zip(n_, m))
    dp = phin - phi
    R = inner_h(dm, dm, h) / mu + inner_h(dp, dp, h) / tau - 2.0 * inner_h(dp, div(dm, h), h)
    return n_, phin, R


# --------------------------------------------------------------------------
# Algorithm 2 (eq. (pdhg)), G^k (eq. (pdhg_stop)) and Appendix B.
# --------------------------------------------------------------------------

def prox_step(m, w, wb, rho, h, mu, tau, p):
    """One iteration of eq. (pdhg) with vphi^k = w and the extrapolated
    vphi-bar^k = wb (tuples of d arrays).  Returns (m', w', wb', G^k)."""
    v = tuple(mi - mu * bi for mi, bi in zip(m, wb))
    u = poisson_neumann(div(v, h) - rho, h)
    a = div_adj(u, h)
    n_ = tuple(vi - ai for vi, ai in zip(v, a))           # projection onto {A m = rho}
    q = project_dual_ball(tuple(wi + tau * ni for wi, ni in zip(w, n_)), p)
    qb = tuple(2.0 * qi - wi for qi, wi in zip(q, w))
    d = tuple(ni - mi for ni, mi in zip(n_, m))
    e = tuple(qi - wi for qi, wi in zip(q, w))
    G = inner_h(d, d, h) / mu + inner_h(e, e, h) / tau + 2.0 * inner_h(e, d, h)
    return n_, q, qb, G


def potential_from_dual(w, h):
    """Appendix B: psi = (A A*)^{-1} A vphi, zero-mean (R8)."""
    return poisson_neumann(div(w, h), h)


def kkt_prox(m, w, rho, h, p):
    """The normalised KKT residual of an Algorithm 2 iterate with the
    potential of Appendix B: D = <psi, rho>_h."""
    psi = potential_from_dual(w, h)
    P = flux_cost(m, h, p)
    r_pri = primal_residual(m, rho, h) / max(P, 1e-300)
    r_dual, _ = _dual_excess(psi, h, p)
    D = inner_h(psi, rho, h)
    return max(r_pri, r_dual, abs(P - D) / max(abs(P), abs(D), 1e-300)), P, D


def evaluate(m, psi, rho, h, p):
    """The certificate for a flux m and usual-sign potential psi: P = f(m),
    D = <psi, rho>_h, lo = D / max(1, max ||grad psi||_q), hi = f of the flux
    made feasible by the minimum-norm correction."""
    res = div(m, h) - rho
    corr = div_adj(poisson_neumann(res, h), h)
    P = flux_cost(m, h, p)
    D = inner_h(psi, rho, h)
    _, gmax = _dual_excess(psi, h, p)
    hi = flux_cost(tuple(mi - ci for mi, ci in zip(m, corr)), h, p)
    return {"P": P, "D": D, "lo": D / max(1.0, gmax), "hi": hi, "grad_max": gmax}


def solve_prox(p0, p1, n, L=1, p=1, stop="fpr", tol=1e-4, alpha=-1.0, max_iters=20000, check_every=1,
               step_scale=0.5):
    """Algorithm 4 in d dimensions: mu = tau = step_scale (R4), vphi-bar =
    vphi at every level start (R5), level 1 from zero, the others from eq.
    (inter_m) for both m and vphi; G^k (stop = "fpr") or the normalised KKT
    residual (stop = "kkt") against tol (h_l/h)^alpha."""
    d = np.asarray(p0).ndim
    sides = level_sides(n, L)
    rhos = prepare_levels(p0, p1, n, L)
    tols = [tol * float(1 << (L - l)) ** alpha for l in range(1, L + 1)]
    out = {"iters": [], "measure": [], "level_w1": [], "status": "ok", "level_seconds": []}
    m = w = None
    mu = tau = step_scale
    for l in range(L):
        nl = sides[l]
        h = 1.0 / nl
        rho = rhos[l]
        t0 = time.perf_counter()
        if m is None:
            m = tuple(np.zeros((nl + 1,) * d) for _ in range(d))
            w = tuple(np.zeros((nl + 1,) * d) for _ in range(d))
        else:
            m = prolong_flux(m)
            w = prolong_flux(w)
        wb = tuple(x.copy() for x in w)
        k = 0
        while True:
            m, w, wb, G = prox_step(m, w, wb, rho, h, mu, tau, p)
            k += 1
            if k % check_every == 0 or k >= max_iters:
                meas = G if stop == "fpr" else kkt_prox(m, w, rho, h, p)[0]
                if meas <= tols[l]:
                    break
                if k >= max_iters:
                    out["status"] = "maxiter"
                    break
        out["iters"].append(k)
        out["measure"].append(float(meas))
        out["level_w1"].append(flux_cost(m, h, p))
        out["level_seconds"].append(time.perf_counter() - t0)
    h = 1.0 / n
    psi = potential_from_dual(w, h)
    ev = evaluate(m, psi, rhos[-1], h, p)
    out.update({"w1": ev["P"], "dual": ev["D"], "lo": ev["lo"], "hi": ev["hi"], "m": m, "vphi": w, "psi": psi,
                "rho": rhos[-1], "tolerances": tols})
    return out


# --------------------------------------------------------------------------
# Sec. 3.3 in d dimensions: both interpolations are products of 1-D factors,
# the potential one linear along every axis (eq. (inter_phi)), the flux one
# nearest-neighbour along the component's own axis (tie to x_i - h_l, R7)
# and linear across (eq. (inter_m)).
# --------------------------------------------------------------------------

def _linear_1d(nc):
    P = np.zeros((2 * nc + 1, nc + 1))
    for I in range(2 * nc + 1):
        if I % 2 == 0:
            P[I, I // 2] = 1.0
        else:
            P[I, (I - 1) // 2] = 0.5
            P[I, (I + 1) // 2] = 0.5
    return P


def _nearest_1d(nc):
    P = np.zeros((2 * nc + 1, nc + 1))
    for I in range(2 * nc + 1):
        P[I, I // 2] = 1.0
    return P


def _apply(M, a, ax):
    return np.moveaxis(np.tensordot(M, a, axes=(1, ax)), 0, ax)


def prolong_potential(c):
    nc = c.shape[0] - 1
    P = _linear_1d(nc)
    f = c
    for ax in range(c.ndim):
        f = _apply(P, f, ax)
    return f


def prolong_flux(cm):
    nc = cm[0].shape[0] - 1
    Pl, Pn = _linear_1d(nc), _nearest_1d(nc)
    out = []
    for i, ci in enumerate(cm):
        f = ci
        for ax in range(ci.ndim):
            f = _apply(Pn if ax == i else Pl, f, ax)
        f = f.copy()
        f[_last(f, i)] = 0.0
        out.append(f)
    return tuple(out)


def restrict_density(f):
    """R6: D^-1 P^T f with P the potential interpolation (per axis)."""
    nf = f.shape[0] - 1
    P = _linear_1d(nf // 2)
    w = P.T @ np.ones(nf + 1)
    c = f
    for ax in range(f.ndim):
        c = _apply(P.T, c, ax)
    for ax in range(f.ndim):
        shape = [1] * f.ndim
        shape[ax] = w.size
        c = c / w.reshape(shape)
    return c


def level_sides(n, L):
    if L < 1 or n % (1 << (L - 1)) != 0:
        raise ValueError("n must be divisible by 2^(L-1)")
    return [n >> (L - l) for l in range(1, L + 1)]


def prepare_levels(p0, p1, n, L):
    """Node masses -> rho_l per level (finest last): rho^k = p^k / h^d after
    renormalising to unit mass, coarse levels by R6, rho_l zero-sum."""
    p0 = np.asarray(p0, dtype=np.float64)
    p1 = np.asarray(p1, dtype=np.float64)
    d = p0.ndim
    if p0.shape != (n + 1,) * d or p1.shape != p0.shape:
        raise ValueError("masses must have shape (n+1,)*d")
    if not (np.all(np.isfinite(p0)) and np.all(np.isfinite(p1))) or np.any(p0 < 0) or np.any(p1 < 0):
        raise ValueError("masses must be finite and non-negative")
    s0, s1 = p0.sum(), p1.sum()
    if s0 <= 0 or abs(s0 - s1) > 1e-9 * s0:
        raise ValueError("masses do not balance")
    sides = level_sides(n, L)
    h = 1.0 / n
    r0 = [None] * L
    r1 = [None] * L
    r0[-1] = p0 / s0 / h ** d
    r1[-1] = p1 / s1 / h ** d
    for l in range(L - 2, -1, -1):
        hl = 1.0 / sides[l]
        for arr in (r0, r1):
            c = restrict_density(arr[l + 1])
            arr[l] = c / (c.sum() * hl ** d)
    rhos = []
    for l in range(L):
        r = r0[l] - r1[l]
        rhos.append(r - r.mean())
    return rhos


# --------------------------------------------------------------------------
# Stop measures and the evaluator (R9), Algorithm 3.
# --------------------------------------------------------------------------

def _dual_excess(psi, h, p):
    gn = pointwise_norm(grad_fwd(psi, h), dual_exponent(p))
    ex = np.maximum(gn - 1.0, 0.0)
    return math.sqrt(float(np.sum(ex * ex)) * h ** psi.ndim), float(gn.max())


def primal_residual(m, rho, h):
    """||A*(A A*)^{-1}(A m - rho)||_{L^2_h}: the norm of the minimum-norm
    flux correction that makes m feasible."""
    corr = div_adj(poisson_neumann(div(m, h) - rho, h), h)
    return math.sqrt(inner_h(corr, corr, h))


def kkt_plain(m, phi, rho, h, p):
    """max(||A*(A A*)^{-1}(A m - rho)|| / P, RMS Lipschitz excess of -phi,
    relative gap) with P = f(m), D = -<phi, rho>_h."""
    P = flux_cost(m, h, p)
    r_pri = primal_residual(m, rho, h) / max(P, 1e-300)
    r_dual, _ = _dual_excess(-phi, h, p)
    D = -inner_h(phi, rho, h)
    return max(r_pri, r_dual, abs(P - D) / max(abs(P), abs(D), 1e-300)), P, D


def evaluate_plain(m, phi, rho, h, p):
    """P = f(m), D = -<phi, rho>_h, lo = D / max(1, max ||grad(-phi)||_q)
    (a feasible potential's dual value, <= W1_h), hi = f of the flux made
    feasible by the minimum-norm correction A*(A A*)^{-1}(A m - rho)."""
    res = div(m, h) - rho
    corr = div_adj(poisson_neumann(res, h), h)
    P = flux_cost(m, h, p)
    D = -inner_h(phi, rho, h)
    _, gmax = _dual_excess(-phi, h, p)
    hi = flux_cost(tuple(mi - ci for mi, ci in zip(m, corr)), h, p)
    return {"P": P, "D": D, "lo": D / max(1.0, gmax), "hi": hi, "grad_max": gmax}


def solve_plain(p0, p1, n, L=1, p=1, stop="fpr", tol=1e-6, alpha=-1.0, max_iters=20000, check_every=1,
                step_scale=0.5):
    """Algorithm 3 in d dimensions: level l stops when R^k (stop = "fpr") or
    the normalised KKT residual (stop = "kkt") is at most
    tol (h_l/h)^alpha, checked every `check_every` iterations and at the
    cap; level 1 starts from zero, the others from eq. (inter_phi)/(inter_m)."""
    d = np.asarray(p0).ndim
    sides = level_sides(n, L)
    rhos = prepare_levels(p0, p1, n, L)
    tols = [tol * float(1 << (L - l)) ** alpha for l in range(1, L + 1)]
    out = {"iters": [], "measure": [], "level_w1": [], "status": "ok", "level_seconds": []}
    m = phi = None
    for l in range(L):
        nl = sides[l]
        h = 1.0 / nl
        rho = rhos[l]
        t0 = time.perf_counter()
        mu, tau = plain_step_sizes(h, d, step_scale)
        if m is None:
            m = tuple(np.zeros((nl + 1,) * d) for _ in range(d))
            phi = np.zeros((nl + 1,) * d)
        else:
            m = prolong_flux(m)
            phi = prolong_potential(phi)
        k = 0
        while True:
            m, phi, R = pd_step(m, phi, rho, h, mu, tau, p)
            k += 1
            if k % check_every == 0 or k >= max_iters:
                meas = R if stop == "fpr" else kkt_plain(m, phi, rho, h, p)[0]
                if meas <= tols[l]:
                    break
                if k >= max_iters:
                    out["status"] = "maxiter"
                    break
        out["iters"].append(k)
        out["measure"].append(float(meas))
        out["level_w1"].append(flux_cost(m, h, p))
        out["level_seconds"].append(time.perf_counter() - t0)
    h = 1.0 / n
    ev = evaluate_plain(m, phi, rhos[-1], h, p)
    out.update({"w1": ev["P"], "dual": ev["D"], "lo": ev["lo"], "hi": ev["hi"], "m": m, "phi": phi,
                "rho": rhos[-1], "tolerances": tols})
    return out

"""Plain FP64 implementation of the multilevel W1 solver, one function per
passage of the paper (arXiv 1810.00118).  Test infrastructure only: see the
package docstring.

Notation follows the paper.  d = 2, Omega = [0,1]^2, a level of side n has
h = 1/n and (n+1)^2 vertex nodes, arrays are indexed [i, j] with i along x1.

* m = (m1, m2): flux.  m1[i, j] lives on the edge (i,j)->(i+1,j) and
  m2[i, j] on (i,j)->(i,j+1); m1[n, :] and m2[:, n] never enter the
  divergence and are identically zero.
* phi: node potential of Algorithm 1 (the paper's sign: W1 = -<phi, rho>_h).
* vphi = (vphi1, vphi2): edge-valued dual variable of Algorithm 2.
* psi: potential of Appendix B, psi = (A A*)^{-1} A vphi; W1 = +<psi, rho>_h.

Readings of the paper taken here (each one is listed in the design notes):
  R1 the divergence's third case applies at x_i = 1 (printed as x_i > 1);
  R2 A* is minus the forward difference, fixed by adjointness under <.,.>_h;
  R3 "((A_h)*A_h)^{-1}" in the projection of Algorithm 2 is the node
     Laplacian (A A*)^{-1}, inverted with a DCT-II (Neumann conditions,
     zero normal flux), the constant mode set to zero;
  R4 step sizes: Algorithm 1 mu = tau = 1/(2||A||) with the Gershgorin bound
     ||A|| <= 2 sqrt(2)/h; Algorithm 2 mu = tau = 1/2;
  R5 in Algorithm 2 the extrapolated dual starts equal to the dual at every
     level start;
  R6 coarse densities come from normalised full weighting (D^-1 P^T, with P
     the potential interpolation) and are renormalised to unit mass;
  R7 the nearest-neighbour tie in the flux interpolation goes to the coarse
     edge that contains the fine edge (coordinate x_i - h_l);
  R8 the potential is reported zero-mean;
  R9 stopping: the paper's fixed-point residual (R^k or G^k) against
     eps_l, or a normalised KKT residual against tol_l; both on a cadence.
     The KKT residual (the paper defines none) is the largest of the
     relative distance of m to {A m = rho} (the norm of the minimum-norm
     correction over f(m)), the RMS Lipschitz excess of the potential and
     the relative primal-dual gap.
"""
from __future__ import annotations

import math
import time

import numpy as np
import scipy.fft

__all__ = [
    "div", "div_adj", "grad_fwd", "pointwise_norm", "inner_h", "flux_cost",
    "shrink", "project_dual_ball", "laplacian_eigenvalues", "poisson_neumann",
    "norm_A_bound", "norm_A_exact", "plain_step_sizes", "prox_step_sizes",
    "pd_step", "prox_step", "potential_from_dual",
    "prolong_potential", "prolong_flux", "restrict_density",
    "level_sides", "level_tolerances", "paper_stop_tolerance",
    "prepare_levels", "min_norm_correction", "primal_residual", "kkt_plain", "kkt_prox", "evaluate", "solve",
]


# --------------------------------------------------------------------------
# Discrete model, Sec. 2.2 ("Discretization") and the norms / inner products
# defined just before Sec. 3.
# --------------------------------------------------------------------------

def div(m1, m2, h):
    """A_h m: the discrete divergence of Sec. 2.2.

    Case by case per axis: m_i(x)/h at x_i = 0, (m_i(x) - m_i(x - h e_i))/h
    inside, -m_i(x - h e_i)/h at x_i = 1 (reading R1).  The flux component on
    the last node of its own axis is not used.
    """
    out = np.zeros(m1.shape, dtype=np.float64)
    out[:-1, :] += m1[:-1, :]      # + m_1(x)/h        where x_1 < 1
    out[1:, :] -= m1[:-1, :]       # - m_1(x - h e_1)/h where x_1 > 0
    out[:, :-1] += m2[:, :-1]
    out[:, 1:] -= m2[:, :-1]
    return out / h


def div_adj(phi, h):
    """A_h^* phi, the adjoint of div under <.,.>_h (reading R2).

    (A* phi)_1[i, j] = (phi[i, j] - phi[i+1, j]) / h for i < n and 0 at i = n;
    likewise for component 2 along j.
    """
    a1 = np.zeros_like(phi, dtype=np.float64)
    a2 = np.zeros_like(phi, dtype=np.float64)
    a1[:-1, :] = (phi[:-1, :] - phi[1:, :]) / h
    a2[:, :-1] = (phi[:, :-1] - phi[:, 1:]) / h
    return a1, a2


def grad_fwd(phi, h):
    """Forward-difference gradient, equal to -A_h^* phi."""
    a1, a2 = div_adj(phi, h)
    return -a1, -a2


def pointwise_norm(v1, v2, p):
    """||(v1(x), v2(x))||_p at every node, p in {1, 2, inf}."""
    if p == 1:
        return np.abs(v1) + np.abs(v2)
    if p == 2:
        return np.sqrt(v1 * v1 + v2 * v2)
    if p == math.inf:
        return np.maximum(np.abs(v1), np.abs(v2))
    raise ValueError("p must be 1, 2 or inf")


def dual_exponent(p):
    """q with 1/p + 1/q = 1 (Sec. 2.1)."""
    return {1: math.inf, 2: 2, math.inf: 1}[p]


def inner_h(a, b, h):
    """<a, b>_h = sum a*b h^d (d = 2); tuples are summed component-wise."""
    if isinstance(a, tuple):
        return sum(inner_h(x, y, h) for x, y in zip(a, b))
    return float(np.sum(a * b) * h * h)


def flux_cost(m1, m2, h, p):
    """f(m_h) = sum_x ||m_h(x)||_p h^d, the objective of eq. (opt_flux_dis)."""
    return float(np.sum(pointwise_norm(m1, m2, p)) * h * h)


# --------------------------------------------------------------------------
# Proximal maps.  Algorithm 1's flux update is the prox of mu*||.||_p per node
# (the argmin in eq. (primaldual)); Algorithm 2's dual update is the
# projection onto the dual-norm unit ball, because f* is the indicator of
# {||vphi(x)||_q <= 1} (the conjugate defined before eq. (minmax_pdhg)).
# --------------------------------------------------------------------------

def _project_l1_ball(v1, v2, r):
    """Euclidean projection of every node's (v1, v2) onto {|y1| + |y2| <= r}.

    The sort-and-threshold method of Duchi et al. (2008), which the paper
    names for the p = inf case (Sec. 4.2, complexity of Algorithms 1 and 3),
    over the d = 2 components of a node: with |v| sorted decreasingly into u
    and partial sums c_j, k is the largest j with u_j > (c_j - r)/j, the
    threshold is theta = (c_k - r)/k and y = sign(v) max(|v| - theta, 0).
    Vectors already in the ball are returned unchanged.
    """
    V = np.stack([np.asarray(v1, dtype=np.float64), np.asarray(v2, dtype=np.float64)], axis=-1)
    A = np.abs(V)
    u = -np.sort(-A, axis=-1)
    c = np.cumsum(u, axis=-1)
    j = np.arange(1, V.shape[-1] + 1, dtype=np.float64)
    k = np.maximum(np.sum(u > (c - r) / j, axis=-1), 1)
    theta = (np.take_along_axis(c, (k - 1)[..., None], axis=-1)[..., 0] - r) / k
    Y = np.sign(V) * np.maximum(A - theta[..., None], 0.0)
    inside = A.sum(axis=-1) <= r
    Y = np.where(inside[..., None], V, Y)
    return Y[..., 0], Y[..., 1]


def shrink(v1, v2, mu, p):
    """argmin_m ||m||_p + ||m - v||^2/(2 mu), per node.

    p = inf by the Moreau decomposition the paper uses for that case
    (Sec. 4.2): prox of mu ||.||_inf at v is v minus the projection of v onto
    the l_1 ball of radius mu.
    """
    if p == math.inf:
        q1, q2 = _project_l1_ball(v1, v2, mu)
        return v1 - q1, v2 - q2
    if p == 1:
        return (np.sign(v1) * np.maximum(np.abs(v1) - mu, 0.0),
                np.sign(v2) * np.maximum(np.abs(v2) - mu, 0.0))
    if p == 2:
        nv = np.sqrt(v1 * v1 + v2 * v2)
        with np.errstate(divide="ignore", invalid="ignore"):
            s = np.where(nv > mu, 1.0 - mu / np.where(nv > 0, nv, 1.0), 0.0)
        return v1 * s, v2 * s
    raise ValueError("shrink implemented for p in {1, 2, inf}")


def project_dual_ball(w1, w2, p):
    """Projection of (w1(x), w2(x)) onto {||.||_q <= 1}, q dual to p."""
    if p == 1:      # q = inf: clamp each component
        return np.clip(w1, -1.0, 1.0), np.clip(w2, -1.0, 1.0)
    if p == 2:      # q = 2: radial
        nw = np.sqrt(w1 * w1 + w2 * w2)
        s = 1.0 / np.maximum(1.0, nw)
        return w1 * s, w2 * s
    if p == math.inf:   # q = 1: the l_1 unit ball
        return _project_l1_ball(w1, w2, 1.0)
    raise ValueError("projection implemented for p in {1, 2, inf}")


# --------------------------------------------------------------------------
# The node Laplacian A A* and its inverse (reading R3).
# --------------------------------------------------------------------------

def laplacian_eigenvalues(n, h):
    """Eigenvalues of A A* for the DCT-II basis of length N = n+1 per axis:
    lam_kl = (4/h^2) (sin^2(pi k/(2N)) + sin^2(pi l/(2N)))."""
    N = n + 1
    s = np.sin(np.pi * np.arange(N) / (2.0 * N)) ** 2 * 4.0 / (h * h)
    return s[:, None] + s[None, :]


def poisson_neumann(r, h):
    """u = (A A*)^{-1} r on the zero-mean subspace (mode (0,0) set to 0).

    The orthonormal DCT-II diagonalises A A*; its inverse is the DCT-III.
    """
    n = r.shape[0] - 1
    lam = laplacian_eigenvalues(n, h)
    rh = scipy.fft.dctn(r, type=2, norm="ortho")
    lam = lam.copy()
    lam[0, 0] = 1.0
    uh = rh / lam
    uh[0, 0] = 0.0
    return scipy.fft.idctn(uh, type=2, norm="ortho")


def norm_A_bound(h, d=2):
    """Gershgorin bound ||A_h|| <= 2 sqrt(d) / h (proof of Theorem 1)."""
    return 2.0 * math.sqrt(d) / h


def norm_A_exact(n, h):
    """||A_h|| = sqrt(largest eigenvalue of A A*) = sqrt(8/h^2 sin^2(pi n/(2(n+1))))."""
    return math.sqrt(8.0 / (h * h)) * math.sin(math.pi * n / (2.0 * (n + 1)))


def plain_step_sizes(h, scale=0.5):
    """mu = tau = scale/||A_h|| with the Gershgorin bound (reading R4);
    scale = 1/2 is the paper's choice for Algorithm 1."""
    s = scale / norm_A_bound(h)
    return s, s


def prox_step_sizes(scale=0.5):
    """mu = tau = scale; 1/2 is the paper's choice for Algorithm 2."""
    return scale, scale


# --------------------------------------------------------------------------
# Algorithm 1 (eq. (primaldual)) and its fixed-point residual (eq. (pd_stop)).
# --------------------------------------------------------------------------

def pd_step(m1, m2, phi, rho, h, mu, tau, p):
    """One iteration of eq. (primaldual).  Returns (m1', m2', phi', R^k)."""
    g1, g2 = grad_fwd(phi, h)
    n1, n2 = shrink(m1 + mu * g1, m2 + mu * g2, mu, p)
    b1, b2 = 2.0 * n1 - m1, 2.0 * n2 - m2
    phin = phi + tau * (div(b1, b2, h) - rho)
    d1, d2, dp = n1 - m1, n2 - m2, phin - phi
    R = (inner_h((d1, d2), (d1, d2), h) / mu + inner_h(dp, dp, h) / tau
         - 2.0 * inner_h(dp, div(d1, d2, h), h))
    return n1, n2, phin, R


# --------------------------------------------------------------------------
# Algorithm 2 (eq. (pdhg)), its residual (eq. (pdhg_stop)) and Appendix B.
# --------------------------------------------------------------------------

def prox_step(m1, m2, w1, w2, wb1, wb2, rho, h, mu, tau, p):
    """One iteration of eq. (pdhg).

    (w1, w2) is vphi^k and (wb1, wb2) the extrapolated vphi-bar^k.
    Returns (m1', m2', w1', w2', wb1', wb2', G^k).
    """
    v1, v2 = m1 - mu * wb1, m2 - mu * wb2
    u = poisson_neumann(div(v1, v2, h) - rho, h)
    a1, a2 = div_adj(u, h)
    n1, n2 = v1 - a1, v2 - a2                      # projection onto {A m = rho}
    q1, q2 = project_dual_ball(w1 + tau * n1, w2 + tau * n2, p)
    qb1, qb2 = 2.0 * q1 - w1, 2.0 * q2 - w2
    d1, d2, e1, e2 = n1 - m1, n2 - m2, q1 - w1, q2 - w2
    G = (inner_h((d1, d2), (d1, d2), h) / mu + inner_h((e1, e2), (e1, e2), h) / tau
         + 2.0 * inner_h((e1, e2), (d1, d2), h))
    return n1, n2, q1, q2, qb1, qb2, G


def potential_from_dual(w1, w2, h):
    """Appendix B: psi = (A A*)^{-1} A vphi, zero-mean (reading R8)."""
    return poisson_neumann(div(w1, w2, h), h)


# --------------------------------------------------------------------------
# Cross-level interpolation, Sec. 3.3: eq. (inter_phi) and eq. (inter_m).
# --------------------------------------------------------------------------

def prolong_potential(c):
    """eq. (inter_phi): average of the coarse nodes in N_l(x) (bilinear).

    Fine node (I, J): both even -> the coarse node itself; one odd -> mean of
    the two coarse neighbours along that axis; both odd -> mean of four.
    """
    nc = c.shape[0] - 1
    f = np.zeros((2 * nc + 1, 2 * nc + 1))
    f[0::2, 0::2] = c
    f[1::2, 0::2] = (c[:-1, :] + c[1:, :]) / 2.0
    f[0::2, 1::2] = (c[:, :-1] + c[:, 1:]) / 2.0
    f[1::2, 1::2] = (c[:-1, :-1] + c[:-1, 1:] + c[1:, :-1] + c[1:, 1:]) / 4.0
    return f


def prolong_flux(c1, c2):
    """eq. (inter_m), also used for vphi: nearest neighbour along the flux's
    own axis (tie to x_i - h_l, reading R7), average of N_l across.

    For m1 at fine (I, J) the coarse along-index is a = floor(I/2); J even
    takes c1[a, J/2], J odd the mean of c1[a, (J-1)/2] and c1[a, (J+1)/2].
    m2 is the mirror image.
    """
    nc = c1.shape[0] - 1
    nf = 2 * nc
    f1 = np.zeros((nf + 1, nf + 1))
    f2 = np.zeros((nf + 1, nf + 1))
    f1[0::2, 0::2] = c1
    f1[1::2, 0::2] = c1[:-1, :]
    f1[0::2, 1::2] = (c1[:, :-1] + c1[:, 1:]) / 2.0
    f1[1::2, 1::2] = (c1[:-1, :-1] + c1[:-1, 1:]) / 2.0
    f2[0::2, 0::2] = c2
    f2[0::2, 1::2] = c2[:, :-1]
    f2[1::2, 0::2] = (c2[:-1, :] + c2[1:, :]) / 2.0
    f2[1::2, 1::2] = (c2[:-1, :-1] + c2[1:, :-1]) / 2.0
    f1[nf, :] = 0.0
    f2[:, nf] = 0.0
    return f1, f2


def _prolong_matrix_1d(nc):
    """1-D factor of the potential interpolation: (2nc+1) x (nc+1)."""
    P = np.zeros((2 * nc + 1, nc + 1))
    for I in range(2 * nc + 1):
        if I % 2 == 0:
            P[I, I // 2] = 1.0
        else:
            P[I, (I - 1) // 2] = 0.5
            P[I, (I + 1) // 2] = 0.5
    return P


def restrict_density(f):
    """Reading R6: coarse = D^{-1} P^T fine, P the bilinear interpolation of
    eq. (inter_phi) and D = diag(P^T 1), i.e. a weighted average of the fine
    nodes around each coarse node (constants are preserved)."""
    nf = f.shape[0] - 1
    P = _prolong_matrix_1d(nf // 2)
    w = P.T @ np.ones(nf + 1)
    return (P.T @ f @ P) / np.outer(w, w)


# --------------------------------------------------------------------------
# Levels and tolerances: h_l = 2^{L-l} h (Sec. 3.2), eq. (tol_formula_propose)
# and eq. (stop_tol) of Sec. 5.
# --------------------------------------------------------------------------

def level_sides(n, L):
    if L < 1 or n % (1 << (L - 1)) != 0 or n // (1 << (L - 1)) < 1:
        raise ValueError("n must be divisible by 2^(L-1)")
    return [n >> (L - l) for l in range(1, L + 1)]


def level_tolerances(eps_L, alpha, n, L):
    """eps_l = eps_L (h_l/h)^alpha for l = 1..L."""
    return [eps_L * (float(1 << (L - l))) ** alpha for l in range(1, L + 1)]


def paper_stop_tolerance(algo, n, multilevel):
    """eq. (stop_tol): the finest-level FPR tolerance used in Sec. 5.3
    (reading eps for Algorithm 4 as eps_L).  algo 1 = plain, 2 = prox."""
    s = (1.0 / n) / (1.0 / 512.0)
    if algo == 1:
        return 1e-6 / 128.0 * s ** 2 if multilevel else 1e-6 / 512.0 * s ** 3
    if multilevel:
        return min(2e-4, 1e-4 / 32.0 * s ** 2)
    return min(2e-4, 1e-4 / 16.0 * s ** 2)


# --------------------------------------------------------------------------
# Input preparation and the density pyramid.
# --------------------------------------------------------------------------

def prepare_levels(p0, p1, n, L):
    """Node masses -> per-level rho_l = rho0_l - rho1_l (finest last).

    rho^k = p^k / h^2 after renormalising p^k to unit mass (Sec. 2.2 samples
    densities on the nodes; sum rho h^2 = 1).  Coarse levels by reading R6,
    each renormalised to unit mass; rho_l is made exactly zero-sum.
    """
    p0 = np.asarray(p0, dtype=np.float64)
    p1 = np.asarray(p1, dtype=np.float64)
    if p0.shape != (n + 1, n + 1) or p1.shape != (n + 1, n + 1):
        raise ValueError("masses must have shape (n+1, n+1)")
    if not (np.all(np.isfinite(p0)) and np.all(np.isfinite(p1))):
        raise ValueError("non-finite mass")
    if np.any(p0 < 0) or np.any(p1 < 0):
        raise ValueError("negative mass")
    s0, s1 = p0.sum(), p1.sum()
    if s0 <= 0 or abs(s0 - s1) > 1e-9 * s0:
        raise ValueError("masses do not balance")
    sides = level_sides(n, L)
    h = 1.0 / n
    r0 = [None] * L
    r1 = [None] * L
    r0[-1] = p0 / s0 / (h * h)
    r1[-1] = p1 / s1 / (h * h)
    for l in range(L - 2, -1, -1):
        hl = 1.0 / sides[l]
        for arr in (r0, r1):
            c = restrict_density(arr[l + 1])
            arr[l] = c / (c.sum() * hl * hl)
    rhos = []
    for l in range(L):
        r = r0[l] - r1[l]
        rhos.append(r - r.mean())
    return rhos


# --------------------------------------------------------------------------
# Stopping measures (reading R9) and the FP64 evaluator.
# --------------------------------------------------------------------------

def _dual_excess(psi, h, p):
    """RMS and max of (||grad psi(x)||_q - 1)_+ and max ||grad psi||_q."""
    g1, g2 = grad_fwd(psi, h)
    gn = pointwise_norm(g1, g2, dual_exponent(p))
    ex = np.maximum(gn - 1.0, 0.0)
    return math.sqrt(float(np.sum(ex * ex)) * h * h), float(gn.max())


def min_norm_correction(m1, m2, rho, h):
    """A*(A A*)^{-1}(A m - rho): the flux change of least L^2_h norm that
    makes m feasible (m minus it satisfies A m = rho).  Its norm is the
    primal part of the normalised KKT residual; m minus it is the feasible
    flux of the certificate's upper bound."""
    return div_adj(poisson_neumann(div(m1, m2, h) - rho, h), h)


def primal_residual(m1, m2, rho, h):
    """||A*(A A*)^{-1}(A m - rho)||_{L^2_h}, the distance of m to the
    feasible set {A m = rho} in the L^2_h norm."""
    c1, c2 = min_norm_correction(m1, m2, rho, h)
    return math.sqrt(inner_h((c1, c2), (c1, c2), h))


def kkt_plain(m1, m2, phi, rho, h, p):
    """Normalised KKT residual of an Algorithm 1 iterate:
    max(||A*(A A*)^{-1}(A m - rho)||_{L^2_h} / P, RMS Lipschitz excess of
    -phi, relative gap) with P = f(m), D = -<phi, rho>_h."""
    P = flux_cost(m1, m2, h, p)
    r_pri = primal_residual(m1, m2, rho, h) / max(P, 1e-300)
    r_dual, _ = _dual_excess(-phi, h, p)
    D = -inner_h(phi, rho, h)
    r_gap = abs(P - D) / max(abs(P), abs(D), 1e-300)
    return max(r_pri, r_dual, r_gap), P, D


def kkt_prox(m1, m2, w1, w2, rho, h, p):
    """Same measure for an Algorithm 2 iterate, the potential psi taken from
    Appendix B: D = <psi, rho>_h."""
    psi = potential_from_dual(w1, w2, h)
    P = flux_cost(m1, m2, h, p)
    r_pri = primal_residual(m1, m2, rho, h) / max(P, 1e-300)
    r_dual, _ = _dual_excess(psi, h, p)
    D = inner_h(psi, rho, h)
    r_gap = abs(P - D) / max(abs(P), abs(D), 1e-300)
    return max(r_pri, r_dual, r_gap), P, D


def evaluate(m1, m2, psi, rho, h, p):
    """FP64 certificate for any flux m and usual-sign potential psi.

    P = f(m); D = <psi, rho>_h;
    hi = f(m - A*(AA*)^{-1}(A m - rho)) (feasible flux, >= W1_h);
    lo = D / max(1, max ||grad psi||_q) (feasible potential, <= W1_h);
    kkt = max(||A*(AA*)^{-1}(A m - rho)||_{L2h} / P, RMS excess, gap).
    """
    m1 = np.asarray(m1, dtype=np.float64)
    m2 = np.asarray(m2, dtype=np.float64)
    psi = np.asarray(psi, dtype=np.float64)
    res = div(m1, m2, h) - rho
    corr = poisson_neumann(res, h)
    c1, c2 = div_adj(corr, h)
    P = flux_cost(m1, m2, h, p)
    D = inner_h(psi, rho, h)
    hi = flux_cost(m1 - c1, m2 - c2, h, p)
    rms, gmax = _dual_excess(psi, h, p)
    lo = D / max(1.0, gmax)
    r_pri = math.sqrt(inner_h((c1, c2), (c1, c2), h)) / max(P, 1e-300)
    r_gap = abs(P - D) / max(abs(P), abs(D), 1e-300)
    return {"P": P, "D": D, "lo": lo, "hi": hi, "kkt": max(r_pri, rms, r_gap),
            "r_pri": r_pri, "r_dual": rms, "r_gap": r_gap, "grad_max": gmax}


# --------------------------------------------------------------------------
# Algorithms 3 and 4: the cascade.
# --------------------------------------------------------------------------

def solve(p0, p1, n, L=1, p=1, algo=1, stop="kkt", tol=1e-6, alpha=-1.0,
          max_iters=20000, check_every=1, step_scale=None, eps_L=None,
          return_fields=True, init=None):
    """Algorithm 3 (algo=1, plain) or Algorithm 4 (algo=2, prox).

    stop = "kkt": stop level l when the normalised KKT residual <= tol_l;
    stop = "fpr": stop when R^k (or G^k) <= eps_l (eq. (pd_stop)/(pdhg_stop)).
    tol_l (or eps_l) = tol (or eps_L) * (h_l/h)^alpha.  Checks run every
    `check_every` iterations and at the cap.  Level 1 starts from zero.
    `max_iters` is one cap for every level or a list of per-level caps,
    coarsest first.  `init` optionally supplies the level-1 start (tests of
    single steps).
    """
    sides = level_sides(n, L)
    caps = [int(max_iters)] * L if np.isscalar(max_iters) else [int(c) for c in max_iters]
    if len(caps) != L or min(caps) < 1:
        raise ValueError("max_iters: one positive cap, or one per level")
    rhos = prepare_levels(p0, p1, n, L)
    base = eps_L if (stop == "fpr" and eps_L is not None) else tol
    tols = level_tolerances(base, alpha, n, L)
    out = {"iters": [], "level_seconds": [], "status": "ok", "measure": [], "level_w1": []}
    state = None
    for l in range(L):
        nl = sides[l]
        h = 1.0 / nl
        rho = rhos[l]
        t0 = time.perf_counter()
        if algo == 1:
            mu, tau = plain_step_sizes(h, 0.5 if step_scale is None else step_scale)
            if state is None:
                if init is not None:
                    m1, m2, phi = (np.array(a, dtype=np.float64) for a in init)
                else:
                    m1 = np.zeros((nl + 1, nl + 1)); m2 = np.zeros_like(m1); phi = np.zeros_like(m1)
            else:
                m1, m2 = prolong_flux(state[0], state[1])
                phi = prolong_potential(state[2])
            k = 0
            while True:
                m1, m2, phi, R = pd_step(m1, m2, phi, rho, h, mu, tau, p)
                k += 1
                if k % check_every == 0 or k >= caps[l]:
                    meas = R if stop == "fpr" else kkt_plain(m1, m2, phi, rho, h, p)[0]
                    if meas <= tols[l]:
                        break
                    if k >= caps[l]:
                        out["status"] = "maxiter"
                        break
            state = (m1, m2, phi)
        else:
            mu, tau = prox_step_sizes(0.5 if step_scale is None else step_scale)
            if state is None:
                if init is not None:
                    m1, m2, w1, w2 = (np.array(a, dtype=np.float64) for a in init)
                else:
                    m1 = np.zeros((nl + 1, nl + 1)); m2 = np.zeros_like(m1)
                    w1 = np.zeros_like(m1); w2 = np.zeros_like(m1)
            else:
                m1, m2 = prolong_flux(state[0], state[1])
                w1, w2 = prolong_flux(state[2], state[3])
            wb1, wb2 = w1.copy(), w2.copy()                  # reading R5
            k = 0
            while True:
                m1, m2, w1, w2, wb1, wb2, G = prox_step(m1, m2, w1, w2, wb1, wb2, rho, h, mu, tau, p)
                k += 1
                if k % check_every == 0 or k >= caps[l]:
                    meas = G if stop == "fpr" else kkt_prox(m1, m2, w1, w2, rho, h, p)[0]
                    if meas <= tols[l]:
                        break
                    if k >= caps[l]:
                        out["status"] = "maxiter"
                        break
            state = (m1, m2, w1, w2)
        out["iters"].append(k)
        out["measure"].append(float(meas))
        # f(m^{K_l}) on this level, the quantity condition (cond_f) of
        # Sec. 5.2 compares with the level optimum
        out["level_w1"].append(flux_cost(state[0], state[1], h, p))
        out["level_seconds"].append(time.perf_counter() - t0)
    h = 1.0 / n
    rho = rhos[-1]
    if algo == 1:
        m1, m2, phi = state
        psi = -(phi - phi.mean())
    else:
        m1, m2, w1, w2 = state
        psi = potential_from_dual(w1, w2, h)
    ev = evaluate(m1, m2, psi, rho, h, p)
    out.update({"w1": ev["P"], "dual": ev["D"], "lo": ev["lo"], "hi": ev["hi"],
                "kkt": ev["kkt"], "levels": sides, "tolerances": tols})
    if return_fields:
        out.update({"m1": m1, "m2": m2, "psi": psi, "rho": rho})
        if algo == 1:
            out["phi"] = state[2]
        else:
            out["vphi1"], out["vphi2"] = state[2], state[3]
    return out

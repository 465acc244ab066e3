"""Oracle of the rational-filter subspace generation (Sec. IV.B, the
subspace-generation subsection; test infrastructure only).

The fine-grid deflation vectors are a fourth-order rational low-pass filter
applied to Gaussian noise (the equation labelled "ratfilt"):

    phi_k  proportional to  prod_{j=0..3} (H + lambda + j eps)^-1 eta_k,

with lambda = 3e-4 and eps = lambda / 3 as the paper's typical values.  The
paper evaluates it with one multi-shift solve; the filter is then the
partial-fraction sum

    prod_j 1 / (x + s_j) = sum_j c_j / (x + s_j),  c_j = prod_{i != j} 1 / (s_i - s_j),

of the shifted solutions.  Optionally the noise is four-dimensional and sits
only on the physical components at the walls: P- at s = 0 and P+ at
s = Ls - 1, the components through which the quark mass couples the two
walls in the kernel's fifth dimension.

Functions
---------
filter_response(x, lam, eps)   the filter as a function of the eigenvalue x
partial_fractions(shifts)      the coefficients c_j
wall_mask(h)                   keep only P- at s = 0 and P+ at s = Ls - 1
multishift_cg(apply, b, ...)   CG for (A + s_j) x_j = b, all j from one Krylov space
rational_filter(op, eta, ...)  the filter by one multi-shift solve and the sum
rational_filter_product(...)   the filter as four successive shifted CG solves
surface_truncate(V, depth)     remove the fifth-dimension interior of subspace vectors

Surface truncation (the closing paragraph of the subsection): the filtered
vectors are bound to the walls, so the interior slices depth <= s < Ls - depth
of the subspace vectors may be set to zero, which cuts the bytes of the
projection to and from the coarse problem by Ls / (2 depth); a depth with
2 depth >= Ls keeps every slice.
"""
from __future__ import annotations

import numpy as np

from .cg import cg
from .gamma import chiral_projectors


def shifts_of(lam, eps, order=4):
    return [lam + j * eps for j in range(order)]


def filter_response(x, lam, eps, order=4):
    """prod_j 1 / (x + lam + j eps)."""
    x = np.asarray(x, dtype=float)
    out = np.ones_like(x)
    for s in shifts_of(lam, eps, order):
        out = out / (x + s)
    return out


def partial_fractions(shifts):
    s = np.asarray(shifts, dtype=float)
    c = np.empty(len(s))
    for j in range(len(s)):
        c[j] = 1.0 / np.prod([s[i] - s[j] for i in range(len(s)) if i != j])
    return c


def wall_mask(h):
    """h (..., Ls, Vh, 4, 3) -> P- h at s = 0, P+ h at s = Ls - 1, zero
    elsewhere (for Ls = 1 both projections of the one slice)."""
    Pp, Pm = chiral_projectors()
    out = np.zeros_like(h)
    out[..., 0, :, :, :] += np.einsum("ab,...bc->...ac", Pm, h[..., 0, :, :, :])
    out[..., -1, :, :, :] += np.einsum("ab,...bc->...ac", Pp, h[..., -1, :, :, :])
    return out


def _dot(a, b):
    return np.vdot(a.ravel(), b.ravel())


def multishift_cg(apply, b, shifts, tol=1e-10, maxiter=100000):
    """Solve (A + s_j) x_j = b for every shift with the Krylov space of the
    smallest one, shifts[0] (it converges last): CG on A + s_0, and for the
    other shifts the collinear residuals r_j = zeta_j r, whose factors obey
    a three-term recurrence in the CG coefficients.  Stops when
    |r| <= tol |b| for the base system.  Returns (xs, iterations)."""
    s0 = shifts[0]
    if any(s < s0 for s in shifts):
        raise ValueError("shifts[0] must be the smallest shift")
    ns = len(shifts)
    x = [np.zeros_like(b) for _ in range(ns)]
    p = [b.copy() for _ in range(ns)]
    r = b.copy()
    zeta = np.ones(ns)       # zeta_k
    zeta_old = np.ones(ns)   # zeta_{k-1}
    alpha_old, beta_old = 1.0, 0.0
    rr = _dot(r, r).real
    stop = tol * tol * rr
    it = 0
    while rr > stop and it < maxiter:
        w = apply(p[0]) + s0 * p[0]
        alpha = rr / _dot(p[0], w).real
        zeta_new = np.ones(ns)
        alphas = np.empty(ns)
        alphas[0] = alpha
        for j in range(1, ns):
            d = shifts[j] - s0
            zeta_new[j] = (zeta[j] * zeta_old[j] * alpha_old /
                           (alpha * beta_old * (zeta_old[j] - zeta[j]) + zeta_old[j] * alpha_old * (1.0 + d * alpha)))
            alphas[j] = alpha * zeta_new[j] / zeta[j]
        for j in range(ns):
            x[j] = x[j] + alphas[j] * p[j]
        r = r - alpha * w
        rr_new = _dot(r, r).real
        beta = rr_new / rr
        p[0] = r + beta * p[0]
        for j in range(1, ns):
            beta_j = beta * (zeta_new[j] / zeta[j]) ** 2
            p[j] = zeta_new[j] * r + beta_j * p[j]
        zeta_old, zeta = zeta, zeta_new
        alpha_old, beta_old = alpha, beta
        rr = rr_new
        it += 1
    return x, it


def rational_filter(op, eta, lam=3e-4, eps=1e-4, tol=1e-10, maxiter=100000, wall=False, normalise=True):
    """phi = prod_j (H + lam + j eps)^-1 eta by one multi-shift solve and the
    partial-fraction sum (eta first wall-masked when wall is set); unit norm
    when normalise is set.  Returns (phi, iterations)."""
    src = wall_mask(eta) if wall else eta
    sh = shifts_of(lam, eps)
    xs, it = multishift_cg(op.H, src, sh, tol=tol, maxiter=maxiter)
    c = partial_fractions(sh)
    phi = sum(cj * xj for cj, xj in zip(c, xs))
    if normalise:
        phi = phi / np.sqrt(_dot(phi, phi).real)
    return phi, it


def rational_filter_product(op, eta, lam=3e-4, eps=1e-4, tol=1e-12, wall=False):
    """The same filter as four successive shifted CG solves (no partial
    fractions), unnormalised."""
    v = wall_mask(eta) if wall else eta
    for s in shifts_of(lam, eps):
        v, _, _ = cg(lambda u, s=s: op.H(u) + s * u, v, tol=tol)
    return v


def surface_truncate(V, depth):
    """V (..., Ls, Vh, 4, 3) with the slices depth <= s < Ls - depth set to
    zero (a copy; unchanged when 2 depth >= Ls)."""
    out = np.array(V, copy=True)
    Ls = out.shape[-4]
    if 2 * depth < Ls:
        out[..., depth:Ls - depth, :, :, :] = 0
    return out

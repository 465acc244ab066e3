"""Oracle HDCG solver layers (test infrastructure only).

* Q = M_SS^-1: promote . (coarse CG on A) . project (Sec. II).
* P_R = 1 - Q H and P_L = 1 - H Q (Luscher's projectors, Sec. II, with
  Q H = 1 - P_R).
* M_IRS(H, N, lambda): exactly N CG iterations on H + lambda from zero
  (Sec. IV.C).
* The generalised PCG of Tang et al. (Fig. "pcg_general", Sec. IV.E) with
  the A-DEF2 row of Table "algos": V_start = Q b + P_R x, M_1 = P_R M_IRS + Q,
  M_2 = M_3 = 1; and the BNN row (M_1 = P_R M_IRS P_L + Q) for the
  equivalence of Sec. IV.E.1.
* Search-direction update: standard (beta = (r', y') / (r, y)) or flexible
  (Notay's FCG with one stored direction, cited but not written out in the
  paper): alpha = (p, r) / (p, w), beta = -(w, y') / (p, w).
* Defect correction: the outer FP64 loop r = b - H x, x += inner(r).
"""
from __future__ import annotations

import numpy as np

from . import blocks as blk
from . import coarse as crs
from .cg import cg, cg_fixed


def _dot(a, b):
    return np.vdot(a.ravel(), b.ravel())


def _nrm(a):
    return float(np.sqrt(_dot(a, a).real))


class TwoLevel:
    """The fine operator together with its blocked subspace and coarse operator."""

    def __init__(self, op, phi, sob, C, A, coarse_tol=1e-12, coarse_maxiter=100000):
        self.op, self.phi, self.sob, self.C, self.A = op, phi, sob, C, A
        self.coarse_tol = coarse_tol
        self.coarse_maxiter = coarse_maxiter
        self.coarse_iters = []

    def project(self, v):
        return blk.project(self.phi, self.sob, v)

    def promote(self, c):
        return blk.promote(self.phi, self.sob, c)

    def coarse_solve(self, c):
        x, it, _ = cg(lambda v: crs.apply(self.A, v, self.C), c, tol=self.coarse_tol,
                      maxiter=self.coarse_maxiter)
        self.coarse_iters.append(it)
        return x

    def Q(self, v):
        return self.promote(self.coarse_solve(self.project(v)))

    def P_R(self, v):
        return v - self.Q(self.op.H(v))

    def P_L(self, v):
        return v - self.op.H(self.Q(v))


def m_irs(op, r, niter, lam):
    """M_IRS(H, N, lambda) r: N CG iterations on (H + lambda) from zero."""
    return cg_fixed(lambda v: op.H(v) + lam * v, r, niter)


def gpcg(tl, b, method="adef2", n_irs=7, lam_irs=1.0, tol=1e-8, maxiter=1000,
         flexible=True, x=None, callback=None, m_irs_fn=None):
    """Generalised PCG (Tang et al.) for the A-DEF2 and BNN rows.  m_irs_fn
    replaces m_irs (same arguments), e.g. by its 16-bit storage form.

    Returns (x, iterations, recursive relative residual)."""
    H = tl.op.H
    mirs = m_irs if m_irs_fn is None else m_irs_fn

    def M_irs(r):
        return mirs(tl.op, r, n_irs, lam_irs)

    if method == "adef2":
        def M1(r):
            z = M_irs(r)
            # P_R M_IRS r + Q r = z - Q (H z - r)
            return z - tl.Q(H(z) - r)
    elif method == "bnn":
        def M1(r):
            return tl.P_R(M_irs(tl.P_L(r))) + tl.Q(r)
    else:
        raise ValueError(method)

    x0 = np.zeros_like(b) if x is None else x
    if method == "adef2":
        x = tl.Q(b) + tl.P_R(x0)  # V_start = Q b + P_R x
    else:
        x = x0.copy()
    r = b - H(x)
    y = M1(r)
    p = y.copy()
    bn = _nrm(b)
    ry = _dot(r, y)
    it = 0
    while it < maxiter and _nrm(r) / bn > tol:
        w = H(p)
        pw = _dot(p, w)
        alpha = (_dot(p, r) if flexible else ry) / pw
        x = x + alpha * p
        r = r - alpha * w
        y = M1(r)
        if flexible:
            beta = -_dot(w, y) / pw
        else:
            ry_new = _dot(r, y)
            beta = ry_new / ry
            ry = ry_new
        p = y + beta * p
        it += 1
        if callback is not None:
            callback(it, x, r, p)
    return x, it, _nrm(r) / bn


def defect_correction(tl, b, tol=1e-8, inner_tol=1e-5, max_outer=50, **kw):
    """x = 0; repeat r = b - H x, stop at |r|/|b| <= tol, else x += inner(r)."""
    x = np.zeros_like(b)
    bn = _nrm(b)
    outers = 0
    inner_its = []
    while True:
        r = b - tl.op.H(x)
        rel = _nrm(r) / bn
        if rel <= tol or outers >= max_outer:
            return x, outers, inner_its, rel
        e, it, _ = gpcg(tl, r, tol=inner_tol, **kw)
        inner_its.append(it)
        x = x + e
        outers += 1

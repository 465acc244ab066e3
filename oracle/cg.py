"""Oracle conjugate gradients (test infrastructure only).

Textbook Hestenes-Stiefel CG on a Hermitian positive-definite operator: the
preconditioned CG of Fig. "pcg" in Sec. IV.A with the preconditioner set to
the identity, which is the plain CG on the red-black normal equations that the
paper compares against (Sec. VI.B, Table "wallclock").  Stop when the
recursive relative residual |r|/|b| reaches tol; then recompute the true
residual and restart from the current x if it is still above tol.
"""
from __future__ import annotations

import numpy as np


def _dot(a, b):
    return np.vdot(a.ravel(), b.ravel())


def cg(apply, b, tol=1e-8, maxiter=100000, x0=None, history=None):
    """Returns (x, iterations, true_relative_residual)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bn = np.sqrt(_dot(b, b).real)
    if bn == 0.0:
        return x, 0, 0.0
    r = b.copy() if x0 is None else b - apply(x)
    it = 0
    while True:
        rr = _dot(r, r).real
        if np.sqrt(rr) / bn <= tol or it >= maxiter:
            return x, it, np.sqrt(rr) / bn
        p = r.copy()
        while it < maxiter:
            w = apply(p)
            alpha = rr / _dot(p, w).real
            x += alpha * p
            r -= alpha * w
            rr_new = _dot(r, r).real
            it += 1
            if history is not None:
                history.append(np.sqrt(rr_new) / bn)
            if np.sqrt(rr_new) / bn <= tol:
                break
            p = r + (rr_new / rr) * p
            rr = rr_new
        # true residual; restart from x when the recursive one has drifted
        r = b - apply(x)


def cg_fixed(apply, b, niter):
    """Exactly niter CG iterations from x = 0 with no early exit (the fixed
    iteration count of the infra-red shifted preconditioner, Sec. IV.C).
    Stops early only if the residual is exactly zero."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = _dot(r, r).real
    for _ in range(niter):
        if rr == 0.0:
            break
        w = apply(p)
        alpha = rr / _dot(p, w).real
        x += alpha * p
        r -= alpha * w
        rr_new = _dot(r, r).real
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x

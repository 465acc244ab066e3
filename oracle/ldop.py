"""Oracle of the second deflation level of the little Dirac operator
(Sec. V.B, "Little Dirac operator deflation"; test infrastructure only).

The coarse operator A (Hermitian positive) is itself deflated by global
coarse vectors, with no further blocking:

* the vectors that come free with the blocked subspace (the global vectors
  of the literature the paper cites): w_k[a][j] = delta_jk / sqrt(Nc), the
  coarse image of the k-th subspace vector summed over all blocks;
* about a hundred more from shifted inverse iteration on A: each a coarse
  noise vector taken through n steps of v <- (A + shift)^-1 v / |.|, the
  solves to a tight residual (the paper: three steps, residual 1e-7).

The third level is one dense matrix: E = W^+ A W for an orthonormal basis W
of those vectors, pre-diagonalised, E = U D U^+, so with Z = W U (still
orthonormal) the coarse-coarse inverse is Z D^-1 Z^+ and costs two
matrix-vector products.  The coarse solve is then deflated CG (the paper's
LittleDopSolverDeflCG): x0 = Z D^-1 Z^+ b, and plain CG whose search
directions are kept A-orthogonal to span(Z),

    p <- r + beta p - Z D^-1 (A Z)^+ r,

A Z stored once so no extra A application is needed.  Coarse vectors are
arrays (..., Nc, Nvec); a basis is (n, Nc, Nvec).
"""
from __future__ import annotations

import numpy as np

from . import coarse as crs
from .cg import cg, cg_fixed


def _flat(V):
    return V.reshape(V.shape[0], -1)


def free_global_vectors(Nc, nvec):
    """w_k[a][j] = delta_jk / sqrt(Nc), k < nvec."""
    W = np.zeros((nvec, Nc, nvec), dtype=np.complex128)
    for k in range(nvec):
        W[k, :, k] = 1.0 / np.sqrt(Nc)
    return W


def inverse_iteration(A, C, V0, n_steps=3, shift=0.0, tol=1e-7):
    """Each coarse vector through n_steps of v <- (A + shift)^-1 v / |.|."""
    out = []
    for v in V0:
        for _ in range(n_steps):
            v, _, _ = cg(lambda u: crs.apply(A, u, C) + shift * u, v, tol=tol)
            v = v / np.linalg.norm(v)
        out.append(v)
    return np.array(out)


def orthonormal_basis(W):
    """An orthonormal basis (n, Nc, Nvec) of the span of the rows of W."""
    Q, _ = np.linalg.qr(_flat(W).T)
    return Q.T.reshape(W.shape)


def third_level(A, C, W):
    """(Z, D, AZ): E = W^+ A W = U D U^+ diagonalised, Z = W U, AZ = A Z."""
    AW = np.array([crs.apply(A, w, C) for w in W])
    E = _flat(W).conj() @ _flat(AW).T
    E = 0.5 * (E + E.conj().T)
    D, U = np.linalg.eigh(E)
    Z = np.einsum("ik,i...->k...", U, W)
    AZ = np.einsum("ik,i...->k...", U, AW)
    return Z, D, AZ


def deflated_cg(A, C, b, Z, D, AZ, tol=1e-8, maxiter=10000):
    """Deflated CG on A x = b from x0 = Z D^-1 Z^+ b, stopping at
    |r| <= tol |b|.  Returns (x, iterations, relative residual)."""
    Zf, AZf = _flat(Z), _flat(AZ)
    bf = b.ravel()

    def apply(v):
        return crs.apply(A, v.reshape(b.shape), C).ravel()

    def defl(r):  # Z D^-1 (A Z)^+ r
        return Zf.T @ ((AZf.conj() @ r) / D)

    x = Zf.T @ ((Zf.conj() @ bf) / D)
    r = bf - apply(x)
    bn = np.linalg.norm(bf)
    rr = np.vdot(r, r).real
    p = r - defl(r)
    it = 0
    while np.sqrt(rr) > tol * bn and it < maxiter:
        w = apply(p)
        alpha = rr / np.vdot(p, w).real
        x = x + alpha * p
        r = r - alpha * w
        rr_new = np.vdot(r, r).real
        p = r + (rr_new / rr) * p - defl(r)
        rr = rr_new
        it += 1
    return x.reshape(b.shape), it, np.sqrt(rr) / bn


# ---------------------------------------------------------------------------
# The truncated operator and the ADEF1 coarse solver (Sec. V.B, "Truncated
# little Dirac operator as preconditioner").  Q_trunc keeps the zero- and
# one-hop terms of A (the site itself and its 8 axis neighbours; still
# Hermitian) plus an infra-red shift; a Chebyshev polynomial of Q_trunc
# approximating 1/x on [lo, hi] is the high-mode preconditioner M, and the
# second level deflates the low modes: ADEF1, M_1 = M P_D + Q with
# P_D = 1 - A Q, Q = Z D^-1 Z^+, A Z stored (no extra A application).

def one_hop_points():
    """Stencil indices l with sum_mu |delta_mu| <= 1 (l = 40 first)."""
    offs = crs.stencil_offsets()
    pts = [l for l in range(crs.NSTENCIL) if np.abs(offs[l]).sum() <= 1]
    pts.remove(40)
    return [40] + pts


def truncate(A, shift=0.0):
    """Q_trunc + shift in the 81-point storage (the dropped terms zero)."""
    T = np.zeros_like(A)
    for l in one_hop_points():
        T[:, l] = A[:, l]
    nvec = A.shape[2]
    T[:, 40] += shift * np.eye(nvec)
    return T


def chebyshev_inverse(apply, r, lo, hi, order):
    """y = p(M) r from the Chebyshev iteration for M y = r started at y = 0:
    the residual r - M y is R_n(M) r with the scaled Chebyshev polynomial
    R_n(x) = T_n((d - x)/c) / T_n(d/c), d = (hi + lo)/2, c = (hi - lo)/2,
    n = order (n - 1 applications of M).  The three-term recurrence of T_n
    gives, with sigma = d/c and omega_k = 2 sigma T_{k-1}(sigma)/T_k(sigma)
    (omega_1 = 2, omega_{k+1} = 1/(1 - omega_k/(4 sigma^2))),
        delta_1 = r/d,  delta_{k+1} = (omega_{k+1}/d) r_k + (omega_{k+1} - 1) delta_k,
        y_k = delta_1 + ... + delta_k,  r_k = r_{k-1} - M delta_k."""
    if order < 1:
        raise ValueError("order must be at least 1")
    d, c = 0.5 * (hi + lo), 0.5 * (hi - lo)
    sigma = d / c
    delta = r / d
    y = delta.copy()
    res = r.copy()
    omega = 2.0
    for _ in range(1, order):
        res = res - apply(delta)
        omega = 1.0 / (1.0 - omega / (4.0 * sigma * sigma))
        delta = (omega / d) * res + (omega - 1.0) * delta
        y = y + delta
    return y


def trunc_cg(T, C, r, order):
    """M_IRS(Q_trunc) r: `order` CG iterations on the shifted truncated
    operator T (truncate(A, shift)) from zero, the fixed-order CG the paper
    offers in place of the Chebyshev polynomial (Sec. V.B, closing paragraph
    of "Truncated little Dirac operator as preconditioner"; the infra-red
    shifted CG of Sec. IV.C)."""
    return cg_fixed(lambda u: crs.apply(T, u, C), r, order)


def coarse_coarse_inverse(Z, D):
    """v -> Z D^-1 Z^+ v on flat vectors."""
    Zf = _flat(Z)
    return lambda v: Zf.T @ ((Zf.conj() @ v) / D)


def adef1_preconditioner(Z, D, AZ, M):
    """r -> M (r - A Z D^-1 Z^+ r) + Z D^-1 Z^+ r (M_1 = M P_D + Q with
    P_D = 1 - A Q), on vectors of the coarse shape."""
    Zf, AZf = _flat(Z), _flat(AZ)

    def M1(r):
        c = (Zf.conj() @ r.ravel()) / D
        return (M((r.ravel() - AZf.T @ c).reshape(r.shape)).ravel() + Zf.T @ c).reshape(r.shape)
    return M1


def adef1_solve(A, C, b, Z, D, AZ, M, tol=1e-8, maxiter=10000):
    """Flexible generalised PCG on A x = b with the ADEF1 preconditioner
    y = M (r - AZ D^-1 Z^+ r) + Z D^-1 Z^+ r, from x0 = Z D^-1 Z^+ b;
    alpha = (p, r)/(p, w), beta = -(w, y)/(p, w).  Stops at |r| <= tol |b|.
    Returns (x, iterations, relative residual)."""
    shape = b.shape
    bf = b.ravel()

    def apply(v):
        return crs.apply(A, v.reshape(shape), C).ravel()

    Q = coarse_coarse_inverse(Z, D)
    M1_ = adef1_preconditioner(Z, D, AZ, M)

    def M1(r):
        return M1_(r.reshape(shape)).ravel()

    x = Q(bf)
    r = bf - apply(x)
    bn = np.linalg.norm(bf)
    y = M1(r)
    p = y.copy()
    it = 0
    while np.linalg.norm(r) > tol * bn and it < maxiter:
        w = apply(p)
        pw = np.vdot(p, w)
        alpha = np.vdot(p, r) / pw
        x = x + alpha * p
        r = r - alpha * w
        it += 1
        if np.linalg.norm(r) <= tol * bn:
            break
        y = M1(r)
        beta = -np.vdot(w, y) / pw
        p = y + beta * p
    return x.reshape(shape), it, np.linalg.norm(r) / bn

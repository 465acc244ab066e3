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
from .cg import cg


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

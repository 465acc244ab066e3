"""Oracle little Dirac operator (test infrastructure only).

A^{ab}_{jk} = <phi^a_j | H | phi^b_k> (Sec. V.A.1).  With blocks of at least
four sites in every direction, spanning the whole fifth dimension, a block
couples only to blocks at most one block away in each direction: 3^4 = 81
stencil points including itself (Sec. V.A).

Stencil index l = sum_mu (delta_mu + 1) 3^mu with delta_mu in {-1, 0, 1},
delta_x fastest, so l = 40 is the site itself.  Storage A[a][l][j][k] =
<phi^a_j | H | phi^{a+delta_l}_k>, and (A c)[a][j] = sum_l sum_k
A[a][l][j][k] c[a+delta_l][k].

Two constructions:
* brute force: H applied to every blocked vector phi^b_k, then projected;
* the Fourier trick of Sec. V.A.1: H applied to 81 phased sums per vector,
  projected, then the 81 x 81 phase matrix M_sl inverted.

Reading of the momenta: the paper writes p_mu = n pi / L_mu; such phases are
not periodic on the coarse torus, so the per-block identity fails on boundary
blocks.  This oracle uses p_mu = 2 pi n m_mu / Lc_mu with n in {-1, 0, 1} and
m_mu = round(Lc_mu / 3), which is periodic and keeps M_sl invertible for
Lc_mu >= 3 (when 3 divides Lc_mu it is the colouring scheme of Sec. V.A.1).
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

from . import blocks as blk

NSTENCIL = 81


def stencil_offsets():
    """delta^l for l = 0..80, shape (81, 4), delta_x fastest."""
    offs = np.zeros((NSTENCIL, 4), dtype=np.int64)
    for l in range(NSTENCIL):
        q = l
        for mu in range(4):
            offs[l, mu] = q % 3 - 1
            q //= 3
    return offs


def coarse_coords(C):
    Cx, Cy, Cz, Ct = C
    a = np.arange(Cx * Cy * Cz * Ct)
    return np.stack([a % Cx, (a // Cx) % Cy, (a // (Cx * Cy)) % Cz, a // (Cx * Cy * Cz)], axis=1)


def coarse_neighbour(C, a_coords, delta):
    c = (a_coords + delta) % np.array(C)
    return c[..., 0] + C[0] * (c[..., 1] + C[1] * (c[..., 2] + C[2] * c[..., 3]))


def neighbour_table(C):
    """nbr[a][l] = coarse index of a + delta_l."""
    cc = coarse_coords(C)
    offs = stencil_offsets()
    return np.stack([coarse_neighbour(C, cc, offs[l]) for l in range(NSTENCIL)], axis=1)


def _blocked_vector(phi, sob, b, k):
    v = np.zeros(phi.shape[1:], dtype=np.complex128)
    v[:, sob[b], :, :] = phi[k][:, sob[b], :, :]
    return v


_POOL_FN = None


def _pool_call(item):
    return _POOL_FN(item)


def _pool_map(fn, items):
    """Independent H applications spread over forked worker processes (each
    returns only its small projected column); results come back in order."""
    global _POOL_FN
    nproc = min(16, os.cpu_count() or 1, len(items))
    if nproc <= 1:
        return [fn(i) for i in items]
    _POOL_FN = fn
    try:
        with mp.get_context("fork").Pool(nproc) as pool:
            return pool.map(_pool_call, items, chunksize=max(1, len(items) // (4 * nproc)))
    finally:
        _POOL_FN = None


def build_brute(op, phi, sob, C):
    """A by applying H to every blocked vector (Nc * Nvec applications)."""
    nc, nvec = sob.shape[0], phi.shape[0]
    cc = coarse_coords(C)
    offs = stencil_offsets()
    A = np.zeros((nc, NSTENCIL, nvec, nvec), dtype=np.complex128)

    def column(bk):
        b, k = bk
        w = op.H(_blocked_vector(phi, sob, b, k))
        return blk.project(phi, sob, w)  # c[a][j] = <phi^a_j, H phi^b_k>

    tasks = [(b, k) for b in range(nc) for k in range(nvec)]
    for (b, k), c in zip(tasks, _pool_map(column, tasks)):
        for l in range(NSTENCIL):
            # b = a + delta_l  <=>  a = b - delta_l
            a = coarse_neighbour(C, cc[b], -offs[l])
            A[a, l, :, k] = c[a]
    return A


def momenta(C):
    """p^s_mu for the 81 momenta, s indexed like l (n_x fastest)."""
    m = np.array([max(1, int(round(L / 3))) for L in C], dtype=np.float64)
    n = stencil_offsets().astype(np.float64)
    return 2.0 * np.pi * n * m / np.array(C, dtype=np.float64)


def build_fourier(op, phi, sob, C):
    """A from 81 phased probes per subspace vector (Sec. V.A.1)."""
    nc, nvec = sob.shape[0], phi.shape[0]
    xb = coarse_coords(C).astype(np.float64)  # block coordinates x^b
    p = momenta(C)  # (81, 4)
    offs = stencil_offsets().astype(np.float64)
    a_of_site, _, _ = blk.block_map(op.dims, tuple(d // c for d, c in zip(op.dims, C)))
    y = np.zeros((NSTENCIL, nc, nvec, nvec), dtype=np.complex128)

    def column(sk):
        s, k = sk
        z = np.exp(1j * xb @ p[s])  # z^s_b
        # phi~_k(p^s) = sum_b z^s_b phi^b_k : a phase per site by its block
        probe = phi[k] * z[a_of_site][None, :, None, None]
        return blk.project(phi, sob, op.H(probe))  # <phi^b_k', H phi~_k(p^s)>

    tasks = [(s, k) for s in range(NSTENCIL) for k in range(nvec)]
    for (s, k), c in zip(tasks, _pool_map(column, tasks)):
        y[s, :, :, k] = np.exp(-1j * xb @ p[s])[:, None] * c
    M = np.exp(1j * p @ offs.T)  # M_sl = exp(i p^s . delta^l)
    Minv = np.linalg.inv(M)
    # A[b][l] = sum_s Minv[l, s] y^s[b]
    return np.einsum("ls,sbjk->bljk", Minv, y)


def apply(A, c, C):
    """(A c)[a][j] = sum_l sum_k A[a][l][j][k] c[a+delta_l][k]; c (..., Nc, Nvec)."""
    nbr = neighbour_table(C)
    out = np.zeros_like(c)
    for l in range(NSTENCIL):
        out += np.einsum("ajk,...ak->...aj", A[:, l], c[..., nbr[:, l], :])
    return out


def to_dense(A, C):
    """The coarse operator as a dense (Nc*Nvec)^2 matrix."""
    nc, _, nvec, _ = A.shape
    nbr = neighbour_table(C)
    D = np.zeros((nc * nvec, nc * nvec), dtype=np.complex128)
    for a in range(nc):
        for l in range(NSTENCIL):
            b = nbr[a, l]
            D[a * nvec:(a + 1) * nvec, b * nvec:(b + 1) * nvec] += A[a, l]
    return D

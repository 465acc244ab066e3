"""Oracle block aggregation (test infrastructure only).

Blocked subspace of Sec. II: phi^b_k equals phi_k on block b and zero
elsewhere; the blocked vectors are orthonormalised block by block
(Gram-Schmidt); P_S = sum |phi^b_k><phi^b_k| acts as project (P^dagger) and
promote (P).  Blocks cover 4D sub-lattices of size B_mu and stretch over the
whole fifth dimension (Sec. V.A).

Block of an odd site: coarse coordinate floor(x_mu / B_mu), coarse index
a = cx + Cx*(cy + Cy*(cz + Cz*ct)).  Inside a block the odd sites are ordered
by their global checkerboard index.
"""
from __future__ import annotations

import numpy as np

from . import geometry as geo


def coarse_dims(dims, block):
    return tuple(d // b for d, b in zip(dims, block))


def block_map(dims, block):
    """For every odd site (cb order): its block index and its rank inside the
    block.  Returns (block_of_site, index_in_block, sites_of_block), the last
    of shape (Nc, n_sites_per_block) holding cb indices in ascending order."""
    c = geo.coords(dims)[geo.parity_sites(dims, 1)]  # (Vh, 4)
    C = coarse_dims(dims, block)
    bc = c // np.array(block)
    a = bc[:, 0] + C[0] * (bc[:, 1] + C[1] * (bc[:, 2] + C[2] * bc[:, 3]))
    nc = int(np.prod(C))
    sites = [np.nonzero(a == blk)[0] for blk in range(nc)]
    n = len(sites[0])
    assert all(len(s) == n for s in sites)
    sob = np.stack(sites)
    idx = np.empty(len(a), dtype=np.int64)
    for blk in range(nc):
        idx[sob[blk]] = np.arange(n)
    return a.astype(np.int64), idx, sob


def block_view(v, sob, blk):
    """The part of half-field(s) v (..., Ls, Vh, 4, 3) on block blk, flattened
    to (..., n_b) in (s, local site, spin, colour) order."""
    part = v[..., :, sob[blk], :, :]
    return part.reshape(part.shape[:-4] + (-1,))


def block_set(v, sob, blk, flat):
    shp = v[..., :, sob[blk], :, :].shape
    v[..., :, sob[blk], :, :] = flat.reshape(shp)


def _mgs(V):
    """Modified Gram-Schmidt on the rows of V (k = 0..n-1), in place."""
    for k in range(V.shape[0]):
        for j in range(k):
            V[k] -= np.vdot(V[j], V[k]) * V[j]
        V[k] /= np.sqrt(np.vdot(V[k], V[k]).real)
    return V


def orthonormalise(phi, sob, passes=2):
    """Block-local Gram-Schmidt of phi (Nvec, Ls, Vh, 4, 3), applied twice."""
    out = phi.copy()
    for blk in range(sob.shape[0]):
        V = block_view(out, sob, blk).copy()
        for _ in range(passes):
            _mgs(V)
        block_set(out, sob, blk, V)
    return out


def to_blocks(v, sob):
    """Half-field(s) (..., Ls, Vh, 4, 3) -> (..., Nc, n_b), each block's part
    flattened in (s, local site, spin, colour) order."""
    g = v[..., :, sob, :, :]  # (..., Ls, Nc, nsb, 4, 3)
    g = np.moveaxis(g, -5, -4)  # (..., Nc, Ls, nsb, 4, 3)
    return g.reshape(g.shape[:-4] + (-1,))


def from_blocks(vb, sob, Ls):
    """Inverse of to_blocks."""
    nc, nsb = sob.shape
    lead = vb.shape[:-2]
    g = vb.reshape(lead + (nc, Ls, nsb, 4, 3))
    g = np.moveaxis(g, -4, -5)  # (..., Ls, Nc, nsb, 4, 3)
    out = np.zeros(lead + (Ls, nc * nsb, 4, 3), dtype=np.complex128)
    out[..., :, sob.ravel(), :, :] = g.reshape(lead + (Ls, nc * nsb, 4, 3))
    return out


def project(phi, sob, psi):
    """c[a][j] = <phi^a_j, psi>; psi (..., Ls, Vh, 4, 3) -> (..., Nc, Nvec)."""
    Pb = to_blocks(phi, sob)  # (Nvec, Nc, n_b)
    vb = to_blocks(psi, sob)  # (..., Nc, n_b)
    return np.einsum("jai,...ai->...aj", Pb.conj(), vb)


def promote(phi, sob, c):
    """psi = sum_{a,k} phi^a_k c[a][k]; c (..., Nc, Nvec) -> half-field(s)."""
    Pb = to_blocks(phi, sob)  # (Nvec, Nc, n_b)
    vb = np.einsum("kai,...ak->...ai", Pb, c)
    return from_blocks(vb, sob, phi.shape[1])

"""Oracle geometry (test infrastructure only).

4D lattice of extents (X, Y, Z, T) with lexicographic site index
lex = x + X*(y + Y*(z + Z*t)); parity = (x+y+z+t) mod 2.  The odd
checkerboard (parity 1) carries the unknowns of the red-black preconditioned
operator (the M_oo ... M_eo structure of the Hermitian red-black operator in
Sec. IV).  A site of parity p has checkerboard index cb = lex >> 1 (X even).

Full-lattice fermion arrays in the oracle have shape
(..., Ls, T, Z, Y, X, 4, 3); half-fields have shape (..., Ls, V/2, 4, 3).
"""
from __future__ import annotations

import numpy as np


def volume(dims) -> int:
    X, Y, Z, T = dims
    return X * Y * Z * T


def coords(dims) -> np.ndarray:
    """Coordinates (x, y, z, t) of every site in lex order, shape (V, 4)."""
    X, Y, Z, T = dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel(), t.ravel()], axis=1)


def parity_sites(dims, p: int) -> np.ndarray:
    """Lex indices of the sites of parity p, ordered by checkerboard index."""
    assert dims[0] % 2 == 0
    c = coords(dims)
    par = c.sum(axis=1) % 2
    sites = np.nonzero(par == p)[0]
    # exactly one of lex 2cb, 2cb+1 has parity p, so sites[cb] >> 1 == cb
    assert np.array_equal(sites >> 1, np.arange(volume(dims) // 2))
    return sites


def embed(half: np.ndarray, dims, p: int) -> np.ndarray:
    """Half-field (..., Ls, Vh, 4, 3) -> full lattice (..., Ls, T, Z, Y, X, 4, 3), zero elsewhere."""
    X, Y, Z, T = dims
    lead = half.shape[:-3]
    full = np.zeros(lead + (volume(dims), 4, 3), dtype=np.complex128)
    full[..., parity_sites(dims, p), :, :] = half
    return full.reshape(lead + (T, Z, Y, X, 4, 3))


def extract(full: np.ndarray, dims, p: int) -> np.ndarray:
    """Full lattice (..., Ls, T, Z, Y, X, 4, 3) -> half-field on parity p."""
    lead = full.shape[:-6]
    f = full.reshape(lead + (volume(dims), 4, 3))
    return f[..., parity_sites(dims, p), :, :]


def neighbours(dims, p: int):
    """Neighbour tables for the sites of parity p (cb order).

    Returns a dict with, for every direction mu:
      fwd[mu], bwd[mu]   cb index (on parity 1-p) of x + mu and x - mu
      fwrap[mu], bwrap[mu]  whether that hop crosses the boundary
      lex                 lex index of each site of parity p
      lex_bwd[mu]         lex index of x - mu (to fetch U_mu(x - mu))
    """
    X, Y, Z, T = dims
    L = np.array(dims)
    sites = parity_sites(dims, p)
    c = coords(dims)[sites]
    out = {"lex": sites, "fwd": [], "bwd": [], "fwrap": [], "bwrap": [], "lex_bwd": []}
    for mu in range(4):
        e = np.zeros(4, dtype=np.int64)
        e[mu] = 1
        cf = (c + e) % L
        cb_ = (c - e) % L
        lf = cf[:, 0] + X * (cf[:, 1] + Y * (cf[:, 2] + Z * cf[:, 3]))
        lb = cb_[:, 0] + X * (cb_[:, 1] + Y * (cb_[:, 2] + Z * cb_[:, 3]))
        out["fwd"].append(lf >> 1)
        out["bwd"].append(lb >> 1)
        out["fwrap"].append(c[:, mu] == L[mu] - 1)
        out["bwrap"].append(c[:, mu] == 0)
        out["lex_bwd"].append(lb)
    return out

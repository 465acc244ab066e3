"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.

This module holds only input generation: gauge links, Gaussian sources,
random starting vectors and SU(3) gauge transformations.  It contains none of
the arithmetic of the method itself (no Dirac operator, no projector, no
solver), so that the CPU oracle and the HIP path can both draw from it without
sharing any computation.

Canonical layouts (the contract between generator, oracle and library):

* gauge   ``U[t][z][y][x][mu][a][b]``  complex128, ``mu`` = x, y, z, t
* odd half-field ``psi[rhs][s][cb][spin][colour]`` complex128 with
  ``cb = lex >> 1`` and ``lex = x + X*(y + Y*(z + Z*t))`` (X even)

Random numbers come from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gell_mann",
    "gauge_field",
    "su3_field",
    "gaussian_half_field",
    "half_field_shape",
    "rng",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0, 0, 1] = l[0, 1, 0] = 1
    l[1, 0, 1] = -1j
    l[1, 1, 0] = 1j
    l[2, 0, 0] = 1
    l[2, 1, 1] = -1
    l[3, 0, 2] = l[3, 2, 0] = 1
    l[4, 0, 2] = -1j
    l[4, 2, 0] = 1j
    l[5, 1, 2] = l[5, 2, 1] = 1
    l[6, 1, 2] = -1j
    l[6, 2, 1] = 1j
    l[7, 0, 0] = l[7, 1, 1] = 1 / np.sqrt(3)
    l[7, 2, 2] = -2 / np.sqrt(3)
    return l


def _exp_i_eps_h(omega: np.ndarray, eps: float) -> np.ndarray:
    """exp(i*eps*H) with H = sum_a omega_a lambda_a / 2 (traceless Hermitian),
    through the eigendecomposition of H so the result is unitary to rounding."""
    h = np.einsum("...a,aij->...ij", omega, gell_mann()) * 0.5
    w, v = np.linalg.eigh(h)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ij,...j,...kj->...ik", v, ph, v.conj())


def gauge_field(dims, eps: float, seed: int) -> np.ndarray:
    """Seeded SU(3) links U = exp(i eps H), H Gaussian traceless Hermitian.

    ``dims`` = (X, Y, Z, T).  Returns complex128 of shape (T, Z, Y, X, 4, 3, 3).
    The eight Gaussian coefficients of each link are drawn in canonical order
    ``standard_normal((T, Z, Y, X, 4, 8))``.
    """
    X, Y, Z, T = dims
    om = rng(seed).standard_normal((T, Z, Y, X, 4, 8))
    return np.ascontiguousarray(_exp_i_eps_h(om, eps))


def su3_field(dims, seed: int, eps: float = 3.0) -> np.ndarray:
    """One random SU(3) matrix per site, shape (T, Z, Y, X, 3, 3)."""
    X, Y, Z, T = dims
    om = rng(seed).standard_normal((T, Z, Y, X, 8))
    return np.ascontiguousarray(_exp_i_eps_h(om, eps))


def half_field_shape(dims, Ls: int, nrhs: int | None = None):
    X, Y, Z, T = dims
    vh = X * Y * Z * T // 2
    s = (Ls, vh, 4, 3)
    return s if nrhs is None else (nrhs,) + s


def gaussian_half_field(dims, Ls: int, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Complex Gaussian odd half-field(s), real and imaginary parts N(0, 1),
    drawn in canonical layout order (real part block first, then imaginary)."""
    shape = half_field_shape(dims, Ls, nrhs)
    g = rng(seed)
    re = g.standard_normal(shape)
    im = g.standard_normal(shape)
    return re + 1j * im


def gaussian_coarse(Nc: int, nvec: int, seed: int, n: int) -> np.ndarray:
    """n complex Gaussian coarse vectors c[k][a][j] (Nc sites, nvec
    components), real and imaginary parts N(0, 1)."""
    g = rng(seed)
    re = g.standard_normal((n, Nc, nvec))
    im = g.standard_normal((n, Nc, nvec))
    return re + 1j * im


def _coarse_index(C, c):
    """Coarse lexicographic index of coordinates c (..., 4), x fastest, on the torus."""
    c = np.mod(c, np.array(C))
    return c[..., 0] + C[0] * (c[..., 1] + C[1] * (c[..., 2] + C[2] * c[..., 3]))


def coarse_stencil_operator(C, nvec: int, seed: int, mass: float = 0.1, fill: float = 0.25) -> np.ndarray:
    """A seeded Hermitian positive-definite block stencil in the layout of the
    little Dirac operator, A[a][l][j][k] with l = sum_mu (delta_mu + 1) 3^mu
    (delta_x fastest, l = 40 the site), A[a][l] = A[a + delta_l][80 - l]^+.

    It is a lattice Laplacian whose hopping matrices on the eight axis
    neighbours are a random pure gauge, U_mu(a) = g_a g_{a+mu}^+ with seeded
    unitary g_a (so the lowest mode sits at mass), (8 + mass) on the
    diagonal, plus a random Hermitian fill on all 81 stencil points whose
    blocks have spectral norm fill * mass / 80 each: the spectrum lies in
    [mass (1 - fill), 16 + mass (1 + fill)].  Coarse extents must be >= 3 so
    the 81 offsets are distinct."""
    C = tuple(int(c) for c in C)
    assert min(C) >= 3
    g = rng(seed)
    nc = int(np.prod(C))
    a = np.arange(nc)
    coords = np.stack([a % C[0], (a // C[0]) % C[1], (a // (C[0] * C[1])) % C[2], a // (C[0] * C[1] * C[2])], 1)
    offs = np.array([[(l // 3 ** mu) % 3 - 1 for mu in range(4)] for l in range(81)])
    A = np.zeros((nc, 81, nvec, nvec), dtype=np.complex128)

    def gauss(*shape):
        return g.standard_normal(shape) + 1j * g.standard_normal(shape)

    def unitary():
        q, r = np.linalg.qr(gauss(nvec, nvec))
        return q * (np.diag(r) / np.abs(np.diag(r)))[None, :]

    gsite = [unitary() for _ in range(nc)]

    for l in range(41):  # one of each pair (l, 80 - l); l = 40 is the site itself
        for site in range(nc):
            B = gauss(nvec, nvec)
            B *= fill * mass / 80 / np.linalg.norm(B, 2)
            if l == 40:
                B = 0.5 * (B + B.conj().T)
            if l == 40:
                A[site, 40] += B + (8.0 + mass) * np.eye(nvec)
                continue
            b = _coarse_index(C, coords[site] + offs[l])
            if int(np.abs(offs[l]).sum()) == 1:  # minus the pure-gauge hop
                B = B - gsite[site] @ gsite[b].conj().T
            A[site, l] += B
            A[b, 80 - l] += B.conj().T
    return A


# Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
# easy as 1, 2, 3", SC 2011): the counter-based generator the library uses
# to draw subspace starting vectors on the device when the caller passes
# none.  Written here from the published definition for the tests that
# reproduce those vectors.
_PHILOX_M = (0xD2511F53, 0xCD9E8D57)
_PHILOX_W = (0x9E3779B9, 0xBB67AE85)
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: uint64 array (..., 4) of 32-bit words; key: two 32-bit words.
    Returns the four 32-bit output words (..., 4) as uint64."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) & _MASK32 for i in range(4)]
    k0, k1 = np.uint64(key[0]) & _MASK32, np.uint64(key[1]) & _MASK32
    m0, m1 = np.uint64(_PHILOX_M[0]), np.uint64(_PHILOX_M[1])
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(_PHILOX_W[0])) & _MASK32
            k1 = (k1 + np.uint64(_PHILOX_W[1])) & _MASK32
        p0 = m0 * c[0]  # 64-bit products of 32-bit words cannot overflow
        p1 = m1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=-1)


def philox_gaussian(n: int, seed: int, offset: int = 0) -> np.ndarray:
    """n complex Gaussian numbers (real and imaginary parts N(0, 1)), number
    i from the Philox4x32-10 block with counter (i lo, i hi, 0, 0) and key
    (seed lo, seed hi), i = offset .. offset + n - 1: two 53-bit uniforms u, v
    from the word pairs (0, 1) and (2, 3), then Box-Muller,
    sqrt(-2 ln(1 - u)) * (cos 2 pi v, sin 2 pi v)."""
    i = np.arange(offset, offset + n, dtype=np.uint64)
    ctr = np.stack([i & _MASK32, i >> np.uint64(32), np.zeros_like(i), np.zeros_like(i)], axis=-1)
    w = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    scale = 2.0 ** -53
    u = (((w[:, 1] << np.uint64(32)) | w[:, 0]) >> np.uint64(11)).astype(np.float64) * scale
    v = (((w[:, 3] << np.uint64(32)) | w[:, 2]) >> np.uint64(11)).astype(np.float64) * scale
    r = np.sqrt(-2.0 * np.log1p(-u))
    return r * np.cos(2.0 * np.pi * v) + 1j * r * np.sin(2.0 * np.pi * v)


def philox_subspace(dims, Ls: int, nvec: int, seed: int) -> np.ndarray:
    """The nvec starting vectors the library draws for hdcg_setup without
    given vectors: canonical Phi[k][s][cb][spin][colour], complex number i of
    the whole array from philox_gaussian."""
    shape = half_field_shape(dims, Ls, nvec)
    return philox_gaussian(int(np.prod(shape)), seed).reshape(shape)

"""Pins of the oracle's Fourier-trick build of the little Dirac operator
(Sec. V.A.1) at the coarse extents the workloads use, where the momenta
p_mu = 2 pi n m_mu / Lc_mu have m_mu > 1 or Lc_mu not a multiple of 3 and the
phase matrix is no longer a plain DFT: Lc = 4 (m = 1), 6 (m = 2) and 8
(m = 3).  The reference is the definition A[a][l][j][k] = <phi^a_j | H |
phi^{a+delta_l}_k> evaluated by brute force on sampled columns (b, k): one H
application of the blocked vector phi^b_k, projected onto every block.  The
sampled blocks include the corner block, whose stencil wraps around the
coarse torus in every direction, so a phase that is not periodic, a wrong
momentum or a wrong inversion of the phase matrix fails here.

Ls = 1 keeps the fine operator cheap (the identity does not depend on Ls)."""
import numpy as np
import pytest

import synth
from oracle import blocks as blk
from oracle import coarse as crs
from oracle.dwf import DWF


def _sampled_columns(op, phi, sob, C, cols):
    """{(b, k): c[a][j] = <phi^a_j, H phi^b_k>} for the sampled columns."""
    out = {}
    for b, k in cols:
        v = np.zeros(phi.shape[1:], dtype=np.complex128)
        v[:, sob[b], :, :] = phi[k][:, sob[b], :, :]
        out[(b, k)] = blk.project(phi, sob, op.H(v))
    return out


def _check(A, cols, C, tol=1e-12):
    cc = crs.coarse_coords(C)
    offs = crs.stencil_offsets()
    scale = max(np.abs(c).max() for c in cols.values())
    for (b, k), c in cols.items():
        for l in range(81):
            a = crs.coarse_neighbour(C, cc[b], -offs[l])  # b = a + delta_l
            err = np.abs(A[a, l, :, k] - c[a]).max()
            assert err <= tol * scale, (b, k, l, err)
        # blocks farther than one step in some direction see nothing of phi^b_k
        near = {int(crs.coarse_neighbour(C, cc[b], -offs[l])) for l in range(81)}
        far = [a for a in range(len(cc)) if a not in near]
        if far:
            assert np.abs(c[far]).max() <= 1e-13 * scale


@pytest.mark.slow
@pytest.mark.parametrize("dims,seed", [
    ((16, 12, 12, 12), 31),   # coarse 4x3x3x3: m = (1, 1, 1, 1), Lc = 4 not a multiple of 3
    ((24, 12, 12, 16), 32),   # coarse 6x3x3x4: m = (2, 1, 1, 1), the configs' 6^3x12 extents
    ((32, 12, 12, 12), 33),   # coarse 8x3x3x3: m = (3, 1, 1, 1), the 8 of a 16^3x32 grid
])
def test_fourier_equals_brute_force_columns(dims, seed):
    Ls, block, nvec = 1, (4, 4, 4, 4), 2
    op = DWF(synth.gauge_field(dims, 0.5, seed), dims, Ls, 1.8, 0.01)
    _, _, sob = blk.block_map(dims, block)
    C = blk.coarse_dims(dims, block)
    phi = blk.orthonormalise(synth.gaussian_half_field(dims, Ls, seed + 100, nrhs=nvec), sob)
    A = crs.build_fourier(op, phi, sob, C)
    nc = sob.shape[0]
    # corner block (wraps in all four directions), a block at the far end of
    # x, and an interior one
    far_x = C[0] - 1
    mid = 1 + C[0] * (1 + C[1] * (1 + C[2] * 1))
    cols = _sampled_columns(op, phi, sob, C, [(0, 0), (far_x, 1), (mid % nc, 0)])
    _check(A, cols, C)
    # Hermiticity A[a][l] = A[a + delta_l][80 - l]^+ over the whole operator
    nbr = crs.neighbour_table(C)
    scale = np.abs(A).max()
    for l in range(81):
        assert np.abs(A[:, l] - np.conj(np.swapaxes(A[nbr[:, l], 80 - l], 1, 2))).max() <= 1e-12 * scale


def test_momenta_reading():
    """m_mu = round(Lc_mu / 3) and the phases are periodic on the coarse
    torus (exp(i p Lc) = 1 for every momentum), with the 3 x 3 phase matrix of
    each direction invertible for Lc >= 3."""
    for C in [(4, 3, 3, 3), (6, 3, 3, 4), (8, 3, 3, 3), (6, 6, 6, 12), (4, 4, 4, 8), (5, 7, 3, 9)]:
        p = crs.momenta(C)
        assert p.shape == (81, 4)
        m = np.array([max(1, round(L / 3)) for L in C])
        n = crs.stencil_offsets()
        assert np.allclose(p, 2 * np.pi * n * m / np.array(C))
        assert np.allclose(np.exp(1j * p * np.array(C)), 1.0, atol=1e-12)
        for mu, L in enumerate(C):
            F = np.exp(1j * 2 * np.pi * m[mu] / L * np.outer([-1, 0, 1], [-1, 0, 1]))
            assert abs(np.linalg.det(F)) > 1e-3

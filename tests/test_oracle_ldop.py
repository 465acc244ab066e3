"""Pins of the oracle's second deflation level (Sec. V.B, "Little Dirac
operator deflation").

- the free global vectors promote to the subspace vectors summed over the
  blocks, and A between them is H between those fine vectors (A = P^+ H P);
- the third level: Z orthonormal, Z^+ A Z = diag(D), and Z D^-1 Z^+ inverts
  A on span(Z);
- deflated CG equals a dense solve; with exact low eigenvectors as Z its
  iteration count obeys the CG bound of the deflated spectrum
  (lambda_max / lambda_{n+1}) and is below plain CG's;
- shifted inverse iteration equals the normalised power of the dense
  shifted inverse, and lowers the Rayleigh quotients of coarse noise.
"""
import numpy as np
import pytest

import synth
from oracle import blocks as blk
from oracle import coarse as crs
from oracle import ldop
from oracle.cg import cg
from oracle.dwf import DWF, inner


@pytest.fixture(scope="module")
def small():
    """6^4 x Ls4, 2^4 blocks, 4 vectors after one inverse-iteration step (so
    that A has the low modes deflation is for)."""
    dims, Ls, block, nvec = (6, 6, 6, 6), 4, (2, 2, 2, 2), 4
    op = DWF(synth.gauge_field(dims, 0.6, 61), dims, Ls, 1.8, 0.01)
    _, _, sob = blk.block_map(dims, block)
    raw = synth.gaussian_half_field(dims, Ls, 62, nrhs=nvec)
    vv = np.array([cg(op.H, v, tol=1e-4)[0] for v in raw])
    phi = blk.orthonormalise(vv, sob)
    C = blk.coarse_dims(dims, block)
    A = crs.build_fourier(op, phi, sob, C)
    return op, phi, sob, C, A


def test_free_vectors_are_the_summed_subspace(small):
    op, phi, sob, C, A = small
    Nc, nvec = A.shape[0], A.shape[2]
    W = ldop.free_global_vectors(Nc, nvec)
    fine = [blk.promote(phi, sob, w) for w in W]
    for k in range(nvec):
        want = phi[k] / np.sqrt(Nc)  # the blocked vectors of k, all blocks
        assert np.abs(fine[k] - want).max() < 1e-13
    for j in range(nvec):
        for k in range(nvec):
            lhs = np.vdot(W[j], crs.apply(A, W[k], C))
            rhs = inner(fine[j], op.H(fine[k]))
            assert abs(lhs - rhs) < 1e-10 * abs(rhs) + 1e-12


def _dense_case(seed, Nc=20, nvec=3):
    rng = np.random.default_rng(seed)
    C = (3, 3, 3, 3)
    Nc = 81
    # an A in the coarse storage whose dense form is Hermitian positive:
    # a diagonal site term plus weak Hermitian hops
    A = np.zeros((Nc, 81, nvec, nvec), dtype=complex)
    nbr = crs.neighbour_table(C)
    for a in range(Nc):
        for l in range(81):
            if l == 40:
                continue
            if l < 40:
                b = nbr[a, l]
                m = 0.05 * (rng.standard_normal((nvec, nvec)) + 1j * rng.standard_normal((nvec, nvec)))
                A[a, l] += m
                A[b, 80 - l] += m.conj().T
    D = crs.to_dense(A, C)
    shift = -np.linalg.eigvalsh(D)[0] + 1e-3
    for a in range(Nc):
        A[a, 40] += shift * np.eye(nvec)
    return A, C


def test_third_level_and_deflated_cg_dense():
    A, C = _dense_case(63)
    Nc, nvec = A.shape[0], A.shape[2]
    Dn = crs.to_dense(A, C)
    ev, V = np.linalg.eigh(Dn)
    rng = np.random.default_rng(64)
    b = (rng.standard_normal((Nc, nvec)) + 1j * rng.standard_normal((Nc, nvec)))
    xd = np.linalg.solve(Dn, b.ravel()).reshape(b.shape)
    nd = 12
    W = ldop.orthonormal_basis(V[:, :nd].T.reshape(nd, Nc, nvec) @ np.eye(nvec))
    Z, Dz, AZ = ldop.third_level(A, C, W)
    Zf = Z.reshape(nd, -1)
    assert np.abs(Zf.conj() @ Zf.T - np.eye(nd)).max() < 1e-12
    assert np.abs(Zf.conj() @ AZ.reshape(nd, -1).T - np.diag(Dz)).max() < 1e-12 * ev.max()
    assert np.allclose(Dz, ev[:nd], rtol=1e-10)
    z = Zf.T @ rng.standard_normal(nd)
    Qz = Zf.T @ ((Zf.conj() @ (Dn @ z)) / Dz)
    assert np.abs(Qz - z).max() < 1e-10 * np.abs(z).max()
    tol = 1e-10
    x, it, rel = ldop.deflated_cg(A, C, b, Z, Dz, AZ, tol=tol)
    assert rel <= tol and np.abs(x - xd).max() < 1e-7 * np.abs(xd).max()
    # exact eigenvectors: CG on the remaining spectrum
    kappa = ev[-1] / ev[nd]
    bound = int(np.ceil(0.5 * np.sqrt(kappa) * np.log(2 / tol))) + 1
    _, it_cg, _ = cg(lambda u: Dn @ u, b.ravel(), tol=tol)
    assert it <= bound and it < it_cg, (it, bound, it_cg)


def test_inverse_iteration_equals_power_of_the_inverse():
    A, C = _dense_case(66)
    Nc, nvec = A.shape[0], A.shape[2]
    Dn = crs.to_dense(A, C)
    rng = np.random.default_rng(67)
    V0 = rng.standard_normal((2, Nc, nvec)) + 1j * rng.standard_normal((2, Nc, nvec))
    shift = 0.05
    Vi = ldop.inverse_iteration(A, C, V0, n_steps=3, shift=shift, tol=1e-13)
    Minv = np.linalg.inv(Dn + shift * np.eye(len(Dn)))
    for v0, v in zip(V0, Vi):
        want = np.linalg.matrix_power(Minv, 3) @ v0.ravel()
        want /= np.linalg.norm(want)
        assert np.abs(v.ravel() - want).max() < 1e-8


def test_deflated_cg_with_free_and_inverse_iteration_vectors(small):
    op, phi, sob, C, A = small
    Nc, nvec = A.shape[0], A.shape[2]
    rng = np.random.default_rng(65)
    V0 = rng.standard_normal((6, Nc, nvec)) + 1j * rng.standard_normal((6, Nc, nvec))
    Vi = ldop.inverse_iteration(A, C, V0, n_steps=3, shift=0.0, tol=1e-9)
    rq0 = [np.vdot(v, crs.apply(A, v, C)).real / np.vdot(v, v).real for v in V0]
    rqi = [np.vdot(v, crs.apply(A, v, C)).real for v in Vi]
    assert np.mean(rqi) < 0.6 * np.mean(rq0), (rqi, rq0)
    W = ldop.orthonormal_basis(np.concatenate([ldop.free_global_vectors(Nc, nvec), Vi]))
    Z, Dz, AZ = ldop.third_level(A, C, W)
    b = rng.standard_normal((Nc, nvec)) + 1j * rng.standard_normal((Nc, nvec))
    x, it, rel = ldop.deflated_cg(A, C, b, Z, Dz, AZ, tol=1e-10)
    xd = np.linalg.solve(crs.to_dense(A, C), b.ravel()).reshape(b.shape)
    assert rel <= 1e-10 and np.abs(x - xd).max() < 1e-7 * np.abs(xd).max()
    _, it_cg, _ = cg(lambda u: crs.apply(A, u, C), b, tol=1e-10)
    assert it < it_cg, (it, it_cg)

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


def test_truncation_keeps_one_hop_terms():
    A, C = _dense_case(68)
    T = ldop.truncate(A, shift=0.3)
    Dn, Dt = crs.to_dense(A, C), crs.to_dense(T, C)
    assert np.abs(Dt - Dt.conj().T).max() < 1e-14
    coords = crs.coarse_coords(C)
    nvec = A.shape[2]
    Cc = np.array(C)
    for a in range(0, A.shape[0], 7):
        for b in range(A.shape[0]):
            d = np.abs(coords[a] - coords[b])
            d = np.minimum(d, Cc - d).sum()  # taxicab hops on the torus
            blk_t = Dt[a * nvec:(a + 1) * nvec, b * nvec:(b + 1) * nvec]
            blk_a = Dn[a * nvec:(a + 1) * nvec, b * nvec:(b + 1) * nvec]
            want = blk_a + (0.3 * np.eye(nvec) if a == b else 0) if d <= 1 else np.zeros_like(blk_a)
            assert np.abs(blk_t - want).max() < 1e-14


def test_chebyshev_residual_polynomial():
    """On an eigenvector with eigenvalue x the iteration leaves
    R_n(x) = T_n((d - x)/c) / T_n(d/c) times it as residual (the definition of
    the Chebyshev iteration), T_n from numpy's Chebyshev series, for x inside
    and outside [lo, hi] and for orders 1, 2 and 16."""
    M, ev, Q = _hpd(30, 69, lo=0.05, hi=60.0)
    lo, hi = 0.5, 45.0
    d, c = 0.5 * (hi + lo), 0.5 * (hi - lo)
    for n in (1, 2, 16):
        Tn = np.zeros(n + 1)
        Tn[n] = 1.0
        norm = np.polynomial.chebyshev.chebval(d / c, Tn)
        for i in range(30):
            v = Q[:, i]
            y = ldop.chebyshev_inverse(lambda u: M @ u, v, lo, hi, n)
            want = np.polynomial.chebyshev.chebval((d - ev[i]) / c, Tn) / norm
            res = v - M @ y
            assert np.abs(res - want * v).max() < 1e-10 * max(1.0, abs(want)), (n, ev[i], want)
    # order 1 is the Jacobi-like step y = r / d
    v = Q[:, 0]
    assert np.allclose(ldop.chebyshev_inverse(lambda u: M @ u, v, lo, hi, 1), v / d, rtol=0, atol=1e-15)


def _hpd(n, seed, lo=1e-3, hi=30.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    ev = np.exp(rng.uniform(np.log(lo), np.log(hi), n))
    return Q @ np.diag(ev) @ Q.conj().T, ev, Q


def test_adef1_solves_and_reduces_iterations(small):
    op, phi, sob, C, A = small
    Nc, nvec = A.shape[0], A.shape[2]
    rng = np.random.default_rng(70)
    V0 = rng.standard_normal((6, Nc, nvec)) + 1j * rng.standard_normal((6, Nc, nvec))
    W = ldop.orthonormal_basis(np.concatenate([ldop.free_global_vectors(Nc, nvec),
                                               ldop.inverse_iteration(A, C, V0, 3, 0.0, 1e-9)]))
    Z, Dz, AZ = ldop.third_level(A, C, W)
    T = ldop.truncate(A, shift=0.1)
    ev = np.linalg.eigvalsh(crs.to_dense(A, C))
    lo, hi = 0.5, 1.1 * ev[-1]

    def M(r):
        return ldop.chebyshev_inverse(lambda u: crs.apply(T, u, C), r, lo, hi, 8)

    b = rng.standard_normal((Nc, nvec)) + 1j * rng.standard_normal((Nc, nvec))
    x, it, rel = ldop.adef1_solve(A, C, b, Z, Dz, AZ, M, tol=1e-10)
    xd = np.linalg.solve(crs.to_dense(A, C), b.ravel()).reshape(b.shape)
    assert rel <= 1e-10 and np.abs(x - xd).max() < 1e-7 * np.abs(xd).max()
    _, it_d, _ = ldop.deflated_cg(A, C, b, Z, Dz, AZ, tol=1e-10)
    assert it < it_d, (it, it_d)


def test_trunc_cg_is_the_fixed_order_cg_on_q_trunc():
    """M_IRS(Q_trunc) (Sec. V.B, with the shifted CG of Sec. IV.C): one
    iteration is the steepest-descent step (r, r) / (r, T r) r; enough
    iterations reach the dense solve of Q_trunc + shift; on an eigenvector of
    T the first iteration is already its exact inverse; zero stays zero."""
    A, C = _dense_case(72)
    T = ldop.truncate(A, shift=0.5)
    Dt = crs.to_dense(T, C)
    ev, U = np.linalg.eigh(Dt)
    assert ev[0] > 0
    rng = np.random.default_rng(73)
    r = rng.standard_normal((A.shape[0], A.shape[2])) + 1j * rng.standard_normal((A.shape[0], A.shape[2]))
    Tr = crs.apply(T, r, C)
    y1 = ldop.trunc_cg(T, C, r, 1)
    want = (np.vdot(r, r) / np.vdot(r, Tr)).real * r
    assert np.abs(y1 - want).max() < 1e-13 * np.abs(want).max()
    yn = ldop.trunc_cg(T, C, r, 300)
    xd = np.linalg.solve(Dt, r.ravel()).reshape(r.shape)
    assert np.abs(yn - xd).max() < 1e-10 * np.abs(xd).max()
    v = U[:, 5].reshape(r.shape)
    assert np.abs(ldop.trunc_cg(T, C, v, 1) - v / ev[5]).max() < 1e-12 * np.abs(v).max() / ev[5]
    assert np.abs(ldop.trunc_cg(T, C, np.zeros_like(r), 4)).max() == 0.0


def test_adef1_with_the_truncated_cg_solves_and_reduces_iterations(small):
    """ADEF1 with M = M_IRS(Q_trunc) (8 CG iterations on Q_trunc + 0.1) in
    place of the Chebyshev polynomial: the flexible coarse solve reaches the
    dense solution, in fewer iterations than deflated CG."""
    op, phi, sob, C, A = small
    Nc, nvec = A.shape[0], A.shape[2]
    rng = np.random.default_rng(74)
    V0 = rng.standard_normal((6, Nc, nvec)) + 1j * rng.standard_normal((6, Nc, nvec))
    W = ldop.orthonormal_basis(np.concatenate([ldop.free_global_vectors(Nc, nvec),
                                               ldop.inverse_iteration(A, C, V0, 3, 0.0, 1e-9)]))
    Z, Dz, AZ = ldop.third_level(A, C, W)
    T = ldop.truncate(A, shift=0.1)
    b = rng.standard_normal((Nc, nvec)) + 1j * rng.standard_normal((Nc, nvec))
    x, it, rel = ldop.adef1_solve(A, C, b, Z, Dz, AZ, lambda r: ldop.trunc_cg(T, C, r, 8), tol=1e-10)
    xd = np.linalg.solve(crs.to_dense(A, C), b.ravel()).reshape(b.shape)
    assert rel <= 1e-10 and np.abs(x - xd).max() < 1e-7 * np.abs(xd).max()
    _, it_d, _ = ldop.deflated_cg(A, C, b, Z, Dz, AZ, tol=1e-10)
    assert it < it_d, (it, it_d)


def test_adef1_is_identity_on_the_deflation_space(small):
    """M_1 A z = z for z in span(Z): Q A z = z because Z^+ A Z = D, and the
    M term then acts on A z - A z = 0 (any M, here a plain scaling)."""
    op, phi, sob, C, A = small
    Nc, nvec = A.shape[0], A.shape[2]
    W = ldop.orthonormal_basis(ldop.free_global_vectors(Nc, nvec))
    Z, Dz, AZ = ldop.third_level(A, C, W)
    M1 = ldop.adef1_preconditioner(Z, Dz, AZ, lambda r: 0.37 * r)
    rng = np.random.default_rng(71)
    coef = rng.standard_normal(len(Z)) + 1j * rng.standard_normal(len(Z))
    z = np.einsum("k,k...->...", coef, Z)
    out = M1(crs.apply(A, z, C))
    assert np.abs(out - z).max() < 1e-11 * np.abs(z).max()
    # and on a vector A-orthogonal to span(Z) it is M alone
    v = rng.standard_normal((Nc, nvec)) + 1j * rng.standard_normal((Nc, nvec))
    v = v - np.einsum("k,k...->...", (Z.reshape(len(Z), -1).conj() @ crs.apply(A, v, C).ravel()) / Dz, Z)
    out = M1(crs.apply(A, v, C))
    assert np.abs(out - 0.37 * crs.apply(A, v, C)).max() < 1e-11 * np.abs(v).max()


def test_chebyshev_minimax_on_the_paper_interval():
    """With the paper's interval [0.5, 45] and order 16 (Table "optimised"),
    the residual factor 1 - x p(x) of the Chebyshev iteration stays within
    1 / T_16(d/c) on the whole interval and reaches it at the 17 Chebyshev
    extrema x_j = d - c cos(j pi / 16) (the minimax property of T_n)."""
    lo, hi, n = 0.5, 45.0, 16
    d, c = 0.5 * (hi + lo), 0.5 * (hi - lo)
    bound = 1.0 / np.cosh(n * np.arccosh(d / c))
    xs = np.concatenate([np.linspace(lo, hi, 997), d - c * np.cos(np.arange(n + 1) * np.pi / n)])
    M = np.diag(xs)
    v = np.ones(len(xs))
    y = ldop.chebyshev_inverse(lambda u: M @ u, v, lo, hi, n)
    res = v - xs * y
    assert np.abs(res).max() <= bound * (1 + 1e-9)
    ext = res[-(n + 1):]
    assert np.allclose(np.abs(ext), bound, rtol=1e-7)
    assert np.all(np.sign(ext[1:]) == -np.sign(ext[:-1]))  # equioscillation

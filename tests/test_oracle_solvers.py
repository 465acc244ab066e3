"""Pins of the oracle's CG, block aggregation, coarse operator and HDCG
layers: dense solves on tiny lattices, the QR factorisation, adjointness,
brute force against the Fourier trick, Hermiticity and translation invariance
of the coarse operator, the projector identities of Sec. II and the A-DEF2
invariants of Sec. IV.E.1."""
import numpy as np
import pytest

import synth
from oracle import blocks as blk
from oracle import coarse as crs
from oracle import geometry as geo
from oracle import hdcg
from oracle.cg import cg, cg_fixed
from oracle.dwf import DWF, inner, norm2


def _dense(apply, shape):
    n = int(np.prod(shape))
    basis = np.eye(n, dtype=complex).reshape((n,) + tuple(shape))
    return apply(basis).reshape(n, n).T


def test_cg_matches_dense_solve():
    dims, Ls = (4, 4, 4, 4), 1
    op = DWF(synth.gauge_field(dims, 0.5, 11), dims, Ls, 1.8, 0.01)
    b = synth.gaussian_half_field(dims, Ls, 12)
    Hd = _dense(op.H, op.half_shape())
    xd = np.linalg.solve(Hd, b.ravel())
    x, it, tr = cg(op.H, b, tol=1e-10)
    assert tr <= 1e-10
    assert np.abs(x.ravel() - xd).max() <= 1e-6 * np.abs(xd).max()


def test_cg_free_field_iteration_bound():
    """A plane-wave source lives in a 4Ls-dimensional invariant subspace, so
    CG needs at most #distinct eigenvalues of K^+K iterations."""
    dims, Ls = (4, 4, 4, 4), 4
    U = np.broadcast_to(np.eye(3), (4, 4, 4, 4, 4, 3, 3)).copy()
    op = DWF(U, dims, Ls, 1.8, 0.01)
    c = geo.coords(dims)[geo.parity_sites(dims, 1)]
    p = np.array([np.pi / 2, 0, np.pi, 3 * np.pi / 4])
    w = synth.rng(3).standard_normal((Ls, 4)) + 0j
    b = np.einsum("v,si,c->svic", np.exp(1j * c @ p), w, np.array([1.0, 0, 0]))
    x, it, tr = cg(op.H, b, tol=1e-12)
    assert tr <= 1e-12 and it <= 4 * Ls + 1


def test_cg_fixed_runs_exact_count_and_converges_to_inverse():
    dims, Ls = (4, 4, 4, 4), 1
    op = DWF(synth.gauge_field(dims, 0.5, 13), dims, Ls, 1.8, 0.01)
    b = synth.gaussian_half_field(dims, Ls, 14)
    lam = 1.0
    Hd = _dense(op.H, op.half_shape()) + lam * np.eye(op.unknowns())
    z = hdcg.m_irs(op, b, 300, lam)
    assert np.abs(Hd @ z.ravel() - b.ravel()).max() < 1e-9 * np.abs(b).max()
    # one iteration is the steepest-descent step alpha b
    z1 = cg_fixed(lambda v: op.H(v) + lam * v, b, 1)
    alpha = norm2(b) / inner(b, op.H(b) + lam * b).real
    assert np.abs(z1 - alpha * b).max() < 1e-15 * np.abs(b).max() * 10


def test_block_map_bit_exact():
    dims, block = (8, 8, 12, 8), (4, 4, 4, 4)
    a, idx, sob = blk.block_map(dims, block)
    C = blk.coarse_dims(dims, block)
    assert C == (2, 2, 3, 2) and sob.shape == (24, 128)
    c = geo.coords(dims)[geo.parity_sites(dims, 1)]
    bc = c // 4
    assert np.array_equal(a, bc[:, 0] + 2 * (bc[:, 1] + 2 * (bc[:, 2] + 3 * bc[:, 3])))
    assert np.array_equal(np.sort(sob.ravel()), np.arange(len(a)))
    assert np.array_equal(sob[a, idx], np.arange(len(a)))
    assert all(np.all(np.diff(row) > 0) for row in sob)


@pytest.fixture(scope="module")
def small_two_level():
    """12^4 x Ls=2, 4^4 blocks (coarse 3^4), Nvec = 2."""
    dims, Ls, block, nvec = (12, 12, 12, 12), 2, (4, 4, 4, 4), 2
    op = DWF(synth.gauge_field(dims, 0.5, 21), dims, Ls, 1.8, 0.01)
    _, _, sob = blk.block_map(dims, block)
    raw = synth.gaussian_half_field(dims, Ls, 22, nrhs=nvec)
    phi = blk.orthonormalise(raw, sob)
    C = blk.coarse_dims(dims, block)
    Af = crs.build_fourier(op, phi, sob, C)
    return op, raw, phi, sob, C, Af


def test_gram_schmidt_equals_qr(small_two_level):
    op, raw, phi, sob, C, _ = small_two_level
    Pr = blk.to_blocks(raw, sob)
    Pp = blk.to_blocks(phi, sob)
    for b in (0, 17, 80):
        Q, R = np.linalg.qr(Pr[:, b, :].T)
        Q = Q * np.sign(np.diag(R).real)[None, :]  # unique QR: positive diagonal
        assert np.abs(Q.T - Pp[:, b, :]).max() < 1e-13
        G = Pp[:, b, :].conj() @ Pp[:, b, :].T
        assert np.abs(G - np.eye(2)).max() < 1e-14


def test_project_promote_adjoint_and_identities(small_two_level):
    op, _, phi, sob, C, _ = small_two_level
    psi = synth.gaussian_half_field(op.dims, op.Ls, 30)
    c = synth.rng(31).standard_normal((81, 2)) + 1j * synth.rng(32).standard_normal((81, 2))
    lhs = np.vdot(c, blk.project(phi, sob, psi))
    rhs = inner(blk.promote(phi, sob, c), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    assert np.abs(blk.project(phi, sob, blk.promote(phi, sob, c)) - c).max() < 1e-13
    Pv = blk.promote(phi, sob, blk.project(phi, sob, psi))
    PPv = blk.promote(phi, sob, blk.project(phi, sob, Pv))
    assert np.abs(PPv - Pv).max() < 1e-13


@pytest.mark.slow
def test_coarse_fourier_equals_brute_force(small_two_level):
    op, _, phi, sob, C, Af = small_two_level
    Ab = crs.build_brute(op, phi, sob, C)
    assert np.abs(Af - Ab).max() < 1e-12 * np.abs(Ab).max()


def test_coarse_hermitian_and_dense_matches_projection(small_two_level):
    op, _, phi, sob, C, A = small_two_level
    nbr = crs.neighbour_table(C)
    for a in (0, 40, 77):
        for l in range(81):
            assert np.abs(A[a, l] - A[nbr[a, l], 80 - l].conj().T).max() < 1e-12 * np.abs(A).max()
    c = synth.rng(40).standard_normal((81, 2)) + 1j * synth.rng(41).standard_normal((81, 2))
    D = crs.to_dense(A, C)
    assert np.abs(crs.apply(A, c, C).ravel() - D @ c.ravel()).max() < 1e-12 * np.abs(D).max()
    # <P c, H P c> = c^+ A c (definition of the little Dirac operator)
    Pc = blk.promote(phi, sob, c)
    assert abs(inner(Pc, op.H(Pc)) - np.vdot(c.ravel(), D @ c.ravel())) < 1e-12 * norm2(Pc) * np.abs(D).max()
    assert np.linalg.eigvalsh(0.5 * (D + D.conj().T)).min() > 0


def test_coarse_translation_invariance_free_field():
    """Unit links, periodic in all directions, the same pattern in every
    block: A[a][l] does not depend on a."""
    dims, Ls, block = (12, 12, 12, 12), 1, (4, 4, 4, 4)
    U = np.broadcast_to(np.eye(3), (12, 12, 12, 12, 4, 3, 3)).copy()
    op = DWF(U, dims, Ls, 1.8, 0.01, bc=(1, 1, 1, 1))
    _, _, sob = blk.block_map(dims, block)
    pat = synth.gaussian_half_field((4, 4, 4, 4), Ls, 50)  # one 4^4 block's odd sites
    # tile: every block takes the same local pattern in local cb order
    _, _, sob_small = blk.block_map((4, 4, 4, 4), block)
    local = blk.to_blocks(pat, sob_small)[0]
    phi = blk.from_blocks(np.broadcast_to(local, (81, local.size))[None], sob, Ls)
    phi = blk.orthonormalise(phi, sob)
    A = crs.build_fourier(op, phi, sob, blk.coarse_dims(dims, block))
    assert np.abs(A - A[0][None]).max() < 1e-12 * np.abs(A).max()
    # the hop reach: a block couples to blocks two away only through 4 hops;
    # with 4^4 blocks every stencil entry is present and nonzero
    assert np.all(np.abs(A[0]).reshape(81, -1).max(axis=1) > 0)


def test_projector_identities(small_two_level):
    op, _, phi, sob, C, A = small_two_level
    tl = hdcg.TwoLevel(op, phi, sob, C, A, coarse_tol=1e-14)
    c = synth.rng(60).standard_normal((81, 2)) + 1j * synth.rng(61).standard_normal((81, 2))
    v = blk.promote(phi, sob, c)
    assert np.abs(tl.Q(op.H(v)) - v).max() < 1e-10 * np.abs(v).max()  # Q H P = P
    psi = synth.gaussian_half_field(op.dims, op.Ls, 62)
    Qpsi = tl.Q(psi)
    assert np.abs(tl.Q(op.H(Qpsi)) - Qpsi).max() < 1e-10 * np.abs(Qpsi).max()  # Q H Q = Q
    PR = tl.P_R(psi)
    assert np.abs(tl.P_R(PR) - PR).max() < 1e-10 * np.abs(PR).max()  # P_R^2 = P_R
    assert np.abs(tl.P_R(Qpsi)).max() < 1e-10 * np.abs(Qpsi).max()  # P_R Q = 0
    # P_L^+ = P_R: <a, P_L b> = <P_R a, b>
    a = synth.gaussian_half_field(op.dims, op.Ls, 63)
    assert abs(inner(a, tl.P_L(psi)) - inner(tl.P_R(a), psi)) < 1e-10 * np.sqrt(norm2(a) * norm2(psi))


@pytest.mark.slow
def test_adef2_invariants_and_bnn_equivalence(small_two_level):
    op, _, phi, sob, C, A = small_two_level
    tl = hdcg.TwoLevel(op, phi, sob, C, A, coarse_tol=1e-14)
    b = synth.gaussian_half_field(op.dims, op.Ls, 70)
    seen = []

    def cb(it, x, r, p):
        seen.append((it, blk.project(phi, sob, r), r.copy(), x.copy()))

    hdcg.gpcg(tl, b, method="adef2", n_irs=3, tol=1e-30, maxiter=4, callback=cb)
    for it, Pr, r, x in seen:
        assert np.abs(Pr).max() <= 1e-10 * np.sqrt(norm2(r))  # Q r_k = 0
        assert np.abs(tl.P_L(r) - r).max() <= 1e-9 * np.abs(r).max()  # P_L r_k = r_k
    # BNN from x = Q b + P_R 0 produces the same iterates
    bnn = []
    hdcg.gpcg(tl, b, method="bnn", n_irs=3, tol=1e-30, maxiter=4, x=tl.Q(b),
              callback=lambda it, x, r, p: bnn.append(x.copy()))
    for (_, _, _, xa), xb in zip(seen, bnn):
        assert np.abs(xa - xb).max() <= 1e-8 * np.abs(xa).max()


@pytest.mark.slow
def test_hdcg_defect_correction_solves(small_two_level):
    op, _, phi, sob, C, A = small_two_level
    tl = hdcg.TwoLevel(op, phi, sob, C, A, coarse_tol=0.04)
    b = synth.gaussian_half_field(op.dims, op.Ls, 80)
    x, outers, inner_its, rel = hdcg.defect_correction(tl, b, tol=1e-8, inner_tol=1e-5, n_irs=4)
    r = b - op.H(x)
    assert np.sqrt(norm2(r) / norm2(b)) <= 1e-8 and outers >= 1



@pytest.mark.slow
def test_standard_and_flexible_pcg_coincide_for_a_fixed_symmetric_preconditioner(small_two_level):
    """Fig. "pcg_general" with its standard update (alpha = (r, y)/(p, w),
    beta = (r', y')/(r, y)) and the flexible one (alpha = (p, r)/(p, w),
    beta = -(w, y')/(p, w)) produce the same iterates in exact arithmetic
    when M_1 is a fixed Hermitian positive operator: (p_k, r_k) = (y_k, r_k)
    because r_k is orthogonal to p_{k-1}, and -(w_k, y_{k+1}) =
    (r_{k+1} - r_k, y_{k+1}) / alpha_k with (r_k, y_{k+1}) = 0.  With an exact
    Q, BNN's M_1 = P_R M P_L + Q is Hermitian for Hermitian M, and A-DEF2
    iterates equal BNN's (Sec. IV.E.1).  M here is the linear Hermitian
    positive polynomial 0.05 + 0.001 H in place of the (nonlinear) M_IRS."""
    op, _, phi, sob, C, A = small_two_level
    tl = hdcg.TwoLevel(op, phi, sob, C, A, coarse_tol=1e-13)
    b = synth.gaussian_half_field(op.dims, op.Ls, 90)

    def poly(o, r, n, lam):
        return 0.05 * r + 0.001 * o.H(r)

    runs = {}
    for method, flex in (("bnn", True), ("bnn", False), ("adef2", False)):
        its = []
        hdcg.gpcg(tl, b, method=method, tol=1e-30, maxiter=4, flexible=flex, m_irs_fn=poly,
                  x=tl.Q(b) if method == "bnn" else None,
                  callback=lambda it, x, r, p: its.append((x.copy(), np.sqrt(norm2(r)))))
        runs[method, flex] = its
    assert len(runs["bnn", True]) == 4
    for (xf, _), (xs, _) in zip(runs["bnn", True], runs["bnn", False]):
        assert np.abs(xf - xs).max() <= 1e-8 * np.abs(xf).max()
    for (xa, _), (xb, _) in zip(runs["adef2", False], runs["bnn", False]):
        assert np.abs(xa - xb).max() <= 1e-8 * np.abs(xa).max()
    # the iteration makes progress (a stalled update would also agree)
    res = [r for _, r in runs["adef2", False]]
    assert res[-1] < 0.5 * np.sqrt(norm2(b))

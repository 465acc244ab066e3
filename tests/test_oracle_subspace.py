"""Pins of the oracle's rational-filter subspace generation (Sec. IV.B,
the equation labelled "ratfilt", Fig. "bandpass").

- the partial-fraction coefficients reproduce the filter's closed form;
- multi-shift CG equals a dense solve of every shifted system (random
  Hermitian positive matrix) and separate CG solves on the domain-wall H;
- on an eigenvector of the operator the filter multiplies by the closed-form
  response at its eigenvalue;
- the multi-shift filter equals four successive shifted solves;
- the wall mask keeps exactly the P- components at s = 0 and the P+ ones at
  s = Ls - 1 (gamma_5 = -1 and +1 there) and is idempotent;
- the filtered vectors are low modes: their Rayleigh quotient drops far
  below that of the noise.
"""
import numpy as np
import pytest

import synth
from oracle import subspace as sub
from oracle.cg import cg
from oracle.dwf import DWF
from oracle.gamma import gamma5


class _Dense:
    """A dense Hermitian positive operator with the oracle's H interface."""

    def __init__(self, M):
        self.M = M

    def H(self, v):
        return self.M @ v


def _hpd(n, seed, lo=1e-3, hi=30.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    ev = np.exp(rng.uniform(np.log(lo), np.log(hi), n))
    return Q @ np.diag(ev) @ Q.conj().T, ev, Q


def test_partial_fractions_reproduce_response():
    lam, eps = 3e-4, 1e-4
    sh = sub.shifts_of(lam, eps)
    c = sub.partial_fractions(sh)
    x = np.concatenate([np.linspace(0.0, 1e-2, 50), np.linspace(0.01, 40, 50)])
    lhs = sum(cj / (x + s) for cj, s in zip(c, sh))
    # the sum cancels: its rounding error is bounded by a few ulps of the
    # largest term, which dominates where the response is small (large x)
    bound = 8 * np.finfo(float).eps * sum(abs(cj) / (x + s) for cj, s in zip(c, sh))
    resp = sub.filter_response(x, lam, eps)
    assert np.all(np.abs(lhs - resp) <= 1e-12 * resp + bound)
    assert np.all(np.abs(lhs - resp)[x < 1e-2] <= 1e-9 * resp[x < 1e-2])
    # two shifts by hand: 1/((x+a)(x+b)) = (1/(x+a) - 1/(x+b)) / (b - a)
    assert np.allclose(sub.partial_fractions([1.0, 3.0]), [0.5, -0.5])


def test_multishift_equals_dense_solves():
    M, _, _ = _hpd(60, 3)
    rng = np.random.default_rng(4)
    b = rng.standard_normal(60) + 1j * rng.standard_normal(60)
    sh = [0.01, 0.05, 0.3, 2.0]
    xs, it = sub.multishift_cg(lambda v: M @ v, b, sh, tol=1e-13)
    for s, x in zip(sh, xs):
        want = np.linalg.solve(M + s * np.eye(60), b)
        assert np.abs(x - want).max() <= 1e-9 * np.abs(want).max(), s
    with pytest.raises(ValueError):
        sub.multishift_cg(lambda v: M @ v, b, [0.5, 0.1])


def test_multishift_equals_separate_cg_on_dwf():
    dims, Ls = (4, 4, 4, 4), 4
    op = DWF(synth.gauge_field(dims, 0.5, 31), dims, Ls, 1.8, 0.05)
    b = synth.gaussian_half_field(dims, Ls, 32)
    sh = [0.02, 0.05, 0.1]
    xs, _ = sub.multishift_cg(op.H, b, sh, tol=1e-12)
    for s, x in zip(sh, xs):
        want, _, _ = cg(lambda u, s=s: op.H(u) + s * u, b, tol=1e-13)
        assert np.abs(x - want).max() <= 1e-8 * np.abs(want).max(), s


def test_filter_on_eigenvector_is_closed_form_response():
    M, ev, Q = _hpd(40, 5, lo=5e-4, hi=10.0)
    k = int(np.argmin(ev))
    v = Q[:, k]
    lam, eps = 3e-4, 1e-4
    phi, _ = sub.rational_filter(_Dense(M), v, lam, eps, tol=1e-14, normalise=False)
    want = sub.filter_response(ev[k], lam, eps) * v
    assert np.abs(phi - want).max() <= 1e-6 * np.abs(want).max()


def test_multishift_filter_equals_product_of_resolvents():
    dims, Ls = (4, 4, 4, 4), 4
    op = DWF(synth.gauge_field(dims, 0.5, 33), dims, Ls, 1.8, 0.01)
    eta = synth.gaussian_half_field(dims, Ls, 34)
    lam, eps = 0.01, 0.01 / 3
    phi, _ = sub.rational_filter(op, eta, lam, eps, tol=1e-12, normalise=False)
    want = sub.rational_filter_product(op, eta, lam, eps, tol=1e-13)
    assert np.abs(phi - want).max() <= 1e-6 * np.abs(want).max()


def test_wall_mask():
    Ls = 5
    h = synth.gaussian_half_field((4, 4, 4, 4), Ls, 35)
    m = sub.wall_mask(h)
    g5 = gamma5()
    assert np.all(m[1:Ls - 1] == 0)
    assert np.allclose(np.einsum("ab,vbc->vac", g5, m[0]), -m[0])
    assert np.allclose(np.einsum("ab,vbc->vac", g5, m[Ls - 1]), m[Ls - 1])
    assert np.array_equal(sub.wall_mask(m), m)
    # the kept components are the input's own
    rest = h - m
    assert np.allclose(np.einsum("ab,vbc->vac", g5, rest[0]), rest[0])
    assert np.allclose(np.einsum("ab,vbc->vac", g5, rest[Ls - 1]), -rest[Ls - 1])


def test_filtered_vectors_are_low_modes():
    dims, Ls = (4, 4, 4, 8), 6
    op = DWF(synth.gauge_field(dims, 0.6, 36), dims, Ls, 1.8, 0.01)
    for wall in (False, True):
        eta = synth.gaussian_half_field(dims, Ls, 37)
        src = sub.wall_mask(eta) if wall else eta
        phi, _ = sub.rational_filter(op, eta, 3e-4, 1e-4, tol=1e-6, wall=wall)
        rq_eta = np.vdot(src, op.H(src)).real / np.vdot(src, src).real
        rq_phi = np.vdot(phi, op.H(phi)).real
        assert rq_phi < 1e-2 * rq_eta, (wall, rq_phi, rq_eta)


def test_surface_truncation():
    """Zero interior, untouched surface, identity when 2 depth >= Ls; the
    block orthonormalisation of truncated vectors keeps the interior zero
    (it only combines vectors within a block); and on the wall-noise
    filtered vectors of a 4^4 x Ls12 operator most of the norm sits on the
    two wall slices, the property the truncation relies on."""
    from oracle import blocks as oblk
    from oracle.dwf import DWF

    dims, Ls = (4, 4, 4, 4), 12
    V = synth.gaussian_half_field(dims, Ls, 420, nrhs=3)
    T = sub.surface_truncate(V, 4)
    assert np.array_equal(T[:, :4], V[:, :4]) and np.array_equal(T[:, Ls - 4:], V[:, Ls - 4:])
    assert not T[:, 4:Ls - 4].any()
    for d in (6, 7, 12):
        assert np.array_equal(sub.surface_truncate(V, d), V)
    Vb = synth.gaussian_half_field((8, 8, 8, 8), 10, 421, nrhs=3)
    _, _, sob = oblk.block_map((8, 8, 8, 8), (4, 4, 4, 4))
    phi = oblk.orthonormalise(sub.surface_truncate(Vb, 3), sob)
    assert not phi[:, 3:7].any()
    F = phi.reshape(3, -1)
    G = F.conj() @ F.T  # all blocks summed: Nblocks x identity
    assert np.abs(G - (2 ** 4) * np.eye(3)).max() < 1e-10
    U = synth.gauge_field(dims, 0.5, 300)
    op = DWF(U, dims, Ls, 1.8, 0.01)
    phi, _ = sub.rational_filter(op, synth.gaussian_half_field(dims, Ls, 400), tol=1e-6, wall=True)
    prof = np.array([np.vdot(phi[s].ravel(), phi[s].ravel()).real for s in range(Ls)])
    assert prof[0] + prof[-1] > 0.5 * prof.sum()

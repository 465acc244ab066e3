"""Pins of the oracle's Mobius (Cayley-form) kernel.

The paper names the kernel (abstract, Sec. I) without writing it out; the
reading is the standard Cayley form with b = 1, c = 0 giving Shamir:
(D psi)_s = (b D_W + 1) psi_s + (c D_W - 1)(P- psi_{s+1} + P+ psi_{s-1}),
D_W = (4 - M5) - Dh/2, -m in place of 1 at the wall couplings.

Pins:
- the Mobius fifth-dimension matrices at (b, c) = (1, 0) equal the Shamir
  ones and C_5 is the identity;
- the Schur complement, on the odd sites, of the full unpreconditioned
  operator D assembled densely from the defining formula above (full-lattice
  hop, explicit shifts and projectors: a construction that shares nothing
  with the red-black factors) equals the oracle's M_pc;
- H is Hermitian and positive, and <a, M_pc b> = <M_pc^+ a, b>;
- M_5^-1 equals the closed form pw[n] = kappa^n / (alpha (1 + m kappa^Ls)),
  kappa = -beta / alpha, on P+ (s >= s', -m otherwise) and its reflection on P-.
"""
import numpy as np
import pytest

import synth
from oracle import geometry as geo
from oracle.dwf import DWF, m5_matrices, mobius_matrices, wilson_hop
from oracle.gamma import chiral_projectors

B5, C5 = 1.5, 0.5


def test_mobius_matrices_at_shamir_point():
    for Ls, M5, m in ((4, 1.8, 0.01), (7, 1.4, 0.3)):
        (Mp, Mm), (Cp, Cm) = mobius_matrices(Ls, M5, m, 1.0, 0.0)
        Sp, Sm = m5_matrices(Ls, M5, m)
        assert np.array_equal(Mp, Sp) and np.array_equal(Mm, Sm)
        assert np.array_equal(Cp, np.eye(Ls)) and np.array_equal(Cm, np.eye(Ls))


def _full_mobius(U, dims, Ls, M5, m, b, c):
    """psi (Ls, T, Z, Y, X, 4, 3) -> D psi, from the defining formula."""
    Pp, Pm = chiral_projectors()

    def dw(f):
        return (4.0 - M5) * f - 0.5 * wilson_hop(U, f, dims, (1, 1, 1, -1))

    def shift_terms(f):
        # P- f_{s+1} + P+ f_{s-1}, with -m at the walls
        g = np.zeros_like(f)
        for s in range(Ls):
            up = f[s + 1] if s < Ls - 1 else -m * f[0]
            dn = f[s - 1] if s > 0 else -m * f[Ls - 1]
            g[s] = np.matmul(Pm, up) + np.matmul(Pp, dn)
        return g

    def D(f):
        k = shift_terms(f)
        return b * dw(f) + f + c * dw(k) - k

    return D


@pytest.mark.parametrize("m", [0.1, 0.0])
def test_mobius_schur_complement_of_full_operator(m):
    dims, Ls, M5 = (2, 2, 2, 4), 3, 1.6
    U = synth.gauge_field(dims, 0.6, 71)
    D = _full_mobius(U, dims, Ls, M5, m, B5, C5)
    V = geo.volume(dims)
    X, Y, Z, T = dims
    N = Ls * V * 12
    cols = []
    for i in range(N):
        e = np.zeros(N, dtype=complex)
        e[i] = 1.0
        cols.append(D(e.reshape(Ls, T, Z, Y, X, 4, 3)).ravel())
    Dm = np.array(cols).T
    # index sets of the two parities, in the half-field order (s, cb, spin, colour)
    idx = np.arange(N).reshape(Ls, V, 4, 3)
    odd = idx[:, geo.parity_sites(dims, 1)].ravel()
    even = idx[:, geo.parity_sites(dims, 0)].ravel()
    S = Dm[np.ix_(odd, odd)] - Dm[np.ix_(odd, even)] @ np.linalg.solve(Dm[np.ix_(even, even)], Dm[np.ix_(even, odd)])
    ref = DWF(U, dims, Ls, M5, m, b=B5, c=C5)
    Nh = len(odd)
    Mpc = np.zeros((Nh, Nh), dtype=complex)
    for i in range(Nh):
        e = np.zeros(Nh, dtype=complex)
        e[i] = 1.0
        Mpc[:, i] = ref.mpc(e.reshape(ref.half_shape())).ravel()
    assert np.abs(S - Mpc).max() < 1e-12 * np.abs(S).max()


def test_mobius_hermitian_positive_and_adjoint():
    dims, Ls = (4, 4, 4, 4), 6
    U = synth.gauge_field(dims, 0.5, 72)
    ref = DWF(U, dims, Ls, 1.8, 0.02, b=B5, c=C5)
    a = synth.gaussian_half_field(dims, Ls, 73)
    b = synth.gaussian_half_field(dims, Ls, 74)
    lhs = np.vdot(a, ref.mpc(b))
    rhs = np.vdot(ref.mpc_dag(a), b)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
    hab = np.vdot(a, ref.H(b))
    hba = np.vdot(b, ref.H(a))
    assert abs(hab - np.conj(hba)) < 1e-11 * abs(hab)
    assert np.vdot(a, ref.H(a)).real > 0
    # genuinely different from Shamir
    sh = DWF(U, dims, Ls, 1.8, 0.02)
    assert np.abs(ref.H(a) - sh.H(a)).max() > 1e-2


@pytest.mark.parametrize("Ls,M5,m", [(8, 1.8, 0.01), (5, 1.3, 0.4)])
def test_mobius_m5_inverse_closed_form(Ls, M5, m):
    (Mp, Mm), _ = mobius_matrices(Ls, M5, m, B5, C5)
    alpha = B5 * (4 - M5) + 1
    beta = C5 * (4 - M5) - 1
    kap = -beta / alpha
    Ip = np.zeros((Ls, Ls))
    for s in range(Ls):
        for t in range(Ls):
            n = (s - t) % Ls
            Ip[s, t] = kap ** n / (alpha * (1 + m * kap ** Ls)) * (1.0 if s >= t else -m)
    assert np.abs(Ip - np.linalg.inv(Mp)).max() < 1e-13
    R = np.eye(Ls)[::-1]
    assert np.abs(R @ Ip @ R - np.linalg.inv(Mm)).max() < 1e-13

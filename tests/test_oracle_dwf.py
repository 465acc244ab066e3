"""Pins of the oracle's domain-wall operator against facts fixed by the
mathematics: Clifford algebra, the free-field closed form in momentum space,
Hermiticity, the adjoint, gauge covariance, the closed-form inverse of the
fifth-dimension matrix, the Ls = 1 reduction to even-odd Wilson, and the exact
reach of a single hop."""
import itertools

import numpy as np
import pytest

import synth
from oracle import geometry as geo
from oracle.dwf import DWF, inner, m5_matrices, wilson_hop
from oracle.gamma import chiral_projectors, gamma5, gammas


def test_gamma_clifford_and_gamma5():
    g = gammas()
    for mu, nu in itertools.product(range(4), range(4)):
        ac = g[mu] @ g[nu] + g[nu] @ g[mu]
        assert np.allclose(ac, 2.0 * (mu == nu) * np.eye(4), atol=0)
    for mu in range(4):
        assert np.array_equal(g[mu], g[mu].conj().T)
    assert np.array_equal(gamma5(), np.diag([1, 1, -1, -1]).astype(complex))
    Pp, Pm = chiral_projectors()
    assert np.allclose(Pp @ Pp, Pp) and np.allclose(Pp @ Pm, 0)


def test_gauge_generator_is_su3():
    U = synth.gauge_field((4, 4, 4, 4), 0.5, 1001)
    I = np.eye(3)
    assert np.abs(U @ U.conj().swapaxes(-1, -2) - I).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14


def test_geometry_checkerboard_bit_exact():
    dims = (4, 6, 4, 8)
    for p in (0, 1):
        s = geo.parity_sites(dims, p)
        c = geo.coords(dims)[s]
        assert np.array_equal(c.sum(1) % 2, np.full(len(s), p))
        assert np.array_equal(s >> 1, np.arange(len(s)))
        lex = c[:, 0] + 4 * (c[:, 1] + 6 * (c[:, 2] + 4 * c[:, 3]))
        assert np.array_equal(lex, s)


def test_hop_gather_equals_roll_form():
    dims, Ls = (4, 4, 6, 4), 3
    op = DWF(synth.gauge_field(dims, 0.6, 3), dims, Ls, 1.8, 0.05, bc=(1, np.exp(0.4j), 1, -1))
    for par, dag in itertools.product((0, 1), (False, True)):
        a = synth.gaussian_half_field(dims, Ls, 10 + par)
        assert np.abs(op.dh(a, par, dag) - op.dh_full(a, par, dag)).max() < 1e-13


@pytest.mark.parametrize("site", [(1, 2, 1, 1), (0, 0, 0, 1), (3, 3, 3, 0)])
def test_point_source_hop_reach(site):
    """M_eo on a point source at odd y lands only on y -/+ mu with
    -1/2 (1 -/+ g_mu) U..., boundary phases where the hop wraps."""
    dims, Ls = (4, 4, 4, 4), 2
    bc = (1, 1, np.exp(0.7j), -1)
    U = synth.gauge_field(dims, 0.8, 5)
    op = DWF(U, dims, Ls, 1.8, 0.01, bc=bc)
    X, Y, Z, T = dims
    y = np.array(site)
    assert y.sum() % 2 == 1
    ylex = y[0] + X * (y[1] + Y * (y[2] + Z * y[3]))
    s0, j, c = 1, 2, 1
    src = np.zeros((Ls, 128, 4, 3), complex)
    src[s0, ylex >> 1, j, c] = 1.0
    out = -0.5 * op.dh_eo(src)
    g = gammas()
    expect = np.zeros_like(out)
    Ul = U.reshape(-1, 4, 3, 3)
    for mu in range(4):
        e = np.eye(4, dtype=int)[mu]
        xm = (y - e) % np.array(dims)
        xp = (y + e) % np.array(dims)
        lm = xm[0] + X * (xm[1] + Y * (xm[2] + Z * xm[3]))
        lp = xp[0] + X * (xp[1] + Y * (xp[2] + Z * xp[3]))
        ph_f = bc[mu] if y[mu] == 0 else 1.0  # hop x=y-mu -> y wraps when y_mu = 0
        ph_b = np.conj(bc[mu]) if y[mu] == dims[mu] - 1 else 1.0
        # forward term at x = y - mu: (1 - g) U_mu(x) psi(x + mu)
        expect[s0, lm >> 1] += -0.5 * ph_f * np.outer((np.eye(4) - g[mu])[:, j], Ul[lm, mu][:, c])
        # backward term at x = y + mu: (1 + g) U_mu(y)^+ psi(y)
        expect[s0, lp >> 1] += -0.5 * ph_b * np.outer((np.eye(4) + g[mu])[:, j], Ul[ylex, mu].conj().T[:, c])
    assert np.abs(out - expect).max() < 1e-15
    nz = set(zip(*np.nonzero(np.abs(out).sum(axis=(2, 3)))))
    assert nz == set(zip(*np.nonzero(np.abs(expect).sum(axis=(2, 3)))))


@pytest.mark.parametrize("Ls,M5,m", [(8, 1.8, 0.01), (16, 1.8, 0.001), (5, 1.2, 0.3), (1, 1.8, 0.01)])
def test_m5_inverse_closed_form(Ls, M5, m):
    Mp, Mm = m5_matrices(Ls, M5, m)
    d = 5.0 - M5
    Ip = np.zeros((Ls, Ls))
    for s, t in itertools.product(range(Ls), range(Ls)):
        n = (s - t) % Ls
        Ip[s, t] = d ** (-1 - n) / (1 + m * d ** (-Ls)) * (1.0 if s >= t else -m)
    Im = Ip[::-1, ::-1]  # R5 M+^-1 R5
    assert np.abs(Ip @ Mp - np.eye(Ls)).max() < 1e-14
    assert np.abs(Im @ Mm - np.eye(Ls)).max() < 1e-14
    op = DWF(synth.gauge_field((4, 4, 4, 4), 0.5, 1), (4, 4, 4, 4), Ls, M5, m)
    assert np.abs(op.Mpi - Ip).max() < 1e-14 and np.abs(op.Mmi - Im).max() < 1e-14


def _op(dims=(4, 4, 4, 4), Ls=4, eps=0.5, seed=1001, bc=(1, 1, 1, -1), mass=0.01):
    return DWF(synth.gauge_field(dims, eps, seed), dims, Ls, 1.8, mass, bc=bc)


def test_hermiticity_positivity_adjoint_and_gamma5R5():
    op = _op(dims=(4, 4, 4, 6), Ls=6, bc=(1, np.exp(0.25j), 1, -1))
    a = synth.gaussian_half_field(op.dims, op.Ls, 1)
    b = synth.gaussian_half_field(op.dims, op.Ls, 2)
    Ha, Hb = op.H(a), op.H(b)
    scale = np.sqrt(inner(Ha, Ha).real * inner(b, b).real)
    assert abs(inner(a, Hb) - np.conj(inner(b, Ha))) < 1e-13 * scale
    assert abs(inner(a, Ha).imag) < 1e-13 * scale and inner(a, Ha).real > 0
    lhs, rhs = inner(a, op.mpc(b)), inner(op.mpc_dag(a), b)
    assert abs(lhs - rhs) < 1e-13 * scale
    # M_pc^+ = Gamma M_pc Gamma with Gamma = gamma5 (x) R5
    G5 = gamma5()

    def Gam(h):
        return np.matmul(G5, h[::-1])

    assert np.abs(op.mpc_dag(a) - Gam(op.mpc(Gam(a)))).max() < 1e-12


def test_gauge_covariance():
    dims = (4, 4, 6, 4)
    op = _op(dims=dims, Ls=4, eps=0.9)
    g = synth.su3_field(dims, 77)
    U2 = op.U.copy()
    X, Y, Z, T = dims
    for mu in range(4):
        gs = np.roll(g, -1, axis=3 - mu)  # g(x + mu); site axes (T, Z, Y, X)
        U2[..., mu, :, :] = g @ op.U[..., mu, :, :] @ gs.conj().swapaxes(-1, -2)
    op2 = DWF(U2, dims, op.Ls, op.M5, op.mass, bc=op.bc)
    go = g.reshape(-1, 3, 3)[geo.parity_sites(dims, 1)]
    psi = synth.gaussian_half_field(dims, op.Ls, 3)

    def gmul(h):
        return np.matmul(h, go.swapaxes(-1, -2))

    lhs = op2.H(gmul(psi))
    rhs = gmul(op.H(psi))
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()


def _free_field_K(p, Ls, M5, m):
    """K(p) = M5 - 1/4 h(p) M5^-1 h(p) on (s, spin), from the definitions:
    h(p) = sum_mu [2 cos p_mu - 2 i g_mu sin p_mu]; the fifth-dimension
    matrix assembled from shift matrices and chiral projectors."""
    g = gammas()
    Pp, Pm = chiral_projectors()
    h = sum(2 * np.cos(p[mu]) * np.eye(4) - 2j * np.sin(p[mu]) * g[mu] for mu in range(4))
    d = 5.0 - M5
    Sup = np.eye(Ls, k=1)  # (S+ psi)_s = psi_{s+1}
    Sdn = np.eye(Ls, k=-1)  # (S- psi)_s = psi_{s-1}
    Cm = np.zeros((Ls, Ls)); Cm[Ls - 1, 0] = m
    Cp = np.zeros((Ls, Ls)); Cp[0, Ls - 1] = m
    M = d * np.eye(4 * Ls) - np.kron(Sup, Pm) - np.kron(Sdn, Pp) + np.kron(Cm, Pm) + np.kron(Cp, Pp)
    Hh = np.kron(np.eye(Ls), h)
    return M - 0.25 * Hh @ np.linalg.inv(M) @ Hh


def _plane_wave(dims, Ls, p, w, u):
    c = geo.coords(dims)[geo.parity_sites(dims, 1)]
    ph = np.exp(1j * c @ np.array(p))
    return np.einsum("v,si,c->svic", ph, w.reshape(Ls, 4), u)


@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 0, 0, 0), (1, 2, 3, 1), (3, 1, 0, 2)])
def test_free_field_plane_waves(n):
    dims, Ls, M5, m = (4, 4, 4, 4), 8, 1.8, 0.01
    U = np.broadcast_to(np.eye(3), (4, 4, 4, 4, 4, 3, 3)).copy()
    op = DWF(U, dims, Ls, M5, m, bc=(1, 1, 1, -1))
    p = [2 * np.pi * n[0] / 4, 2 * np.pi * n[1] / 4, 2 * np.pi * n[2] / 4, (2 * n[3] + 1) * np.pi / 4]
    K = _free_field_K(p, Ls, M5, m)
    lam, W = np.linalg.eigh(K.conj().T @ K)
    u = np.array([0.3, -0.5j, 0.8])
    for i in (0, 1, len(lam) // 2, len(lam) - 1):
        psi = _plane_wave(dims, Ls, p, W[:, i], u)
        r = op.H(psi)
        assert np.abs(r - lam[i] * psi).max() < 1e-12 * max(1.0, lam[i])


@pytest.mark.slow
def test_free_field_full_spectrum():
    """Dense spectrum of H on 4^4 x Ls=2 equals the union over the half
    Brillouin zone of spec(K^+ K), three-fold for colour."""
    dims, Ls, M5, m = (4, 4, 4, 4), 2, 1.8, 0.1
    U = np.broadcast_to(np.eye(3), (4, 4, 4, 4, 4, 3, 3)).copy()
    op = DWF(U, dims, Ls, M5, m)
    n = op.unknowns()
    basis = np.eye(n, dtype=complex).reshape((n,) + op.half_shape())
    Hd = op.H(basis).reshape(n, n).T
    ev = np.linalg.eigvalsh(0.5 * (Hd + Hd.conj().T))
    allev = []
    for nn in itertools.product(range(4), repeat=4):
        p = [2 * np.pi * nn[0] / 4, 2 * np.pi * nn[1] / 4, 2 * np.pi * nn[2] / 4, (2 * nn[3] + 1) * np.pi / 4]
        K = _free_field_K(p, Ls, M5, m)
        allev.extend(np.linalg.eigvalsh(K.conj().T @ K))
    union = np.sort(np.repeat(allev, 3))[::2]  # p and p + pi(1,1,1,1) coincide on odd sites
    assert len(union) == n
    assert np.abs(np.sort(ev) - union).max() < 1e-12 * ev.max()


def test_ls1_reduces_to_even_odd_wilson():
    """Ls = 1: D5 = (1 + m) and H is the even-odd Wilson normal operator with
    diagonal 5 - M5 + m: compare M_pc with the dense Schur complement of the
    full Wilson matrix."""
    dims, M5, m = (4, 4, 4, 4), 1.8, 0.05
    U = synth.gauge_field(dims, 0.6, 9)
    op = DWF(U, dims, 1, M5, m)
    V = 256
    basis = np.eye(V * 12, dtype=complex).reshape(V * 12, 1, 4, 4, 4, 4, 4, 3)
    D = (5 - M5 + m) * np.eye(V * 12) - 0.5 * wilson_hop(U, basis, dims, op.bc).reshape(V * 12, V * 12).T
    idx = lambda sites: (sites[:, None] * 12 + np.arange(12)[None, :]).ravel()
    e, o = idx(geo.parity_sites(dims, 0)), idx(geo.parity_sites(dims, 1))
    S = D[np.ix_(o, o)] - D[np.ix_(o, e)] @ np.linalg.solve(D[np.ix_(e, e)], D[np.ix_(e, o)])
    nh = V // 2 * 12
    b = np.eye(nh, dtype=complex).reshape((nh, 1, V // 2, 4, 3))
    Mpc = op.mpc(b).reshape(nh, nh).T
    assert np.abs(Mpc - S).max() < 1e-13 * np.abs(S).max()

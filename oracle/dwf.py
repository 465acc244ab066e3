"""Oracle domain-wall operator (test infrastructure only).

Follows the Hermitian red-black operator of Sec. IV (the equation defining
H = (M_oo - M_oe M_ee^-1 M_eo)^dagger (M_oo - M_oe M_ee^-1 M_eo)).  The paper
cites the domain-wall kernel without writing it out; this oracle takes Shamir's
form with Wilson parameter r = 1:

  D_DW = (4 - M5) - Dh/2 + D5,
  (Dh psi)(x) = sum_mu [(1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu)],
  (D5 psi)_s  = psi_s - P- psi_{s+1} [s<Ls-1] - P+ psi_{s-1} [s>0]
                + m P- psi_0 [s=Ls-1] + m P+ psi_{Ls-1} [s=0].

Hence M_ee = M_oo = M_5 := (5 - M5) + (D5 - 1), M_eo = -Dh_eo/2,
M_oe = -Dh_oe/2 and M_pc = M_5 - (1/4) Dh_oe M_5^-1 Dh_eo on odd sites.
M_pc^dagger is composed from the adjoint of every factor.  A boundary phase
zeta_mu multiplies the hop that crosses x_mu = L_mu - 1 -> 0 (zeta_mu^* the
reverse hop).

Deliberately plain: full 4x4 spin matrices (no spin projection), full-lattice
arrays with np.roll for neighbours, dense Ls x Ls matrices for the fifth
dimension, np.linalg.inv for M_5^-1.

Mobius (Cayley-form) kernel, which the paper names (abstract, Sec. I) but
does not write out; the reading follows the standard form of the cited
literature, with b = 1, c = 0 giving Shamir:

  (D psi)_s = (b D_W + 1) psi_s + (c D_W - 1) (P- psi_{s+1} + P+ psi_{s-1}),
  D_W = (4 - M5) - Dh/2, and -m in place of 1 for the wall couplings.

With K = P- S+ + P+ S- (the two chiral shifts, -m at the wrap) this is
D = (alpha + beta K) - (1/2) Dh (b + c K), alpha = b (4 - M5) + 1,
beta = c (4 - M5) - 1.  Hence M_ee = M_oo = M_5 := alpha + beta K,
M_eo = -(1/2) Dh_eo C_5, M_oe = -(1/2) Dh_oe C_5 with C_5 := b + c K applied
before the hop, and M_pc = M_5 - (1/4) Dh_oe C_5 M_5^-1 Dh_eo C_5.
"""
from __future__ import annotations

import numpy as np

from . import geometry as geo
from .gamma import chiral_projectors, gammas

# axis of direction mu (x, y, z, t) in arrays ending in (T, Z, Y, X, spin, colour)
# or (T, Z, Y, X, 3, 3) for a single link direction
_AX = {0: -3, 1: -4, 2: -5, 3: -6}


def _colour(U, psi):
    """out[..., site, i, a] = sum_b U[site, a, b] psi[..., site, i, b]."""
    return np.matmul(psi, U.swapaxes(-1, -2))


def _colour_sites(U, h):
    """out[..., v, i, a] = sum_b U[v, a, b] h[..., v, i, b] for site-indexed links."""
    return np.matmul(h, U.swapaxes(-1, -2))


def _spin(G, psi):
    """out[..., i, c] = sum_j G[i, j] psi[..., j, c]."""
    return np.matmul(G, psi)


def _shift(f, mu, direction, zeta, L):
    """direction=+1: returns g(x) = f(x+mu) with zeta applied where the hop
    crosses the boundary; direction=-1: g(x) = f(x-mu) with conj(zeta)."""
    ax = _AX[mu]
    g = np.roll(f, -direction, axis=ax)
    idx = [slice(None)] * g.ndim
    if direction > 0:
        idx[g.ndim + ax] = L - 1
        g[tuple(idx)] *= zeta
    else:
        idx[g.ndim + ax] = 0
        g[tuple(idx)] *= np.conj(zeta)
    return g


def wilson_hop(U, psi_full, dims, bc, dagger=False):
    """Dh (or Dh^dagger, which swaps the two projectors) on a full-lattice field.

    U: (T, Z, Y, X, 4, 3, 3); psi_full: (..., Ls, T, Z, Y, X, 4, 3)."""
    g = gammas()
    one = np.eye(4)
    out = np.zeros_like(psi_full)
    for mu in range(4):
        L = dims[mu]
        Umu = U[..., mu, :, :]
        fwd = _colour(Umu, _shift(psi_full, mu, +1, bc[mu], L))
        # U_mu(x - mu)^dagger psi(x - mu), phase conj(zeta) on the wrapped hop
        Ub = np.roll(Umu, 1, axis=_AX[mu]).conj().swapaxes(-1, -2)
        bwd = _colour(Ub, _shift(psi_full, mu, -1, bc[mu], L))
        if not dagger:
            out += _spin(one - g[mu], fwd) + _spin(one + g[mu], bwd)
        else:
            out += _spin(one + g[mu], fwd) + _spin(one - g[mu], bwd)
    return out


def m5_matrices(Ls, M5, mass):
    """Dense Ls x Ls real matrices of M_5 on the P+ and P- chiral halves."""
    d = 5.0 - M5
    Mp = d * np.eye(Ls)
    Mm = d * np.eye(Ls)
    for s in range(Ls - 1):
        Mm[s, s + 1] -= 1.0  # - P- psi_{s+1}
    for s in range(1, Ls):
        Mp[s, s - 1] -= 1.0  # - P+ psi_{s-1}
    Mm[Ls - 1, 0] += mass  # + m P- psi_0 at s = Ls-1
    Mp[0, Ls - 1] += mass  # + m P+ psi_{Ls-1} at s = 0
    return Mp, Mm


def mobius_matrices(Ls, M5, mass, b, c):
    """Dense Ls x Ls matrices (P+ half, P- half) of M_5 = alpha + beta K and
    C_5 = b + c K for the Mobius kernel; K is S- (s-1) on P+ and S+ (s+1) on
    P-, each with -m on its wrapped entry."""
    Kp = np.zeros((Ls, Ls))
    Km = np.zeros((Ls, Ls))
    for s in range(Ls):
        if s > 0:
            Kp[s, s - 1] = 1.0
        else:
            Kp[0, Ls - 1] = -mass
        if s < Ls - 1:
            Km[s, s + 1] = 1.0
        else:
            Km[Ls - 1, 0] = -mass
    alpha = b * (4.0 - M5) + 1.0
    beta = c * (4.0 - M5) - 1.0
    one = np.eye(Ls)
    return (alpha * one + beta * Kp, alpha * one + beta * Km), (b * one + c * Kp, b * one + c * Km)


def apply_5d(Mp, Mm, half):
    """Apply Mp (x) P+ + Mm (x) P- to a half-field (..., Ls, Vh, 4, 3)."""
    Pp, Pm = chiral_projectors()

    def along_s(M, f):
        # out[..., s, v, i, c] = sum_t M[s, t] f[..., t, v, i, c]
        g = np.moveaxis(f, -4, -1)
        return np.moveaxis(np.matmul(g, M.T), -1, -4)

    return along_s(Mp, _spin(Pp, half)) + along_s(Mm, _spin(Pm, half))


class DWF:
    """Domain-wall operator on the odd checkerboard: Shamir, or Mobius when
    (b, c) is given other than (1, 0)."""

    def __init__(self, U, dims, Ls, M5, mass, bc=(1, 1, 1, -1), b=1.0, c=0.0):
        self.U = np.asarray(U, dtype=np.complex128)
        self.dims = tuple(dims)
        self.Ls = int(Ls)
        self.M5 = float(M5)
        self.mass = float(mass)
        self.bc = tuple(complex(z) for z in bc)
        self.b, self.c = float(b), float(c)
        self.mobius = (self.b, self.c) != (1.0, 0.0)
        if self.mobius:
            (self.Mp, self.Mm), (self.Cp, self.Cm) = mobius_matrices(self.Ls, self.M5, self.mass, self.b, self.c)
        else:
            self.Mp, self.Mm = m5_matrices(self.Ls, self.M5, self.mass)
        self.Mpi = np.linalg.inv(self.Mp)
        self.Mmi = np.linalg.inv(self.Mm)

    # site-local fifth-dimension factors ------------------------------------
    def m5(self, h):
        return apply_5d(self.Mp, self.Mm, h)

    def m5_dag(self, h):
        return apply_5d(self.Mp.T, self.Mm.T, h)

    def m5_inv(self, h):
        return apply_5d(self.Mpi, self.Mmi, h)

    def m5_inv_dag(self, h):
        return apply_5d(self.Mpi.T, self.Mmi.T, h)

    def c5(self, h):
        return apply_5d(self.Cp, self.Cm, h) if self.mobius else h

    def c5_dag(self, h):
        return apply_5d(self.Cp.T, self.Cm.T, h) if self.mobius else h

    # checkerboard hops -----------------------------------------------------
    def _tables(self, out_parity):
        key = "_nb%d" % out_parity
        if not hasattr(self, key):
            nb = geo.neighbours(self.dims, out_parity)
            Uf = self.U.reshape(-1, 4, 3, 3)
            t = {"fwd": nb["fwd"], "bwd": nb["bwd"], "Uf": [], "Ubd": [], "phf": [], "phb": []}
            for mu in range(4):
                t["Uf"].append(Uf[nb["lex"], mu])  # U_mu(x)
                t["Ubd"].append(Uf[nb["lex_bwd"][mu], mu].conj().swapaxes(-1, -2))  # U_mu(x-mu)^+
                t["phf"].append(np.where(nb["fwrap"][mu], self.bc[mu], 1.0)[:, None, None])
                t["phb"].append(np.where(nb["bwrap"][mu], np.conj(self.bc[mu]), 1.0)[:, None, None])
            setattr(self, key, t)
        return getattr(self, key)

    def dh(self, h, src_parity, dagger=False):
        """Dh (or Dh^dagger, projector signs swapped) from parity src_parity to
        the other parity; h has shape (..., Ls, Vh, 4, 3)."""
        t = self._tables(1 - src_parity)
        g = gammas()
        one = np.eye(4)
        out = np.zeros_like(h)
        for mu in range(4):
            fwd = t["phf"][mu] * _colour_sites(t["Uf"][mu], h[..., t["fwd"][mu], :, :])
            bwd = t["phb"][mu] * _colour_sites(t["Ubd"][mu], h[..., t["bwd"][mu], :, :])
            pf, pb = (one - g[mu], one + g[mu]) if not dagger else (one + g[mu], one - g[mu])
            out += _spin(pf, fwd) + _spin(pb, bwd)
        return out

    def dh_full(self, h, src_parity, dagger=False):
        """Same operator through the full-lattice np.roll form (cross-check)."""
        full = geo.embed(h, self.dims, src_parity)
        out = wilson_hop(self.U, full, self.dims, self.bc, dagger=dagger)
        return geo.extract(out, self.dims, 1 - src_parity)

    def dh_eo(self, h_odd, dagger=False):
        return self.dh(h_odd, 1, dagger)

    def dh_oe(self, h_even, dagger=False):
        return self.dh(h_even, 0, dagger)

    # preconditioned operator ------------------------------------------------
    def mpc(self, h):
        """M_pc = M_5 - (1/4) Dh_oe C_5 M_5^-1 Dh_eo C_5 on odd half-fields
        (C_5 = 1 for Shamir)."""
        t = self.m5_inv(self.dh_eo(self.c5(h)))
        return self.m5(h) - 0.25 * self.dh_oe(self.c5(t))

    def mpc_dag(self, h):
        """M_pc^dagger = M_5^+ - (1/4) C_5^+ (Dh_eo)^+ (M_5^-1)^+ C_5^+ (Dh_oe)^+,
        with (Dh_oe)^+ = (Dh^+)_eo and (Dh_eo)^+ = (Dh^+)_oe."""
        t = self.m5_inv_dag(self.c5_dag(self.dh_eo(h, dagger=True)))
        return self.m5_dag(h) - 0.25 * self.c5_dag(self.dh_oe(t, dagger=True))

    def H(self, h):
        """The Hermitian red-black operator M_pc^dagger M_pc."""
        return self.mpc_dag(self.mpc(h))

    def unknowns(self):
        return self.Ls * geo.volume(self.dims) // 2 * 12

    def half_shape(self):
        return (self.Ls, geo.volume(self.dims) // 2, 4, 3)


def inner(a, b):
    """<a, b> = sum conj(a) b over all indices."""
    return np.vdot(a.ravel(), b.ravel())


def norm2(a):
    return float(np.vdot(a.ravel(), a.ravel()).real)

"""Oracle of 16-bit field storage in the M_IRS preconditioner (test
infrastructure only).

Sec. VI.E (Table "sloppy") keeps the single-precision arithmetic of M_IRS but
cuts every word the preconditioner communicates to 16 bits: the 8-bit
exponent and 7 of the 23 mantissa bits, i.e. bfloat16.  The one-GPU reading
here stores every field of the M_IRS CG -- its iterate, residual, search
direction and H times the search direction, and the two half-fields that one
application of M_pc leaves behind -- as bfloat16 values, with the arithmetic
between two stores carried out at full precision.  The paper truncates;
this reading rounds to the nearest bfloat16 value, ties to an even
significand, which halves the largest error and has no bias.

round_bf16 is that rounding, written from its definition (an 8-bit
significand, exponents as float32).  mpc_bf16 / mpc_dag_bf16 apply the two
half-steps of M_pc (Sec. IV: t = M_5^-1 Dh_eo x, then M_pc x = M_5 x -
(1/4) Dh_oe t) and their adjoints, rounding each stored half-field; m_irs_bf16
is the fixed-iteration CG of Sec. IV.C with its vectors rounded after every
update.  Shamir's kernel only: the Mobius kernel adds C_5 factors whose place
relative to the stored half-fields is an implementation choice.
"""
from __future__ import annotations

import numpy as np

_SIG_BITS = 8  # bfloat16 significand: 7 stored bits and the implicit one


def round_bf16(a):
    """Each real and imaginary part of `a` rounded to the nearest bfloat16
    value (ties to an even significand), returned in a's dtype (float64 or
    complex128).  Values must lie in float32's normal range or be zero."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        return round_bf16(a.real) + 1j * round_bf16(a.imag)
    x = a.astype(np.float64)
    nz = x != 0.0
    if np.any(np.abs(x[nz]) < 2.0 ** -126) or np.any(np.abs(x) > 3.0e38):
        raise ValueError("round_bf16: value outside float32's normal range")
    m, e = np.frexp(x)  # x = m 2^e, 0.5 <= |m| < 1
    # m has 8 significant bits after scaling by 2^8; np.rint ties to even
    q = np.rint(np.ldexp(m, _SIG_BITS))
    return np.ldexp(q, e - _SIG_BITS)


def trunc_bf16(a):
    """Each real and imaginary part of `a` (float32 values) cut to bfloat16 by
    dropping the low 16 bits of its float32 word: the truncation of Sec. VI.E
    (rounding toward zero)."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        return trunc_bf16(a.real) + 1j * trunc_bf16(a.imag)
    m, e = np.frexp(a.astype(np.float32).astype(np.float64))
    return np.ldexp(np.trunc(np.ldexp(m, _SIG_BITS)), e - _SIG_BITS)


def mpc_bf16(op, h):
    """M_pc h with the even half-field t and the result stored in 16 bits
    (returns the stored result and the unrounded one)."""
    if op.mobius:
        raise ValueError("mpc_bf16 covers Shamir's kernel only")
    t = round_bf16(op.m5_inv(op.dh_eo(h)))
    y = op.m5(h) - 0.25 * op.dh_oe(t)
    return round_bf16(y), y


def mpc_dag_bf16(op, h):
    """M_pc^+ h with the same two stores."""
    if op.mobius:
        raise ValueError("mpc_dag_bf16 covers Shamir's kernel only")
    t = round_bf16(op.m5_inv_dag(op.dh_eo(h, dagger=True)))
    return round_bf16(op.m5_dag(h) - 0.25 * op.dh_oe(t, dagger=True))


def H_bf16(op, h):
    """H h = M_pc^+ M_pc h through 16-bit storage; also returns |M_pc h|^2 of
    the unrounded M_pc h (the (p, H p) a CG takes from the operator)."""
    chi, chi_exact = mpc_bf16(op, h)
    return mpc_dag_bf16(op, chi), float(np.vdot(chi_exact.ravel(), chi_exact.ravel()).real)


def _nrm(a):
    return float(np.vdot(a.ravel(), a.ravel()).real)


def m_irs_bf16(op, b, niter, lam, trunc=False):
    """M_IRS(H, N, lambda) b (Sec. IV.C): exactly N CG iterations on
    H + lambda from zero, every vector stored in 16 bits.  The norms are
    those of the values before they are stored; the scalars are FP64.
    trunc: cut the CG's vectors by truncation (the paper's choice) instead of
    rounding them (H keeps rounding)."""
    rnd = trunc_bf16 if trunc else round_bf16
    r = rnd(b)
    p = r.copy()
    x = np.zeros_like(r)
    rr = _nrm(r)
    pp = rr
    for _ in range(niter):
        w, pap = H_bf16(op, p)
        alpha = rr / (pap + lam * pp)
        x = rnd(x + alpha * p)
        r_new = r - alpha * (w + lam * p)
        rr_new = _nrm(r_new)
        r = rnd(r_new)
        p_new = r + (rr_new / rr) * p
        pp = _nrm(p_new)
        p = rnd(p_new)
        rr = rr_new
    return x

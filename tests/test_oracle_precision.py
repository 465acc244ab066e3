"""Pins of the oracle's 16-bit storage (bfloat16 rounding, H and M_IRS with
16-bit fields; Sec. VI.E, Table "sloppy").

- round_bf16 against hand-worked cases (ties to even at 1 + 2^-8 and
  1 + 3 2^-8) and, on random float32 values, against a construction from the
  float32 bit pattern (the two candidates obtained by clearing the low 16
  bits and by stepping one 2^16 unit up in magnitude, nearer one kept, ties to
  the even pattern) that shares nothing with frexp / rint;
- with the rounding replaced by the identity, H_bf16 is the oracle's H and
  m_irs_bf16 is its FP64 M_IRS (so no term of either is dropped);
- with the rounding in place, the error of H_bf16 sits at the level one
  bfloat16 rounding per stored field gives (so the rounding does happen);
- Table "sloppy": M_IRS in 16 bits, rounded or truncated as the paper does,
  leaves the A-DEF2 iteration count as in FP64 (within one iteration) on a
  small two-level problem;
- truncation equals clearing the low 16 bits of the float32 word.
"""
import numpy as np
import pytest

import synth
from oracle import blocks as blk
from oracle import coarse as crs
from oracle import hdcg
from oracle import precision as prc
from oracle.dwf import DWF, norm2

U_BF16 = 2.0 ** -8  # unit roundoff of an 8-bit significand


def test_round_bf16_hand_cases():
    x = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -20, -1.5, 0.0,
                  3 * 2.0 ** 100, -(1 + 2.0 ** -7 + 2.0 ** -9)])
    want = np.array([1.0, 1.0, 1 + 2.0 ** -6, 1 + 2.0 ** -7, -1.5, 0.0, 3 * 2.0 ** 100, -(1 + 2.0 ** -7)])
    assert np.array_equal(prc.round_bf16(x), want)
    z = prc.round_bf16(np.array([(1 + 2.0 ** -8) + 1j * (1 + 3 * 2.0 ** -8)]))
    assert z[0] == 1.0 + 1j * (1 + 2.0 ** -6)


def _bf16_from_bits(f32):
    """Nearest bfloat16 of each float32 from its bit pattern."""
    u = f32.view(np.uint32).astype(np.uint64)
    lo = u & 0xFFFF0000
    hi = lo + 0x10000
    vlo = lo.astype(np.uint32).view(np.float32).astype(np.float64)
    vhi = hi.astype(np.uint32).view(np.float32).astype(np.float64)
    x = f32.astype(np.float64)
    dlo, dhi = np.abs(x - vlo), np.abs(vhi - x)
    even_lo = ((lo >> 16) & 1) == 0
    take_lo = (dlo < dhi) | ((dlo == dhi) & even_lo)
    return np.where(take_lo, vlo, vhi)


def test_round_bf16_matches_bit_pattern_construction():
    rng = np.random.default_rng(5)
    f = (rng.standard_normal(200000) * np.exp(rng.uniform(-30, 30, 200000))).astype(np.float32)
    # add exact ties: low 16 bits 0x8000 with both parities of bit 16
    t = rng.integers(0x3F000000, 0x40800000, 2000, dtype=np.uint32)
    t = (t & 0xFFFF0000) | 0x8000
    f = np.concatenate([f, t.view(np.float32)])
    got = prc.round_bf16(f.astype(np.float64))
    assert np.array_equal(got, _bf16_from_bits(f))
    rel = np.abs(got - f) / np.abs(f.astype(np.float64))
    assert rel.max() <= U_BF16
    assert np.array_equal(prc.round_bf16(got), got)


def test_trunc_bf16_drops_low_bits():
    rng = np.random.default_rng(6)
    f = (rng.standard_normal(100000) * np.exp(rng.uniform(-20, 20, 100000))).astype(np.float32)
    want = (f.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)
    got = prc.trunc_bf16(f.astype(np.float64))
    assert np.array_equal(got, want)
    assert np.all(np.abs(got) <= np.abs(f)) and np.abs(got - f).max() > 0


@pytest.fixture(scope="module")
def op_small():
    dims, Ls = (4, 4, 4, 8), 6
    return DWF(synth.gauge_field(dims, 0.5, 91), dims, Ls, 1.8, 0.02)


def test_identity_rounding_gives_fp64_oracle(op_small, monkeypatch):
    op = op_small
    x = synth.gaussian_half_field(op.dims, op.Ls, 92)
    monkeypatch.setattr(prc, "round_bf16", lambda a: a)
    y, pap = prc.H_bf16(op, x)
    assert np.array_equal(y, op.H(x))
    assert abs(pap - norm2(op.mpc(x))) <= 1e-13 * pap
    z = prc.m_irs_bf16(op, x, 5, 0.7)
    ref = hdcg.m_irs(op, x, 5, 0.7)
    assert np.abs(z - ref).max() <= 1e-12 * np.abs(ref).max()


def test_h_bf16_error_at_rounding_level(op_small):
    op = op_small
    x = prc.round_bf16(synth.gaussian_half_field(op.dims, op.Ls, 93))
    y, _ = prc.H_bf16(op, x)
    ref = op.H(x)
    rel = np.sqrt(norm2(y - ref) / norm2(ref))
    # four stored fields, each off by at most U_BF16 relative per value
    assert 0.1 * U_BF16 < rel < 4 * U_BF16
    with pytest.raises(ValueError):
        prc.H_bf16(DWF(synth.gauge_field(op.dims, 0.5, 91), op.dims, op.Ls, 1.8, 0.02, b=1.5, c=0.5), x)


def test_sloppy_mirs_keeps_iteration_count():
    """One A-DEF2 solve to 1e-5 (the inner solve of the defect correction)
    with M_IRS in FP64 and in 16 bits: the iteration counts agree to one."""
    dims, Ls, block, nvec = (6, 6, 6, 6), 4, (2, 2, 2, 2), 4
    op = DWF(synth.gauge_field(dims, 0.5, 21), dims, Ls, 1.8, 0.01)
    _, _, sob = blk.block_map(dims, block)
    phi = blk.orthonormalise(synth.gaussian_half_field(dims, Ls, 22, nrhs=nvec), sob)
    C = blk.coarse_dims(dims, block)
    tl = hdcg.TwoLevel(op, phi, sob, C, crs.build_fourier(op, phi, sob, C), coarse_tol=0.04)
    b = synth.gaussian_half_field(dims, Ls, 80)
    its = {}

    def truncating(op_, r_, n_, lam_):
        return prc.m_irs_bf16(op_, r_, n_, lam_, trunc=True)

    for name, fn in (("fp64", None), ("bf16", prc.m_irs_bf16), ("bf16-trunc", truncating)):
        x, it, rel = hdcg.gpcg(tl, b, n_irs=4, tol=1e-5, m_irs_fn=fn)
        assert rel <= 1e-5 and np.sqrt(norm2(b - op.H(x)) / norm2(b)) <= 2e-5
        its[name] = it
    assert abs(its["bf16"] - its["fp64"]) <= 1 and abs(its["bf16-trunc"] - its["fp64"]) <= 1, its

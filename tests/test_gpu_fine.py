"""GPU parity of the fine operator, BLAS-1 and FP64 CG against the oracle.

Tolerances: FP64 applications 1e-12 relative (max-norm); complex64
applications 5e-6 (a sum of ~100 terms of O(1) magnitude in float32,
eps 6e-8); integer layouts bit-exact; CG true residual <= 1e-8."""
import numpy as np
import pytest

import synth
from oracle.cg import cg
from oracle.dwf import DWF
from oracle import geometry as geo
from tests.gpu_util import banner, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1402_2585_amd as hd  # noqa: E402

CASES = {
    "cfg1-4^4xLs8": ((4, 4, 4, 4), 8, 0.5, (1, 1, 1, -1), 0.01),
    "ragged-6x4x4x8xLs5": ((6, 4, 4, 8), 5, 0.8, (1, 1, 1, -1), 0.1),
    "phases-8x4x6x4xLs3": ((8, 4, 6, 4), 3, 0.9, (1, np.exp(0.3j), -1, np.exp(-0.7j)), 0.05),
    "ls1-4x4x4x6": ((4, 4, 4, 6), 1, 0.7, (1, 1, 1, -1), 0.02),
    "ls12-4x4x6x4": ((4, 4, 6, 4), 12, 0.6, (1, 1, 1, -1), 0.003),
}


def _make(name, seed=1):
    dims, Ls, eps, bc, mass = CASES[name]
    U = synth.gauge_field(dims, eps, 100 + seed)
    return dims, Ls, U, bc, mass, hd.FineOperator(U, dims, Ls, 1.8, mass, bc), DWF(U, dims, Ls, 1.8, mass, bc)


@pytest.mark.parametrize("name", list(CASES))
def test_layout_roundtrip_bit_exact(name):
    banner(f"layout {name}")
    dims, Ls, U, bc, mass, op, ref = _make(name)
    for prec, dt in ((hd.DWF_C128, np.complex128), (hd.DWF_C64, np.complex64)):
        b = synth.gaussian_half_field(dims, Ls, 7, nrhs=2).astype(dt)
        back = op.to_canonical(op.to_native(b, prec), prec, nrhs=2).cpu().numpy()
        assert np.array_equal(back, b)
    op.close()


@pytest.mark.parametrize("name", list(CASES))
def test_mpc_and_H_c128(name):
    banner(f"mpc/H c128 {name}")
    dims, Ls, U, bc, mass, op, ref = _make(name)
    b = synth.gaussian_half_field(dims, Ls, 11)
    nb = op.to_native(b)
    for dag in (0, 1):
        got = op.to_canonical(op.mpc(nb, dagger=dag)).cpu().numpy()
        want = ref.mpc_dag(b) if dag else ref.mpc(b)
        assert rel_err(got, want) < 1e-12, (dag, rel_err(got, want))
    got = op.to_canonical(op.H(nb)).cpu().numpy()
    assert rel_err(got, ref.H(b)) < 1e-12
    op.close()


@pytest.mark.parametrize("name", ["cfg1-4^4xLs8", "ragged-6x4x4x8xLs5", "phases-8x4x6x4xLs3"])
def test_H_c64(name):
    banner(f"H c64 {name}")
    dims, Ls, U, bc, mass, op, ref = _make(name)
    b = synth.gaussian_half_field(dims, Ls, 12)
    nb = op.to_native(b, hd.DWF_C64)
    got = op.to_canonical(op.H(nb, hd.DWF_C64), hd.DWF_C64).cpu().numpy()
    err = rel_err(got, ref.H(b))
    print(f"c64 rel err {err:.2e}", flush=True)
    assert err < 5e-6
    op.close()


def test_multi_rhs_matches_single():
    banner("H c128 nrhs=3")
    dims, Ls, U, bc, mass, op, ref = _make("ragged-6x4x4x8xLs5")
    b = synth.gaussian_half_field(dims, Ls, 13, nrhs=3)
    nb = op.to_native(b)
    got = op.to_canonical(op.H(nb, nrhs=3), nrhs=3).cpu().numpy()
    for r in range(3):
        assert rel_err(got[r], ref.H(b[r])) < 1e-12
    op.close()


def test_free_field_plane_wave_through_gpu():
    banner("free-field plane wave 4^4xLs8")
    from tests.test_oracle_dwf import _free_field_K, _plane_wave

    dims, Ls, M5, m = (4, 4, 4, 4), 8, 1.8, 0.01
    U = np.broadcast_to(np.eye(3), (4, 4, 4, 4, 4, 3, 3)).copy()
    op = hd.FineOperator(U, dims, Ls, M5, m)
    p = [np.pi / 2, np.pi, 0.0, 3 * np.pi / 4]
    K = _free_field_K(p, Ls, M5, m)
    lam, W = np.linalg.eigh(K.conj().T @ K)
    for i in (0, len(lam) - 1):
        psi = _plane_wave(dims, Ls, p, W[:, i], np.array([0.2, 0.7j, -0.4]))
        got = op.to_canonical(op.H(op.to_native(psi))).cpu().numpy()
        assert rel_err(got, lam[i] * psi) < 1e-12
    op.close()


def test_gauge_covariance_through_gpu():
    banner("gauge covariance 4x4x6x4xLs4")
    dims, Ls = (4, 4, 6, 4), 4
    U = synth.gauge_field(dims, 0.9, 5)
    g = synth.su3_field(dims, 77)
    U2 = U.copy()
    for mu in range(4):
        gs = np.roll(g, -1, axis=3 - mu)
        U2[..., mu, :, :] = g @ U[..., mu, :, :] @ gs.conj().swapaxes(-1, -2)
    op, op2 = hd.FineOperator(U, dims, Ls, 1.8, 0.01), hd.FineOperator(U2, dims, Ls, 1.8, 0.01)
    go = g.reshape(-1, 3, 3)[geo.parity_sites(dims, 1)]
    psi = synth.gaussian_half_field(dims, Ls, 3)
    gpsi = np.matmul(psi, go.swapaxes(-1, -2))
    lhs = op2.to_canonical(op2.H(op2.to_native(gpsi))).cpu().numpy()
    rhs = np.matmul(op.to_canonical(op.H(op.to_native(psi))).cpu().numpy(), go.swapaxes(-1, -2))
    assert rel_err(lhs, rhs) < 1e-12
    op.close()
    op2.close()


@pytest.mark.parametrize("prec", [hd.DWF_C128, hd.DWF_C64])
def test_blas_against_numpy(prec):
    banner(f"blas prec={prec}")
    dims, Ls, U, bc, mass, op, ref = _make("ragged-6x4x4x8xLs5")
    dt = np.complex128 if prec == hd.DWF_C128 else np.complex64
    tol = 1e-13 if prec == hd.DWF_C128 else 1e-6
    f = [synth.gaussian_half_field(dims, Ls, 20 + i, nrhs=2).astype(dt) for i in range(4)]
    x, r, p, w = [op.to_native(a, prec) for a in f]
    n2 = hd.dwf_norm2(op.h, x, prec, 2)
    want = np.array([np.vdot(f[0][i].astype(complex), f[0][i].astype(complex)).real for i in range(2)])
    assert np.abs(n2 - want).max() <= 1e-13 * want.max()
    n2b = hd.dwf_norm2(op.h, x, prec, 2)
    assert np.array_equal(n2, n2b)  # deterministic reduction
    d = hd.dwf_dot(op.h, x, r, prec, 2)
    wd = np.array([np.vdot(f[0][i].astype(complex), f[1][i].astype(complex)) for i in range(2)])
    assert np.abs(d - wd).max() <= 1e-12 * np.abs(wd).max() + 1e-9
    alpha = [0.3, -1.7]
    rr = hd.dwf_cg_update(op.h, x, r, p, w, alpha, prec, 2)
    xs = op.to_canonical(x, prec, 2).cpu().numpy()
    rs = op.to_canonical(r, prec, 2).cpu().numpy()
    for i in range(2):
        ex = f[0][i].astype(complex) + alpha[i] * f[2][i]
        er = f[1][i].astype(complex) - alpha[i] * f[3][i]
        assert rel_err(xs[i], ex) < tol and rel_err(rs[i], er) < tol
        assert abs(rr[i] - np.vdot(rs[i].astype(complex), rs[i].astype(complex)).real) < 1e-12 * rr[i]
    beta = [0.25, 2.0]
    hd.dwf_xpay(op.h, p, r, beta, prec, 2)
    ps = op.to_canonical(p, prec, 2).cpu().numpy()
    for i in range(2):
        assert rel_err(ps[i], rs[i].astype(complex) + beta[i] * f[2][i]) < tol
    op.close()


def test_cg_solve_config1_against_oracle():
    banner("cg_solve fp64 config 1 (4^4 x Ls8, m=0.01, eps=0.5)")
    dims, Ls, M5, mass = (4, 4, 4, 4), 8, 1.8, 0.01
    U = synth.gauge_field(dims, 0.5, 1001)
    b = synth.gaussian_half_field(dims, Ls, 1100)
    op = hd.FineOperator(U, dims, Ls, M5, mass)
    ref = DWF(U, dims, Ls, M5, mass)
    nb = op.to_native(b)
    x = op.new_field(zero=True)
    rc, st = hd.cg_solve(op.h, x, nb, 1, 1e-8, 5000)
    assert rc == 0 and st["converged"] == 1
    xc = op.to_canonical(x).cpu().numpy()
    r = b - ref.H(xc)
    assert np.sqrt(np.vdot(r, r).real / np.vdot(b, b).real) <= 1e-8
    xr, it, _ = cg(ref.H, b, tol=1e-8)
    print(f"gpu its {st['iterations']} oracle its {it}", flush=True)
    # the host checks convergence two iterations behind the GPU, so up to two
    # extra iterations can run
    assert it - 2 <= st["iterations"] <= it + 4
    assert np.sqrt(np.vdot(xc - xr, xc - xr).real / np.vdot(xr, xr).real) < 1e-5
    op.close()


@pytest.mark.parametrize("inner_tol", [1e-5, 1e-2])
def test_cg_solve_mixed_against_oracle(inner_tol):
    banner(f"cg_solve_mixed config 1 inner_tol={inner_tol}")
    dims, Ls, M5, mass = (4, 4, 4, 4), 8, 1.8, 0.01
    U = synth.gauge_field(dims, 0.5, 1001)
    b = synth.gaussian_half_field(dims, Ls, 1100, nrhs=2)
    op = hd.FineOperator(U, dims, Ls, M5, mass)
    ref = DWF(U, dims, Ls, M5, mass)
    x = op.new_field(nrhs=2, zero=True)
    rc, st = hd.cg_solve_mixed(op.h, x, op.to_native(b), 2, 1e-10, inner_tol, 5000)
    assert rc == 0 and st["converged"] == 1 and st["restarts"] >= 1
    xc = op.to_canonical(x, nrhs=2).cpu().numpy()
    for r in range(2):
        res = b[r] - ref.H(xc[r])
        assert np.sqrt(np.vdot(res, res).real / np.vdot(b[r], b[r]).real) <= 1e-10
    # zero source
    z = op.new_field(zero=True)
    rc, st = hd.cg_solve_mixed(op.h, op.new_field(), z, 1, 1e-8)
    assert rc == 0 and st["iterations"] == 0
    op.close()


def test_cg_solve_more_hop_workgroups_than_reduction_slots():
    """24^3 x 48 gives 82944 hop workgroups (4 sites each), more than the
    65536 slots of the BLAS reductions: the fused |M_pc p|^2 of the CG must
    still be summed over all of them."""
    banner("cg_solve fp64 24^3x48 x Ls2 (fused norm over 82944 workgroups)")
    dims, Ls, M5, mass = (24, 24, 24, 48), 2, 1.8, 0.2
    U = synth.gauge_field(dims, 0.5, 1201)
    b = synth.gaussian_half_field(dims, Ls, 1202)
    op = hd.FineOperator(U, dims, Ls, M5, mass)
    x = op.new_field(zero=True)
    rc, st = hd.cg_solve(op.h, x, op.to_native(b), 1, 1e-8, 2000)
    assert rc == 0 and st["converged"] == 1
    xc = op.to_canonical(x).cpu().numpy()
    op.close()
    r = b - DWF(U, dims, Ls, M5, mass).H(xc)
    assert np.sqrt(np.vdot(r, r).real / np.vdot(b, b).real) <= 1e-8


def test_cg_solve_zero_source_and_maxiter():
    banner("cg_solve edge cases")
    dims, Ls = (4, 4, 4, 4), 4
    op = hd.FineOperator(synth.gauge_field(dims, 0.5, 3), dims, Ls, 1.8, 0.01)
    x = op.new_field(zero=True)
    z = op.new_field(zero=True)
    rc, st = hd.cg_solve(op.h, x, z, 1, 1e-8, 100)
    assert rc == 0 and st["iterations"] == 0
    b = op.to_native(synth.gaussian_half_field(dims, Ls, 4))
    rc, st = hd.cg_solve(op.h, x, b, 1, 1e-8, 3)
    assert rc == hd.DWF_NOT_CONVERGED and st["converged"] == 0
    op.close()


def test_config2_full_size_H():
    """Config 2 (16^4 x Ls16, eps 0.7) at full size in the launch shape the
    benchmark times: c128 to 1e-12, c64 to 5e-6."""
    banner("H config 2 full size 16^4xLs16")
    dims, Ls, M5, mass = (16, 16, 16, 16), 16, 1.8, 0.01
    U = synth.gauge_field(dims, 0.7, 2001)
    b = synth.gaussian_half_field(dims, Ls, 2100)
    op = hd.FineOperator(U, dims, Ls, M5, mass)
    want = DWF(U, dims, Ls, M5, mass).H(b)
    got = op.to_canonical(op.H(op.to_native(b))).cpu().numpy()
    assert rel_err(got, want) < 1e-12
    got64 = op.to_canonical(op.H(op.to_native(b, hd.DWF_C64), hd.DWF_C64), hd.DWF_C64).cpu().numpy()
    assert rel_err(got64, want) < 5e-6
    op.close()


# Launch shapes of the hop kernel (dwf_set_hop_shape: bx, by, bz, bt, remap,
# lds_kb, nt, morton, phases): every ordering and load-phase path must give
# the same operator as the oracle.
SHAPES = {
    "default": None,
    "linear": (0, 0, 0, 0, 1, 0, 1, 1, 4),
    "two-phases": (2, 2, 1, 1, 1, 0, 1, 1, 2),
    "lexicographic-2^4-plain-stores": (2, 2, 2, 2, 0, 0, 0, 0, 4),
    "morton-1x2x2x1-no-remap": (1, 2, 2, 1, 0, 0, 1, 1, 4),
    "regions-morton-2x2x1x1": (2, 2, 1, 1, 1, 0, 1, 2, 4),
    "regions-planes-2^4": (2, 2, 2, 2, 1, 0, 1, 3, 4),
}


@pytest.mark.parametrize("shape", list(SHAPES))
def test_hop_launch_shapes_ls16(shape):
    banner(f"launch shape {shape}")
    dims, Ls = (8, 8, 4, 8), 16
    U = synth.gauge_field(dims, 0.7, 150)
    op = hd.FineOperator(U, dims, Ls, 1.8, 0.02)
    if SHAPES[shape] is not None:
        hd.dwf_set_hop_shape(op.h, SHAPES[shape])
    ref = DWF(U, dims, Ls, 1.8, 0.02)
    b = synth.gaussian_half_field(dims, Ls, 151)
    want = ref.H(b)
    got = op.to_canonical(op.H(op.to_native(b))).cpu().numpy()
    assert rel_err(got, want) < 1e-12
    got64 = op.to_canonical(op.H(op.to_native(b, hd.DWF_C64), hd.DWF_C64), hd.DWF_C64).cpu().numpy()
    assert rel_err(got64, want) < 5e-6
    op.close()


@pytest.mark.parametrize("order", [2, 3, 4])
@pytest.mark.parametrize("block", [(2, 2, 1, 1), (1, 2, 2, 1)])
def test_hop_region_orders_on_a_block_grid_of_odd_extents(order, block):
    """The table orders (eight per-XCD regions by bisection, Morton or
    t-planes inside) on a lattice whose block grid is not a power of two
    (3 x 3 x 4 x 6 blocks of 2x2x1x1, 6 x 3 x 2 x 6 of 1x2x2x1; regions of
    unequal size): every site is computed once, with the arithmetic of every
    other order, so H matches the oracle (complex128) and equals, bit for bit,
    the lexicographic order's H in complex128, complex64 and 16-bit storage."""
    dims, Ls = (12, 6, 4, 6), 16
    banner(f"region order {order} block {block} on {dims} x Ls{Ls}")
    U = synth.gauge_field(dims, 0.7, 152)
    op = hd.FineOperator(U, dims, Ls, 1.8, 0.02)
    lex = hd.FineOperator(U, dims, Ls, 1.8, 0.02)
    hd.dwf_set_hop_shape(op.h, tuple(block) + (1, 0, 1, order, 4))
    hd.dwf_set_hop_shape(lex.h, tuple(block) + (0, 0, 1, 0, 4))
    assert hd.dwf_get_hop_shape(op.h, hd.DWF_C128)[0][7] == order
    b = synth.gaussian_half_field(dims, Ls, 153)
    want = DWF(U, dims, Ls, 1.8, 0.02).H(b)
    x = op.to_native(b)
    got = op.H(x)
    assert rel_err(op.to_canonical(got).cpu().numpy(), want) < 1e-12
    assert torch.equal(got, lex.H(x))
    x64 = op.to_native(b, hd.DWF_C64)
    assert torch.equal(op.H(x64, hd.DWF_C64), lex.H(x64, hd.DWF_C64))
    x16, _ = _bf16_input(op, b)
    assert torch.equal(op.H(x16, hd.DWF_BF16), lex.H(x16, hd.DWF_BF16))
    op.close()
    lex.close()


def test_dwf_tune_hop_runs_the_autotuner_once():
    """dwf_tune_hop tunes one (storage, one / several RHS) slot on scratch
    fields: afterwards dwf_get_hop_shape reports it tuned, every candidate
    tried has a positive time (the several-RHS candidates only for the
    several-RHS slot), and H with the chosen shape matches the oracle."""
    dims, Ls = (8, 8, 4, 8), 16
    banner("dwf_tune_hop")
    U = synth.gauge_field(dims, 0.7, 159)
    op = hd.FineOperator(U, dims, Ls, 1.8, 0.02)
    assert not hd.dwf_get_hop_shape(op.h, hd.DWF_C64, 1)[2]
    for n in (1, 3):
        hd.dwf_tune_hop(op.h, hd.DWF_C64, n)
        shape, ms, tuned = hd.dwf_get_hop_shape(op.h, hd.DWF_C64, n)
        print(n, shape, [round(m, 4) for m in ms], flush=True)
        assert tuned and len(ms) >= 13 and all(m > 0 for m in ms[:13])
        assert all((m > 0) == (n > 1) for m in ms[13:])
    assert not hd.dwf_get_hop_shape(op.h, hd.DWF_BF16, 1)[2]
    b = synth.gaussian_half_field(dims, Ls, 160)
    got = op.to_canonical(op.H(op.to_native(b, hd.DWF_C64), hd.DWF_C64), hd.DWF_C64).cpu().numpy()
    assert rel_err(got, DWF(U, dims, Ls, 1.8, 0.02).H(b)) < 5e-6
    op.close()


@pytest.mark.parametrize("mobius", [False, True])
def test_hop_several_rhs_per_workgroup_bitwise(mobius):
    """rg > 1: one workgroup applies a stage to several right-hand sides one
    after another on the links it staged once.  H on 5 right-hand sides
    (groups of 4 and 1, and of 5 with rg = 16) equals, bit for bit, the one
    right-hand side per workgroup form in complex128, complex64 and 16-bit
    storage (Shamir and Mobius: the adjoint Mobius stage has an LDS buffer of
    its own then); M_IRS on 3 right-hand sides, whose CG takes (p, H p) from
    the fused norms of the same stages, gives the same result in complex64
    and 16-bit fields."""
    dims, Ls, nr = (8, 8, 4, 8), 16, 5
    banner(f"several RHS per workgroup, mobius={mobius}")
    U = synth.gauge_field(dims, 0.7, 154)
    kw = dict(b5=1.5, c5=0.5) if mobius else {}
    ops = {rg: hd.FineOperator(U, dims, Ls, 1.8, 0.02, **kw) for rg in (1, 4, 16)}
    for rg, o in ops.items():
        hd.dwf_set_hop_shape(o.h, (2, 2, 1, 1, 1, 0, 0, 4, 0, rg))
    b = synth.gaussian_half_field(dims, Ls, 155, nrhs=nr)
    op1 = ops[1]
    want = DWF(U, dims, Ls, 1.8, 0.02, **({"b": 1.5, "c": 0.5} if mobius else {})).H(b[2])
    for prec in (hd.DWF_C128, hd.DWF_C64, hd.DWF_BF16):
        x = _bf16_input(op1, b)[0] if prec == hd.DWF_BF16 else op1.to_native(b, prec)
        ref = op1.H(x, prec, nrhs=nr)
        for rg in (4, 16):
            assert torch.equal(ops[rg].H(x, prec, nrhs=nr), ref), (prec, rg)
        if prec == hd.DWF_C128:
            got = op1.to_canonical(ref, nrhs=nr).cpu().numpy()[2]
            assert rel_err(got, want) < 1e-12
    for o in ops.values():
        o.close()
    # M_IRS on 3 right-hand sides (its CG takes (p, H p) from the fused norm
    # of the stages), complex64 and 16-bit fields
    dims = (12, 12, 12, 12)
    U = synth.gauge_field(dims, 0.7, 156)
    raw = synth.gaussian_half_field(dims, Ls, 157, nrhs=4)
    r = synth.gaussian_half_field(dims, Ls, 158, nrhs=3)
    outs = {}
    for rg in (1, 4):
        o = hd.FineOperator(U, dims, Ls, 1.8, 0.02, **kw)
        hd.dwf_set_hop_shape(o.h, (2, 2, 1, 1, 1, 0, 0, 4, 0, rg))
        h = hd.HDCG(o, (4, 4, 4, 4), raw)
        for iprec in (hd.DWF_C64, hd.DWF_BF16):
            h.set_params(irs_prec=iprec)
            z = o.new_field(hd.DWF_C64, 3, zero=True)
            hd.hdcg_mirs(h.h, z, o.to_native(r, hd.DWF_C64), 3)
            outs[(rg, iprec)] = z
        h.close()
        o.close()
    for iprec in (hd.DWF_C64, hd.DWF_BF16):
        assert torch.equal(outs[(1, iprec)], outs[(4, iprec)]), iprec


# Mobius (Cayley-form) kernel: (b5, c5) other than Shamir's (1, 0)
MOBIUS = {
    "4^4xLs8-b1.5-c0.5": ((4, 4, 4, 4), 8, 1.5, 0.5, 0.02, (1, 1, 1, -1)),
    "8x4x6x4xLs5-b2-c1-phases": ((8, 4, 6, 4), 5, 2.0, 1.0, 0.1, (1, np.exp(0.3j), -1, np.exp(-0.7j))),
    "8x8x4x8xLs16-b1.5-c0.5": ((8, 8, 4, 8), 16, 1.5, 0.5, 0.01, (1, 1, 1, -1)),
    "4x4x4x6xLs1-b1.2-c0.3": ((4, 4, 4, 6), 1, 1.2, 0.3, 0.05, (1, 1, 1, -1)),
}


@pytest.mark.parametrize("name", list(MOBIUS))
def test_mobius_mpc_and_H(name):
    banner(f"mobius {name}")
    dims, Ls, b5, c5, mass, bc = MOBIUS[name]
    U = synth.gauge_field(dims, 0.6, 160)
    op = hd.FineOperator(U, dims, Ls, 1.8, mass, bc, b5=b5, c5=c5)
    ref = DWF(U, dims, Ls, 1.8, mass, bc, b=b5, c=c5)
    b = synth.gaussian_half_field(dims, Ls, 161)
    nb = op.to_native(b)
    for dag in (0, 1):
        got = op.to_canonical(op.mpc(nb, dagger=dag)).cpu().numpy()
        want = ref.mpc_dag(b) if dag else ref.mpc(b)
        assert rel_err(got, want) < 1e-12, (dag, rel_err(got, want))
    want = ref.H(b)
    assert rel_err(op.to_canonical(op.H(nb)).cpu().numpy(), want) < 1e-12
    got64 = op.to_canonical(op.H(op.to_native(b, hd.DWF_C64), hd.DWF_C64), hd.DWF_C64).cpu().numpy()
    assert rel_err(got64, want) < 5e-6
    op.close()


def test_mobius_cg_solve_against_oracle():
    banner("mobius cg_solve 4^4 x Ls8")
    dims, Ls, b5, c5, mass = (4, 4, 4, 4), 8, 1.5, 0.5, 0.02
    U = synth.gauge_field(dims, 0.5, 162)
    b = synth.gaussian_half_field(dims, Ls, 163)
    op = hd.FineOperator(U, dims, Ls, 1.8, mass, b5=b5, c5=c5)
    x = op.new_field(zero=True)
    rc, st = hd.cg_solve(op.h, x, op.to_native(b), 1, 1e-9, 5000)
    assert rc == 0
    r = b - DWF(U, dims, Ls, 1.8, mass, b=b5, c=c5).H(op.to_canonical(x).cpu().numpy())
    assert np.sqrt(np.vdot(r, r).real / np.vdot(b, b).real) <= 1e-9
    op.close()


def test_mobius_rejects_unstable_fifth_dimension():
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 0.5, 164)
    with pytest.raises(hd.HdcgError):
        hd.FineOperator(U, dims, 8, 1.8, 0.01, b5=0.1, c5=2.0)  # |beta| > |alpha|


# 16-bit (bfloat16) storage of fine fields: the form M_IRS takes with
# irs_prec = DWF_BF16 (Sec. VI.E, Table "sloppy").  Against the oracle that
# rounds the same stored fields, the only differences are rounding decisions
# that FP32 (kernel) and FP64 (oracle) arithmetic take apart, each one unit in
# the last bfloat16 place, so: norm-wise 2e-4 (vs ~2e-3 for one missing or
# extra rounding: unit roundoff 2^-8 = 3.9e-3), and element-wise 2^-6 of the
# value plus 2^-8 of the largest value.
from oracle import precision as prc  # noqa: E402

BF16_CASES = ["cfg1-4^4xLs8", "ragged-6x4x4x8xLs5", "phases-8x4x6x4xLs3", "ls12-4x4x6x4"]


def _bf16_input(op, b):
    """b rounded through complex64 and then the library's bfloat16 store."""
    n64 = op.to_native(b, hd.DWF_C64)
    nrhs = b.size // (op.Vh * op.Ls * 12)
    return op.convert(n64, hd.DWF_BF16, hd.DWF_C64, nrhs), n64


def _from_bf16(op, x16, nrhs=1):
    return op.to_canonical(op.convert(x16, hd.DWF_C64, hd.DWF_BF16, nrhs), hd.DWF_C64, nrhs).cpu().numpy()


def _check_bf16(got, want):
    got = np.asarray(got, np.complex128)
    nerr = np.sqrt(np.vdot(got - want, got - want).real / np.vdot(want, want).real)
    d = np.abs(got - want)
    bound = 2.0 ** -6 * np.abs(want) + 2.0 ** -8 * np.abs(want).max()
    return nerr, bool(np.all(d <= bound))


def test_bf16_convert_is_round_to_nearest_even():
    banner("bf16 convert 6x4x4x8xLs5 nrhs=2")
    dims, Ls, U, bc, mass, op, ref = _make("ragged-6x4x4x8xLs5")
    b = synth.gaussian_half_field(dims, Ls, 17, nrhs=2).astype(np.complex64)
    x16, _ = _bf16_input(op, b)
    assert x16.dtype == torch.bfloat16 and x16.numel() == 2 * b.size
    got = _from_bf16(op, x16, 2)
    assert np.array_equal(got.astype(np.complex128), prc.round_bf16(b.astype(np.complex128)))
    nrm = hd.dwf_norm2(op.h, x16, hd.DWF_BF16, 2)
    want = [np.vdot(g, g).real for g in got.astype(np.complex128)]
    assert np.allclose(nrm, want, rtol=1e-12, atol=0)
    with pytest.raises(hd.HdcgError):
        hd.dwf_convert(op.h, x16, hd.DWF_BF16, op.to_native(b[0]), hd.DWF_C128, 1)
    op.close()


@pytest.mark.parametrize("name", BF16_CASES)
def test_bf16_mpc_and_H_against_rounding_oracle(name):
    banner(f"mpc/H bf16 {name}")
    dims, Ls, U, bc, mass, op, ref = _make(name)
    b = synth.gaussian_half_field(dims, Ls, 18).astype(np.complex64)
    x16, _ = _bf16_input(op, b)
    xin = prc.round_bf16(b.astype(np.complex128))
    for dag in (0, 1):
        got = _from_bf16(op, op.mpc(x16, hd.DWF_BF16, dagger=dag))
        want = prc.mpc_dag_bf16(ref, xin) if dag else prc.mpc_bf16(ref, xin)[0]
        nerr, elem_ok = _check_bf16(got, want)
        print(f"dagger={dag} norm-wise {nerr:.2e}", flush=True)
        assert nerr < 2e-4 and elem_ok
    got = _from_bf16(op, op.H(x16, hd.DWF_BF16))
    nerr, elem_ok = _check_bf16(got, prc.H_bf16(ref, xin)[0])
    print(f"H norm-wise {nerr:.2e}", flush=True)
    assert nerr < 2e-4 and elem_ok
    # and against the exact FP64 H: the error one rounding per stored field gives
    exact = ref.H(xin)
    e = np.sqrt(np.vdot(got - exact, got - exact).real / np.vdot(exact, exact).real)
    assert 2.0 ** -8 / 10 < e < 4 * 2.0 ** -8
    op.close()


def test_bf16_mobius_H_within_rounding_bound():
    banner("H bf16 mobius 8x8x4x8xLs16")
    dims, Ls, b5, c5, mass, bc = MOBIUS["8x8x4x8xLs16-b1.5-c0.5"]
    U = synth.gauge_field(dims, 0.6, 165)
    op = hd.FineOperator(U, dims, Ls, 1.8, mass, bc, b5=b5, c5=c5)
    ref = DWF(U, dims, Ls, 1.8, mass, bc, b=b5, c=c5)
    b = synth.gaussian_half_field(dims, Ls, 166).astype(np.complex64)
    x16, _ = _bf16_input(op, b)
    xin = prc.round_bf16(b.astype(np.complex128))
    got = _from_bf16(op, op.H(x16, hd.DWF_BF16))
    exact = ref.H(xin)
    e = np.sqrt(np.vdot(got - exact, got - exact).real / np.vdot(exact, exact).real)
    print(f"mobius bf16 H norm-wise {e:.2e}", flush=True)
    assert e < 4 * 2.0 ** -8
    op.close()


def test_bf16_full_size_H_config2():
    """16^4 x Ls16 in the launch shape the benchmark times, against the
    rounding oracle on every site."""
    banner("H bf16 config 2 full size 16^4xLs16")
    dims, Ls, M5, mass = (16, 16, 16, 16), 16, 1.8, 0.01
    U = synth.gauge_field(dims, 0.7, 2001)
    b = synth.gaussian_half_field(dims, Ls, 2100).astype(np.complex64)
    op = hd.FineOperator(U, dims, Ls, M5, mass)
    x16, _ = _bf16_input(op, b)
    got = _from_bf16(op, op.H(x16, hd.DWF_BF16))
    want = prc.H_bf16(DWF(U, dims, Ls, M5, mass), prc.round_bf16(b.astype(np.complex128)))[0]
    nerr, elem_ok = _check_bf16(got, want)
    print(f"config 2 bf16 H norm-wise {nerr:.2e}", flush=True)
    assert nerr < 2e-4 and elem_ok
    op.close()

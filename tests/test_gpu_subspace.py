"""GPU parity of the rational-filter subspace generation (Sec. IV.B,
equation "ratfilt"): multi-shift CG against the oracle's shifted solves, and
the filtered, wall-masked, block-normalised subspace of hdcg_setup against
the oracle's.

Tolerances: each shifted solution to 1e-7 relative (max-norm) of the exact
one when the base residual is 1e-10 (the error is at most the residual over
the smallest eigenvalue of H + s, which is above 1e-3 here); the filtered
subspace to 1e-6 (both sides stop a multi-shift solve at 1e-10, the GPU up to
two iterations later, and the partial-fraction sum amplifies the remaining
difference by at most max|c_j| / max response, about 1e2 here); a full
solve on the filtered subspace reaches the FP64 residual."""
import numpy as np
import pytest

import synth
from oracle import blocks as oblk
from oracle import subspace as osub
from oracle.cg import cg
from oracle.dwf import DWF
from tests.gpu_util import banner, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1402_2585_amd as hd  # noqa: E402


@pytest.mark.parametrize("dims,Ls,nrhs,shifts", [
    ((4, 4, 4, 4), 8, 2, [0.01, 0.03, 0.1, 0.5]),
    ((6, 4, 4, 8), 5, 1, [3e-4, 4e-4, 5e-4, 6e-4]),
    ((4, 4, 6, 4), 3, 3, [0.2]),
])
def test_multishift_cg_against_shifted_solves(dims, Ls, nrhs, shifts):
    banner(f"multishift {dims} Ls{Ls} nrhs={nrhs} shifts={shifts}")
    U = synth.gauge_field(dims, 0.5, 400)
    op = hd.FineOperator(U, dims, Ls, 1.8, 0.02)
    ref = DWF(U, dims, Ls, 1.8, 0.02)
    b = synth.gaussian_half_field(dims, Ls, 401, nrhs=nrhs)
    x = op.new_field(nrhs=nrhs * len(shifts))
    rc, st = hd.dwf_multishift_cg(op.h, x, op.to_native(b), shifts, nrhs, tol=1e-10, maxiter=5000)
    print(rc, st, flush=True)
    assert rc == 0 and st["converged"] == 1
    got = op.to_canonical(x, nrhs=nrhs * len(shifts)).cpu().numpy().reshape((len(shifts), nrhs) + op.canonical_shape)
    bb = b.reshape((nrhs,) + op.canonical_shape)
    for j, s in enumerate(shifts):
        for r in range(nrhs):
            want, _, _ = cg(lambda u, s=s: ref.H(u) + s * u, bb[r], tol=1e-13)
            err = rel_err(got[j, r], want)
            assert err < 1e-7, (j, r, err)
    op.close()


def test_multishift_rejects_bad_shifts():
    dims, Ls = (4, 4, 4, 4), 4
    op = hd.FineOperator(synth.gauge_field(dims, 0.5, 402), dims, Ls, 1.8, 0.02)
    b = op.to_native(synth.gaussian_half_field(dims, Ls, 403))
    x = op.new_field(nrhs=2)
    with pytest.raises(hd.HdcgError):
        hd.dwf_multishift_cg(op.h, x, b, [0.5, 0.1])  # base shift not the smallest
    with pytest.raises(hd.HdcgError):
        hd.dwf_multishift_cg(op.h, x, b, [0.1] * 9)   # more than 8 shifts
    op.close()


def test_rational_filter_subspace_against_oracle():
    """hdcg_setup with subspace_gen = 1 and wall noise: the wall-masked,
    filtered noise, block-normalised, against the oracle's (one vector: the
    oracle's filter costs about 20 s of CPU here)."""
    dims, Ls, block, nvec, wall = (12, 12, 12, 12), 2, (4, 4, 4, 4), 1, True
    banner(f"rational-filter subspace 12^4 x Ls2 nvec={nvec} wall={wall}")
    lam, eps = 0.1, 0.1 / 3
    U = synth.gauge_field(dims, 0.5, 410)
    raw = synth.gaussian_half_field(dims, Ls, 411, nrhs=nvec)
    op = hd.FineOperator(U, dims, Ls, 1.8, 0.01)
    h = hd.HDCG(op, block, raw, subspace_gen=1, rat_lo=lam, rat_eps=eps, rat_tol=1e-10, rat_maxiter=5000,
                wall_noise=int(wall))
    ref = DWF(U, dims, Ls, 1.8, 0.01)
    filt = np.stack([osub.rational_filter(ref, raw[k], lam, eps, tol=1e-10, wall=wall)[0] for k in range(nvec)])
    _, _, sob = oblk.block_map(dims, block)
    want = oblk.orthonormalise(filt, sob)
    got = h.subspace().cpu().numpy()
    err = rel_err(got, want)
    print(f"filtered subspace rel err {err:.2e}", flush=True)
    assert err < 1e-6
    h.close()
    op.close()


def test_hdcg_solve_with_rational_filter_subspace():
    """The paper's filter (lambda = 3e-4, eps = lambda/3, residual 1e-6, wall
    noise) as the subspace of a full solve, beside the raw noise it starts
    from (iteration counts printed; with Ls = 2 and 4 vectors the two deflate
    about equally -- the comparison that matters is the benchmark's at
    16^3 x 32 x 16 with 24 vectors)."""
    dims, Ls, block, nvec = (12, 12, 12, 12), 2, (4, 4, 4, 4), 4
    banner("hdcg_solve with the rational-filter subspace 12^4 x Ls2")
    U = synth.gauge_field(dims, 0.5, 300)
    raw = synth.gaussian_half_field(dims, Ls, 301, nrhs=nvec)
    op = hd.FineOperator(U, dims, Ls, 1.8, 0.01)
    ref = DWF(U, dims, Ls, 1.8, 0.01)
    b = synth.gaussian_half_field(dims, Ls, 358)
    its = {}
    for name, kw in (("noise", {}), ("filter", dict(subspace_gen=1, wall_noise=1))):
        h = hd.HDCG(op, block, raw, **kw)
        x = op.new_field()
        rc, st = hd.hdcg_solve(h.h, x, op.to_native(b), 1, 1e-8)
        print(name, st, flush=True)
        assert rc == 0 and st["converged"] == 1
        r = b - ref.H(op.to_canonical(x).cpu().numpy())
        assert np.sqrt(np.vdot(r, r).real / np.vdot(b, b).real) <= 1e-8
        its[name] = st["inner_iterations"]
        h.close()
    print("A-DEF2 iterations", its, flush=True)
    with pytest.raises(hd.HdcgError):
        hd.HDCG(op, block, raw, subspace_gen=1, rat_lo=-1.0)
    op.close()


def test_surface_truncated_subspace():
    """Surface-depth truncation (Sec. IV.B, closing paragraph of the
    subspace-generation subsection) on 12^4 x Ls12, Nvec 4, 4^4 blocks, depth
    4: the subspace equals the oracle's block-orthonormalised truncated
    vectors (1e-12) with an exactly zero interior; project and promote
    through the surface-only copies (complex64, and bf16 against the
    oracle's rounding of the same subspace: 2e-5) on 1, 2 and 6 right-hand
    sides (streaming and tiled kernels) equal the oracle's, the promoted
    interior exactly zero over a prefilled output; HDCG with it reaches the
    FP64 residual 1e-8."""
    from oracle import precision as prc

    dims, Ls, block, nvec, depth = (12, 12, 12, 12), 12, (4, 4, 4, 4), 4, 4
    banner(f"surface-truncated subspace {dims} Ls{Ls} depth {depth}")
    U = synth.gauge_field(dims, 0.5, 430)
    raw = synth.gaussian_half_field(dims, Ls, 431, nrhs=nvec)
    op = hd.FineOperator(U, dims, Ls, 1.8, 0.02)
    ref = DWF(U, dims, Ls, 1.8, 0.02)
    h = hd.HDCG(op, block, raw, n_ii=0, surface_depth=depth)
    _, _, sob = oblk.block_map(dims, block)
    phi = oblk.orthonormalise(osub.surface_truncate(raw, depth), sob)
    got = h.subspace().cpu().numpy()
    assert rel_err(got, phi) < 1e-12
    assert not got[:, depth:Ls - depth].any()
    phi16 = prc.round_bf16(phi)
    for prec, P in ((hd.DWF_C64, phi), (hd.DWF_BF16, phi16)):
        for nr in (1, 2, 6):
            v = synth.gaussian_half_field(dims, Ls, 432 + nr, nrhs=nr).astype(np.complex64)
            c = h.new_coarse(hd.DWF_C64, nrhs=nr)
            hd.hdcg_project(h.h, c, op.to_native(v, hd.DWF_C64), prec, nr)
            want = oblk.project(P, sob, v.astype(np.complex128).reshape((nr,) + v.shape[-4:]))
            err_p = rel_err(c.cpu().numpy(), want)
            cc = synth.gaussian_coarse(h.Nc, nvec, 440 + nr, nr).astype(np.complex64)
            f = op.new_field(hd.DWF_C64, nrhs=nr)
            f.fill_(1.0)
            hd.hdcg_promote(h.h, f, torch.from_numpy(cc).to("cuda"), prec, nr)
            gotp = op.to_canonical(f, hd.DWF_C64, nrhs=nr).cpu().numpy().reshape((nr,) + v.shape[-4:])
            want = osub.surface_truncate(oblk.promote(P, sob, cc.astype(np.complex128)), depth)
            err_q = rel_err(gotp, want)
            print(f"prec={prec} nrhs={nr}: project {err_p:.2e}, promote {err_q:.2e}", flush=True)
            assert err_p < 2e-5 and err_q < 2e-5
            assert not gotp[:, depth:Ls - depth].any()
    b = synth.gaussian_half_field(dims, Ls, 450)
    for pprec in (hd.DWF_C64, hd.DWF_BF16):
        h.set_params(phi_prec=pprec)
        x = op.new_field()
        rc, st = hd.hdcg_solve(h.h, x, op.to_native(b), 1, 1e-8)
        print(f"hdcg_solve, surface subspace, phi_prec={pprec}", st, flush=True)
        assert rc == 0 and st["converged"] == 1
        r = b - ref.H(op.to_canonical(x).cpu().numpy())
        assert np.sqrt(np.vdot(r, r).real / np.vdot(b, b).real) <= 1e-8
    with pytest.raises(hd.HdcgError):
        hd.HDCG(op, block, raw, n_ii=0, surface_depth=3)
    h.close()
    op.close()

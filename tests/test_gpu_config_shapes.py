"""GPU parity at the shapes the HDCG workloads run: Ls = 16 fine fields,
Nvec = 24 on a coarse 4x3x3x3 grid and Nvec = 48 on a coarse 6x3x3x3 grid
(Fourier momenta with m = 1 on an extent that 3 does not divide, and m = 2),
so that the instantiations the 16^3x32 and 24^3x48 workloads execute are
compared with the oracle: the block kernels on 24576-entry block panels with
Nvec > 16 (several vector groups of the orthonormalisation, several 16-vector
tiles of the block dot products), the MFMA mat-vec with two and three
16-row M tiles, and the persistent coarse CG on them.

The full oracle operator would take Nc * Nvec applications of H per shape, so
the GPU's build is checked on sampled columns: for a sampled (b, k) the
oracle applies H to its own orthonormalised phi^b_k and projects onto its own
phi^a_j for blocks a around b (including stencil entries that wrap around the
coarse torus).  The coarse kernels are checked on a seeded Hermitian
positive-definite stencil operator (synth) imported into the handle, against
the oracle's mat-vec and a dense solve.  End-to-end solves at the
12^3x24 x Ls8, Nvec 8 configuration and at the full 16^3x32 x Ls16, Nvec 24
workload are checked with one application of the oracle's H.

Tolerances as in the other GPU tests: FP64 1e-12 (max-norm, relative to the
largest entry), complex64 2e-5, bf16 1e-2, fp16 2e-3; solves to their
stated residuals.
"""
import multiprocessing as mp

import numpy as np
import pytest

import synth
from oracle import blocks as oblk
from oracle import coarse as ocrs
from oracle import precision as oprc
from oracle.dwf import DWF
from synth.configs import WORKLOADS
from tests.gpu_util import banner, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1402_2585_amd as hd  # noqa: E402

SHAPES = {
    # name: dims, Ls, nvec, eps, mass, seed
    "16x12^3xLs16-n24": ((16, 12, 12, 12), 16, 24, 0.7, 0.003, 410),
    "24x12^3xLs16-n48": ((24, 12, 12, 12), 16, 48, 0.7, 0.001, 420),
}
BLOCK = (4, 4, 4, 4)


def _coarse_index(C, c):
    c = np.mod(np.asarray(c), np.array(C))
    return int(c[0] + C[0] * (c[1] + C[1] * (c[2] + C[2] * c[3])))


@pytest.fixture(scope="module", params=list(SHAPES))
def shape(request):
    name = request.param
    dims, Ls, nvec, eps, mass, seed = SHAPES[name]
    banner(f"setup {name}")
    U = synth.gauge_field(dims, eps, seed)
    raw = synth.gaussian_half_field(dims, Ls, seed + 1, nrhs=nvec)
    op = hd.FineOperator(U, dims, Ls, 1.8, mass)
    h = hd.HDCG(op, BLOCK, raw, n_ii=0)
    ref = DWF(U, dims, Ls, 1.8, mass)
    _, _, sob = oblk.block_map(dims, BLOCK)
    C = oblk.coarse_dims(dims, BLOCK)
    cc = ocrs.coarse_coords(C)
    # sampled columns (b, k): the corner block (its stencil wraps in every
    # direction) and the far end in x; the blocks a checked around each
    cols = [(0, 0), (C[0] - 1, nvec - 1)]
    rows = {}
    for b, _ in cols:
        rows[b] = sorted({_coarse_index(C, cc[b] + d) for d in
                          ((0, 0, 0, 0), (-1, 0, 0, 0), (1, 0, 0, 0), (0, 0, 0, 1), (-1, -1, -1, -1), (1, 1, 0, -1))})
    blocks = sorted({b for b, _ in cols} | {a for r in rows.values() for a in r})
    phi = oblk.orthonormalise(raw, sob[blocks])  # the oracle's subspace on the sampled blocks
    del raw
    yield dict(name=name, dims=dims, Ls=Ls, nvec=nvec, op=op, h=h, ref=ref, sob=sob, C=C, cols=cols, rows=rows,
               blocks=blocks, phi=phi)
    h.close()
    op.close()


def _block_part(v, sob, b):
    """(..., Ls, nsb, 4, 3) part of half-field(s) v on block b."""
    return v[..., :, sob[b], :, :]


def test_subspace_on_sampled_blocks(shape):
    t = shape
    banner(f"subspace {t['name']}")
    P = t["h"].subspace()  # on the GPU, canonical
    for b in t["blocks"]:
        got = P[:, :, torch.from_numpy(t["sob"][b]).to("cuda")].cpu().numpy()
        want = _block_part(t["phi"], t["sob"], b)
        assert rel_err(got, want) < 1e-12, b


def test_coarse_operator_sampled_columns(shape):
    """A[a][l][j][k] = <phi^a_j | H | phi^{a+delta_l}_k> of the GPU's
    Fourier-trick build against the oracle's H on sampled columns."""
    t = shape
    banner(f"coarse A sampled columns {t['name']}")
    A = t["h"].coarse_matrix()
    C, sob, phi = t["C"], t["sob"], t["phi"]
    cc = ocrs.coarse_coords(C)
    offs = ocrs.stencil_offsets()
    for b, k in t["cols"]:
        v = np.zeros(phi.shape[1:], dtype=np.complex128)
        v[:, sob[b]] = phi[k][:, sob[b]]
        w = t["ref"].H(v)
        scale = 0.0
        got, want = [], []
        for a in t["rows"][b]:
            d = (cc[b] - cc[a] + 1) % np.array(C) - 1  # b = a + delta_l on the torus
            l = int(sum((d[mu] + 1) * 3 ** mu for mu in range(4)))
            assert np.array_equal(ocrs.coarse_neighbour(C, cc[a], offs[l]), b)
            pa = oblk.block_view(phi, sob, a)  # (nvec, n_b)
            want.append(pa.conj() @ oblk.block_view(w, sob, a))
            got.append(A[a, l, :, k].cpu().numpy())
            scale = max(scale, np.abs(want[-1]).max())
        err = max(np.abs(g - w_).max() for g, w_ in zip(got, want)) / scale
        print(f"column ({b}, {k}): rel err {err:.2e}", flush=True)
        assert err < 1e-12


def test_project_promote_on_sampled_blocks(shape):
    t = shape
    banner(f"project / promote {t['name']}")
    op, h, sob, phi = t["op"], t["h"], t["sob"], t["phi"]
    nr = 2
    psi = synth.gaussian_half_field(t["dims"], t["Ls"], 430, nrhs=nr)
    c = synth.gaussian_coarse(h.Nc, h.nvec, 431, nr)
    phi16 = oprc.round_bf16(phi)
    for prec, tol, P in ((hd.DWF_C128, 1e-12, phi), (hd.DWF_C64, 2e-5, phi), (hd.DWF_BF16, 2e-5, phi16)):
        vprec = hd.DWF_C128 if prec == hd.DWF_C128 else hd.DWF_C64
        src = psi if vprec == hd.DWF_C128 else psi.astype(np.complex64)
        out = h.new_coarse(vprec, nr)
        hd.hdcg_project(h.h, out, op.to_native(src, vprec), prec, nr)
        got = out.cpu().numpy()
        fine = op.new_field(vprec, nr)
        cin = c if vprec == hd.DWF_C128 else c.astype(np.complex64)
        hd.hdcg_promote(h.h, fine, torch.from_numpy(cin).to("cuda"), prec, nr)
        fc = op.to_canonical(fine, vprec, nr)
        for b in t["blocks"]:
            pb = oblk.block_view(P, sob, b)  # (nvec, n_b)
            want_c = np.einsum("ji,ri->rj", pb.conj(), oblk.block_view(src.astype(np.complex128), sob, b))
            assert rel_err(got[:, b], want_c) < tol, (prec, b)
            want_f = np.einsum("ji,rj->ri", pb, cin[:, b].astype(np.complex128))
            got_f = fc[:, :, torch.from_numpy(sob[b]).to("cuda")].cpu().numpy().reshape(nr, -1)
            assert rel_err(got_f, want_f) < tol, (prec, b)


def test_project_promote_many_rhs_bf16(shape):
    """The 16-bit-subspace project and promote for 17 right-hand sides (the
    MFMA kernels: one full group of 16 and a ragged group of one; promote
    with two 8-RHS column tiles) against the oracle on the sampled blocks,
    to the complex64 tolerance: the kernels carry the complex64 operand as
    three bf16 terms, exact to 2^-24, so only the summation order differs
    from an FP32 computation."""
    t = shape
    banner(f"project / promote, 17 RHS, bf16 subspace {t['name']}")
    op, h, sob, phi = t["op"], t["h"], t["sob"], t["phi"]
    nr = 17
    psi = synth.gaussian_half_field(t["dims"], t["Ls"], 470, nrhs=nr).astype(np.complex64)
    c = synth.gaussian_coarse(h.Nc, h.nvec, 471, nr).astype(np.complex64)
    phi16 = oprc.round_bf16(phi)
    out = h.new_coarse(hd.DWF_C64, nr)
    hd.hdcg_project(h.h, out, op.to_native(psi, hd.DWF_C64), hd.DWF_BF16, nr)
    got = out.cpu().numpy()
    fine = op.new_field(hd.DWF_C64, nr)
    hd.hdcg_promote(h.h, fine, torch.from_numpy(c).to("cuda"), hd.DWF_BF16, nr)
    fc = op.to_canonical(fine, hd.DWF_C64, nr)
    for b in t["blocks"]:
        pb = oblk.block_view(phi16, sob, b)  # (nvec, n_b)
        want_c = np.einsum("ji,ri->rj", pb.conj(), oblk.block_view(psi.astype(np.complex128), sob, b))
        err_c = rel_err(got[:, b], want_c)
        want_f = np.einsum("ji,rj->ri", pb, c[:, b].astype(np.complex128))
        got_f = fc[:, :, torch.from_numpy(sob[b]).to("cuda")].cpu().numpy().reshape(nr, -1)
        err_f = rel_err(got_f, want_f)
        print(f"block {b}: project {err_c:.2e}, promote {err_f:.2e}", flush=True)
        assert err_c < 2e-5 and err_f < 2e-5, b


def test_coarse_kernels_on_seeded_operator(shape):
    """coarse_apply (complex128, complex64 on the VALU for one right-hand side
    and on the FP32 MFMA for several, bf16 and fp16 MFMA; 1, 3, 9, 16 and 17
    right-hand sides: one and two N tiles, full and partial, and a second
    launch row of 16) on a seeded Hermitian positive-definite stencil
    operator imported into the handle, against the oracle's mat-vec."""
    t = shape
    banner(f"coarse apply on seeded operator {t['name']}")
    h = t["h"]
    A = synth.coarse_stencil_operator(t["C"], h.nvec, 440)
    hd.hdcg_import_coarse(h.h, torch.from_numpy(A).to("cuda"))
    assert rel_err(h.coarse_matrix().cpu().numpy(), A) == 0.0
    for nr in (1, 3, 9, 16, 17):
        c = synth.gaussian_coarse(h.Nc, h.nvec, 441 + nr, nr)
        want = ocrs.apply(A, c, t["C"])
        for prec, tol in ((hd.DWF_C128, 1e-12), (hd.DWF_C64, 2e-5), (hd.DWF_BF16, 1e-2), (hd.DWF_F16, 2e-3)):
            vt = torch.complex128 if prec == hd.DWF_C128 else torch.complex64
            inp = torch.from_numpy(c).to("cuda", vt).contiguous()
            out = torch.zeros_like(inp)
            hd.coarse_apply(h.h, out, inp, prec, nr)
            err = rel_err(out.cpu().numpy(), want)
            print(f"nrhs {nr} prec {prec}: rel err {err:.2e}", flush=True)
            assert err < tol, (nr, prec)


def test_mfma_tile_candidates_and_autotuner(shape):
    """Every tile the autotuner chooses from (16x16x16 and gfx950 16x16x32
    MFMA forms, 4 or 8 waves, 2 or 4 K steps in flight) gives the oracle's
    mat-vec to the 16-bit tolerance for 1, 3 and 16 right-hand sides; the
    autotuner's pick is one of them and its timings are reported."""
    t = shape
    banner(f"MFMA tile candidates {t['name']}")
    h = t["h"]
    A = synth.coarse_stencil_operator(t["C"], h.nvec, 445)
    hd.hdcg_import_coarse(h.h, torch.from_numpy(A).to("cuda"))
    for nr in (1, 3, 16):
        c = synth.gaussian_coarse(h.Nc, h.nvec, 446 + nr, nr)
        want = ocrs.apply(A, c, t["C"])
        inp = torch.from_numpy(c).to("cuda", torch.complex64).contiguous()
        for prec, tol in ((hd.DWF_BF16, 1e-2), (hd.DWF_F16, 2e-3)):
            for cand in range(6):
                h.set_params(mfma_tile=cand)
                out = torch.zeros_like(inp)
                hd.coarse_apply(h.h, out, inp, prec, nr)
                err = rel_err(out.cpu().numpy(), want)
                assert err < tol, (nr, prec, cand, err)
            h.set_params(mfma_tile=-1)
            tile, ms = hd.hdcg_mfma_tile(h.h, prec, nr)
            assert tile[0] in (16, 32) and tile[1] in (4, 8) and tile[2] in (2, 4)
            assert len(ms) == 6 and min(m for m in ms if m >= 0) > 0
            if h.nvec % 8 == 0:
                assert all(m > 0 for m in ms[3:5]) or nr == 1  # the 16x16x32 candidates were timed
            print(f"nrhs {nr} prec {prec}: tile {tile}, ms {[round(m, 4) for m in ms]}", flush=True)


def test_truncated_operator_16bit_on_seeded_operator(shape):
    """Q_trunc + 0.3 (Sec. V.B) in complex64 and in the 16-bit MFMA storage
    (m1_prec bf16 / fp16: nine matrices per site, per-matrix scales) on 1, 3
    and 16 right-hand sides against the oracle's truncated operator
    (complex64 2e-5, bf16 1e-2, fp16 2e-3, as the 81-point mat-vec); the
    Chebyshev polynomial of order 6 on [0.5, Gershgorin bound] and 6
    iterations of the truncated CG with each storage against the oracle's
    (complex64 1e-4, bf16 3e-2, fp16 5e-3)."""
    from oracle import ldop as oldop

    t = shape
    banner(f"16-bit truncated operator {t['name']}")
    h = t["h"]
    A = synth.coarse_stencil_operator(t["C"], h.nvec, 450)
    hd.hdcg_import_coarse(h.h, torch.from_numpy(A).to("cuda"))
    shift = 0.3
    T = oldop.truncate(A, shift)
    # an upper bound of the spectrum of the Hermitian T: the largest absolute row sum
    rows = np.zeros((h.Nc, h.nvec))
    for l in oldop.one_hop_points():
        rows += np.abs(T[:, l]).sum(axis=2)
    hi = float(rows.max())
    tols = {hd.DWF_C64: (2e-5, 1e-4), hd.DWF_BF16: (1e-2, 3e-2), hd.DWF_F16: (2e-3, 5e-3)}
    try:
        for mp, (tol_mv, tol_pre) in tols.items():
            h.set_params(m1_prec=mp, m1_shift=shift, m1_lo=0.5, m1_hi=hi, m1_order=6)
            for nr in (1, 3, 16):
                c = synth.gaussian_coarse(h.Nc, h.nvec, 451 + nr, nr)
                want = ocrs.apply(T, c, t["C"])
                inp = torch.from_numpy(c).to("cuda", torch.complex64).contiguous()
                out = torch.zeros_like(inp)
                hd.hdcg_trunc_apply(h.h, out, inp, hd.DWF_C64, nr)
                err = rel_err(out.cpu().numpy(), want)
                print(f"Q_trunc m1_prec {mp} nrhs {nr}: rel err {err:.2e}", flush=True)
                assert err < tol_mv, (mp, nr)
            r = synth.gaussian_coarse(h.Nc, h.nvec, 460, 3)
            inp = torch.from_numpy(r).to("cuda", torch.complex64).contiguous()
            want = np.array([oldop.chebyshev_inverse(lambda u: ocrs.apply(T, u, t["C"]), ri, 0.5, hi, 6) for ri in r])
            y = torch.zeros_like(inp)
            hd.hdcg_chebyshev(h.h, y, inp, hd.DWF_C64, 3)
            err = rel_err(y.cpu().numpy(), want)
            print(f"Chebyshev order 6, m1_prec {mp}: rel err {err:.2e}", flush=True)
            assert err < tol_pre, mp
            want = np.array([oldop.trunc_cg(T, t["C"], ri, 6) for ri in r])
            y = torch.zeros_like(inp)
            hd.hdcg_trunc_cg(h.h, y, inp, hd.DWF_C64, 3)
            err = rel_err(y.cpu().numpy(), want)
            print(f"truncated CG 6 iterations, m1_prec {mp}: rel err {err:.2e}", flush=True)
            assert err < tol_pre, mp
    finally:
        h.set_params(m1_prec=hd.DWF_C64, m1_shift=0.0, m1_hi=0.0, m1_order=16)


def test_coarse_solves_on_seeded_operator(shape):
    """Coarse CG (complex64 VALU and bf16 / fp16 MFMA storage) on a seeded
    operator against a dense solve: one right-hand side, and 5 and 16 at once
    in the batched persistent kernel, whose per-right-hand-side masks give
    uneven iteration counts (a zero source takes none).  The 16-bit runs use a better-conditioned operator
    (mass 1, condition ~ 17) so that the rounding of A (relative 2^-9 for
    bf16) stays below the solve tolerance in the solution."""
    t = shape
    banner(f"coarse solves on seeded operator {t['name']}")
    h, C = t["h"], t["C"]
    for mass, precs, tol, check in ((0.1, (hd.DWF_C64,), 1e-5, 2e-3), (1.0, (hd.DWF_BF16, hd.DWF_F16), 1e-3, 3e-2)):
        A = synth.coarse_stencil_operator(C, h.nvec, 450, mass=mass)
        hd.hdcg_import_coarse(h.h, torch.from_numpy(A).to("cuda"))
        D = ocrs.to_dense(A, C)
        for nr in (1, 5, 16):
            b = synth.gaussian_coarse(h.Nc, h.nvec, 451 + nr, nr)
            if nr == 16:
                # right-hand sides of different spectral content, so that their
                # solves need different iteration counts: zero, a rescaled one,
                # D^j v (high modes weighted up), a point source
                b[3] = 0.0
                b[7] *= 1e-3
                for j, r in enumerate((10, 11, 12, 13), start=1):
                    v = b[r].ravel()
                    for _ in range(j):
                        v = D @ v
                    b[r] = v.reshape(b[r].shape)
                b[14] = 0.0
                b[14, 5, 2] = 1.0
            xw = np.linalg.solve(D, b.reshape(nr, -1).T).T
            for prec in precs:
                x = torch.zeros((nr, h.Nc, h.nvec), dtype=torch.complex64, device="cuda")
                rc, it = hd.hdcg_coarse_solve(h.h, x, torch.from_numpy(b).to("cuda", torch.complex64), prec, nr, tol,
                                              5000)
                assert rc == 0 and it > 0
                its = hd.hdcg_coarse_iterations(h.h, nr)
                assert max(its) == it, (its, it)  # one persistent solve: it runs until the last converges
                if nr == 16:
                    assert its[3] == 0 and len(set(its)) > 2, its  # the zero source, uneven counts
                xg = x.cpu().numpy().reshape(nr, -1).astype(np.complex128)
                for r in range(nr):
                    nb = np.linalg.norm(b[r])
                    if nb == 0.0:
                        assert np.abs(xg[r]).max() == 0.0
                        continue
                    res = np.linalg.norm(b[r].ravel() - D @ xg[r]) / nb
                    err = np.linalg.norm(xg[r] - xw[r]) / np.linalg.norm(xw[r])
                    assert res < check and err < check * 20, (mass, prec, nr, r, res, err)
                print(f"mass {mass} prec {prec} nrhs {nr}: {it} iterations, per RHS {its}", flush=True)


# ------------------------------------------------------------ end to end --
def _solve_and_check(op, h, ref, dims, Ls, seed, nr=1, tol=1e-8):
    b = synth.gaussian_half_field(dims, Ls, seed, nrhs=nr if nr > 1 else None)
    x = op.new_field(nrhs=nr)
    rc, st = hd.hdcg_solve(h.h, x, op.to_native(b), nr, tol)
    print(st, flush=True)
    assert rc == 0 and st["converged"] == 1
    xc = op.to_canonical(x, nrhs=nr).cpu().numpy()
    for r in range(nr):
        br = b[r] if nr > 1 else b
        xr = xc[r] if nr > 1 else xc
        res = br - ref.H(xr)
        rel = np.sqrt(np.vdot(res, res).real / np.vdot(br, br).real)
        print(f"rhs {r}: oracle true residual {rel:.3e}", flush=True)
        assert rel <= tol * (1 + 1e-3)
    return st


@pytest.mark.parametrize("flexible", [1, 0])
def test_mini_hdcg_solve_checked_by_oracle(flexible):
    """12^3x24 x Ls8, m 0.01, eps 0.5, 4^4 blocks (coarse 3^3x6), Nvec 8, two
    inverse-iteration steps, n_irs 7, lambda 1, coarse tolerance 0.04; the
    flexible and the standard search-direction updates of Fig.
    "pcg_general"."""
    dims, Ls, nvec = (12, 12, 12, 24), 8, 8
    banner(f"mini HDCG 12^3x24 x Ls8 Nvec8 flexible={flexible}")
    U = synth.gauge_field(dims, 0.5, 460)
    raw = synth.gaussian_half_field(dims, Ls, 461, nrhs=nvec)
    op = hd.FineOperator(U, dims, Ls, 1.8, 0.01)
    h = hd.HDCG(op, BLOCK, raw, n_ii=2, tol_ii=1e-3, flexible=flexible)
    ref = DWF(U, dims, Ls, 1.8, 0.01)
    _solve_and_check(op, h, ref, dims, Ls, 462, nr=1)
    _solve_and_check(op, h, ref, dims, Ls, 463, nr=3)
    h.close()
    op.close()


def test_config3_hdcg_solve_checked_by_oracle():
    """The 16^3x32 x Ls16, m = 0.003 workload (Nvec 24, three inverse-
    iteration steps to 1e-3): the GPU's solution has an FP64 true residual
    of at most 1e-8 under the oracle's H."""
    w = WORKLOADS[3]
    banner("config 3 HDCG solve, oracle residual")
    U = synth.gauge_field(w.dims, w.eps, w.gauge_seed)
    V = np.concatenate([synth.gaussian_half_field(w.dims, w.Ls, w.subspace_seed(k), nrhs=1) for k in range(w.nvec)])
    op = hd.FineOperator(U, w.dims, w.Ls, w.M5, w.mass)
    h = hd.HDCG(op, w.block, V, n_ii=3, tol_ii=1e-3, maxiter_ii=500)
    del V
    ref = DWF(U, w.dims, w.Ls, w.M5, w.mass)
    _solve_and_check(op, h, ref, w.dims, w.Ls, w.source_seed(0))
    h.close()
    op.close()


_LS_JOB = None


def _oracle_H_block(b):
    ref, phi, sob = _LS_JOB
    v = np.zeros(phi.shape, dtype=np.complex128)
    v[:, sob[b]] = phi[:, sob[b]]
    return ref.H(v)


def test_inverse_iteration_step_pinned_by_oracle_H():
    """One inverse-iteration step (Sec. II: phi' = (H + lambda_ii)^-1 phi,
    normalised; here lambda_ii = 0) with Nvec = 1: the block
    orthonormalisation then only rescales phi' block by block, so phi' =
    sum_b n_b Phi_b for unknown n_b, and H phi' must reproduce the starting
    vector up to one overall factor.  The least-squares residual
    min_n |sum_b n_b H Phi_b - v| / |v|, with H the oracle's, is therefore at
    most the step's solve tolerance (1e-6, complex64 CG) plus complex64
    rounding; a step that applied H, or no step, leaves a residual of order
    one since the 81 vectors H Phi_b span only 81 directions."""
    global _LS_JOB
    dims, Ls = (12, 12, 12, 12), 2
    banner("inverse iteration step against the oracle's H")
    U = synth.gauge_field(dims, 0.5, 470)
    v = synth.gaussian_half_field(dims, Ls, 471, nrhs=1)
    op = hd.FineOperator(U, dims, Ls, 1.8, 0.05)
    h = hd.HDCG(op, BLOCK, v, n_ii=1, tol_ii=1e-6, maxiter_ii=5000)
    Phi = h.subspace().cpu().numpy()[0]
    h.close()
    op.close()
    ref = DWF(U, dims, Ls, 1.8, 0.05)
    _, _, sob = oblk.block_map(dims, BLOCK)
    _LS_JOB = (ref, Phi, sob)
    try:
        with mp.get_context("fork").Pool(min(16, mp.cpu_count())) as pool:
            cols = pool.map(_oracle_H_block, range(sob.shape[0]))
    finally:
        _LS_JOB = None
    G = np.stack([c.ravel() for c in cols], axis=1)
    n, *_ = np.linalg.lstsq(G, v[0].ravel(), rcond=None)
    res = np.linalg.norm(G @ n - v[0].ravel()) / np.linalg.norm(v[0])
    print(f"least-squares residual {res:.2e}", flush=True)
    assert res < 1e-5
    # the step changed the vector: Phi is not the starting vector rescaled per block
    overlap = max(abs(np.vdot(Phi[:, sob[b]], v[0][:, sob[b]])) / np.linalg.norm(v[0][:, sob[b]])
                  for b in range(sob.shape[0]))
    assert overlap < 0.99

"""The no-allocation coarse solve (hdcg_coarse_solve_noalloc) against the
allocating entry point (hdcg_coarse_solve) on the same handles and inputs,
on two calls in a row, the second with a smaller input (a handle with fewer
coarse sites and fewer right-hand sides), complex64 and bf16 storage.  Both
run the same persistent kernel with the same launch shape and deterministic
reductions, so the solutions agree bit for bit; they are also held to the
complex64 solve tolerance against the oracle's dense solve of the coarse
operator the oracle builds itself."""
import numpy as np
import pytest

import synth
from oracle import blocks as oblk
from oracle import coarse as ocrs
from oracle.dwf import DWF
from tests.gpu_util import banner

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1402_2585_amd as hd  # noqa: E402

CASES = [
    # dims, Ls, nvec, nrhs, seed: the second call has fewer coarse sites and right-hand sides
    ((16, 12, 12, 12), 2, 8, 5, 490),
    ((12, 12, 12, 12), 2, 4, 2, 495),
]


def _handle(dims, Ls, nvec, seed):
    U = synth.gauge_field(dims, 0.5, seed)
    raw = synth.gaussian_half_field(dims, Ls, seed + 1, nrhs=nvec)
    op = hd.FineOperator(U, dims, Ls, 1.8, 0.05)
    h = hd.HDCG(op, (4, 4, 4, 4), raw)
    ref = DWF(U, dims, Ls, 1.8, 0.05)
    _, _, sob = oblk.block_map(dims, (4, 4, 4, 4))
    C = oblk.coarse_dims(dims, (4, 4, 4, 4))
    A = ocrs.build_brute(ref, oblk.orthonormalise(raw, sob), sob, C)
    return op, h, ocrs.to_dense(A, C)


def test_noalloc_coarse_solve_matches_allocating_entry_point():
    for dims, Ls, nvec, nr, seed in CASES:
        banner(f"no-allocation coarse solve {dims} Ls{Ls} nvec {nvec} nrhs {nr}")
        op, h, D = _handle(dims, Ls, nvec, seed)
        b = synth.gaussian_coarse(h.Nc, nvec, seed + 2, nr)
        b[nr - 1] *= 1e-2
        bt = torch.from_numpy(b).to("cuda", torch.complex64)
        # the 16-bit storage is built by a call that may allocate
        hd.coarse_apply(h.h, h.new_coarse(hd.DWF_C64, nr), bt, hd.DWF_BF16, nr)
        for prec, tol in ((hd.DWF_C64, 1e-5), (hd.DWF_BF16, 1e-3)):
            x_ref = torch.zeros_like(bt)
            rc, it = hd.hdcg_coarse_solve(h.h, x_ref, bt, prec, nr, tol, 5000)
            assert rc == 0
            x = torch.full_like(bt, float("nan"))  # every entry must be written
            rc2, it2 = hd.hdcg_coarse_solve_noalloc(h.h, x, bt, prec, nr, tol, 5000)
            assert rc2 == 0 and it2 == it, (it, it2)
            xa, xr = x.cpu().numpy(), x_ref.cpu().numpy()
            assert np.array_equal(xa, xr), np.abs(xa - xr).max()
            for r in range(nr):
                res = np.linalg.norm(b[r].ravel() - D @ xa[r].ravel().astype(complex)) / np.linalg.norm(b[r])
                assert res < (3e-4 if prec == hd.DWF_C64 else 2e-2), (prec, r, res)
            print(f"prec {prec}: {it} iterations, equal to the allocating call", flush=True)
        # argument checks happen before any device work
        with pytest.raises(hd.HdcgError):
            hd.hdcg_coarse_solve_noalloc(h.h, x, bt, hd.DWF_C64, 17, 1e-5, 100)
        with pytest.raises(hd.HdcgError):
            hd.hdcg_coarse_solve_noalloc(h.h, x, bt, hd.DWF_C128, nr, 1e-5, 100)
        with pytest.raises(hd.HdcgError):  # fp16 storage not built on this handle
            hd.hdcg_coarse_solve_noalloc(h.h, x, bt, hd.DWF_F16, nr, 1e-5, 100)
        h.close()
        op.close()

"""GPU tests of the batched solve: up to 16 right-hand sides in one group
(every operator pass and one persistent coarse solve shared by all of
them), the preconditioner replayed from a captured HIP graph, the phase
times of Fig. "pie" and the per-right-hand-side statistics of hdcg_stats.

A graph replay must give exactly what the same work launched one kernel at a
time gives (the kernels and their order are the same and every reduction is
deterministic), so the solution with the graph is compared bit for bit with
the one without, on a solve whose inner iterations replay the graph many
times with the program's own eager work and host synchronisations in
between; every solution is also checked with the oracle's H.
"""
import numpy as np
import pytest

import synth
from oracle.dwf import DWF
from tests.gpu_util import banner

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1402_2585_amd as hd  # noqa: E402

DIMS, LS, BLOCK, NVEC = (12, 12, 12, 12), 4, (4, 4, 4, 4), 8


@pytest.fixture(scope="module")
def setup():
    banner("batch / graph setup 12^4 x Ls4, Nvec 8")
    U = synth.gauge_field(DIMS, 0.5, 480)
    raw = synth.gaussian_half_field(DIMS, LS, 481, nrhs=NVEC)
    op = hd.FineOperator(U, DIMS, LS, 1.8, 0.01)
    h = hd.HDCG(op, BLOCK, raw, n_ii=1, tol_ii=1e-3, coarse_prec=hd.DWF_BF16)
    ref = DWF(U, DIMS, LS, 1.8, 0.01)
    yield op, h, ref
    h.close()
    op.close()


def _oracle_residuals(op, ref, x, b, nr):
    xc = op.to_canonical(x, nrhs=nr).cpu().numpy().reshape((nr,) + b.shape[-4:])
    out = []
    for r in range(nr):
        res = b[r] - ref.H(xc[r])
        out.append(float(np.sqrt(np.vdot(res, res).real / max(np.vdot(b[r], b[r]).real, 1e-300))))
    return out


@pytest.mark.parametrize("cprec", [hd.DWF_C64, hd.DWF_BF16])
def test_graph_replay_equals_eager(setup, cprec):
    op, h, ref = setup
    banner(f"graph replay vs eager, coarse_prec {cprec}")
    nr = 3
    b = synth.gaussian_half_field(DIMS, LS, 482, nrhs=nr)
    bn = op.to_native(b)
    xs, sts = {}, {}
    for graph in (1, 0):
        h.set_params(graph=graph, coarse_prec=cprec, coarse_persistent=1)
        x = op.new_field(nrhs=nr)
        rc, st = hd.hdcg_solve(h.h, x, bn, nr, 1e-8)
        assert rc == 0 and st["converged"] == 1
        xs[graph], sts[graph] = x.cpu().numpy(), st
        print(graph, {k: st[k] for k in ("inner_iterations", "coarse_iterations", "graph_replays")}, flush=True)
    assert sts[1]["graph_replays"] > 3 and sts[0]["graph_replays"] == 0
    assert np.array_equal(xs[1], xs[0])  # bit for bit
    for k in ("outer_iterations", "inner_iterations", "coarse_solves", "coarse_iterations"):
        assert sts[1][k] == sts[0][k], k
    assert sts[1]["coarse_iterations_rhs"] == sts[0]["coarse_iterations_rhs"]
    for rel in _oracle_residuals(op, ref, torch.from_numpy(xs[1]).to("cuda"), b, nr):
        assert rel <= 1e-8 * (1 + 1e-3)
    h.set_params(graph=1, coarse_prec=hd.DWF_C64)


def test_batch_of_16_with_zero_source_and_stats(setup):
    """16 right-hand sides in one group (one of them zero): every one reaches
    1e-8 under the oracle's H, the per-right-hand-side statistics are filled,
    and the phase times add up to at most the solve time."""
    op, h, ref = setup
    banner("16 right-hand sides in one batch, phase timing")
    nr = 16
    b = synth.gaussian_half_field(DIMS, LS, 483, nrhs=nr)
    b[5] = 0.0
    h.set_params(phase_timing=1)
    x = op.new_field(nrhs=nr)
    rc, st = hd.hdcg_solve(h.h, x, op.to_native(b), nr, 1e-8)
    h.set_params(phase_timing=0)
    print({k: v for k, v in st.items() if not k.endswith("_rhs")}, flush=True)
    assert rc == 0 and st["converged"] == 1 and st["group_size"] == 16 and st["nrhs"] == 16
    assert len(st["coarse_iterations_rhs"]) == 16 and len(st["true_residual_rhs"]) == 16
    assert st["true_residual_rhs"][5] == 0.0
    assert max(st["true_residual_rhs"]) == st["true_residual"] <= 1e-8
    assert st["coarse_iterations_rhs"][5] == 0 and min(st["coarse_iterations_rhs"][:5]) > 0
    phases = [st[k] for k in ("t_fine_dp", "t_fine_sp", "t_coarse", "t_project_promote", "t_linalg", "t_convert")]
    assert all(t > 0 for t in phases) and sum(phases) <= st["seconds"]
    assert st["graph_replays"] == 0  # timing replaces the graph
    xc = op.to_canonical(x, nrhs=nr).cpu().numpy()
    assert np.abs(xc[5]).max() == 0.0
    for r in (0, 15):
        res = b[r] - ref.H(xc[r])
        assert np.sqrt(np.vdot(res, res).real / np.vdot(b[r], b[r]).real) <= 1e-8 * (1 + 1e-3)


def test_setup_without_vectors_draws_philox_starting_vectors():
    """hdcg_setup with no vectors draws them on the device from the seed
    (Philox4x32-10, Box-Muller); synth.philox_subspace draws the same numbers
    on the host from the generator's published definition, so the
    orthonormalised subspace equals the oracle's orthonormalisation of those
    (1e-12), and a solve on it converges."""
    from oracle import blocks as oblk

    dims, Ls, nvec, seed = (12, 12, 12, 12), 2, 4, 77
    banner("hdcg_setup with vectors drawn on the device")
    U = synth.gauge_field(dims, 0.5, 490)
    op = hd.FineOperator(U, dims, Ls, 1.8, 0.05)
    h = hd.HDCG(op, BLOCK, None, nvec=nvec, seed=seed)
    raw = synth.philox_subspace(dims, Ls, nvec, seed)
    _, _, sob = oblk.block_map(dims, BLOCK)
    want = oblk.orthonormalise(raw, sob)
    got = h.subspace().cpu().numpy()
    err = np.abs(got - want).max() / np.abs(want).max()
    print(f"subspace from the device generator: rel err {err:.2e}", flush=True)
    assert err < 1e-12
    h2 = hd.HDCG(op, BLOCK, None, nvec=nvec, seed=seed + 1)
    assert np.abs(h2.subspace().cpu().numpy() - got).max() > 0.5 * np.abs(got).max()  # another seed, other vectors
    h2.close()
    ref = DWF(U, dims, Ls, 1.8, 0.05)
    b = synth.gaussian_half_field(dims, Ls, 491)
    x = op.new_field()
    rc, st = hd.hdcg_solve(h.h, x, op.to_native(b), 1, 1e-8)
    assert rc == 0
    r = b - ref.H(op.to_canonical(x).cpu().numpy())
    assert np.sqrt(np.vdot(r, r).real / np.vdot(b, b).real) <= 1e-8 * (1 + 1e-3)
    h.close()
    op.close()

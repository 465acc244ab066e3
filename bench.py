"""Benchmark: M_pc^+ M_pc GB/s on one MI355X (16^4 x Ls16 domain-wall
operator, FP64 complex), with the roofline of the hop kernel and the CPU
oracle timed on a bounded sample; plus HDCG against plain FP64 CG time to a
1e-8 residual on the 16^3x32 x Ls16 workload (skip with --no-hdcg) and on
the 24^3x48 x Ls16 workload with one and with 16 right-hand sides (skip
with --no-big).

Prints ONE JSON line.  Inputs are seeded synthetic SU(3) gauge fields and
Gaussian sources already resident in HBM when the timed region starts.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
_T0 = time.perf_counter()


def log(msg):
    """Progress on stderr (stdout carries only the JSON line)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes_H(dims, Ls, nrhs, cbytes, gbytes=None):
    """Bytes one application of M_pc^+ M_pc must move: four hop stages, each
    reading its input half-field and writing its output (8 transfers), two
    centre re-reads (the M_5 terms of stages 2 and 4), one full gauge read per
    stage (V sites x 4 links x 9 complex, shared by all right-hand sides).
    cbytes / gbytes: bytes per complex of the fields / the links (16-bit
    fields keep complex64 links)."""
    X, Y, Z, T = dims
    V = X * Y * Z * T
    half = V // 2 * Ls * 12
    return 10 * half * nrhs * cbytes + 4 * V * 36 * (cbytes if gbytes is None else gbytes)


def flops_H(dims, Ls, nrhs):
    """5616 flops per odd 5D site (4 Wilson hops of 1320, two M_5^-1 at 96,
    two M_5 at 48, two subtractions at 24)."""
    X, Y, Z, T = dims
    return 5616 * (X * Y * Z * T // 2) * Ls * nrhs


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("fine_op.hip", "fine_op.h", "common.h"):
        h.update(open(os.path.join(ROOT, "paper_1402_2585_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(prec_tag):
    """HBM bytes per hop launch from the committed rocprofv3 --pmc summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or None
    when the kernel sources changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", "hop_kernel_16^4xLs16_pmc.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("source_hash") != kernel_source_hash():
        return None
    v = d.get(prec_tag)
    return None if v is None else v.get("bytes_per_launch")


def time_H(op, hd, prec, steps, warmup, nrhs=1, reps=1):
    """Median over `reps` repetitions of `steps` ping-pong applications of H,
    each timed with HIP events on torch's current stream (where the library
    launches); returns ms per application."""
    import torch

    x = op.new_field(prec, nrhs)
    y = op.new_field(prec, nrhs)
    x.copy_(torch.randn(x.shape, dtype=x.dtype, device="cuda"))
    s = torch.cuda.current_stream()
    for _ in range(warmup):
        hd.mpc_dag_mpc_apply(op.h, y, x, prec, nrhs)
        hd.mpc_dag_mpc_apply(op.h, x, y, prec, nrhs)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        a, b = x, y
        for _ in range(steps):
            hd.mpc_dag_mpc_apply(op.h, b, a, prec, nrhs)  # ping-pong
            a, b = b, a
        e1.record(s)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / steps)
    return sorted(times)[len(times) // 2]


def copy_bandwidth(torch, mib=2048, reps=10):
    """Device-to-device copy of `mib` MiB (read + write bytes per second): the
    measured second denominator of the roofline."""
    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * n * 4 / (ms * 1e-3) / 1e9


def mall_busting(hd, torch, steps=10):
    """H at 32^3 x 64 x Ls16, whose fields (1.6 GB per complex64 half-field)
    do not fit the 256 MB Infinity Cache: GB/s in complex128 and complex64."""
    import synth

    dims, Ls = (32, 32, 32, 64), 16
    U = synth.gauge_field(dims, 0.7, 2201)
    op = hd.FineOperator(U, dims, Ls, 1.8, 0.01)
    out = {"workload": "mpcdagmpc 32^3x64 x Ls16, 1 RHS"}
    for name, prec, cb in (("c128", hd.DWF_C128, 16), ("c64", hd.DWF_C64, 8)):
        ms = time_H(op, hd, prec, steps, 2, reps=3)
        out[name] = {"gbs": round(algorithmic_bytes_H(dims, Ls, 1, cb) / (ms * 1e-3) / 1e9, 1),
                     "ms_per_application": round(ms, 4)}
    op.close()
    return out


def _host_info():
    """CPU model, logical CPUs of the host and CPUs this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "usable_cpus": usable}


_CPU_JOB = None


def _oracle_H_once(seed):
    """One oracle application of H at the bench workload on a source of its
    own, with the BLAS / OpenMP pools of this process held to one thread."""
    from threadpoolctl import threadpool_limits

    import synth

    ref, dims, Ls = _CPU_JOB
    b = synth.gaussian_half_field(dims, Ls, seed)
    with threadpool_limits(limits=1):
        t = time.perf_counter()
        ref.H(b)
        return time.perf_counter() - t


def cpu_baseline(dims, Ls, eps, mass, n_single=2, max_workers=16):
    """The oracle, untouched, on the host (the bounded sample): FP64
    applications of H at the full workload size, first n_single of them one
    after another on one thread, then one per worker process on every usable
    core at once (at most max_workers, the machine's CPU share); returns the
    single-thread seconds per application, the all-core applications per
    second and the worker count."""
    import multiprocessing as mp

    import synth
    from oracle.dwf import DWF

    global _CPU_JOB
    U = synth.gauge_field(dims, eps, 2001)
    _CPU_JOB = (DWF(U, dims, Ls, 1.8, mass), dims, Ls)
    single = sum(_oracle_H_once(2100 + i) for i in range(n_single)) / n_single
    workers = max(1, min(_host_info()["usable_cpus"], max_workers))
    t = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        pool.map(_oracle_H_once, [2200 + i for i in range(workers)], chunksize=1)
    wall = time.perf_counter() - t
    _CPU_JOB = None
    return single, workers / wall, workers, wall


def hdcg_vs_cg(hd, torch, tol=1e-8):
    """The metric's second half on the 16^3x32 x Ls16, m=0.003 workload: plain
    FP64 CG, mixed-precision CG (complex64 CG inside FP64 defect correction)
    and HDCG (Nvec=24, 4^4 blocks, 3 inverse-iteration steps each to
    1e-3, complex64 coarse operator and inner solver, FP64 defect correction)
    from the same seeded source, each to a 1e-8 FP64 true residual, on this
    GPU; then the same HDCG with 16-bit M_IRS fields and with the second
    deflation level of the coarse operator."""
    import numpy as np

    import synth
    from synth.configs import WORKLOADS

    w = WORKLOADS[3]
    U = synth.gauge_field(w.dims, w.eps, w.gauge_seed)
    op = hd.FineOperator(U, w.dims, w.Ls, w.M5, w.mass)
    b = op.to_native(synth.gaussian_half_field(w.dims, w.Ls, w.source_seed(0)))
    tune_hop(hd, op, (1, 8))
    x = op.new_field(zero=True)
    log("16^3x32: FP64 CG")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc_cg, st_cg = hd.cg_solve(op.h, x, b, 1, tol, 50000)
    torch.cuda.synchronize()
    t_cg = time.perf_counter() - t0
    xm = op.new_field(zero=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc_m, st_m = hd.cg_solve_mixed(op.h, xm, b, 1, tol, 1e-5, 50000)
    torch.cuda.synchronize()
    t_mixed = time.perf_counter() - t0
    del xm
    V = np.stack([synth.gaussian_half_field(w.dims, w.Ls, w.subspace_seed(k)) for k in range(w.nvec)])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = hd.HDCG(op, w.block, V, n_ii=3, tol_ii=1e-3, maxiter_ii=500)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    log(f"16^3x32 HDCG setup: {t_setup:.1f} s")
    x2 = op.new_field(zero=True)
    # solved twice from x = 0: the first solve also allocates the workspace
    # (reported as seconds_first_solve), the second is the headline
    t_hc, _ = _timed(torch, lambda: hd.hdcg_solve(h.h, x2, b, 1, tol))
    x2.zero_()
    t_h, (rc_h, st_h) = _timed(torch, lambda: hd.hdcg_solve(h.h, x2, b, 1, tol))
    bb = hd.dwf_norm2(op.h, b, hd.DWF_C128)[0]

    def true_residual(xs):
        # independent FP64 true residual of a solution on the GPU operator
        r = op.H(xs)
        hd.dwf_xpay(op.h, r, b, [-1.0], hd.DWF_C128)  # r = b - H x
        return float(np.sqrt(hd.dwf_norm2(op.h, r, hd.DWF_C128)[0] / bb))

    rel = true_residual(x2)
    # the same solve with M_IRS on 16-bit fields (Sec. VI.E, Table "sloppy")
    h.set_params(irs_prec=hd.DWF_BF16)
    x3 = op.new_field(zero=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc_b, st_b = hd.hdcg_solve(h.h, x3, b, 1, tol)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    rel_b = true_residual(x3)
    # second deflation level of the coarse operator (Sec. V.B): the 24 free
    # global vectors and 128 more after 3 inverse-iteration steps to 1e-7
    n_extra = 128
    noise = torch.from_numpy(synth.gaussian_coarse(h.Nc, w.nvec, w.coarse_seed, n_extra)).to("cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hd.hdcg_ldop_setup(h.h, n_extra, noise, 0.0, 3, 1e-7)
    torch.cuda.synchronize()
    t_ldop = time.perf_counter() - t0
    del noise
    ldop = {"global_vectors": w.nvec + n_extra, "setup_seconds": round(t_ldop, 3)}
    # the last two: the coarse solves by ADEF1 with the Chebyshev inverse of
    # the one-hop truncated operator (Sec. V.B; Table "optimised" uses order
    # 16), interval [0.5, 1.05 x estimated largest eigenvalue]
    # (ldop_m1 = 2: M_IRS(Q_trunc), 8 CG iterations; m1_prec: storage of Q_trunc)
    for name, iprec, pprec, m1, order, m1p in (
            ("c64_mirs", hd.DWF_C64, hd.DWF_C64, 0, 16, hd.DWF_C64),
            ("bf16_mirs", hd.DWF_BF16, hd.DWF_C64, 0, 16, hd.DWF_C64),
            ("bf16_mirs_bf16_subspace", hd.DWF_BF16, hd.DWF_BF16, 0, 16, hd.DWF_C64),
            ("bf16_mirs_bf16_subspace_adef1_cheb16", hd.DWF_BF16, hd.DWF_BF16, 1, 16, hd.DWF_C64),
            ("bf16_mirs_bf16_subspace_adef1_cheb8", hd.DWF_BF16, hd.DWF_BF16, 1, 8, hd.DWF_C64),
            ("bf16_mirs_bf16_subspace_adef1_cheb8_bf16_qtrunc", hd.DWF_BF16, hd.DWF_BF16, 1, 8, hd.DWF_BF16),
            ("bf16_mirs_bf16_subspace_adef1_trunc_cg8", hd.DWF_BF16, hd.DWF_BF16, 2, 8, hd.DWF_C64),
            ("bf16_mirs_bf16_subspace_adef1_trunc_cg8_bf16_qtrunc", hd.DWF_BF16, hd.DWF_BF16, 2, 8, hd.DWF_BF16)):
        h.set_params(irs_prec=iprec, ldop_defl=1, phi_prec=pprec, ldop_m1=m1, m1_order=order, m1_prec=m1p)
        x5 = op.new_field(zero=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc5, st5 = hd.hdcg_solve(h.h, x5, b, 1, tol)
        torch.cuda.synchronize()
        t5 = time.perf_counter() - t0
        log(f"16^3x32 HDCG {name}: {t5:.3f} s")
        ldop[name] = {"seconds": round(t5, 4), "outer": st5["outer_iterations"], "inner": st5["inner_iterations"],
                      "coarse_iterations": st5["coarse_iterations"], "true_residual": true_residual(x5),
                      "status": rc5, "speedup_solve_vs_cg": round(t_cg / t5, 3)}
        del x5
    h.close()
    op.close()
    return {
        "workload": "16^3x32 x Ls16, M5=1.8, m=0.003, eps=0.7, Nvec=24, 4^4 blocks (coarse 4^3x8), "
                    "inverse iteration 3 steps to 1e-3",
        "cg_fp64": {"seconds": round(t_cg, 4), "iterations": st_cg["iterations"], "matmuls": st_cg["matmuls"],
                    "true_residual": st_cg["true_residual"], "status": rc_cg},
        "cg_mixed": {"seconds": round(t_mixed, 4), "iterations_c64": st_m["iterations"],
                     "corrections_fp64": st_m["restarts"], "matmuls": st_m["matmuls"],
                     "true_residual": st_m["true_residual"], "status": rc_m},
        "hdcg": {"seconds": round(t_h, 4), "seconds_first_solve": round(t_hc, 4), "setup_seconds": round(t_setup, 3),
                 "outer": st_h["outer_iterations"], "inner": st_h["inner_iterations"],
                 "coarse_iterations": st_h["coarse_iterations"], "matmuls_fp64": st_h["matmuls_fp64"],
                 "matmuls_fp32": st_h["matmuls_fp32"], "true_residual": rel, "status": rc_h},
        "hdcg_bf16_mirs": {"seconds": round(t_b, 4), "outer": st_b["outer_iterations"],
                           "inner": st_b["inner_iterations"], "coarse_iterations": st_b["coarse_iterations"],
                           "true_residual": rel_b, "status": rc_b,
                           "speedup_vs_c64_mirs": round(t_h / t_b, 3),
                           "speedup_solve_vs_cg": round(t_cg / t_b, 3),
                           "speedup_solve_vs_mixed_cg": round(t_mixed / t_b, 3)},
        "hdcg_ldop_deflation": ldop,
        "speedup_solve": round(t_cg / t_h, 3),
        "speedup_solve_vs_mixed_cg": round(t_mixed / t_h, 3),
        "break_even_rhs": (round(t_setup / (t_cg - t_h), 1) if t_cg > t_h else None),
    }


def tune_hop(hd, op, counts):
    """Run the hop launch-shape autotuner for every field storage and the
    given right-hand-side counts before anything is timed (its trials are a
    one-time cost per operator, as a serving process would pay at start)."""
    for n in counts:
        for prec in (hd.DWF_C128, hd.DWF_C64, hd.DWF_BF16):
            hd.dwf_tune_hop(op.h, prec, n)
    hd.dwf_release_workspace(op.h)


def _timed(torch, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, out


def hdcg_24(hd, torch, tol=1e-8):
    """The 24^3x48 x Ls16, m = 0.001 workloads on one operator and one
    subspace: config 4 (one right-hand side; Nvec = 48, 4^4 blocks, the
    coarse operator in bf16 on MFMA with FP32 accumulation, FP64
    orthonormalisation and true residual) and config 5 (16 right-hand sides
    sharing the subspace, solved as one batch: per iteration one persistent
    coarse-CG launch for all 16 with per-RHS masks, the preconditioner
    replayed from a captured graph, autotuned MFMA tiles), each to a 1e-8
    FP64 true residual, against plain FP64 CG on the same GPU from the same
    sources (config 5: four batches of four) and, for config 4, the
    mixed-precision CG; then both HDCG legs again with the second deflation
    level of the coarse operator.  Each HDCG leg solves twice from x = 0 and reports
    both: the first solve of a batch size also allocates its workspace and
    tunes the MFMA tiles for it; the second is the headline.  The 48
    starting vectors are drawn on the device
    (Philox4x32-10, seed 4500; three inverse-iteration steps, complex64 CG to
    1e-3, at most 100 iterations); M_IRS and the subspace copy inside Q are
    stored in bf16; the FP64 subspace is released after setup (memory for
    the 16-RHS batch).  Residuals are recomputed with the library's FP64 H
    (the parity tests check such solutions against the oracle's H)."""
    import numpy as np

    import synth
    from synth.configs import WORKLOADS

    w4, w5 = WORKLOADS[4], WORKLOADS[5]
    op = hd.FineOperator(synth.gauge_field(w4.dims, w4.eps, w4.gauge_seed), w4.dims, w4.Ls, w4.M5, w4.mass)
    fe = op.Vh * w4.Ls * 12

    def source(seed):
        return torch.from_numpy(synth.gaussian_half_field(w4.dims, w4.Ls, seed)).to("cuda")

    b4 = op.to_native(source(w4.source_seed(0)))
    b5 = op.new_field(nrhs=w5.nrhs)
    for r in range(w5.nrhs):
        b5[r * fe:(r + 1) * fe] = op.to_native(source(w5.source_seed(r)))

    def true_residuals(x, b, nr):
        out = []
        for r in range(nr):
            xr, br = x[r * fe:(r + 1) * fe], b[r * fe:(r + 1) * fe]
            res = op.H(xr)
            hd.dwf_xpay(op.h, res, br, [-1.0], hd.DWF_C128)
            out.append(float(np.sqrt(hd.dwf_norm2(op.h, res, hd.DWF_C128)[0] / hd.dwf_norm2(op.h, br, hd.DWF_C128)[0])))
        return out

    tune_hop(hd, op, (1, w5.nrhs))
    log("24^3x48: sources on the device, hop shapes tuned")
    x = op.new_field(zero=True)
    t_cg4, (rc, st_cg4) = _timed(torch, lambda: hd.cg_solve(op.h, x, b4, 1, tol, 50000))
    log(f"config 4 FP64 CG: {t_cg4:.2f} s")
    x.zero_()
    t_mx4, (rcm, st_mx4) = _timed(torch, lambda: hd.cg_solve_mixed(op.h, x, b4, 1, tol, 1e-5, 50000))
    log(f"config 4 mixed CG: {t_mx4:.2f} s")
    x5 = op.new_field(nrhs=w5.nrhs, zero=True)
    t_cg5, its5, rel_cg5 = 0.0, 0, 0.0
    for r0 in range(0, w5.nrhs, 4):
        xs, bs = x5[r0 * fe:(r0 + 4) * fe], b5[r0 * fe:(r0 + 4) * fe]
        dt, (rc5, st5) = _timed(torch, lambda: hd.cg_solve(op.h, xs, bs, 4, tol, 50000))
        t_cg5 += dt
        log(f"config 5 FP64 CG, right-hand sides {r0}-{r0 + 3}: {dt:.2f} s")
        its5 = max(its5, st5["iterations"])
        rel_cg5 = max(rel_cg5, st5["true_residual"])
    hd.dwf_release_workspace(op.h)
    t_setup, h = _timed(torch, lambda: hd.HDCG(op, w4.block, None, nvec=w4.nvec, seed=4500, n_ii=3, tol_ii=1e-3,
                                               maxiter_ii=100, coarse_prec=hd.DWF_BF16, irs_prec=hd.DWF_BF16,
                                               phi_prec=hd.DWF_BF16, keep_subspace_fp64=0))
    log(f"24^3x48 HDCG setup: {t_setup:.1f} s")
    # each leg solves twice from x = 0: the first solve of a batch size also
    # allocates that size's workspace and runs the MFMA tile autotuner for it
    # (one-time costs per handle); the second is the per-solve cost when a
    # handle serves many batches
    x.zero_()
    t_h4c, _ = _timed(torch, lambda: hd.hdcg_solve(h.h, x, b4, 1, tol))
    x.zero_()
    t_h4, (rch4, st_h4) = _timed(torch, lambda: hd.hdcg_solve(h.h, x, b4, 1, tol))
    log(f"config 4 HDCG solve: {t_h4:.3f} s (first solve {t_h4c:.3f} s)")
    rel4 = true_residuals(x, b4, 1)[0]
    x5.zero_()
    t_h5c, _ = _timed(torch, lambda: hd.hdcg_solve(h.h, x5, b5, w5.nrhs, tol))
    x5.zero_()
    t_h5, (rch5, st_h5) = _timed(torch, lambda: hd.hdcg_solve(h.h, x5, b5, w5.nrhs, tol))
    log(f"config 5 HDCG solve (16 RHS): {t_h5:.3f} s (first solve {t_h5c:.3f} s)")
    rel5 = true_residuals(x5, b5, w5.nrhs)
    tile1, _ = hd.hdcg_mfma_tile(h.h, hd.DWF_BF16, 1)
    tile16, _ = hd.hdcg_mfma_tile(h.h, hd.DWF_BF16, 16)
    # second deflation level of the coarse operator (Sec. V.B): the 48 free
    # global vectors and 128 more from three shifted inverse-iteration steps
    # (complex128 coarse CG to 1e-7, groups of 16) on seeded coarse noise;
    # every coarse solve is then deflated CG.  Both legs again, twice each.
    n_extra = 128
    noise = torch.from_numpy(synth.gaussian_coarse(h.Nc, w4.nvec, w4.coarse_seed, n_extra)).to("cuda")
    t_ldop, _ = _timed(torch, lambda: hd.hdcg_ldop_setup(h.h, n_extra, noise, 0.0, 3, 1e-7))
    del noise
    log(f"24^3x48 second deflation level: {t_ldop:.1f} s")
    x.zero_()
    t_l4c, _ = _timed(torch, lambda: hd.hdcg_solve(h.h, x, b4, 1, tol))
    x.zero_()
    t_l4, (rcl4, st_l4) = _timed(torch, lambda: hd.hdcg_solve(h.h, x, b4, 1, tol))
    log(f"config 4 HDCG solve with the second level: {t_l4:.3f} s (first solve {t_l4c:.3f} s)")
    rell4 = true_residuals(x, b4, 1)[0]
    x5.zero_()
    t_l5c, _ = _timed(torch, lambda: hd.hdcg_solve(h.h, x5, b5, w5.nrhs, tol))
    x5.zero_()
    t_l5, (rcl5, st_l5) = _timed(torch, lambda: hd.hdcg_solve(h.h, x5, b5, w5.nrhs, tol))
    log(f"config 5 HDCG solve (16 RHS) with the second level: {t_l5:.3f} s (first solve {t_l5c:.3f} s)")
    rell5 = true_residuals(x5, b5, w5.nrhs)
    h.close()
    op.close()

    def hstats(st):
        return {k: st[k] for k in ("outer_iterations", "inner_iterations", "coarse_solves", "coarse_iterations",
                                   "matmuls_fp64", "matmuls_fp32", "matmuls_bf16", "group_size", "graph_replays")}

    return {
        "workload": "24^3x48 x Ls16, M5=1.8, m=0.001, eps=0.7, Nvec=48, 4^4 blocks (coarse 6^3x12), inverse "
                    "iteration 3 steps to 1e-3 (at most 100 its), bf16 MFMA coarse operator, bf16 M_IRS fields "
                    "and subspace in Q",
        "setup_seconds": round(t_setup, 2),
        "mfma_tiles": {"nrhs_1": tile1, "nrhs_16": tile16},
        "config4": {
            "cg_fp64": {"seconds": round(t_cg4, 3), "iterations": st_cg4["iterations"],
                        "true_residual": st_cg4["true_residual"], "status": rc},
            "cg_mixed": {"seconds": round(t_mx4, 3), "iterations_c64": st_mx4["iterations"],
                         "true_residual": st_mx4["true_residual"], "status": rcm},
            "hdcg": dict(seconds=round(t_h4, 3), seconds_first_solve=round(t_h4c, 3), true_residual=rel4,
                         status=rch4, **hstats(st_h4)),
            "speedup_solve_vs_cg": round(t_cg4 / t_h4, 3),
            "speedup_solve_vs_mixed_cg": round(t_mx4 / t_h4, 3),
            "hdcg_second_level": dict(seconds=round(t_l4, 3), seconds_first_solve=round(t_l4c, 3),
                                      true_residual=rell4, status=rcl4, speedup_solve_vs_cg=round(t_cg4 / t_l4, 3),
                                      speedup_solve_vs_mixed_cg=round(t_mx4 / t_l4, 3), **hstats(st_l4)),
        },
        "config5": {
            "nrhs": w5.nrhs,
            "cg_fp64": {"seconds": round(t_cg5, 3), "max_iterations": its5, "true_residual": rel_cg5},
            "hdcg": dict(seconds=round(t_h5, 3), seconds_first_solve=round(t_h5c, 3), true_residual_max=max(rel5),
                         status=rch5,
                         coarse_iterations_rhs=st_h5["coarse_iterations_rhs"], **hstats(st_h5)),
            "speedup_solve_vs_cg": round(t_cg5 / t_h5, 3),
            "break_even_rhs": (round(t_setup / (t_cg5 - t_h5) * w5.nrhs, 1) if t_cg5 > t_h5 else None),
            "hdcg_second_level": dict(seconds=round(t_l5, 3), seconds_first_solve=round(t_l5c, 3),
                                      true_residual_max=max(rell5), status=rcl5,
                                      coarse_iterations_rhs=st_l5["coarse_iterations_rhs"],
                                      speedup_solve_vs_cg=round(t_cg5 / t_l5, 3),
                                      break_even_rhs=(round((t_setup + t_ldop) / (t_cg5 - t_l5) * w5.nrhs, 1)
                                                      if t_cg5 > t_l5 else None),
                                      **hstats(st_l5)),
        },
        "second_level": {"global_vectors": w4.nvec + n_extra, "setup_seconds": round(t_ldop, 2)},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-hdcg", action="store_true", help="skip HDCG vs CG at 16^3x32xLs16")
    ap.add_argument("--no-extra", action="store_true", help="skip the copy bandwidth and the 32^3x64 H")
    ap.add_argument("--no-big", action="store_true", help="skip HDCG vs CG at 24^3x48xLs16 (1 and 16 RHS)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver and its kernels run on one GPU; multi-GPU sharding is a design only, so --gpus must be 1"}))
        sys.exit(2)

    import torch

    import paper_1402_2585_amd as hd
    import synth

    dims, Ls, eps, mass = (16, 16, 16, 16), 16, 0.7, 0.01
    U = synth.gauge_field(dims, eps, 2001)
    op = hd.FineOperator(U, dims, Ls, 1.8, mass)
    torch.cuda.synchronize()
    by128 = algorithmic_bytes_H(dims, Ls, 1, 16)
    by64 = algorithmic_bytes_H(dims, Ls, 1, 8)
    fl = flops_H(dims, Ls, 1)

    log("16^4: timing H")
    # timed region: `steps` applications of H in FP64 complex
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms128 = time_H(op, hd, hd.DWF_C128, args.steps, args.warmup)
    wall = time.perf_counter() - t0
    ms64 = time_H(op, hd, hd.DWF_C64, args.steps, args.warmup)
    # outside the timed region: the median of 5 further repetitions
    med128 = time_H(op, hd, hd.DWF_C128, args.steps, 0, reps=5)
    med64 = time_H(op, hd, hd.DWF_C64, args.steps, 0, reps=5)
    gbs128 = by128 / (ms128 * 1e-3) / 1e9
    gbs64 = by64 / (ms64 * 1e-3) / 1e9

    out = {
        "metric": "M_pc^dagger M_pc GB/s (HDCG hot path, 1 GPU)",
        "value": round(gbs128, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms128, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded SU(3) links eps=0.7, Gaussian sources)",
        "config": {"workload": "mpcdagmpc 16^4 x Ls16, M5=1.8, m=0.01, 1 RHS, ping-pong",
                   "lattice": list(dims), "Ls": Ls, "nrhs": 1},
        "gflops": round(fl / (ms128 * 1e-3) / 1e9, 1),
        "c64": {"gbs": round(gbs64, 1), "ms_per_application": round(ms64, 5),
                "gflops": round(fl / (ms64 * 1e-3) / 1e9, 1), "frac_of_hbm_peak": round(gbs64 / HBM_PEAK_GBS, 3),
                "traffic": traffic_from_profiles("c64")},
        "roofline": {
            "kernel": "hop_kernel (4 launches per application; per-launch average)",
            "bound": "hbm",
            "achieved": round(gbs128, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(gbs128 / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profiles("c128"),
            "algorithmic_bytes_per_launch": by128 / 4,
            "avg_launch_ms": round(ms128 / 4, 5),
        },
        "timed_wall_s": round(wall, 3),
        "median_of_5": {"c128_ms_per_application": round(med128, 5), "c64_ms_per_application": round(med64, 5),
                        "c128_gbs": round(by128 / (med128 * 1e-3) / 1e9, 1),
                        "c64_gbs": round(by64 / (med64 * 1e-3) / 1e9, 1)},
    }
    log(f"H c128 {ms128:.4f} ms, c64 {ms64:.4f} ms")
    if not args.no_extra:
        # the Mobius kernel (b5 = 1.5, c5 = 0.5) on the same workload
        opm = hd.FineOperator(U, dims, Ls, 1.8, mass, b5=1.5, c5=0.5)
        msm = time_H(opm, hd, hd.DWF_C128, args.steps, 2)
        msm64 = time_H(opm, hd, hd.DWF_C64, args.steps, 2)
        opm.close()
        # 16-bit fields (the M_IRS storage of irs_prec = DWF_BF16), complex64 links
        ms16 = time_H(op, hd, hd.DWF_BF16, args.steps, 2)
        by16 = algorithmic_bytes_H(dims, Ls, 1, 4, 8)
        out["bf16"] = {"gbs": round(by16 / (ms16 * 1e-3) / 1e9, 1), "ms_per_application": round(ms16, 5),
                       "speedup_vs_c64": round(ms64 / ms16, 3),
                       "frac_of_hbm_peak": round(by16 / (ms16 * 1e-3) / 1e9 / HBM_PEAK_GBS, 3),
                       "traffic": traffic_from_profiles("bf16")}
        out["mobius"] = {"b5": 1.5, "c5": 0.5,
                         "c128": {"gbs": round(by128 / (msm * 1e-3) / 1e9, 1), "ms_per_application": round(msm, 5)},
                         "c64": {"gbs": round(by64 / (msm64 * 1e-3) / 1e9, 1), "ms_per_application": round(msm64, 5)}}
        log("copy bandwidth and 32^3x64")
        cb = copy_bandwidth(torch)
        out["roofline"]["copy_gbs_measured"] = round(cb, 1)
        out["roofline"]["frac_of_copy"] = round(gbs128 / cb, 4)
        out["mall_busting"] = mall_busting(hd, torch)
    if not args.no_hdcg:
        out["hdcg_vs_cg"] = hdcg_vs_cg(hd, torch)
    if not args.no_big:
        out["hdcg_vs_cg_24^3x48"] = hdcg_24(hd, torch)
    if not args.no_cpu:
        # the oracle forks its workers: release this process's device handles
        # first, and start no GPU work in the children
        log("CPU oracle baseline")
        single, apps_per_s, workers, wall = cpu_baseline(dims, Ls, eps, mass)
        out["cpu_baseline"] = {
            "value": round(by128 * apps_per_s / 1e9, 4), "unit": "GB/s", "cores": workers, "kind": "oracle",
            "sample": f"{workers} FP64 applications of H at 16^4 x Ls16, one per worker process on "
                      f"{workers} cores at once ({wall:.1f} s wall; numpy, BLAS held to 1 thread per process)",
            "single_thread": {"value": round(by128 / single / 1e9, 4), "unit": "GB/s", "cores": 1,
                              "seconds_per_application": round(single, 2)},
            "host": _host_info()}
    op.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Workload driver for profiler runs (rocprofv3 --kernel-trace / --pmc).

  python3 -m paper_1402_2585_amd.prof_driver --what H --prec c128 --reps 5
  python3 -m paper_1402_2585_amd.prof_driver --what copy --mib 1024 --reps 5
  python3 -m paper_1402_2585_amd.prof_driver --what hdcg --workload 3 --coarse c64
  python3 -m paper_1402_2585_amd.prof_driver --what mfma --workload 4 --Ls 1 --reps 20
  python3 -m paper_1402_2585_amd.prof_driver --what coarse_cg --workload 4 --Ls 1 --reps 10

`H` applies M_pc^+ M_pc to a seeded source on the 16^4 x Ls16 workload (or
--dims/--Ls); `copy` runs a plain device-to-device copy kernel of known size,
which calibrates the FETCH_SIZE / WRITE_SIZE counters (bytes reported per
byte actually moved); `hdcg` sets up HDCG on a numbered synthetic workload
(inverse iteration with the given steps / tolerance / cap) and runs one
solve to a 1e-8 FP64 true residual, printing the solver statistics;
`lanczos` estimates the extreme eigenvalues of H on a numbered workload (the
conditioning that sets the plain-CG iteration count) from --steps Lanczos
steps with full reorthogonalisation, H applied by the library in FP64;
`coarse_cg` times the coarse mat-vec in every storage and the persistent
coarse CG per iteration for 1-16 right-hand sides on a seeded Hermitian,
diagonally dominant stencil operator with the workload's coarse shape.
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--what", choices=["H", "copy", "hdcg", "lanczos", "coarse", "mfma", "coarse_cg"], default="H")
    ap.add_argument("--steps", type=int, default=80)
    ap.add_argument("--workload", type=int, default=3)
    ap.add_argument("--coarse", choices=["c64", "bf16", "f16"], default="c64")
    ap.add_argument("--irs", choices=["c64", "bf16"], default="c64", help="storage of the M_IRS fields")
    ap.add_argument("--phi", choices=["c64", "bf16"], default="c64", help="storage of the subspace in Q")
    ap.add_argument("--ldop", type=int, default=0,
                    help="extra global coarse vectors of the second deflation level (0: none)")
    ap.add_argument("--nrhs_solve", type=int, default=1, help="right-hand sides of the HDCG solve")
    ap.add_argument("--m1_order", type=int, default=0,
                    help="with --ldop: coarse solves by ADEF1 with a Chebyshev inverse of this order (0: deflated CG)")
    ap.add_argument("--variants", action="store_true",
                    help="solve five times on one setup: as given, 16-bit M_IRS fields, both again after "
                         "building the second deflation level (--ldop vectors, default 128), and with the "
                         "subspace of Q in 16 bits as well")
    ap.add_argument("--cg", action="store_true", help="also time the plain FP64 CG on the same source(s)")
    ap.add_argument("--surface_depth", type=int, default=0,
                    help="keep only the subspace's s < d and s >= Ls - d slices (0: all)")
    ap.add_argument("--seeded", action="store_true",
                    help="the subspace starting vectors drawn by the library (Philox, seed 1000 cfg + 500)")
    ap.add_argument("--phase_timing", action="store_true", help="report the solve's phase times (Fig. pie)")
    ap.add_argument("--no_graph", action="store_true", help="launch the preconditioner kernel by kernel")
    ap.add_argument("--n_ii", type=int, default=3)
    ap.add_argument("--tol_ii", type=float, default=1e-3)
    ap.add_argument("--maxiter_ii", type=int, default=500)
    ap.add_argument("--prec", choices=["c128", "c64"], default="c128")
    ap.add_argument("--dims", type=int, nargs=4, default=[16, 16, 16, 16])
    ap.add_argument("--Ls", type=int, default=16)
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--mib", type=int, default=1024)
    a = ap.parse_args()

    import torch

    if a.what == "copy":
        n = a.mib * 1024 * 1024 // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(a.reps):
            y.copy_(x)
        torch.cuda.synchronize()
        print(f"copy {a.mib} MiB x {a.reps}", flush=True)
        return

    import synth

    if a.what == "hdcg":
        run_hdcg(a, torch, synth)
        return
    if a.what == "lanczos":
        run_lanczos(a, torch, synth)
        return
    if a.what == "coarse":
        run_coarse(a, torch, synth)
        return
    if a.what == "mfma":
        run_mfma(a, torch, synth)
        return
    if a.what == "coarse_cg":
        run_coarse_cg(a, torch, synth)
        return

    dims = tuple(a.dims)
    dt = torch.complex128 if a.prec == "c128" else torch.complex64
    # every torch operation happens before the library launches its first kernel
    U = torch.from_numpy(synth.gauge_field(dims, 0.7, 2001)).to("cuda")
    b = torch.from_numpy(synth.gaussian_half_field(dims, a.Ls, 2100, nrhs=a.nrhs)).to(dtype=dt).to("cuda")
    torch.cuda.synchronize()
    print("inputs on device", flush=True)

    import paper_1402_2585_amd as hd

    prec = hd.DWF_C128 if a.prec == "c128" else hd.DWF_C64
    h = hd.dwf_create(U, dims, a.Ls, 1.8, 0.01)
    nbytes = hd.dwf_field_bytes(h, prec, a.nrhs)
    x = torch.empty(nbytes // b.element_size(), dtype=dt, device="cuda")
    y = torch.empty_like(x)
    hd.dwf_import(h, x, b, prec, a.nrhs)
    print("operator created", flush=True)
    for _ in range(a.reps):
        hd.mpc_dag_mpc_apply(h, y, x, prec, a.nrhs)
        hd.mpc_dag_mpc_apply(h, x, y, prec, a.nrhs)
    hd.dwf_norm2(h, x, prec, a.nrhs)  # synchronises the stream
    hd.dwf_destroy(h)
    print(f"H {a.prec} dims={dims} Ls={a.Ls} nrhs={a.nrhs} x {2 * a.reps}", flush=True)


def run_hdcg(a, torch, synth):
    import numpy as np

    from synth.configs import WORKLOADS

    w = WORKLOADS[a.workload]
    # every torch operation on the inputs happens before the library's first launch
    U = torch.from_numpy(synth.gauge_field(w.dims, w.eps, w.gauge_seed)).to("cuda")
    V = None if a.seeded else torch.from_numpy(np.stack([synth.gaussian_half_field(w.dims, w.Ls, w.subspace_seed(k))
                                                         for k in range(w.nvec)])).to("cuda")
    bsrc = torch.from_numpy(synth.gaussian_half_field(w.dims, w.Ls, w.source_seed(0))).to("cuda")
    torch.cuda.synchronize()
    print("inputs on device", flush=True)

    import paper_1402_2585_amd as hd

    cprec = {"c64": hd.DWF_C64, "bf16": hd.DWF_BF16, "f16": hd.DWF_F16}[a.coarse]
    op = hd.FineOperator(U, w.dims, w.Ls, w.M5, w.mass)
    b = op.to_native(bsrc)
    # the hop autotuner's trials before the setup, so that a traced solve
    # phase holds only the solve's own launches
    for n in sorted({1, 8, a.nrhs_solve}):
        for p in (hd.DWF_C128, hd.DWF_C64, hd.DWF_BF16):
            hd.dwf_tune_hop(op.h, p, n)
    hd.dwf_release_workspace(op.h)
    iprec = {"c64": hd.DWF_C64, "bf16": hd.DWF_BF16}[a.irs]
    pprec = {"c64": hd.DWF_C64, "bf16": hd.DWF_BF16}[a.phi]
    h = hd.HDCG(op, w.block, V, nvec=w.nvec, seed=w.subspace_seed(0), n_ii=a.n_ii, tol_ii=a.tol_ii,
                maxiter_ii=a.maxiter_ii, coarse_prec=cprec, irs_prec=iprec, phi_prec=pprec,
                surface_depth=a.surface_depth, verbose=1, keep_subspace_fp64=0 if a.seeded else 1,
                phase_timing=1 if a.phase_timing else 0, graph=0 if a.no_graph else 1)
    del V
    print("setup done", flush=True)
    if a.variants:
        run_variants(a, torch, synth, hd, w, op, h, b)
        h.close()
        op.close()
        return
    if a.ldop > 0:
        noise = torch.from_numpy(synth.gaussian_coarse(h.Nc, w.nvec, w.coarse_seed, a.ldop)).to("cuda")
        hd.hdcg_ldop_setup(h.h, a.ldop, noise, 0.0, 3, 1e-7)
        del noise
        print(f"second deflation level: {w.nvec + a.ldop} global vectors", flush=True)
        if a.m1_order > 0:
            h.set_params(ldop_m1=1, m1_order=a.m1_order)
            lo, hi = hd.hdcg_m1_interval(h.h)
            print(f"ADEF1, Chebyshev order {a.m1_order} on [{lo}, {hi:.3f}]", flush=True)
    if a.nrhs_solve > 1:
        b = op.new_field(nrhs=a.nrhs_solve)
        n1 = b.numel() // a.nrhs_solve
        for r in range(a.nrhs_solve):
            src = torch.from_numpy(synth.gaussian_half_field(w.dims, w.Ls, w.source_seed(r))).to("cuda")
            b[r * n1:(r + 1) * n1] = op.to_native(src)
    x = op.new_field(zero=True, nrhs=a.nrhs_solve)
    rc, st = hd.hdcg_solve(h.h, x, b, a.nrhs_solve, 1e-8)
    print(f"hdcg workload {a.workload} coarse {a.coarse} M_IRS fields {a.irs} subspace {a.phi} ldop {a.ldop} "
          f"m1_order {a.m1_order} surface_depth {a.surface_depth} "
          f"nrhs {a.nrhs_solve}: "
          f"status {rc} {st}", flush=True)
    h.close()
    op.close()


def run_variants(a, torch, synth, hd, w, op, h, b):
    import time

    import numpy as np

    nr = a.nrhs_solve
    if nr > 1:
        bs = torch.from_numpy(np.stack([synth.gaussian_half_field(w.dims, w.Ls, w.source_seed(r))
                                        for r in range(nr)])).to("cuda")
        b = op.to_native(bs)
        del bs
    if a.cg:
        x = op.new_field(zero=True, nrhs=nr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in range(nr):
            n1 = x.numel() // nr
            rc, st = hd.cg_solve(op.h, x[r * n1:(r + 1) * n1], b[r * n1:(r + 1) * n1], 1, 1e-8, 50000)
        torch.cuda.synchronize()
        print(f"plain FP64 CG, {nr} right-hand side(s) one after another: {time.perf_counter() - t0:.3f} s", flush=True)
        del x

    def solve(name):
        x = op.new_field(zero=True, nrhs=nr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st = hd.hdcg_solve(h.h, x, b, nr, 1e-8)
        torch.cuda.synchronize()
        print(f"variant {name}: {time.perf_counter() - t0:.3f} s, status {rc} {st}", flush=True)

    solve("as given")
    h.set_params(irs_prec=hd.DWF_BF16)
    solve("16-bit M_IRS fields")
    n_extra = a.ldop if a.ldop > 0 else 128
    noise = torch.from_numpy(synth.gaussian_coarse(h.Nc, w.nvec, w.coarse_seed, n_extra)).to("cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hd.hdcg_ldop_setup(h.h, n_extra, noise, 0.0, 3, 1e-7)
    torch.cuda.synchronize()
    print(f"second deflation level: {w.nvec + n_extra} global vectors, {time.perf_counter() - t0:.2f} s", flush=True)
    del noise
    solve("16-bit M_IRS fields + second level")
    h.set_params(phi_prec=hd.DWF_BF16)
    solve("16-bit M_IRS fields + second level + 16-bit subspace in Q")
    h.set_params(ldop_m1=1)
    lo, hi = hd.hdcg_m1_interval(h.h)
    print(f"ADEF1 Chebyshev interval [{lo}, {hi:.3f}]", flush=True)
    for order in (16, 8, 4):
        h.set_params(m1_order=order)
        solve(f"16-bit M_IRS fields + second level (ADEF1, Chebyshev order {order}) + 16-bit subspace in Q")
    h.set_params(ldop_m1=0, m1_order=16, irs_prec=hd.DWF_C64, phi_prec=hd.DWF_C64)
    solve("second level")


def run_coarse(a, torch, synth):
    """Times the coarse-grid kernels of a numbered workload (subspace: the
    starting vectors drawn on the device from the workload's seed,
    orthonormalised, no inverse iteration): the little Dirac operator
    mat-vec, its one-hop truncation and the Chebyshev inverse (order 16 on
    [0.5, 45]) on one right-hand side, and the project / promote of the
    solve's subspace copies on one and on --nrhs_solve right-hand sides;
    complex64 vectors, --reps each."""
    import time

    from synth.configs import WORKLOADS

    w = WORKLOADS[a.workload]
    U = torch.from_numpy(synth.gauge_field(w.dims, w.eps, w.gauge_seed)).to("cuda")
    torch.cuda.synchronize()
    import paper_1402_2585_amd as hd

    op = hd.FineOperator(U, w.dims, w.Ls, w.M5, w.mass)
    del U
    # both subspace copies (complex64, bf16) are built before the FP64 one is released
    h = hd.HDCG(op, w.block, None, nvec=w.nvec, seed=w.subspace_seed(0), n_ii=0, keep_subspace_fp64=0,
                phi_prec=hd.DWF_BF16)
    h.set_params(m1_lo=0.5, m1_hi=45.0, m1_order=16)
    x = torch.from_numpy(synth.gaussian_coarse(h.Nc, h.nvec, w.coarse_seed, 1)).to(torch.complex64).to("cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    print(f"coarse grid Nc {h.Nc} nvec {h.nvec}", flush=True)
    nr = max(1, a.nrhs_solve)
    f = torch.randn(nr * op.new_field(hd.DWF_C64).numel(), dtype=torch.complex64, device="cuda")
    g = torch.empty_like(f)
    ym = torch.randn(nr * h.Nc * h.nvec, dtype=torch.complex64, device="cuda")
    torch.cuda.synchronize()
    cases = [("A mat-vec", lambda: hd.coarse_apply(h.h, y, x, hd.DWF_C64)),
             ("Q_trunc mat-vec", lambda: hd.hdcg_trunc_apply(h.h, y, x, hd.DWF_C64)),
             ("Chebyshev order 16", lambda: hd.hdcg_chebyshev(h.h, y, x, hd.DWF_C64))]
    for n in sorted({1, nr}):
        cases += [(f"project, complex64 subspace, {n} RHS", lambda n=n: hd.hdcg_project(h.h, ym, f, hd.DWF_C64, n)),
                  (f"project, bf16 subspace, {n} RHS", lambda n=n: hd.hdcg_project(h.h, ym, f, hd.DWF_BF16, n)),
                  (f"promote, complex64 subspace, {n} RHS", lambda n=n: hd.hdcg_promote(h.h, g, ym, hd.DWF_C64, n)),
                  (f"promote, bf16 subspace, {n} RHS", lambda n=n: hd.hdcg_promote(h.h, g, ym, hd.DWF_BF16, n))]
    for name, fn in cases:
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.reps):
            fn()
        torch.cuda.synchronize()
        print(f"{name}: {(time.perf_counter() - t0) / a.reps * 1e3:.3f} ms", flush=True)
    h.close()
    op.close()


def run_mfma(a, torch, synth):
    """The 16-bit MFMA mat-vec of the little Dirac operator on the coarse grid
    of a numbered workload (Nc, Nvec as there; the fine lattice keeps the
    workload's 4D extents with Ls = --Ls, which does not change the coarse
    shape), on a random operator imported into the handle: for bf16 and fp16
    storage and 1, 8 and 16 right-hand sides, the autotuned tile and the time
    of every candidate, and the matrix bytes per launch over the time."""
    import time

    from synth.configs import WORKLOADS

    import paper_1402_2585_amd as hd

    w = WORKLOADS[a.workload]
    U = torch.from_numpy(synth.gauge_field(w.dims, w.eps, w.gauge_seed)).to("cuda")
    op = hd.FineOperator(U, w.dims, a.Ls, w.M5, w.mass)
    h = hd.HDCG(op, w.block, None, nvec=w.nvec, seed=w.subspace_seed(0))
    g = torch.Generator(device="cuda").manual_seed(5)
    A = torch.randn((h.Nc, 81, h.nvec, h.nvec), dtype=torch.complex128, device="cuda", generator=g)
    hd.hdcg_import_coarse(h.h, A)
    del A
    kst = (2 * 81 * h.nvec + 15) // 16
    mbytes = h.Nc * kst * h.nvec * 16 * 2  # fragment-ordered 16-bit storage
    print(f"coarse grid Nc {h.Nc} nvec {h.nvec}: 16-bit matrix {mbytes / 1e9:.3f} GB", flush=True)
    for prec, pname in ((hd.DWF_BF16, "bf16"), (hd.DWF_F16, "fp16")):
        for nr in (1, 8, 16):
            x = torch.randn((nr, h.Nc, h.nvec), dtype=torch.complex64, device="cuda", generator=g)
            y = torch.empty_like(x)
            tile, ms = hd.hdcg_mfma_tile(h.h, prec, nr)
            hd.coarse_apply(h.h, y, x, prec, nr)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(a.reps):
                hd.coarse_apply(h.h, y, x, prec, nr)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / a.reps
            vb = 2 * h.Nc * h.nvec * nr * 8
            flops = 8 * h.Nc * 81 * h.nvec * h.nvec * nr
            print(f"{pname} nrhs {nr}: tile {tile} {dt * 1e3:.4f} ms, {(mbytes + vb) / dt / 1e9:.1f} GB/s, "
                  f"{flops / dt / 1e12:.2f} TFLOP/s; candidates ms {[round(m, 4) for m in ms]}", flush=True)
    h.close()
    op.close()


def run_coarse_cg(a, torch, synth):
    """The coarse mat-vec and the persistent coarse CG on the coarse grid of a
    numbered workload (the fine lattice with Ls = --Ls, which does not change
    the coarse shape), on a seeded Hermitian, diagonally dominant stencil
    operator built on the device and imported into the handle: the
    standalone mat-vec for complex128, complex64 and bf16 storage and 1, 8
    and 16 right-hand sides (--reps each), and the persistent CG's time per
    iteration for complex64 and bf16 and 1, 2, 8 and 16 right-hand sides, as
    the difference of fixed-count solves of 12 and 4 iterations over 8
    (tolerance 1e-30, so every right-hand side runs to the cap)."""
    import time

    from synth.configs import WORKLOADS

    import paper_1402_2585_amd as hd

    w = WORKLOADS[a.workload]
    U = torch.from_numpy(synth.gauge_field(w.dims, w.eps, w.gauge_seed)).to("cuda")
    op = hd.FineOperator(U, w.dims, a.Ls, w.M5, w.mass)
    h = hd.HDCG(op, w.block, None, nvec=w.nvec, seed=w.subspace_seed(0), n_ii=0)
    # A[a][l] = B_l(a) for the 40 stencil points before the site, A[a + d_l][80 - l]
    # = B_l(a)^+ (Hermitian), 8 on the site's diagonal: diagonally dominant
    C = [w.dims[i] // w.block[i] for i in range(4)]
    nc, nv = h.Nc, h.nvec
    g = torch.Generator(device="cuda").manual_seed(460)
    ai = torch.arange(nc, device="cuda")
    co = torch.stack([ai % C[0], (ai // C[0]) % C[1], (ai // (C[0] * C[1])) % C[2], ai // (C[0] * C[1] * C[2])], 1)
    A = torch.zeros((nc, 81, nv, nv), dtype=torch.complex128, device="cuda")
    for l in range(40):
        off = torch.tensor([(l // 3 ** mu) % 3 - 1 for mu in range(4)], device="cuda")
        c2 = (co + off) % torch.tensor(C, device="cuda")
        nb = c2[:, 0] + C[0] * (c2[:, 1] + C[1] * (c2[:, 2] + C[2] * c2[:, 3]))
        B = 1e-3 * torch.randn((nc, nv, nv), dtype=torch.complex128, device="cuda", generator=g)
        A[:, l] = B
        A[nb, 80 - l] = B.conj().transpose(1, 2)
    A[:, 40] = 8.0 * torch.eye(nv, dtype=torch.complex128, device="cuda")
    hd.hdcg_import_coarse(h.h, A)
    del A
    abytes = {hd.DWF_C128: 16, hd.DWF_C64: 8, hd.DWF_BF16: 4}
    names = {hd.DWF_C128: "complex128", hd.DWF_C64: "complex64", hd.DWF_BF16: "bf16"}
    print(f"coarse grid Nc {h.Nc} nvec {h.nvec}", flush=True)
    for prec in (hd.DWF_C128, hd.DWF_C64, hd.DWF_BF16):
        vt = torch.complex128 if prec == hd.DWF_C128 else torch.complex64
        for nr in (1, 8, 16):
            x = torch.randn((nr, h.Nc, h.nvec), dtype=vt, device="cuda", generator=g)
            y = torch.empty_like(x)
            hd.coarse_apply(h.h, y, x, prec, nr)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(a.reps):
                hd.coarse_apply(h.h, y, x, prec, nr)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / a.reps
            mb = h.Nc * 81 * h.nvec * h.nvec * abytes[prec]
            print(f"mat-vec {names[prec]} nrhs {nr}: {dt * 1e3:.3f} ms, matrix {mb / dt / 1e9:.0f} GB/s", flush=True)
    for prec in (hd.DWF_C64, hd.DWF_BF16):
        h.set_params(coarse_prec=prec)
        for nr in (1, 2, 8, 16):
            b = torch.randn((nr, h.Nc, h.nvec), dtype=torch.complex64, device="cuda", generator=g)
            x = torch.zeros_like(b)
            hd.hdcg_coarse_solve(h.h, x, b, prec, nr, 1e-30, 4)
            ts = {}
            for mi in (4, 12):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rc, it = hd.hdcg_coarse_solve(h.h, x, b, prec, nr, 1e-30, mi)
                torch.cuda.synchronize()
                ts[mi] = time.perf_counter() - t0
                assert it == mi, (rc, it, mi)
            print(f"persistent coarse CG {names[prec]} nrhs {nr}: {(ts[12] - ts[4]) / 8 * 1e3:.3f} ms per iteration",
                  flush=True)
    h.close()
    op.close()


def run_lanczos(a, torch, synth):
    import numpy as np

    from synth.configs import WORKLOADS

    w = WORKLOADS[a.workload]
    U = torch.from_numpy(synth.gauge_field(w.dims, w.eps, w.gauge_seed)).to("cuda")
    b = torch.from_numpy(synth.gaussian_half_field(w.dims, w.Ls, w.source_seed(0))).to("cuda")
    torch.cuda.synchronize()

    import paper_1402_2585_amd as hd

    op = hd.FineOperator(U, w.dims, w.Ls, w.M5, w.mass)
    v = op.to_native(b)
    v /= torch.linalg.vector_norm(v)
    Q = [v.clone()]
    alpha, beta = [], []
    for j in range(a.steps):
        wv = op.H(Q[-1])
        al = torch.vdot(Q[-1], wv).real
        wv -= al * Q[-1]
        if j > 0:
            wv -= beta[-1] * Q[-2]
        for q in Q:  # full reorthogonalisation
            wv -= torch.vdot(q, wv) * q
        be = torch.linalg.vector_norm(wv)
        alpha.append(float(al))
        beta.append(float(be))
        Q.append(wv / be)
        if len(Q) > 2 and j % 20 == 19:
            print(f"lanczos step {j + 1}", flush=True)
    T = np.diag(alpha) + np.diag(beta[:-1], 1) + np.diag(beta[:-1], -1)
    ev = np.linalg.eigvalsh(T)
    print(f"lanczos workload {a.workload} {w.dims} Ls={w.Ls} m={w.mass}: steps {a.steps} "
          f"lambda_min {ev[0]:.6e} lambda_max {ev[-1]:.6e} ratio {ev[-1] / ev[0]:.1f}", flush=True)
    op.close()


if __name__ == "__main__":
    main()

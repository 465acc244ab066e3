"""Summaries of rocprofv3 result databases (the rocpd SQLite files that
`rocprofv3 --kernel-trace` and `rocprofv3 --pmc` write), for the profile
notes under profiles/.

  python3 paper_1402_2585_amd/prof_summary.py trace <run_results.db> [--match S] [--grid N]
  python3 paper_1402_2585_amd/prof_summary.py pmc <run_results.db> [--match S] [--grid N]
  python3 paper_1402_2585_amd/prof_summary.py hop-json <dir> --out profiles/hop_kernel_16^4xLs16_pmc.json [--shapes S]
  python3 paper_1402_2585_amd/prof_summary.py solve <run_results.db> [--top N]

`solve` summarises the solve phase of a traced `prof_driver.py --what hdcg`
run: the dispatches after the last kernel that only the setup launches (the
Gram, Cholesky, inverse-DFT, probe and second-level build kernels), their
span from first start to last end, the time kernels were busy (the union of
the dispatch intervals), and per kernel the workgroups x grid.y, calls, total
and average time, largest total first.

`trace` prints, per kernel name (optionally only names containing S and
dispatches whose grid has N work-items in x), the dispatch count and the
average / minimum / maximum duration in microseconds.  `pmc` prints, per
kernel name and counter, the dispatch count and the average counter value
per dispatch.  Both print a markdown table; --json prints the same rows as
JSON instead.
"""
from __future__ import annotations

import argparse
import json
import sqlite3
from collections import defaultdict


def trace_rows(db, match=None, grid=None):
    c = sqlite3.connect(db)
    rows = defaultdict(list)
    for name, dur, gx in c.execute("select name, duration, grid_x from kernels"):
        if match and match not in name:
            continue
        if grid is not None and gx != grid:
            continue
        rows[name].append(dur / 1000.0)
    return [{"kernel": k, "calls": len(v), "avg_us": sum(v) / len(v), "min_us": min(v), "max_us": max(v)}
            for k, v in sorted(rows.items())]


def pmc_rows(db, match=None, grid=None):
    c = sqlite3.connect(db)
    acc = defaultdict(lambda: defaultdict(list))
    for name, counter, value, gx in c.execute(
            "select kernel_name, counter_name, value, grid_size_x from counters_collection"):
        if match and match not in name:
            continue
        if grid is not None and gx != grid:
            continue
        acc[name][counter].append(value)
    out = []
    for k in sorted(acc):
        for cn in sorted(acc[k]):
            v = acc[k][cn]
            out.append({"kernel": k, "counter": cn, "dispatches": len(v), "avg": sum(v) / len(v)})
    return out


def hop_json(dirs, out_path, root, shapes=None):
    """The hop kernel's HBM traffic per launch on 16^4 x Ls16 from the
    FETCH_SIZE / WRITE_SIZE runs (dirs: {tag: (fetch_db, write_db)} for
    c128, c64, bf16 and the copy-kernel calibration 'copy'), scaled by what
    the same counters read for the copy kernel of 1 GiB read + 1 GiB write;
    tagged with the hash of the kernel sources it was taken on."""
    import hashlib
    import os

    def avg(db, counter, match):
        vals = [r["avg"] for r in pmc_rows(db, match) if r["counter"] == counter]
        return vals

    gib_kib = 1024.0 * 1024.0
    fscale = gib_kib / avg(dirs["copy"][0], "FETCH_SIZE", "copy_kernel")[0]
    wscale = gib_kib / avg(dirs["copy"][1], "WRITE_SIZE", "copy_kernel")[0]
    h = hashlib.sha256()
    for f in ("fine_op.hip", "fine_op.h", "common.h"):
        h.update(open(os.path.join(root, "paper_1402_2585_amd", "csrc", f), "rb").read())
    V, Ls = 16 ** 4, 16
    half = V // 2 * Ls * 12
    out = {"source_hash": h.hexdigest()[:16],
           "workload": "H = M_pc^+ M_pc on 16^4 x Ls16, 1 RHS",
           "launch_shapes": shapes or {},
           "calibration": {"fetch_scale": fscale, "write_scale": wscale,
                           "copy_kernel": "hdcg_prof copy 1024 3: 1 GiB read + 1 GiB write per launch"}}
    for tag, cb, gb in (("c128", 16, 16), ("c64", 8, 8), ("bf16", 4, 8)):
        fetch_db, write_db = dirs[tag]
        def epi(name):  # the third template argument of hop_kernel<R, DAG, EPI, NPH, LS, MOB, T>
            return name[name.index("hop_kernel<") + len("hop_kernel<"):].split(",")[2].strip()

        f_inv = [r["avg"] for r in pmc_rows(fetch_db, "hop_kernel") if r["counter"] == "FETCH_SIZE" and epi(r["kernel"]) == "0"]
        f_sub = [r["avg"] for r in pmc_rows(fetch_db, "hop_kernel") if r["counter"] == "FETCH_SIZE" and epi(r["kernel"]) == "1"]
        w = [r["avg"] for r in pmc_rows(write_db, "hop_kernel") if r["counter"] == "WRITE_SIZE"]
        fi, fs, ww = sum(f_inv) / len(f_inv), sum(f_sub) / len(f_sub), sum(w) / len(w)
        per_launch = ((fi + fs) / 2 * fscale + ww * wscale) * 1024.0
        alg = (10 * half * cb + 4 * V * 36 * gb) / 4
        out[tag] = {"bytes_per_launch": per_launch, "algorithmic_bytes_per_launch": alg,
                    "amplification": per_launch / alg,
                    "fetch_kib_per_dispatch": {"m5inv_stage": fi, "m5sub_stage": fs},
                    "write_kib_per_dispatch": ww}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


SETUP_KERNELS = ("k_chol_inv", "k_gs_apply", "k_idft_dim", "k_probe", "k_philox_gaussian", "k_blockmap",
                 "k_transpose", "k_phi_layout", "k_phi_bf16", "k_phi_surface", "k_free_vectors", "k_surface_zero",
                 "k_gram", "k_expand", "k_frag", "k_scales", "k_rho")


def solve_rows(db, setup_kernels=SETUP_KERNELS):
    c = sqlite3.connect(db)
    rows = list(c.execute("select name, start, end, grid_x, grid_y, workgroup_x from kernels order by start"))
    last = -1
    for i, (name, *_rest) in enumerate(rows):
        if any(k in name for k in setup_kernels):
            last = i
    sol = rows[last + 1:]
    if not sol:
        return None
    span = (max(r[2] for r in sol) - min(r[1] for r in sol)) / 1e6
    busy, cur_s, cur_e = 0, None, None
    for _, st, en, *_r in sol:
        if cur_e is None or st > cur_e:
            if cur_e is not None:
                busy += cur_e - cur_s
            cur_s, cur_e = st, en
        else:
            cur_e = max(cur_e, en)
    busy += cur_e - cur_s
    per = defaultdict(list)
    shape = {}
    for name, st, en, gx, gy, wx in sol:
        per[name].append((en - st) / 1e3)
        shape[name] = (gx // max(wx, 1), gy)
    table = sorted(({"kernel": k, "workgroups": shape[k][0], "grid_y": shape[k][1], "calls": len(v),
                     "total_ms": sum(v) / 1e3, "avg_us": sum(v) / len(v)} for k, v in per.items()),
                   key=lambda r: -r["total_ms"])
    return {"span_ms": span, "busy_ms": busy / 1e6, "dispatches": len(sol), "kernels": table}


def short(name, n=110):
    name = name.replace("hdk::", "").replace("(anonymous namespace)::", "")
    i = name.find("(")
    if i > 0:
        name = name[:i]
    return name if len(name) <= n else name[:n] + "..."


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["trace", "pmc", "hop-json", "solve"])
    ap.add_argument("db", help="result database, or for hop-json the directory holding the runs "
                               "fetch_<tag>/, write_<tag>/ (tag c128, c64, bf16, copy), each with run_results.db")
    ap.add_argument("--out", default=None, help="hop-json: output path")
    ap.add_argument("--shapes", default=None,
                    help="hop-json: the launch shapes the runs used, e.g. 'c128=2,2,1,1,1,0,0,4,0,1;c64=...'")
    ap.add_argument("--match", default=None)
    ap.add_argument("--grid", type=int, default=None)
    ap.add_argument("--json", action="store_true")
    ap.add_argument("--top", type=int, default=25, help="solve: kernels listed")
    a = ap.parse_args()
    if a.what == "solve":
        r = solve_rows(a.db)
        if r is None:
            raise SystemExit("no dispatches after the setup")
        if a.json:
            print(json.dumps(r, indent=1))
            return
        print(f"Solve phase (after the setup's last kernel): span {r['span_ms']:.1f} ms, kernels busy "
              f"{r['busy_ms']:.1f} ms, {r['dispatches']} dispatches.\n")
        print("| kernel | workgroups x grid.y | calls | total ms | avg us |\n|---|---|---|---|---|")
        for k in r["kernels"][:a.top]:
            print(f"| `{short(k['kernel'])}` | {k['workgroups']} x {k['grid_y']} | {k['calls']} | "
                  f"{k['total_ms']:.2f} | {k['avg_us']:.1f} |")
        return
    if a.what == "hop-json":
        import os

        d = {t: (os.path.join(a.db, f"fetch_{t}", "run_results.db"), os.path.join(a.db, f"write_{t}", "run_results.db"))
             for t in ("c128", "c64", "bf16", "copy")}
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        shapes = dict(kv.split("=", 1) for kv in a.shapes.split(";")) if a.shapes else None
        print(json.dumps(hop_json(d, a.out, root, shapes), indent=1))
        return
    rows = (trace_rows if a.what == "trace" else pmc_rows)(a.db, a.match, a.grid)
    if a.json:
        print(json.dumps(rows, indent=1))
        return
    if a.what == "trace":
        print("| kernel | calls | avg us | min us | max us |\n|---|---|---|---|---|")
        for r in rows:
            print(f"| `{short(r['kernel'])}` | {r['calls']} | {r['avg_us']:.2f} | {r['min_us']:.2f} | {r['max_us']:.2f} |")
    else:
        print("| kernel | counter | dispatches | average per dispatch |\n|---|---|---|---|")
        for r in rows:
            print(f"| `{short(r['kernel'])}` | {r['counter']} | {r['dispatches']} | {r['avg']:.6g} |")


if __name__ == "__main__":
    main()

"""Summaries of rocprofv3 output (rocpd SQLite databases) for the engine.

    python -m paper_2303_01471_amd.profiling kernels DB [--isolated] [--largest-grid]
        per-kernel dispatch count, total / mean / min / max duration (the
        --kernel-trace --stats view), one line per kernel; --isolated keeps only
        dispatches that overlapped no other one, --largest-grid only each kernel's
        dispatches of its largest grid
    python -m paper_2303_01471_amd.profiling counters DB
        mean value per dispatch of every collected counter, per kernel
    python -m paper_2303_01471_amd.profiling traffic FETCH_DB:WRITE_DB:POINTS_JSON [...] --copy-bytes B --source-hash H
        HBM bytes per grid point of every pass kernel from FETCH_SIZE and
        WRITE_SIZE, each scaled by what the same counter reads for one
        elementwise kernel that reads and writes B bytes in the same run; one
        triple per benchmark run (its two counter databases and its points-per-
        dispatch map), merged into one JSON (profiles/traffic.json format)

Dispatch sizes (grid points per launch) come from the kernel arguments of the
pass kernels as recorded by the benchmark (every instance active, steps capped).
"""
from __future__ import annotations

import argparse
import collections
import json
import re
import sqlite3
import sys


def _short(name: str) -> str:
    n = name.replace("(anonymous namespace)::", "").split("(")[0]
    for pre in ("void ", "qhd::"):
        n = n.replace(pre, "")
    return n.strip()


def _isolated(rows):
    """indices of the dispatches whose [start, end) overlaps no other dispatch"""
    order = sorted(range(len(rows)), key=lambda i: rows[i][1])
    keep = set()
    max_end = None  # latest end among the dispatches started before
    for pos, i in enumerate(order):
        st, en = rows[i][1], rows[i][2]
        nxt = rows[order[pos + 1]][1] if pos + 1 < len(order) else None
        if (max_end is None or max_end <= st) and (nxt is None or nxt >= en):
            keep.add(i)
        max_end = en if max_end is None else max(max_end, en)
    return keep


def kernel_stats(db: str, isolated: bool = False, largest_grid: bool = False):
    """Per-kernel duration statistics; with ``isolated`` only over dispatches that ran
    alone on the device (no other dispatch overlapping them), the view of the library's
    serialised timing chunks; with ``largest_grid`` only over each kernel's dispatches of
    its largest grid (a batch's launches, not those of single-instance runs of the same
    kernel)."""
    con = sqlite3.connect(db)
    cols = [r[1] for r in con.execute("pragma table_info(kernels)")]
    st = "start" if "start" in cols else "start_ns"
    en = "end" if "end" in cols else "end_ns"
    grid = "grid_x * grid_y * grid_z" if "grid_x" in cols else "0"
    rows = con.execute(f'select name, "{st}", "{en}", {grid} from kernels').fetchall()
    keep = _isolated(rows) if isolated else set(range(len(rows)))
    if largest_grid:
        big = collections.defaultdict(int)
        for r in rows:
            big[_short(r[0])] = max(big[_short(r[0])], r[3])
        keep = {i for i in keep if rows[i][3] == big[_short(rows[i][0])]}
    rows = [(rows[i][0], rows[i][2] - rows[i][1]) for i in sorted(keep)]
    agg = collections.defaultdict(list)
    for name, dur in rows:
        agg[_short(name)].append(dur)
    out = []
    for k, v in agg.items():
        out.append(dict(kernel=k, calls=len(v), total_ns=sum(v), mean_ns=sum(v) / len(v), min_ns=min(v),
                        max_ns=max(v)))
    out.sort(key=lambda r: -r["total_ns"])
    return out


def counter_means(db: str):
    con = sqlite3.connect(db)
    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    for name, cname, val, d in con.execute(
            "select kernel_name, counter_name, value, dispatch_id from counters_collection"):
        k = _short(name)
        agg[k][cname] += val
        disp[k].add(d)
    return {k: {c: v / len(disp[k]) for c, v in d.items()} for k, d in agg.items()}, \
        {k: len(v) for k, v in disp.items()}


# pass kernel -> (family name used by the library's timing, algorithmic bytes per point);
# the 2-D kernels' third template argument is the model (0 QHD, 1 QAA), a last boolean
# one whether the fourth-order stage arithmetic is compiled in
def _model_suffix(m, i=2):
    return "_qaa" if (m.re.groups >= i and m.group(i) == "1") else ""


_FAMILY = [
    (re.compile(r"k_row_pass_2d<(\d+), \d+(?:, (\d+))?(?:, (?:true|false))?>"),
     lambda m: f"row_pass_2d{_model_suffix(m)}/n{m.group(1)}", 24.0),
    (re.compile(r"k_col_pass_(?:2d|tw)<(\d+), \d+(?:, (\d+))?(?:, (?:true|false))?>"),
     lambda m: f"col_pass_2d{_model_suffix(m)}/n{m.group(1)}", 16.0),
    (re.compile(r"k_col_pass_split<(\d+),"), lambda m: f"col_pass_2d/n{m.group(1)}", 16.0),
    (re.compile(r"k_lf_row_2d<(\d+), \d+>"), lambda m: f"row_pass_2d_qaa_lf/n{m.group(1)}", 20.0),
    (re.compile(r"k_lf_col_2d<(\d+), \d+>"), lambda m: f"col_pass_2d_qaa_lf/n{m.group(1)}", 20.0),
    (re.compile(r"k_line_pass_1d<(\d+),"), lambda m: f"line_pass_1d/n{m.group(1)}", 24.0),
    # 3-D: the x-pass (psi read and written, f read) and the (y, z)-plane pass
    (re.compile(r"k_xpass_3d<(\d+),"), lambda m: f"xpass_3d/n{m.group(1)}", 24.0),
    (re.compile(r"k_plane(?:_direct)?_3d<(\d+), (\d+),"), lambda m: f"plane_3d/n{m.group(1)}x{m.group(2)}", 16.0),
    # matrix-core DFT passes (128^3): AXIS 0 MODE 1 is the x-pass, MODE 0 the y-pass, MODE 2 the z-pass
    (re.compile(r"k_mfma_pass_3d<0, 1>"), lambda m: "xpass_3d_mfma/n128", 24.0),
    (re.compile(r"k_mfma_pass_3d<1, 0>"), lambda m: "ypass_3d_mfma/n128", 16.0),
    (re.compile(r"k_mfma_pass_3d<2, 2>"), lambda m: "zpass_3d_mfma/n128", 16.0),
]

# relaxed-QP kernels of one step (psi read and written per axis pass, f read once)
_RQP_STEP = re.compile(r"k_rqp_(?:fused|axis_staged|axis_direct)\b")


def family_of(kernel: str):
    """(family name, algorithmic bytes per point) of a pass kernel, or None."""
    for rx, fam, bpp in _FAMILY:
        m = rx.search(kernel)
        if m:
            return fam(m), bpp
    return None


def traffic(fetch_db: str, write_db: str, copy_bytes: float, points_per_dispatch: dict,
            source_hash: str) -> dict:
    fe, nfe = counter_means(fetch_db)
    wr, nwr = counter_means(write_db)
    # the calibration kernel: the run's only torch elementwise launch, which reads and
    # writes copy_bytes once
    copy_k = [k for k in fe if "elementwise" in k.lower()]
    if len(copy_k) != 1 or nfe[copy_k[0]] != 1 or nwr.get(copy_k[0]) != 1:
        raise SystemExit(f"expected exactly one calibration dispatch, found {[(k, nfe[k]) for k in copy_k]}")
    ck = copy_k[0]
    f_scale = copy_bytes / (fe[ck]["FETCH_SIZE"] * 1024.0)
    w_scale = copy_bytes / (wr[ck]["WRITE_SIZE"] * 1024.0)
    out = {"source_hash": source_hash, "copy_kernel": ck, "copy_bytes": copy_bytes,
           "fetch_scale": f_scale, "write_scale": w_scale, "kernels": {}}
    # a family's kernel is its most-dispatched instantiation (the one the workload runs;
    # other variants are autotuning trials)
    best = {}
    for k in fe:
        fb = family_of(k)
        if fb and (fb[0] not in best or nfe[k] > nfe[best[fb[0]]]):
            best[fb[0]] = k
    for k, v in fe.items():
        fb = family_of(k)
        if fb and best[fb[0]] == k:
            name, bpp = fb
            pts = points_per_dispatch.get(name)
            if not pts:
                continue
            fetch = v["FETCH_SIZE"] * 1024.0 * f_scale
            write = wr.get(k, {}).get("WRITE_SIZE", 0.0) * 1024.0 * w_scale
            out["kernels"][name] = {"kernel": k, "points_per_dispatch": pts,
                                    "fetch_bytes_per_point": fetch / pts,
                                    "write_bytes_per_point": write / pts,
                                    "hbm_bytes_per_point": (fetch + write) / pts,
                                    "algorithmic_bytes_per_point": bpp}
    # relaxed QP: all step kernels together (one fused pass per step, then one pass per
    # remaining axis), bytes per lattice point and step
    rq = sorted(k for k in fe if _RQP_STEP.search(k))
    pts = points_per_dispatch.get("rqp_step")
    steps = sum(nfe[k] for k in rq if "fused" in k)
    if rq and pts and steps:
        fetch = sum(fe[k]["FETCH_SIZE"] * nfe[k] for k in rq) * 1024.0 * f_scale
        write = sum(wr.get(k, {}).get("WRITE_SIZE", 0.0) * nwr.get(k, 0) for k in rq) * 1024.0 * w_scale
        out["kernels"]["rqp_step"] = {"kernel": " + ".join(rq), "points_per_dispatch": pts, "steps": steps,
                                      "fetch_bytes_per_point": fetch / (pts * steps),
                                      "write_bytes_per_point": write / (pts * steps),
                                      "hbm_bytes_per_point": (fetch + write) / (pts * steps),
                                      "algorithmic_bytes_per_point": points_per_dispatch.get("rqp_bytes_per_point")}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("kernels")
    a.add_argument("db")
    a.add_argument("--isolated", action="store_true",
                   help="only dispatches that overlap no other dispatch (serialised timing chunks)")
    a.add_argument("--largest-grid", action="store_true",
                   help="only each kernel's dispatches of its largest grid (the batch's launches)")
    b = sub.add_parser("counters")
    b.add_argument("db")
    c = sub.add_parser("traffic")
    c.add_argument("runs", nargs="+", help="FETCH_DB:WRITE_DB:POINTS_JSON (points: family -> points per dispatch)")
    c.add_argument("--copy-bytes", type=float, required=True)
    c.add_argument("--source-hash", required=True)
    args = ap.parse_args(argv)
    if args.cmd == "kernels":
        print(f"{'calls':>8} {'total_ms':>10} {'mean_us':>10} {'min_us':>9} {'max_us':>9}  kernel")
        for r in kernel_stats(args.db, args.isolated, args.largest_grid):
            print(f"{r['calls']:8d} {r['total_ns'] / 1e6:10.3f} {r['mean_ns'] / 1e3:10.2f} "
                  f"{r['min_ns'] / 1e3:9.2f} {r['max_ns'] / 1e3:9.2f}  {r['kernel']}")
    elif args.cmd == "counters":
        means, n = counter_means(args.db)
        for k, d in sorted(means.items()):
            print(f"{k} dispatches={n[k]} " + " ".join(f"{c}={v:.1f}" for c, v in sorted(d.items())))
    else:
        merged = None
        for run in args.runs:
            fdb, wdb, pfile = run.split(":")
            with open(pfile) as fh:
                pts = json.load(fh)
            t = traffic(fdb, wdb, args.copy_bytes, pts, args.source_hash)
            t["runs"] = [{k: t[k] for k in ("copy_kernel", "fetch_scale", "write_scale")} | {"fetch_db": fdb}]
            if merged is None:
                merged = t
            else:
                merged["kernels"].update(t["kernels"])
                merged["runs"] += t["runs"]
        json.dump(merged, sys.stdout, indent=1)
        print()


if __name__ == "__main__":
    main()

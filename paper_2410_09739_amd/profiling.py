"""Turn rocprofv3 CSV output into the short text summaries kept with the
measurements.

Three commands:

``kernel-stats STATS_CSV OUT.md --title T --cmd C [--trace TRACE_CSV]``
    Table of the ``*_kernel_stats.csv`` written by
    ``rocprofv3 --kernel-trace --stats --output-format csv`` (with the trace
    CSV: one row per kernel and launch grid).

``counters DIR OUT.md --title T --cmd C [--match NAME]``
    Mean of every counter per dispatch of a ``rocprofv3 --pmc`` run, one row
    per kernel and grid size.

``traffic --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR --out OUT.md --cmd C ...``
    HBM bytes per launch of the stream-collide kernel of every storage form,
    from one ``--pmc FETCH_SIZE`` and one ``--pmc WRITE_SIZE`` run of the bench
    (counter values in KiB per dispatch), each scaled by what the same counter
    reads for a plain device copy of known size.  The result is written as
    markdown with one fenced JSON block that the bench reads back; the block
    records a hash of the kernel sources so that a stale measurement is never
    reported for a changed kernel.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_2410_09739_amd/csrc/stream_collide.hpp", "paper_2410_09739_amd/csrc/fpc_collide.hpp",
                  "paper_2410_09739_amd/csrc/d3q27.hpp", "paper_2410_09739_amd/csrc/lattice.hpp"]
# storage form id (template argument of k_stream_collide) -> (name, bytes per population)
FORMS = {0: ("f64", 8), 1: ("f32", 4), 2: ("f16dev", 2), 3: ("bf16dev", 2), 4: ("f16dev_rne", 2),
         5: ("bf16dev_rne", 2)}
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def _code_only(text: str) -> str:
    """C/C++ source without comments, whitespace runs collapsed to one space
    (string and character literals kept as they are)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash() -> str:
    """Hash of the code of the stream-collide kernel sources: comments and
    layout do not count, so that only a change to the code itself marks a
    traffic measurement as stale."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def _counter_means(d: str) -> dict[str, list[float]]:
    path = next(os.path.join(d, f) for f in sorted(os.listdir(d)) if f.endswith("counter_collection.csv"))
    vals: dict[str, list[float]] = defaultdict(list)
    with open(path) as fh:
        for r in csv.DictReader(fh):
            vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return vals


def _counter_means_by_name(d: str) -> dict[str, dict[str, list[float]]]:
    """kernel -> counter -> values per dispatch (a run collecting several counters)."""
    path = next(os.path.join(d, f) for f in sorted(os.listdir(d)) if f.endswith("counter_collection.csv"))
    vals: dict[str, dict[str, list[float]]] = defaultdict(lambda: defaultdict(list))
    with open(path) as fh:
        for r in csv.DictReader(fh):
            vals[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return vals


def _copy_factor(d: str, nbytes: int) -> float:
    """Bytes that one KiB of the counter stands for, from a copy of ``nbytes``."""
    v = _counter_means(d)[COPY_KERNEL]
    big = [x for x in v if x > 0.25 * max(v)]
    return nbytes / (sum(big) / len(big))


def traffic(args) -> dict:
    nodes = args.nx * args.ny * args.nz
    cf = _copy_factor(args.copy_fetch, args.copy_bytes)
    cw = _copy_factor(args.copy_write, args.copy_bytes)
    fetch, write = _counter_means(args.fetch), _counter_means(args.write)
    dram = _counter_means_by_name(args.dram) if getattr(args, "dram", None) else {}
    forms = {}
    for name in fetch:
        m = re.match(r"void k_stream_collide<(\d+),", name)
        if not m or name not in write:
            continue
        form, sb = FORMS[int(m.group(1))]
        fk = sum(fetch[name]) / len(fetch[name])
        wk = sum(write[name]) / len(write[name])
        hbm = fk * cf + wk * cw
        alg = nodes * 54 * sb
        forms[form] = {"kernel": name, "launches": len(fetch[name]), "fetch_kib": round(fk, 3),
                       "write_kib": round(wk, 3), "hbm_bytes_per_launch": round(hbm),
                       "algorithmic_bytes_per_launch": alg, "traffic_over_algorithmic": round(hbm / alg, 5)}
        if name in dram:
            # DRAM requests counted in 32-byte units (a 64- or 128-byte request counts 2 or 4):
            # bytes with no calibration
            rd = dram[name].get("TCC_EA0_RDREQ_DRAM_32B_sum", [])
            wr = dram[name].get("TCC_EA0_WRREQ_WRITE_DRAM_32B_sum", [])
            if rd and wr:
                b = 32.0 * (sum(rd) / len(rd) + sum(wr) / len(wr))
                forms[form]["dram_32b_read_bytes"] = round(32.0 * sum(rd) / len(rd))
                forms[form]["dram_32b_write_bytes"] = round(32.0 * sum(wr) / len(wr))
                forms[form]["dram_32b_over_algorithmic"] = round(b / alg, 5)
    return {"kernel_source_sha": kernel_source_hash(), "workload": args.workload,
            "shape": [args.nx, args.ny, args.nz], "nodes": nodes,
            "copy_factor_fetch_bytes_per_kib": round(cf, 3), "copy_factor_write_bytes_per_kib": round(cw, 3),
            "forms": forms}


def write_traffic_md(res: dict, out: str, cmds: list[str]) -> None:
    with open(out, "w") as fo:
        fo.write(f"# HBM traffic of the fused stream-collide kernel, {res['workload']}\n\n")
        fo.write("FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from separate rocprofv3 --pmc runs, "
                 "each scaled by the bytes per KiB that the same counter shows for a plain device "
                 f"copy of known size (fetch {res['copy_factor_fetch_bytes_per_kib']} B/KiB, "
                 f"write {res['copy_factor_write_bytes_per_kib']} B/KiB).  Algorithmic bytes per "
                 "launch: 27 reads + 27 writes of the stored population per node.\n\n")
        fo.write("Commands (run from the repository root):\n\n```\n" + "\n".join(cmds) + "\n```\n\n")
        dram = all("dram_32b_over_algorithmic" in r for r in res["forms"].values())
        if dram:
            fo.write("Cross-check without a calibration: the DRAM read and write requests in 32-byte units "
                     "(TCC_EA0_RDREQ_DRAM_32B_sum, TCC_EA0_WRREQ_WRITE_DRAM_32B_sum, one further run) "
                     "times 32 bytes.\n\n")
        fo.write("| form | fetch KiB | write KiB | HBM bytes / launch | algorithmic | ratio |"
                 + (" DRAM 32-B units x 32 / algorithmic |" if dram else "") + "\n"
                 "|---|---|---|---|---|---|" + ("---|" if dram else "") + "\n")
        for f, r in res["forms"].items():
            fo.write(f"| {f} | {r['fetch_kib']:.1f} | {r['write_kib']:.1f} | {r['hbm_bytes_per_launch']} | "
                     f"{r['algorithmic_bytes_per_launch']} | {r['traffic_over_algorithmic']:.4f} |"
                     + (f" {r['dram_32b_over_algorithmic']:.4f} |" if dram else "") + "\n")
        fo.write("\n```json\n" + json.dumps(res, indent=1) + "\n```\n")


def read_traffic_md(path: str) -> dict | None:
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        m = re.search(r"```json\n(.*?)\n```", fh.read(), re.S)
    return json.loads(m.group(1)) if m else None


def kernel_stats(args) -> None:
    """Per-kernel table from ``*_kernel_stats.csv``; with ``--trace`` (the
    ``*_kernel_trace.csv`` of the same run) one row per kernel and grid size,
    so that launches of one kernel on different lattices are told apart."""
    rows = []
    if args.trace:
        groups: dict[tuple, list[float]] = defaultdict(list)
        with open(args.trace) as fh:
            for r in csv.DictReader(fh):
                grid = "x".join(r[f"Grid_Size_{d}"] for d in "XYZ")
                groups[(r["Kernel_Name"], grid)].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
        total = sum(sum(v) for v in groups.values())
        for (name, grid), v in groups.items():
            rows.append((name, grid, len(v), sum(v) / 1e3, sum(v) / len(v) / 1e3, 100.0 * sum(v) / total))
        rows.sort(key=lambda r: -r[3])
    else:
        with open(args.stats) as fh:
            for r in csv.DictReader(fh):
                rows.append((r["Name"], "", int(r["Calls"]), float(r["TotalDurationNs"]) / 1e3,
                             float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    with open(args.out, "w") as fo:
        fo.write(f"# {args.title}\n\nCommand (run from the repository root):\n\n```\n{args.cmd}\n```\n\n")
        if args.note:
            fo.write(args.note + "\n\n")
        fo.write("| kernel | grid (threads) | calls | total (us) | average (us) | % |\n|---|---|---|---|---|---|\n")
        for name, grid, calls, tot, avg, pct in rows[: args.rows]:
            n = name if len(name) < 120 else name[:117] + "..."
            fo.write(f"| `{n}` | {grid} | {calls} | {tot:.1f} | {avg:.3f} | {pct:.2f} |\n")


def counters(args) -> None:
    """Mean of every counter per dispatch, one row per kernel and grid size,
    from the ``*_counter_collection.csv`` of a ``rocprofv3 --pmc`` run."""
    path = next(os.path.join(args.dir, f) for f in sorted(os.listdir(args.dir)) if f.endswith("counter_collection.csv"))
    vals: dict[tuple, dict[str, list[float]]] = defaultdict(lambda: defaultdict(list))
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if args.match and args.match not in r["Kernel_Name"]:
                continue
            vals[(r["Kernel_Name"], r["Grid_Size"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    names = sorted({c for v in vals.values() for c in v})
    with open(args.out, "w") as fo:
        fo.write(f"# {args.title}\n\nCommand (run from the repository root):\n\n```\n{args.cmd}\n```\n\n")
        if args.note:
            fo.write(args.note + "\n\n")
        fo.write("| kernel | grid (threads) | dispatches | " + " | ".join(names) + " |\n")
        fo.write("|---|---|---|" + "---|" * len(names) + "\n")
        for (name, grid), v in sorted(vals.items()):
            k = name.split("(")[0].replace("void ", "")
            n = max(len(x) for x in v.values())
            cells = [f"{sum(v[c]) / len(v[c]):.0f}" if v.get(c) else "" for c in names]
            fo.write(f"| `{k}` | {grid} | {n} | " + " | ".join(cells) + " |\n")


def main() -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    k = sub.add_parser("kernel-stats")
    k.add_argument("stats")
    k.add_argument("out")
    k.add_argument("--title", required=True)
    k.add_argument("--cmd", required=True)
    k.add_argument("--rows", type=int, default=16)
    k.add_argument("--trace", default=None, help="the run's *_kernel_trace.csv: split rows by grid size")
    k.add_argument("--note", default="")
    t = sub.add_parser("traffic")
    for a in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--out"):
        t.add_argument(a, required=True)
    t.add_argument("--copy-bytes", type=int, default=1 << 31)
    t.add_argument("--nx", type=int, default=256)
    t.add_argument("--ny", type=int, default=128)
    t.add_argument("--nz", type=int, default=128)
    t.add_argument("--workload", default="channel 256x128x128 (walls, body force)")
    t.add_argument("--cmd", action="append", default=[])
    t.add_argument("--dram", default=None, help="a --pmc run of TCC_EA0_RDREQ_DRAM_32B_sum and "
                   "TCC_EA0_WRREQ_WRITE_DRAM_32B_sum (cross-check)")
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("out")
    c.add_argument("--title", required=True)
    c.add_argument("--cmd", required=True)
    c.add_argument("--note", default="")
    c.add_argument("--match", default="", help="keep kernels whose name contains this")
    a = ap.parse_args()
    if a.cmd_name == "kernel-stats":
        kernel_stats(a)
    elif a.cmd_name == "counters":
        counters(a)
    else:
        res = traffic(a)
        write_traffic_md(res, a.out, a.cmd)
        print(json.dumps(res))


if __name__ == "__main__":
    main()

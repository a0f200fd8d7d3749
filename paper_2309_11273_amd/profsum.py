"""Summaries of rocprofv3 output for the committed profile records.

  python -m paper_2309_11273_amd.profsum stats  CSV --command CMD
      kernel-trace statistics (--kernel-trace --stats) as a markdown table
  python -m paper_2309_11273_amd.profsum pmc    CSV [CSV ...] --command CMD [--command CMD ...]
      per-kernel averages of the counters of --pmc runs as a markdown table
  python -m paper_2309_11273_amd.profsum traffic --fetch CSV --write CSV --workload NAME
                                                 --copy-bytes N --out JSON
      HBM bytes per launch of every solver kernel from a FETCH_SIZE run and a
      WRITE_SIZE run (KiB per dispatch), each scaled by what the same counter
      reads for a plain read-and-write kernel of N bytes each way launched
      in the same process; merged into the JSON file under
      "<kernel>@<workload>" with the hash of the kernel's sources
  python -m paper_2309_11273_amd.profsum tail   TRACE_CSV --last N
      average duration of the last N dispatches of every solver kernel in a
      --kernel-trace run (the eager profiled steps that close a bench run,
      which bench.py times with HIP events for the roofline's kernel_ms)
  python -m paper_2309_11273_amd.profsum requests --csv CSV --workload NAME
                                                  --copy-bytes N --out JSON
      exact read bytes per launch from a run of the read-request counters by
      size (TCC_EA0_RDREQ_32B_sum, _64B_sum, _128B_sum): 32, 64 and 128
      bytes per request.  On gfx950 FETCH_SIZE counts a 128-byte request as
      64 bytes (its 128-byte term, TCC_BUBBLE, reads zero), so the copy
      reference's scale (2, all its reads are 128-byte requests) is exact
      only for kernels that issue 128-byte requests alone.  Added to the
      JSON entries taken on the same kernel source as "read_bytes_exact" and
      "bytes_per_launch_exact" (with the WRITE_SIZE bytes, which count every
      write request at its size)

Nothing here touches the GPU.
"""

from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")

# source files each solver kernel is compiled from
KERNEL_SOURCES = {
    "k_tpass1_f32": ["kernels_tiled.hip", "tile_common.h"], "k_tpass2_f32": ["kernels_tiled.hip", "tile_common.h"],
    "k_tpass1_f64": ["kernels_tiled64.hip", "tile_common.h"], "k_tpass2_f64": ["kernels_tiled64.hip", "tile_common.h"],
    "k_tdsum": ["kernels_tiled.hip", "tile_common.h"],
    "k_pass1_f32": ["kernels_f32.hip"], "k_pass2_f32": ["kernels_f32.hip"],
    "k_pass1_f64": ["kernels.hip"], "k_pass2_f64": ["kernels.hip"],
    "k_fac_extension": ["factored.hip", "factored.h", "tile_common.h"],
    "k_fac_dilatation": ["factored.hip", "factored.h", "tile_common.h"],
    "k_fac_force": ["factored.hip", "factored.h", "tile_common.h"],
    "k_fac_rows": ["factored.hip", "factored.h", "tile_common.h"],
    "k_fin_pass1": ["finite.hip", "finite.h"], "k_fin_pass2": ["finite.hip", "finite.h"],
    "k_adr_sums": ["adr.hip", "adr.h"], "k_adr_reduce": ["adr.hip", "adr.h"], "k_adr_update": ["adr.hip", "adr.h"],
}

# the known-size reference kernel bench.py --copy-mb launches (torch.mul out=)
COPY_KERNEL_MARK = "MulFunctor"


def kernel_source_hash(kname: str) -> str:
    """Hash of the sources a kernel is compiled from (and the shared header)."""
    h = hashlib.sha256()
    for fname in KERNEL_SOURCES[kname] + ["kernels.h"]:
        with open(os.path.join(CSRC, fname), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(full: str) -> str:
    """'void pdk::k_tpass1_f32<3, true>(...)' -> 'k_tpass1_f32<3, true>'."""
    n = full.split("(")[0].replace("void ", "").strip()
    return n.split("::")[-1] if n.startswith("pdk::") else n


def base_name(full: str) -> str:
    return short_name(full).split("<")[0]


def stats_md(path: str, command: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = [f"Command: `{command}`", "",
           "| kernel | calls | average (us) | min (us) | max (us) | total (ms) | % |",
           "|---|---|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out) + "\n"


def tail_md(trace_csv: str, last: int) -> str:
    per = collections.defaultdict(list)
    for r in csv.DictReader(open(trace_csv)):
        k = short_name(r["Kernel_Name"])
        if k.startswith("k_"):
            per[k].append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    out = ["| kernel | dispatches | last | average of the last (us) |", "|---|---|---|---|"]
    for k in sorted(per, key=lambda k: -sum(d for _, d in per[k])):
        d = [x[1] for x in sorted(per[k])[-last:]]
        out.append(f"| `{k}` | {len(per[k])} | {len(d)} | {sum(d) / len(d) / 1e3:.2f} |")
    return "\n".join(out) + "\n"


def counter_means(paths):
    """{kernel short name: {counter: mean value per dispatch}}."""
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for p in paths:
        for r in csv.DictReader(open(p)):
            acc[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in acc.items()}


def pmc_md(paths, commands) -> str:
    m = counter_means(paths)
    counters = sorted({c for d in m.values() for c in d})
    out = [f"Command: `{c}`" for c in commands] + ["", "Mean per dispatch.", "",
                                                    "| kernel | " + " | ".join(counters) + " |",
                                                    "|---|" + "---|" * len(counters)]
    for k in sorted(m):
        if not (k.startswith("k_") or COPY_KERNEL_MARK in k):
            continue
        name = "copy reference (torch.mul)" if COPY_KERNEL_MARK in k else f"`{k}`"
        out.append(f"| {name} | " + " | ".join(f"{m[k].get(c, float('nan')):.0f}" for c in counters) + " |")
    return "\n".join(out) + "\n"


def traffic(fetch_csv: str, write_csv: str, copy_bytes: int, workload: str, out_json: str) -> dict:
    fm, wm = counter_means([fetch_csv]), counter_means([write_csv])
    ref = [k for k in fm if COPY_KERNEL_MARK in k]
    if not ref:
        raise SystemExit("no reference copy kernel in the FETCH_SIZE run")
    kf = copy_bytes / (fm[ref[0]]["FETCH_SIZE"] * 1024.0)
    kw = copy_bytes / (wm[ref[0]]["WRITE_SIZE"] * 1024.0)
    db = json.load(open(out_json)) if os.path.exists(out_json) else {}
    for k in fm:
        b = base_name(k)
        if b not in KERNEL_SOURCES or k not in wm:
            continue
        fetch = fm[k]["FETCH_SIZE"] * 1024.0 * kf
        write = wm[k]["WRITE_SIZE"] * 1024.0 * kw
        db[f"{b}@{workload}"] = {"bytes_per_launch": int(fetch + write), "fetch_bytes": int(fetch),
                                 "write_bytes": int(write), "fetch_scale": round(kf, 4),
                                 "write_scale": round(kw, 4), "source_sha": kernel_source_hash(b)}
    with open(out_json, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
        f.write("\n")
    return db


REQ_COUNTERS = {"TCC_EA0_RDREQ_32B_sum": 32, "TCC_EA0_RDREQ_64B_sum": 64, "TCC_EA0_RDREQ_128B_sum": 128}


def requests(req_csv: str, copy_bytes: int, workload: str, out_json: str) -> dict:
    m = counter_means([req_csv])
    exact = {k: sum(v[c] * b for c, b in REQ_COUNTERS.items()) for k, v in m.items()
             if all(c in v for c in REQ_COUNTERS)}
    ref = [k for k in exact if COPY_KERNEL_MARK in k]
    if not ref:
        raise SystemExit("no reference copy kernel in the request-size run")
    ratio = exact[ref[0]] / copy_bytes
    if abs(ratio - 1.0) > 0.01:
        raise SystemExit(f"request-size bytes of the copy reference are {ratio:.4f} x its size")
    db = json.load(open(out_json)) if os.path.exists(out_json) else {}
    for k, rd in exact.items():
        b = base_name(k)
        e = db.get(f"{b}@{workload}")
        if b not in KERNEL_SOURCES or not e or e.get("source_sha") != kernel_source_hash(b):
            continue
        e["read_bytes_exact"] = int(rd)
        e["bytes_per_launch_exact"] = int(rd + e["write_bytes"])
    with open(out_json, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
        f.write("\n")
    return db


def main(argv=None):
    ap = argparse.ArgumentParser(prog="profsum")
    sp = ap.add_subparsers(dest="cmd", required=True)
    a = sp.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--command", required=True)
    b = sp.add_parser("pmc")
    b.add_argument("csv", nargs="+")
    b.add_argument("--command", action="append", required=True)
    c = sp.add_parser("traffic")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--copy-bytes", type=int, required=True)
    c.add_argument("--workload", required=True)
    c.add_argument("--out", required=True)
    t = sp.add_parser("tail")
    t.add_argument("csv")
    t.add_argument("--last", type=int, required=True)
    r = sp.add_parser("requests")
    r.add_argument("--csv", required=True)
    r.add_argument("--copy-bytes", type=int, required=True)
    r.add_argument("--workload", required=True)
    r.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        sys.stdout.write(stats_md(args.csv, args.command))
    elif args.cmd == "pmc":
        sys.stdout.write(pmc_md(args.csv, args.command))
    elif args.cmd == "tail":
        sys.stdout.write(tail_md(args.csv, args.last))
    elif args.cmd == "traffic":
        json.dump(traffic(args.fetch, args.write, args.copy_bytes, args.workload, args.out), sys.stdout, indent=1)
        sys.stdout.write("\n")
    else:
        json.dump(requests(args.csv, args.copy_bytes, args.workload, args.out), sys.stdout, indent=1)
        sys.stdout.write("\n")


if __name__ == "__main__":
    main()

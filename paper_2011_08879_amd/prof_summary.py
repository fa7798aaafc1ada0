"""Summaries of rocprofv3 runs over the SpMV sweep's marked launch groups.

`bench.py --profile-sweep groups.json` launches every sweep SpMV in a group of
its own, opened by a small COPY kernel whose grid (256 (k+1) threads) names
group k, and ends with a 1 GiB COPY.  This module reads the CSV output of
rocprofv3 (`--output-format csv`): the kernel trace for durations and the
counter collection for HBM traffic, attributes every dispatch to its group and
writes a Markdown table and the JSON file bench.py reads its traffic figures
from.

HBM bytes come from two gfx950 L2 counters that count DRAM-bound requests in
32-byte units whatever the request size: TCC_EA0_RDREQ_DRAM_32B (reads) and
TCC_EA0_WRREQ_WRITE_DRAM_32B (writes), summed over all L2 channels of all
XCDs; bytes = 32 x count.  The 1 GiB COPY checks them.  (The derived
FETCH_SIZE counts a 128-byte read as 64 bytes on gfx950, hence half the bytes
of a streaming read.)

Usage:
  python -m paper_2011_08879_amd.prof_summary --trace G0.json:T.csv \\
      --pmc G1.json:C1.csv [--pmc G2.json:C2.csv ...] --md OUT.md --json OUT.json \\
      --command "..."
  python -m paper_2011_08879_amd.prof_summary stats KERNEL_STATS.csv [TOP]
  python -m paper_2011_08879_amd.prof_summary counters COUNTER_COLLECTION.csv NAME_PART
"""
from __future__ import annotations

import argparse
import collections
import csv
import json
import os

READ_32B = "TCC_EA0_RDREQ_DRAM_32B_sum"
WRITE_32B = "TCC_EA0_WRREQ_WRITE_DRAM_32B_sum"
MARKER = "stream_copy_kernel"


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError("none of %s in %s" % (names, list(row)))


def read_trace(path):
    """[(kernel, grid_threads, duration_ns)] in dispatch order."""
    out = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            start = int(_col(r, "Start_Timestamp"))
            end = int(_col(r, "End_Timestamp"))
            disp = int(_col(r, "Dispatch_Id", "Correlation_Id"))
            grid = int(_col(r, "Grid_Size", "Grid_Size_X"))
            out.append((disp, _col(r, "Kernel_Name"), grid, end - start))
    out.sort()
    return [t[1:] for t in out]


def read_counters(path):
    """[(kernel, grid_threads, {counter: value})] in dispatch order."""
    d = collections.OrderedDict()
    with open(path) as fh:
        for r in csv.DictReader(fh):
            disp = int(_col(r, "Dispatch_Id", "Correlation_Id"))
            e = d.setdefault(disp, [_col(r, "Kernel_Name"), int(_col(r, "Grid_Size")), {}])
            e[2][_col(r, "Counter_Name")] = float(_col(r, "Counter_Value"))
    return [tuple(d[k]) for k in sorted(d)]


def split_groups(dispatches, n_groups):
    """Dispatches after marker k (a COPY of grid 256 (k+1)) up to the next
    marker belong to group k; the group after the last SpMV group is the
    calibration copy."""
    groups = [[] for _ in range(n_groups)]
    cur = None
    for item in dispatches:
        name, grid = item[0], item[1]
        if MARKER in name and grid % 256 == 0 and 1 <= grid // 256 <= n_groups:
            cur = grid // 256 - 1
            continue
        if cur is not None:
            groups[cur].append(item)
    return groups


def _short(name):
    name = name.replace("void ", "").replace("gko::", "").replace("(anonymous namespace)::", "")
    return name.split("(")[0]


def _groups(path):
    with open(path) as fh:
        return json.load(fh)


def _keep(k, ng, disp):
    """The calibration group counts only the COPY itself (not the fill of its
    source array)."""
    return [d for d in disp if k < ng - 1 or MARKER in d[0]]


def summarize(trace_run, pmc_runs):
    """trace_run: (groups json, kernel trace csv) or None; pmc_runs: list of
    (groups json, counter csv), each run with its own launch count."""
    meta = _groups(trace_run[0] if trace_run else pmc_runs[0][0])
    names = [g["name"] for g in meta["groups"]]
    ng = len(names)  # the last group is the calibration copy
    res = {"source_sha256": meta["source_sha256"], "kernels": {}}
    trace = None
    if trace_run:
        trace = [_keep(k, ng, d) for k, d in enumerate(split_groups(read_trace(trace_run[1]), ng))]
    pmc = collections.defaultdict(lambda: collections.defaultdict(float))
    for gpath, path in pmc_runs:
        m = _groups(gpath)
        assert [g["name"] for g in m["groups"]] == names, "runs of different group lists"
        assert m["source_sha256"] == meta["source_sha256"], "runs on different sources"
        for k, disp in enumerate(split_groups(read_counters(path), ng)):
            launches = m["groups"][k]["launches"]
            for kern, grid, ctr in _keep(k, ng, disp):
                for c, v in ctr.items():
                    pmc[k][c] += v / launches
    for k, g in enumerate(meta["groups"]):
        launches = g["launches"]
        row = {"alg_bytes": g["alg_bytes"], "launches": launches}
        if trace is not None:
            per = collections.OrderedDict()
            for kern, grid, ns in trace[k]:
                key = "%s[grid %d]" % (_short(kern), grid)
                per.setdefault(key, []).append(ns)
            row["dispatches"] = {kk: {"per_launch": len(v) / launches,
                                      "avg_us": round(sum(v) / len(v) / 1e3, 2)}
                                 for kk, v in per.items()}
            row["trace_us"] = round(sum(ns for _, _, ns in trace[k]) / launches / 1e3, 2)
        if READ_32B in pmc[k]:
            row["read_bytes"] = int(round(pmc[k][READ_32B] * 32))
        if WRITE_32B in pmc[k]:
            row["write_bytes"] = int(round(pmc[k][WRITE_32B] * 32))
        if "read_bytes" in row and "write_bytes" in row:
            row["traffic_bytes"] = row["read_bytes"] + row["write_bytes"]
            row["traffic_over_alg"] = round(row["traffic_bytes"] / g["alg_bytes"], 4)
        for c, v in pmc[k].items():
            if c not in (READ_32B, WRITE_32B):
                row.setdefault("counters_per_launch", {})[c] = v
        res["kernels"][g["name"]] = row
    cal = res["kernels"].pop("copy_1GiB")
    res["calibration"] = {"copy_bytes": meta["groups"][-1]["alg_bytes"] // 2, **{
        k: cal[k] for k in ("read_bytes", "write_bytes", "trace_us") if k in cal}}
    return res


def to_markdown(res, command):
    lines = ["| matrix/format | kernels (avg us per dispatch) | trace us | alg MB | HBM read MB |"
             " HBM write MB | traffic / alg |", "|---|---|---:|---:|---:|---:|---:|"]
    for name, r in res["kernels"].items():
        ks = "; ".join("%s %.1f" % (k, v["avg_us"]) for k, v in r.get("dispatches", {}).items())
        lines.append("| %s | %s | %s | %.1f | %s | %s | %s |" % (
            name, ks, r.get("trace_us", "-"), r["alg_bytes"] / 1e6,
            "%.1f" % (r["read_bytes"] / 1e6) if "read_bytes" in r else "-",
            "%.1f" % (r["write_bytes"] / 1e6) if "write_bytes" in r else "-",
            r.get("traffic_over_alg", "-")))
    c = res["calibration"]
    cal = ("Calibration: the library's COPY kernel moving %d bytes in and out (%s us) read %s "
           "and wrote %s bytes by these counters." % (
               c["copy_bytes"], c.get("trace_us", "-"), c.get("read_bytes", "-"),
               c.get("write_bytes", "-")))
    head = ["# SpMV sweep (FP64): kernel durations and HBM traffic", "",
            "Workload: one SpMV y = A x per group on the 27-point stencil 128^3 (n = 2,097,152, "
            "nnz = 55,742,968) and the lognormal random matrix (n = 10^6, mean 16, longest row "
            "10,000), each format as the sweep stores it, and the random-gather probe (y[i] = "
            "x[idx[i]], 16M uniform int32 indices into an 8 MB FP64 x, index and output "
            "streamed); one MI355X (gfx950). Durations: "
            "kernel trace, mean per dispatch. HBM bytes per SpMV: 32 x "
            "(TCC_EA0_RDREQ_DRAM_32B_sum, TCC_EA0_WRREQ_WRITE_DRAM_32B_sum), no scale factor.",
            "", "Kernel sources (sha256 over csrc/): `%s`." % res["source_sha256"], "",
            "Commands (repo root, `export TMPDIR=/tmp`):", "", "```", command, "```", "", cal, ""]
    return "\n".join(head + lines + sq_table(res)) + "\n"


# Shader counters per SpMV, summed over all CUs: instructions issued by kind,
# cycles with LDS instructions active and lost to bank conflicts, and the
# GPU's active cycles (GRBM_GUI_ACTIVE, summed over the 8 XCDs).
SQ_COLUMNS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_VMEM_RD", "SQ_ACTIVE_INST_LDS",
              "SQ_LDS_BANK_CONFLICT", "SQ_WAIT_INST_ANY", "SQ_BUSY_CYCLES", "GRBM_GUI_ACTIVE")


def sq_table(res):
    rows = [(n, r.get("counters_per_launch", {})) for n, r in res["kernels"].items()]
    if not any("SQ_INSTS_VALU" in c for _, c in rows):
        return []
    out = ["", "Shader counters per SpMV (one pass of their own; sums over all CUs):", "",
           "| matrix/format | " + " | ".join(SQ_COLUMNS) + " |",
           "|---|" + "---:|" * len(SQ_COLUMNS)]
    for n, c in rows:
        out.append("| %s | " % n + " | ".join(
            "%.4g" % c[k] if k in c else "-" for k in SQ_COLUMNS) + " |")
    return out


def kernel_stats_table(path, top=25):
    """Markdown table of rocprofv3's kernel_stats.csv: the `top` kernels by
    total time (calls, total ms, mean us, share)."""
    rows = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            rows.append((float(r["TotalDurationNs"]), int(r["Calls"]), float(r["AverageNs"]),
                         float(r["Percentage"]), _short(r["Name"])))
    rows.sort(reverse=True)
    out = ["| kernel | calls | total ms | mean us | share % |", "|---|---:|---:|---:|---:|"]
    for tot, calls, avg, pct, name in rows[:top]:
        out.append("| %s | %d | %.2f | %.2f | %.2f |" % (name, calls, tot / 1e6, avg / 1e3, pct))
    return "\n".join(out) + "\n"


def kernel_counters_table(path, match):
    """Per kernel instantiation whose name contains `match`: dispatches and
    the mean of every counter over them (counter CSV of rocprofv3)."""
    per = collections.OrderedDict()
    for kern, grid, ctr in read_counters(path):
        if match not in kern:
            continue
        e = per.setdefault("%s[grid %d]" % (_short(kern), grid), [0, {}])
        e[0] += 1
        for c, v in ctr.items():
            e[1][c] = e[1].get(c, 0.0) + v
    names = sorted({c for _, (n, d) in per.items() for c in d})
    out = ["| kernel | dispatches | " + " | ".join(names) + " |",
           "|---|---:|" + "---:|" * len(names)]
    for k, (n, d) in per.items():
        out.append("| %s | %d | " % (k, n) + " | ".join("%.4g" % (d.get(c, 0.0) / n) for c in names)
                   + " |")
    return "\n".join(out) + "\n"


def main():
    import sys
    if len(sys.argv) > 1 and sys.argv[1] == "stats":
        print(kernel_stats_table(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 25))
        return
    if len(sys.argv) > 1 and sys.argv[1] == "counters":
        print(kernel_counters_table(sys.argv[2], sys.argv[3]))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", default="", help="GROUPS.json:kernel_trace.csv")
    ap.add_argument("--pmc", action="append", default=[], help="GROUPS.json:counter_collection.csv")
    ap.add_argument("--md", default="")
    ap.add_argument("--json", default="")
    ap.add_argument("--command", default="")
    a = ap.parse_args()
    res = summarize(a.trace.split(":", 1) if a.trace else None,
                    [p.split(":", 1) for p in a.pmc])
    if a.json:
        with open(a.json, "w") as fh:
            json.dump(res, fh, indent=1)
    md = to_markdown(res, a.command)
    if a.md:
        with open(a.md, "w") as fh:
            fh.write(md)
    print(md)


if __name__ == "__main__":
    main()

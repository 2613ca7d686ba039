"""Turns rocprofv3 CSV output into the short text summaries kept in profiles/.

  python -m paper_2103_10116_amd.profile_summary stats <kernel_trace.csv> <out.md> "<command>"
  python -m paper_2103_10116_amd.profile_summary traffic <fetch_counter.csv> \
      <write_counter.csv> <out.txt> "<command>"

`stats` lists every kernel (grouped by name and grid size) with its call
count and mean / median duration.  `traffic` records FETCH_SIZE and
WRITE_SIZE per dispatch (KiB) for the SpMV kernels, the scale factors
measured on the HBM probe's copy kernel (1 GiB read + 1 GiB written), and
the SHA-256 of spmv.hip at measurement time, so that a later reader can tell
whether the counters still describe the current kernels.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SPMV_SRC = os.path.join(HERE, "csrc", "spmv.hip")


def spmv_source_sha() -> str:
    with open(SPMV_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _short(name: str) -> str:
    return name.replace("mxs::(anonymous namespace)::", "").replace("mxs::", "") \
        .replace("void ", "").split("(")[0]


def stats(trace_csv: str, out: str, command: str, top: int = 30,
          always=("k_csr", "k_coo", "k_ell")) -> None:
    """Per-kernel summary: the `top` kernel/grid pairs by total time, then
    every SpMV kernel (names starting with one of `always`) not among them."""
    rows = list(csv.DictReader(open(trace_csv)))
    agg = collections.defaultdict(list)
    for r in rows:
        key = (_short(r["Kernel_Name"]), int(r["Grid_Size_X"]), int(r["Workgroup_Size_X"]))
        agg[key].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1000.0)
    lines = ["# rocprofv3 kernel trace summary", "", f"Command: `{command}`", "",
             "| kernel | grid (threads) | wg | calls | mean us | median us | total ms |",
             "|---|---|---|---|---|---|---|"]
    ranked = sorted(agg.items(), key=lambda kv: -sum(kv[1]))
    shown = ranked[:top] + [kv for kv in ranked[top:] if kv[0][0].startswith(tuple(always))]
    for (name, grid, wg), v in shown:
        v = sorted(v)
        lines.append(f"| `{name}` | {grid} | {wg} | {len(v)} | {sum(v)/len(v):.2f} | "
                     f"{v[len(v)//2]:.2f} | {sum(v)/1e3:.3f} |")
    if len(ranked) > len(shown):
        rest = [t for kv in ranked if kv not in shown for t in kv[1]]
        lines.append(f"| ({len(ranked) - len(shown)} more kernel/grid pairs) | | | {len(rest)} | | | "
                     f"{sum(rest)/1e3:.3f} |")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _counters(path):
    rows = list(csv.DictReader(open(path)))
    agg = collections.defaultdict(list)
    for r in rows:
        agg[(_short(r["Kernel_Name"]), int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    return {k: sorted(v)[len(v) // 2] for k, v in agg.items()}


def traffic(fetch_csv: str, write_csv: str, out: str, command: str) -> None:
    fe = _counters(fetch_csv)
    wr = _counters(write_csv)
    copy = [k for k in fe if k[0] == "k_probe_copy1"]
    gib_kib = float(1 << 20)
    fscale = gib_kib / fe[copy[0]] if copy else 1.0
    wscale = gib_kib / wr[copy[0]] if copy else 1.0
    lines = ["# HBM traffic per dispatch from rocprofv3 --pmc (median over dispatches)",
             f"# command (FETCH_SIZE run; the WRITE_SIZE run is the same with --pmc WRITE_SIZE):",
             f"#   {command}",
             "# scale factors from the probe's copy kernel (1 GiB read, 1 GiB written):",
             f"fetch_scale {fscale:.4f}", f"write_scale {wscale:.4f}",
             f"spmv_source_sha256 {spmv_source_sha()}",
             "# kernel grid fetch_kib write_kib scaled_bytes"]
    for k in sorted(fe):
        name, grid = k
        if not (name.startswith("k_csr") or name.startswith("k_coo") or name.startswith("k_ell")
                or name.startswith("k_probe")):
            continue
        f_ = fe[k]
        w_ = wr.get(k, 0.0)
        total = (f_ * fscale + w_ * wscale) * 1024.0
        lines.append(f"{name.replace(' ', '')} {grid} {f_:.1f} {w_:.1f} {total:.0f}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def load_traffic(path: str) -> dict:
    """{(kernel, grid): bytes} if the file matches the current spmv.hip."""
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return {}
    sha = None
    out = {}
    for ln in lines:
        if ln.startswith("spmv_source_sha256"):
            sha = ln.split()[1]
        elif ln and not ln.startswith("#") and not ln.startswith(("fetch_scale", "write_scale")):
            p = ln.split()
            if len(p) == 5:
                out[(p[0], int(p[1]))] = float(p[4])
    return out if sha == spmv_source_sha() else {}


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
    else:
        raise SystemExit(__doc__)

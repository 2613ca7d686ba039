"""Turns rocprofv3 CSV output into the short text summaries kept in profiles/.

  python -m paper_2103_10116_amd.profile_summary stats <kernel_trace.csv> <out.md> "<command>"
  python -m paper_2103_10116_amd.profile_summary traffic <fetch_counter.csv> \
      <write_counter.csv> <out.txt> "<command>" [probe_bytes]
  python -m paper_2103_10116_amd.profile_summary counters <out.txt> "<command>" \
      <pass1.csv> [<pass2.csv> ...]

`stats` lists every kernel (grouped by name and grid size) with its call
count and mean / median duration.  `traffic` records FETCH_SIZE and
WRITE_SIZE per dispatch (KiB) for the SpMV and CG kernels, the scale factors
measured on the HBM probe's copy kernel (it reads and writes probe_bytes,
the probe's array size), and the SHA-256 of spmv.hip at measurement time, so that a later reader can tell
whether the counters still describe the current kernels.  `counters` merges
the passes of one workload (one counter set per run) into one table per
kernel and grid, with the ratios derived from them: L2 hit rate, mean
latency of the vector cache's L2 reads and of the L2's reads beyond it (by
Little's law from the accumulated in-flight level), the share of those that
went to DRAM, resident waves per CU, and the shares of time the address unit
was stalled by the vector cache and the vector cache waited on pending
misses.
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
          always=("k_csr", "k_coo", "k_ell", "k_cg")) -> None:
    """Per-kernel summary: the `top` kernel/grid pairs by total time, then
    every SpMV or CG kernel (names starting with one of `always`) not among
    them."""
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


def traffic(fetch_csv: str, write_csv: str, out: str, command: str,
            probe_bytes: int = 1 << 30) -> None:
    """probe_bytes: the array size of the probe run in the same command (its
    copy kernel reads and writes that many bytes)."""
    fe = _counters(fetch_csv)
    wr = _counters(write_csv)
    copy = [k for k in fe if k[0] == "k_probe_copy1"]
    probe_kib = float(probe_bytes) / 1024.0
    fscale = probe_kib / fe[copy[0]] if copy else 1.0
    wscale = probe_kib / wr[copy[0]] if copy else 1.0
    lines = ["# HBM traffic per dispatch from rocprofv3 --pmc (median over dispatches)",
             f"# command (FETCH_SIZE run; the WRITE_SIZE run is the same with --pmc WRITE_SIZE):",
             f"#   {command}",
             f"# scale factors from the probe's copy kernel ({probe_bytes / 2**30:g} GiB read, "
             f"{probe_bytes / 2**30:g} GiB written):",
             f"fetch_scale {fscale:.4f}", f"write_scale {wscale:.4f}",
             f"spmv_source_sha256 {spmv_source_sha()}",
             "# kernel grid fetch_kib write_kib scaled_bytes"]
    for k in sorted(fe):
        name, grid = k
        if not name.startswith(("k_csr", "k_coo", "k_ell", "k_panel", "k_cg", "k_probe")):
            continue
        f_ = fe[k]
        w_ = wr.get(k, 0.0)
        total = (f_ * fscale + w_ * wscale) * 1024.0
        lines.append(f"{name.replace(' ', '')} {grid} {f_:.1f} {w_:.1f} {total:.0f}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _counters_all(paths):
    """{(kernel, grid): {counter: median over dispatches}} over several runs."""
    out = collections.defaultdict(dict)
    for path in paths:
        agg = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            agg[(_short(r["Kernel_Name"]), int(r["Grid_Size"]), r["Counter_Name"])].append(
                float(r["Counter_Value"]))
        for (k, g, c), v in agg.items():
            out[(k, g)][c] = sorted(v)[len(v) // 2]
    return out


def _derived(c: dict, num_cu: int = 256) -> dict:
    d = {}
    if "TCC_HIT_sum" in c and "TCC_MISS_sum" in c:
        t = c["TCC_HIT_sum"] + c["TCC_MISS_sum"]
        d["l2_hit_rate"] = c["TCC_HIT_sum"] / t if t else 0.0
    if c.get("TCP_TCC_READ_REQ_sum"):
        if "TCP_TCC_READ_REQ_LATENCY_sum" in c:
            d["l2_read_latency_cycles"] = c["TCP_TCC_READ_REQ_LATENCY_sum"] / c["TCP_TCC_READ_REQ_sum"]
    if c.get("TCC_EA0_RDREQ_sum"):
        if "TCC_EA0_RDREQ_LEVEL_sum" in c:
            d["beyond_l2_read_latency_cycles"] = c["TCC_EA0_RDREQ_LEVEL_sum"] / c["TCC_EA0_RDREQ_sum"]
        if "TCC_EA0_RDREQ_DRAM_sum" in c:
            d["beyond_l2_reads_to_dram"] = c["TCC_EA0_RDREQ_DRAM_sum"] / c["TCC_EA0_RDREQ_sum"]
    busy = c.get("GRBM_GUI_ACTIVE")
    if busy:
        xcd = busy / 8.0  # the GUI-active count is summed over the 8 XCDs
        if "SQ_WAVE_CYCLES" in c:
            # wave-cycles are counted in units of 4 cycles
            d["resident_waves_per_cu"] = 4.0 * c["SQ_WAVE_CYCLES"] / (xcd * num_cu)
        if "SQ_WAIT_INST_ANY" in c and c.get("SQ_WAVE_CYCLES"):
            d["wave_time_waiting"] = c["SQ_WAIT_INST_ANY"] / c["SQ_WAVE_CYCLES"]
        if "TA_ADDR_STALLED_BY_TC_CYCLES_sum" in c:
            d["ta_stalled_by_vector_cache"] = c["TA_ADDR_STALLED_BY_TC_CYCLES_sum"] / num_cu / xcd
        if "TCP_PENDING_STALL_CYCLES_sum" in c:
            d["vector_cache_pending_stall"] = c["TCP_PENDING_STALL_CYCLES_sum"] / num_cu / xcd
        if "TA_BUSY_avr" in c:
            d["ta_busy"] = c["TA_BUSY_avr"] / xcd
    return d


def counters(out: str, command: str, paths, prefixes=("k_",)) -> None:
    table = _counters_all(paths)
    lines = ["# rocprofv3 --pmc counters per dispatch (median over dispatches), one pass per run",
             f"# command (each pass: --pmc <its counters>): {command}",
             f"# spmv_source_sha256 {spmv_source_sha()}", ""]
    for (name, grid), c in sorted(table.items()):
        if not name.startswith(tuple(prefixes)):
            continue
        lines.append(f"## {name.replace(' ', '')} grid {grid}")
        for k in sorted(c):
            lines.append(f"  {k} {c[k]:.6g}")
        for k, v in _derived(c).items():
            lines.append(f"  = {k} {v:.4g}")
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
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5],
                int(sys.argv[6]) if len(sys.argv) > 6 else 1 << 30)
    elif sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3], sys.argv[4:])
    else:
        raise SystemExit(__doc__)

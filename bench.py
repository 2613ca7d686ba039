"""Benchmark of the SpMV + Krylov hot path on one MI355X.

One timed step = one SpMV y = A x in each of the four formats (CSR, COO,
ELL, hybrid) and both value types (FP64, FP32) on the 27-point stencil
matrix of a 128^3 grid (n = 2,097,152, nnz = 55,742,968), inputs resident
in HBM.  `value` is the step's algorithmic bytes divided by its time.
Alongside, the run measures the attainable HBM bandwidth, every format on
the power-law matrices (n = 2^20, MALL flushed between repetitions), the
Krylov solvers on the 128^3 Poisson and convection-diffusion matrices,
iterative refinement against plain FP64 CG, and the CPU oracle on a
bounded sample.  Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--sections ...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# the all-core host baseline keeps its OpenMP threads next to each other;
# set before any OpenMP runtime reads the environment
os.environ.setdefault("OMP_PROC_BIND", "close")

METRIC = "SpMV GB/s & % HBM roofline; CG solves/s + p99 latency, batched vs plain"
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# algorithmic bytes per product (each array counted once)
# ---------------------------------------------------------------------------
def spmv_bytes(fmt, desc, vb, xb, beta_nonzero=False):
    n, nnz = desc["nrows"], desc["nnz"]
    vec = n * xb * (3 if beta_nonzero else 2)  # x read, y write (+ y read)
    if fmt == "csr":
        return nnz * (vb + 4) + 4 * (n + 1) + vec
    if fmt == "coo":
        return nnz * (vb + 8) + vec
    # ELL and HYB: useful bytes, i.e. the entries they hold, plus vectors
    if fmt == "ell":
        return nnz * (vb + 4) + vec
    K, stride, cn = desc["ell_width"], desc["ell_stride"], desc["coo_nnz"]
    return (nnz - cn) * (vb + 4) + cn * (vb + 8) + vec


def ell_streamed_bytes(desc, vb, xb):
    return desc["ell_width"] * desc["ell_stride"] * (vb + 4) + 2 * desc["nrows"] * xb


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "spmv_stencil27_128_traffic.txt")


# The paper's own measurements on Intel GPUs, quoted as context only (other
# hardware, SuiteSparse matrices): sections "Bandwidth Tests and Roofline
# Performance Model", "SpMV Performance Analysis", "Krylov Solver
# Performance Analysis" and "Platform Portability".
PAPER_CONTEXT = {
    "hardware": {"gen9": "Intel Gen9 UHD P630, 41.6 GB/s theoretical, ~37 GB/s BabelStream",
                 "gen12": "Intel Gen12 Iris Xe Max (DG1), 68 GB/s theoretical, ~58 GB/s BabelStream"},
    "spmv_gen9_fp64_gflops": {"csr": 5.1, "coo": 3.8, "csr_roofline": 6.0, "coo_roofline": 4.6},
    "spmv_gen12_fp32": "CSR and COO close to their roofline bounds (14.5 / 9.7 GFLOP/s)",
    "krylov_1000_iters_gflops": {"gen9_fp64": [1.5, 2.5], "gen12_fp32": [5.0, 9.0]},
    "spmv_fraction_of_peak_bw": {"nvidia_and_gen12": 0.9, "radeon_vii_and_gen9": [0.6, 0.7]},
}


def fastest_refinement(rows):
    """The unpreconditioned refinement variant with the shortest solve (the
    comparison with plain FP64 CG is between unpreconditioned solvers), and
    the literal scheme's own figure beside it."""
    cand = {k: v for k, v in rows.items()
            if k.startswith("ir_") and "jacobi" not in k and v.get("status") == 0}
    if not cand:
        return None
    best = min(cand, key=lambda k: cand[k]["time_s"])
    lit = rows.get("ir_f32", {})
    return {"variant": best, "speedup_vs_plain": cand[best]["speedup_vs_plain"],
            "literal_ir_f32_speedup_vs_plain": lit.get("speedup_vs_plain")}


def measured_traffic(fmt, dt, info, max_row):
    """HBM bytes per launch of this SpMV from the committed rocprofv3 --pmc
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel factors), or
    None when the summary predates the current kernels or lacks them."""
    from paper_2103_10116_amd import profile_summary
    table = profile_summary.load_traffic(TRAFFIC_FILE)
    if not table:
        return None
    t = "double,double" if dt == "f64" else "float,float"
    vb = 8 if dt == "f64" else 4
    npl = {256: 4, 512: 8, 1024: 16}.get(info["block_nnz"], 8)
    # the library streams the arrays of a matrix above 256 MiB non-temporally
    # (a template flag of the kernel: part of its name)
    big = lambda nbytes: "true" if nbytes > 256 * (1 << 20) else "false"
    nt_csr = big(info["nnz"] * (4 + vb))
    nt_coo = big(info["coo_nnz"] * (8 + vb))
    nt_ell = big(info["ell_width"] * info["ell_stride"] * (4 + vb))
    wpg = info["waves_per_group"]
    chunked = -(-info["blocks"] // wpg) * 64 * wpg  # threads of the stream/COO grid
    keys = []
    ck = info["csr_kernel"]
    if fmt == "csr" and ck == 4:  # products through LDS
        nt = nt_csr if info["block_nnz"] == 512 else "false"
        keys.append((f"k_csr_pr<{t},{info['block_nnz']},false,{wpg},{nt}>", chunked))
    if fmt == "csr" and ck == 3:  # rows from LDS, two waves per group, G lanes per row
        g = info["lanes_per_row"]
        st = 16 if -(-max_row // g) > 8 else 8  # a lane's entries per step
        nt = nt_csr if info["block_nnz"] == 1024 else "false"
        keys.append((f"k_csr_rl<{t},{info['block_nnz']},false,2,{g},{st},{nt}>",
                     -(-info["blocks"] // 2) * 128))
    if fmt == "csr" and ck == 1:
        keys.append((f"k_csr<{t},{npl},false,{wpg}>", chunked))
    if fmt == "csr" and info["lanes_per_row"] == 1:
        keys.append((f"k_csr_row<{t},false>", -(-info["nrows"] // 256) * 256))
    coo = "k_coo_runs" if info["coo_kernel"] == 2 else "k_coo"
    if coo == "k_coo":
        nt = nt_coo if npl <= 8 else "false"
        coo_args = lambda accum: f"{t},{npl},{accum},{wpg},{nt}"
    else:
        coo_args = lambda accum: f"{t},{npl},{accum},{wpg}"
    if fmt == "coo":
        keys.append((f"{coo}<{coo_args('false')}>", chunked))
    if fmt in ("ell", "hyb"):
        w = 1
        while w < 16 and (info["ell_width"] + w - 1) // w > 256:
            w *= 2
        keys.append((f"k_ell<{t},{w},{nt_ell if w == 1 else 'false'}>", info["ell_stride"] * w))
    if fmt == "hyb" and info["coo_nnz"]:
        keys.append((f"{coo}<{coo_args('true')}>", chunked))
    if not keys or any(k not in table for k in keys):
        return None
    return int(sum(table[k] for k in keys))


class Timer:
    """HIP events on the ctx stream (torch's current stream)."""

    def __init__(self, torch):
        self.torch = torch

    def time(self, fn, reps, flush=None):
        torch = self.torch
        times = []
        if flush is None:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            e1.synchronize()
            return e0.elapsed_time(e1) / reps * 1e-3, None
        for _ in range(reps):
            flush()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1) * 1e-3)
        return float(np.mean(times)), float(np.median(times))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sections", default="probe,spmv,tune,zipf,krylov,ir,pagerank,serve,cpu")
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--plain-requests", type=int, default=10000)
    ap.add_argument("--grid", type=int, default=128, help="stencil grid side (128 = full size)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): sharding over "
              "several GPUs is a design, not built", file=sys.stderr)
        sys.exit(2)
    sections = set(args.sections.split(","))

    import torch
    from paper_2103_10116_amd import inputs as I
    from paper_2103_10116_amd import mxs

    dev = torch.device("cuda:0")
    ctx = mxs.Context(0)
    timer = Timer(torch)
    out = {"metric": METRIC, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic"}
    extra = {"paper_context": PAPER_CONTEXT}
    # GPU solutions (host copies) of the solver rows, keyed by system: the
    # CPU leg solves the same systems with the oracle and reports each row's
    # distance to the oracle's solution
    sols = {}

    # ---------------- HBM probe ----------------
    peak_meas = None
    if "probe" in sections:
        bw = mxs.hbm_probe(ctx, 4 << 30, 5)   # 4 GiB arrays, far beyond the 256 MB cache
        peak_meas = bw["best_gbs"]
        extra["hbm_probe_gbs"] = {k: round(v, 1) for k, v in bw.items()}
        log("hbm probe", extra["hbm_probe_gbs"])

    # ---------------- SpMV step on the 27-point stencil ----------------
    N = args.grid
    log(f"generating 27-point stencil {N}^3")
    A = I.stencil27(N)
    x64 = I.uniform_vector(A.n, I.VECTOR_SEED)
    M = mxs.Matrix.from_host(ctx, A)
    xd = {"f64": torch.from_numpy(x64).to(dev), "f32": torch.from_numpy(x64.astype(np.float32)).to(dev)}
    yd = {"f64": torch.zeros(A.n, dtype=torch.float64, device=dev),
          "f32": torch.zeros(A.n, dtype=torch.float32, device=dev)}
    mats = {}
    for fmt in ("csr", "coo", "ell", "hyb"):
        for dt in ("f64", "f32"):
            mats[(fmt, dt)] = M if (fmt, dt) == ("csr", "f64") else M.convert(fmt, dt)
    per = {}
    step_bytes = 0
    for (fmt, dt), B in mats.items():
        vb = 8 if dt == "f64" else 4
        nbytes = spmv_bytes(fmt, B.info(), vb, vb)
        step_bytes += nbytes
        fn = lambda B=B, dt=dt: mxs.spmv(ctx, B, xd[dt], yd[dt])
        for _ in range(args.warmup):
            fn()
        t, _ = timer.time(fn, max(args.steps, 10))
        per[f"{fmt}_{dt}"] = {"us": round(t * 1e6, 2), "GBs": round(nbytes / t / 1e9, 1),
                              "bytes": nbytes,
                              "frac_spec": round(nbytes / t / 1e9 / PEAK_HBM_GBS, 4)}
        if peak_meas:
            per[f"{fmt}_{dt}"]["frac_measured"] = round(nbytes / t / 1e9 / peak_meas, 4)
        log(f"stencil27 {fmt} {dt}: {t*1e6:.1f} us  {nbytes/t/1e9:.0f} GB/s")

    def step():
        for (fmt, dt), B in mats.items():
            mxs.spmv(ctx, B, xd[dt], yd[dt])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / args.steps
    value = step_bytes / (ms_step * 1e-3) / 1e9
    out.update({"value": round(value, 1), "ms_per_step": round(ms_step, 4)})
    out["config"] = {"workload": f"SpMV y=Ax, 27-point stencil {N}^3 (n={A.n}, nnz={A.nnz}), "
                                 "CSR+COO+ELL+HYB x FP64+FP32 per step",
                     "n": A.n, "nnz": A.nnz, "step_bytes": step_bytes,
                     "wall_s_timed": round(wall, 4)}
    # dominant kernel: the slowest of the step
    dom = max(per, key=lambda k: per[k]["us"])
    d = per[dom]
    fmt_d, dt_d = dom.split("_")
    out["roofline"] = {"bound": "hbm", "kernel": f"spmv_{dom}", "achieved": d["GBs"],
                       "peak": PEAK_HBM_GBS, "unit": "GB/s",
                       "frac": round(d["GBs"] / PEAK_HBM_GBS, 4),
                       "bytes_per_launch": d["bytes"], "us_per_launch": d["us"],
                       "traffic": measured_traffic(fmt_d, dt_d, mats[(fmt_d, dt_d)].info(),
                                                   int(A.row_lengths().max()))}
    if peak_meas:
        out["roofline"]["measured_peak"] = round(peak_meas, 1)
        out["roofline"]["frac_measured"] = round(d["GBs"] / peak_meas, 4)
    extra["stencil27_per_kernel"] = per
    # complex values (CSR only): the same pattern with U[-1,1] imaginary parts
    cx = {}
    zval = A.val + 1j * I.uniform_vector(A.nnz, I.VECTOR_SEED + 1)
    Mz = mxs.Matrix.from_host_complex(ctx, A.n, A.ncols, A.rowptr, A.col, zval)
    for dtz, tdt, vbz in (("c128", torch.complex128, 16), ("c64", torch.complex64, 8)):
        Bz = Mz if dtz == "c128" else Mz.convert("csr", dtz)
        xz = torch.from_numpy(x64 + 0.5j * x64).to(tdt).to(dev)
        yz = torch.zeros(A.n, dtype=tdt, device=dev)
        fn = lambda Bz=Bz, xz=xz, yz=yz: mxs.spmv(ctx, Bz, xz, yz)
        for _ in range(args.warmup):
            fn()
        t, _ = timer.time(fn, max(args.steps, 10))
        nbz = A.nnz * (vbz + 4) + 4 * (A.n + 1) + 2 * A.n * vbz
        cx[f"csr_{dtz}"] = {"us": round(t * 1e6, 2), "GBs": round(nbz / t / 1e9, 1), "bytes": nbz,
                            "GFLOPs": round(8 * A.nnz / t / 1e9, 1),
                            "kernel": Bz.info()["csr_kernel"]}
        log(f"stencil27 csr {dtz}: {t*1e6:.1f} us  {nbz/t/1e9:.0f} GB/s")
        if Bz is not Mz:
            Bz.close()
    Mz.close()
    extra["stencil27_complex"] = cx
    # the byte rule makes the hybrid all ELL on this matrix (K_h = 27); a
    # forced width of 20 measures its COO part at full size (7 entries of
    # every interior row)
    hs = {}
    for dt in ("f64", "f32"):
        vb = 8 if dt == "f64" else 4
        Bh = M.convert("hyb", dt, ell_width=20)
        inf = Bh.info()
        nbh = spmv_bytes("hyb", inf, vb, vb)
        fn = lambda Bh=Bh, dt=dt: mxs.spmv(ctx, Bh, xd[dt], yd[dt])
        for _ in range(args.warmup):
            fn()
        t, _ = timer.time(fn, max(args.steps, 10))
        hs[f"hyb_w20_{dt}"] = {"us": round(t * 1e6, 2), "GBs": round(nbh / t / 1e9, 1),
                               "bytes": nbh, "ell_width": inf["ell_width"],
                               "coo_nnz": inf["coo_nnz"]}
        if peak_meas:
            hs[f"hyb_w20_{dt}"]["frac_measured"] = round(nbh / t / 1e9 / peak_meas, 4)
        log(f"stencil27 hyb (width 20) {dt}: {t*1e6:.1f} us  {nbh/t/1e9:.0f} GB/s")
        Bh.close()
    extra["stencil27_hyb_forced_width"] = hs
    for k in list(mats):
        if k != ("csr", "f64"):
            mats[k].close()
    del mats

    # ---------------- the SpMV autotuner against AUTO on the same matrix ------
    if "tune" in sections:
        from paper_2103_10116_amd import autotune
        tuned = {}
        for fmt in ("csr", "coo"):
            for dt in ("f64", "f32"):
                opts = autotune.tune_spmv(ctx, M, dt, fmt=fmt, refresh=True)
                row = {"tuned_opts": opts}
                for label, o in (("auto", {}), ("tuned", opts)):
                    B = M.convert(fmt, dt, **o)
                    fn = lambda B=B, dt=dt: mxs.spmv(ctx, B, xd[dt], yd[dt])
                    for _ in range(args.warmup):
                        fn()
                    t, _ = timer.time(fn, max(args.steps, 10))
                    row[f"{label}_us"] = round(t * 1e6, 2)
                    row[f"{label}_kernel"] = {k: B.info()[k] for k in
                                              ("csr_kernel", "coo_kernel", "block_nnz",
                                               "lanes_per_row", "waves_per_group")}
                    B.close()
                row["tuned_over_auto"] = round(row["auto_us"] / row["tuned_us"], 3)
                tuned[f"{fmt}_{dt}"] = row
                log(f"autotune stencil27 {fmt} {dt}: auto {row['auto_us']} us, tuned "
                    f"{row['tuned_us']} us {opts}")
        extra["stencil27_spmv_autotune"] = tuned

    # ---------------- power-law matrices, cold (MALL flushed) ----------------
    if "zipf" in sections:
        zres = {}
        for label, s in (("zipf_s2.0", 2.0), ("zipf_s1.79_mean16", 1.79)):
            log(f"generating {label}")
            Z = I.zipf_random(2 ** 20, s, 4096)
            Zm = mxs.Matrix.from_host(ctx, Z)
            zx = {"f64": torch.from_numpy(I.uniform_vector(Z.n, I.VECTOR_SEED)).to(dev)}
            zx["f32"] = zx["f64"].float()
            zy = {"f64": torch.zeros(Z.n, dtype=torch.float64, device=dev),
                  "f32": torch.zeros(Z.n, dtype=torch.float32, device=dev)}
            r = {"nnz": Z.nnz, "max_row": int(Z.row_lengths().max())}
            # columns uniform over all of x: every entry's x load is a cache
            # line of its own, so the random-gather rate bounds the product
            gp = {dt: mxs.gather_probe(ctx, Z.ncols, Z.nnz, vb, 5) for dt, vb in (("f64", 8), ("f32", 4))}
            gp_slice = {}
            r["gather_probe_per_s"] = {dt: round(v / 1e9, 2) for dt, v in gp.items()}
            for fmt in ("csr", "coo", "hyb", "ell"):
                for dt in ("f64", "f32"):
                    B = Zm if (fmt, dt) == ("csr", "f64") else Zm.convert(fmt, dt)
                    vb = 8 if dt == "f64" else 4
                    info = B.info()
                    nbytes = spmv_bytes(fmt, info, vb, vb)
                    fn = lambda B=B, dt=dt: mxs.spmv(ctx, B, zx[dt], zy[dt])
                    fn()
                    t_cold, med = timer.time(fn, 10, flush=lambda: mxs.flush_cache(ctx, 1 << 30))
                    t_warm, _ = timer.time(fn, 10)
                    e = {"cold_us": round(t_cold * 1e6, 2), "cold_GBs": round(nbytes / t_cold / 1e9, 1),
                         "warm_us": round(t_warm * 1e6, 2), "warm_GBs_cache_assisted": round(nbytes / t_warm / 1e9, 1),
                         "bytes": nbytes}
                    # bound: the x gathers at the probe's rate, or the rest of
                    # the bytes at the measured HBM rate, whichever is longer;
                    # with column panels each XCD gathers from one slice of x,
                    # so the probe is taken on an x of the slice's size
                    t_b = (nbytes - Z.ncols * vb) / (peak_meas * 1e9) if peak_meas else 0.0
                    t_g = Z.nnz / gp[dt]
                    panels = info.get("col_panels", 0) if fmt in ("csr", "coo", "hyb") else 0
                    e["gather_bound_full_x_us"] = round(max(t_g, t_b) * 1e6, 2)
                    if panels > 1:
                        key = (dt, panels)
                        if key not in gp_slice:
                            gp_slice[key] = mxs.gather_probe(ctx, -(-Z.ncols // panels), Z.nnz,
                                                             vb, 5)
                        # the hybrid's ELL part gathers over the whole x, its
                        # COO part from the slices
                        sliced = info["coo_nnz"] if fmt == "hyb" else Z.nnz
                        t_g = (Z.nnz - sliced) / gp[dt] + sliced / gp_slice[key]
                        e["col_panels"] = panels
                    e["gather_bound_us"] = round(max(t_g, t_b) * 1e6, 2)
                    e["frac_of_gather_bound"] = round(max(t_g, t_b) / t_cold, 3)
                    if fmt == "ell":
                        e["ell_width"] = info["ell_width"]
                        e["streamed_bytes_if_fully_read"] = ell_streamed_bytes(info, vb, vb)
                    if fmt == "hyb":
                        e["ell_width"] = info["ell_width"]
                        e["coo_nnz"] = info["coo_nnz"]
                    r[f"{fmt}_{dt}"] = e
                    log(f"{label} {fmt} {dt}: cold {t_cold*1e6:.1f} us {nbytes/t_cold/1e9:.0f} GB/s, "
                        f"warm {t_warm*1e6:.1f} us, gather bound {e['gather_bound_us']:.1f} us")
                    if B is not Zm:
                        B.close()
            # y = A x + y (beta = 1: y is read as well), cold, FP64
            for fmt in ("csr", "coo"):
                B = Zm if fmt == "csr" else Zm.convert(fmt, "f64")
                nbytes = spmv_bytes(fmt, B.info(), 8, 8, beta_nonzero=True)
                fn = lambda B=B: mxs.spmv(ctx, B, zx["f64"], zy["f64"], 1.0, 1.0)
                fn()
                t_cold, _ = timer.time(fn, 10, flush=lambda: mxs.flush_cache(ctx, 1 << 30))
                r[f"{fmt}_f64_beta1"] = {"cold_us": round(t_cold * 1e6, 2),
                                         "cold_GBs": round(nbytes / t_cold / 1e9, 1),
                                         "bytes": nbytes}
                log(f"{label} {fmt} f64 beta=1: cold {t_cold*1e6:.1f} us")
                if B is not Zm:
                    B.close()
            Zm.close()
            zres[label] = r
        extra["powerlaw_2p20"] = zres

    # ---------------- Krylov solvers ----------------
    if "krylov" in sections:
        kr = {}
        # 2D Poisson 64x64, b = A * ones (small: launch/latency bound)
        P = I.poisson2d(64)
        Pm = mxs.Matrix.from_host(ctx, P)
        ones = torch.ones(P.n, dtype=torch.float64, device=dev)
        b = torch.zeros(P.n, dtype=torch.float64, device=dev)
        mxs.spmv(ctx, Pm, ones, b)
        xs = torch.zeros_like(b)
        for solver in ("cg", "pipecg"):
            lat = []
            for i in range(25):
                xs.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = mxs.solve(ctx, solver, Pm, b, xs, tol=1e-10)
                lat.append(time.perf_counter() - t0)
            lat = np.array(lat[3:])
            row = f"{solver}_poisson2d_64"
            kr[row] = {"iters": r.iters, "relres_true": r.relres_true,
                       "solves_per_s": round(1.0 / lat.mean(), 1),
                       "p50_ms": round(np.percentile(lat, 50) * 1e3, 3),
                       "p99_ms": round(np.percentile(lat, 99) * 1e3, 3)}
            sols.setdefault("poisson2d_64", {})[("krylov", row)] = xs.cpu().numpy()
            log(row, kr[row])
        # 3D problems at 128^3; the product of each matrix is also timed cold
        # (256 MB cache flushed before each launch) and warm (back to back, as
        # inside a solver, where the previous iteration leaves part of the
        # matrix and vectors in the cache)
        spmv_cw = {}
        for name, gen, solver in (("cg_poisson3d", I.poisson3d, "cg"),
                                  ("pipecg_poisson3d", I.poisson3d, "pipecg"),
                                  ("bicgstab_convdiff3d", I.convdiff3d, "bicgstab"),
                                  ("cgs_convdiff3d", I.convdiff3d, "cgs"),
                                  ("gmres30_convdiff3d", I.convdiff3d, "gmres")):
            Q = gen(N)
            system = "poisson3d_%d" % N if gen is I.poisson3d else "convdiff3d_%d" % N
            Qm = mxs.Matrix.from_host(ctx, Q)
            xstar = torch.from_numpy(I.uniform_vector(Q.n, I.VECTOR_SEED)).to(dev)
            bq = torch.zeros(Q.n, dtype=torch.float64, device=dev)
            mxs.spmv(ctx, Qm, xstar, bq)
            xq = torch.zeros_like(bq)
            csr_b = Q.nnz * 12 + 4 * (Q.n + 1) + 16 * Q.n
            if system not in spmv_cw:
                yq = torch.zeros_like(bq)
                fn = lambda Qm=Qm, yq=yq: mxs.spmv(ctx, Qm, xstar, yq)
                fn()
                t_cold, _ = timer.time(fn, 10, flush=lambda: mxs.flush_cache(ctx, 1 << 30))
                t_warm, _ = timer.time(fn, 20)
                spmv_cw[system] = {
                    "bytes": csr_b, "csr_kernel": Qm.info()["csr_kernel"],
                    "cold_us": round(t_cold * 1e6, 2), "cold_GBs": round(csr_b / t_cold / 1e9, 1),
                    "warm_us": round(t_warm * 1e6, 2),
                    "warm_GBs_cache_assisted": round(csr_b / t_warm / 1e9, 1)}
                if peak_meas:
                    spmv_cw[system]["cold_frac_measured"] = round(csr_b / t_cold / 1e9 / peak_meas, 4)
                log(system, "spmv cold/warm", spmv_cw[system])
            ts = []
            for rep in range(3):
                xq.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = mxs.solve(ctx, solver, Qm, bq, xq, tol=1e-10, restart=30)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            t = float(np.median(ts))
            err = float(torch.linalg.norm(xq - xstar) / torch.linalg.norm(xstar))
            sols.setdefault(system, {})[("krylov", name)] = xq.cpu().numpy()
            # fixed 1000 iterations (no convergence test can stop it), for
            # GFLOP/s and GB/s under the per-iteration models: CG 2nnz+10n
            # flops and B_csr+64n bytes; BiCGSTAB 4nnz+20n and 2B_csr+120n
            # when the products form r_hat.v and (t.s, t.t) (rows-from-LDS
            # CSR: r_hat read by the first product), else 2B_csr+144n;
            # pipelined CG 2nnz+16n and B_csr+104n (q, z, w, s, r, p, x read,
            # z, s, p, x, r, w written); CGS 4nnz+19n and 2B_csr+128n (the
            # product forms r_hat.v), else 2B_csr+136n;
            # GMRES(30) step j 2nnz+8(j+1)n+3n
            # and B_csr+(4(j+1)+9)8n, averaged over j = 0..29
            n_, z_ = Q.n, Q.nnz
            own_dots = Qm.info()["csr_kernel"] == mxs.CSR_ROWS_LDS
            fl, by = {"cg": (2 * z_ + 10 * n_, csr_b + 64 * n_),
                      "pipecg": (2 * z_ + 16 * n_, csr_b + 104 * n_),
                      "bicgstab": (4 * z_ + 20 * n_,
                                   2 * csr_b + (120 if own_dots else 144) * n_),
                      "cgs": (4 * z_ + 19 * n_, 2 * csr_b + (128 if own_dots else 136) * n_),
                      "gmres": (2 * z_ + 8 * 15.5 * n_ + 3 * n_,
                                csr_b + (4 * 15.5 + 9) * 8 * n_)}[solver]
            xq.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rf = mxs.solve(ctx, solver, Qm, bq, xq, tol=0.0, max_iters=1000, restart=30,
                           raise_on_error=False)
            torch.cuda.synchronize()
            tf = time.perf_counter() - t0
            itf = max(rf.iters, 1)
            fixed = {"iters": rf.iters, "status": rf.status, "time_s": round(tf, 4),
                     "ms_per_iter": round(tf / itf * 1e3, 4),
                     "GFLOPs": round(fl * itf / tf / 1e9, 1),
                     "GBs_model": round(by * itf / tf / 1e9, 1),
                     "frac_spec": round(by * itf / tf / 1e9 / PEAK_HBM_GBS, 4)}
            if peak_meas:
                fixed["frac_measured"] = round(by * itf / tf / 1e9 / peak_meas, 4)
                # an iteration re-reads the matrix (217 MB) and the vectors:
                # part of it is served by the 256 MB cache, so this fraction
                # is cache-assisted; the cold product gives the HBM figure
                fixed["cache_assisted"] = True
            kr[name] = {"n": Q.n, "nnz": Q.nnz, "iters": r.iters, "restarts": r.restarts,
                        "relres_true": r.relres_true, "err_vs_xstar": err,
                        "time_s": round(t, 4), "solves_per_s": round(1 / t, 2),
                        "ms_per_iter": round(t / max(r.iters, 1) * 1e3, 4),
                        "spmv_bytes": csr_b, "fixed_1000_iters": fixed}
            log(name, kr[name])
            Qm.close()
        kr["spmv_cold_vs_warm"] = spmv_cw
        extra["krylov"] = kr

    # ---------------- iterative refinement vs plain FP64 CG ----------------
    if "ir" in sections:
        irr = {}
        for name, gen in (("poisson3d_%d" % N, lambda: I.poisson3d(N)),
                          ("random_spd_2p20", lambda: I.random_spd(2 ** 20))):
            log("IR", name)
            Q = gen()
            Qm = mxs.Matrix.from_host(ctx, Q)
            xstar = torch.from_numpy(I.uniform_vector(Q.n, I.VECTOR_SEED)).to(dev)
            bq = torch.zeros(Q.n, dtype=torch.float64, device=dev)
            mxs.spmv(ctx, Qm, xstar, bq)
            xq = torch.zeros_like(bq)
            nxs = float(torch.linalg.norm(xstar))
            store = sols.setdefault(name, {})

            def run(label, fn, reps=3):
                # full solves from x = 0, median wall time of `reps`
                ts = []
                for _ in range(reps):
                    xq.zero_()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    res = fn()
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                store[("iterative_refinement", label)] = xq.cpu().numpy()
                return res, float(np.median(ts)), float(torch.linalg.norm(xq - xstar)) / nxs

            r, t_plain, err = run("plain_f64_cg", lambda: mxs.solve(
                ctx, "cg", Qm, bq, xq, tol=1e-10, raise_on_error=False))
            e = {"plain_f64_cg": {"iters": r.iters, "status": r.status,
                                  "time_s": round(t_plain, 4), "relres_true": r.relres_true,
                                  "err_vs_xstar": err}}
            # preconditioned CG (Jacobi; block Jacobi with 8-row blocks)
            pcs = {"jacobi": mxs.Precond(ctx, Qm, "jacobi"),
                   "block8": mxs.Precond(ctx, Qm, "block_jacobi", 8)}
            for pname, P in pcs.items():
                rp_, t_p, err = run(f"pcg_{pname}_f64", lambda P=P: mxs.solve(
                    ctx, "cg", Qm, bq, xq, tol=1e-10, raise_on_error=False, precond=P))
                e[f"pcg_{pname}_f64"] = {
                    "iters": rp_.iters, "status": rp_.status, "time_s": round(t_p, 4),
                    "relres_true": rp_.relres_true, "speedup_vs_plain": round(t_plain / t_p, 3),
                    "err_vs_xstar": err}
            for low in ("f32", "f16"):
                L = Qm.convert("csr", low)
                ri, t_ir, err = run(f"ir_{low}_jacobi_inner", lambda L=L: mxs.solve_ir(
                    ctx, Qm, L, bq, xq, tol=1e-10, raise_on_error=False, precond=pcs["jacobi"]))
                e[f"ir_{low}_jacobi_inner"] = {
                    "outer": ri.outer_iters, "inner_total": ri.inner_iters_total,
                    "status": ri.status, "relres_true": ri.relres_true,
                    "time_s": round(t_ir, 4), "speedup_vs_plain": round(t_plain / t_ir, 3),
                    "speedup_vs_pcg_jacobi": round(e["pcg_jacobi_f64"]["time_s"] / t_ir, 3),
                    "err_vs_xstar": err}
                L.close()
            for P in pcs.values():
                P.close()
            for low in ("f32", "f16"):
                for carry, variant in ((False, False), (False, True), (True, False),
                                       (True, True)):
                    L = Qm.convert("csr", low)
                    label = (f"ir_{low}{'_carry' if carry else ''}"
                             f"{'_laststep' if variant else ''}")
                    ri, t_ir, err = run(label, lambda L=L, variant=variant, carry=carry:
                                        mxs.solve_ir(ctx, Qm, L, bq, xq, tol=1e-10,
                                                     last_step_variant=variant,
                                                     carry_direction=carry,
                                                     raise_on_error=False))
                    e[label] = {
                        "outer": ri.outer_iters, "inner_total": ri.inner_iters_total,
                        "status": ri.status, "relres_true": ri.relres_true,
                        "time_s": round(t_ir, 4), "speedup_vs_plain": round(t_plain / t_ir, 3),
                        "err_vs_xstar": err}
                    L.close()
            e["fastest_refinement"] = fastest_refinement(e)
            irr[name] = e
            log(name, json.dumps(e))
            Qm.close()
        extra["iterative_refinement"] = irr

    # ---------------- PageRank over the SpMV ----------------
    if "pagerank" in sections:
        prr = {}
        for label, s_ in (("powerlaw_2p20_s1.79", 1.79), ("powerlaw_2p20_s2.0", 2.0)):
            Gh = I.powerlaw_graph(2 ** 20, s_)
            g = mxs.Graph(ctx, Gh)
            xg = torch.zeros(Gh.n, dtype=torch.float64, device=dev)
            e = {"n": Gh.n, "edges": Gh.nnz}
            for fmt in ("csr", "coo", "hyb"):
                op = None if fmt == "csr" else g.transition().convert(fmt, "f64")
                mxs.pagerank(ctx, g, xg, 0.85, 1e-10, op=op)  # warm-up
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = mxs.pagerank(ctx, g, xg, 0.85, 1e-10, op=op)
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
                # per step: the SpMV (format bytes, FP64) + the update (z, x
                # read, x written, one mask byte)
                d = (op or g.transition()).info()
                sp = spmv_bytes(fmt, d, 8, 8)
                step_b = sp + 25 * Gh.n
                e[fmt] = {"iters": r.iters, "delta": r.delta, "time_s": round(t, 4),
                          "ms_per_iter": round(t / r.iters * 1e3, 4),
                          "GBs_model": round(step_b * r.iters / t / 1e9, 1),
                          "bytes_per_step": step_b}
                if op is not None:
                    op.close()
            prr[label] = e
            log("pagerank", label, json.dumps(e))
            g.close()
        extra["pagerank"] = prr

    # ---------------- batched CG serving vs plain CG ----------------
    if "serve" in sections:
        from paper_2103_10116_amd import autotune, serve
        # threads per system of each size class, timed on this GPU (cached)
        t0 = time.perf_counter()
        classes = autotune.tune_batch_classes(ctx, log=log)
        t_tune = time.perf_counter() - t0
        count = args.serve_requests
        closed = I.serving_stream(count, rate=0.0)
        log(f"generating {count} serving systems")
        systems = serve.build_systems(closed)
        sv = {"requests": count, "tol": 1e-10,
              "system": "weighted 5-point Laplacian, m x m grid, m ~ U{8..96}, diagonal shift U[0,1]",
              "classes": [{"max_n": c[0], "threads": c[1]} for c in classes],
              "tune_s": round(t_tune, 2)}
        bkw = dict(budget_bytes=4 << 30, max_slots=2048, iters_per_step=32, classes=classes,
                   staging_bytes=4 << 30)
        # untimed warm-up of both paths (first launches of their kernels)
        serve.run_batched(ctx, closed[:256], systems, **bkw)
        serve.run_batched(ctx, closed[:256], systems, mode="ir32", **bkw)
        serve.run_plain(ctx, closed[:16], systems)
        rb = serve.run_batched(ctx, closed, systems, **bkw)
        sv["batched_closed"] = rb.summary()
        log("batched closed", sv["batched_closed"])
        mu_b = rb.solves_per_s
        # the same requests with FP32 storage inside FP64 refinement
        rbi = serve.run_batched(ctx, closed, systems, mode="ir32", **bkw)
        sv["batched_ir32_closed"] = rbi.summary()
        log("batched ir32 closed", sv["batched_ir32_closed"])
        # admission by footprint: a budget far below what the slots could hold
        # (the systems average ~0.37 MB), so requests wait for memory
        small = dict(bkw, budget_bytes=256 << 20)
        rs = serve.run_batched(ctx, closed, systems, **small)
        sv["batched_closed_budget_256MiB"] = rs.summary()
        log("batched closed, 256 MiB budget", sv["batched_closed_budget_256MiB"])
        nplain = min(count, args.plain_requests)
        rp = serve.run_plain(ctx, closed[:nplain], systems)
        sv["plain_closed"] = rp.summary()
        log("plain closed", sv["plain_closed"])
        mu_p = rp.solves_per_s
        # one open stream both paths can sustain (half the plain path's capacity)
        lam = 0.5 * mu_p
        s_open = I.serving_stream(nplain, rate=lam)
        sv["open_stream_plain_rate"] = {"rate_per_s": round(lam, 2), "requests": nplain,
                                        "batched": serve.run_batched(ctx, s_open, systems, **bkw).summary(),
                                        "plain": serve.run_plain(ctx, s_open, systems).summary()}
        log("open stream at 0.5 x plain capacity", sv["open_stream_plain_rate"])
        # the batched path near its own saturation (the plain path cannot
        # keep up with it: its queue would grow without bound)
        lam_b = 0.9 * mu_b
        s_hi = I.serving_stream(count, rate=lam_b)
        sv["open_stream_batched_rate"] = {"rate_per_s": round(lam_b, 2), "requests": count,
                                          "batched": serve.run_batched(ctx, s_hi, systems, **bkw).summary()}
        log("open stream at 0.9 x batched capacity", sv["open_stream_batched_rate"])
        sv["speedup_solves_per_s"] = round(mu_b / mu_p, 2)
        extra["serving"] = sv

    # ---------------- CPU oracle baseline ----------------
    if "cpu" in sections:
        import oracle
        from concurrent.futures import ThreadPoolExecutor
        hw = _cpu_info()
        nt = hw["threads_used"]
        xs64 = I.uniform_vector(A.n, I.VECTOR_SEED)
        b_csr = spmv_bytes("csr", {"nrows": A.n, "nnz": A.nnz}, 8, 8)

        def spmv_rate(threads, budget_s):
            oracle.use_threads(threads)
            t0 = time.perf_counter()
            reps = 0
            while True:
                oracle.spmv_csr(A, xs64)
                reps += 1
                if time.perf_counter() - t0 > budget_s:
                    break
            return (time.perf_counter() - t0) / reps, reps

        t1, reps1 = spmv_rate(1, 6.0)
        tn, repsn = spmv_rate(nt, 3.0)
        out["cpu_baseline"] = {
            "value": round(b_csr / tn / 1e9, 3), "unit": "GB/s", "cores": nt, "kind": "oracle",
            "sample": f"FP64 CSR products of the 27-point {N}^3 matrix (accurate row sums): "
                      f"{repsn} on {nt} threads ({tn:.4f} s each; OpenMP build of the oracle "
                      f"source, rows split statically) and {reps1} on 1 thread ({t1:.3f} s each)",
            "single_thread_value": round(b_csr / t1 / 1e9, 3),
            "cpu": hw["model"], "physical_cores": hw["physical_cores"],
            "omp_proc_bind": os.environ.get("OMP_PROC_BIND"),
            "logical_cpus": hw["logical_cpus"]}
        log("cpu baseline", out["cpu_baseline"])
        # the oracle's solvers on the same workloads, 1 thread and all
        # threads: whole solves where they take well under a second, else a
        # few iterations timed and reported per iteration
        co = {"cpu": hw["model"], "physical_cores": hw["physical_cores"], "threads": nt,
              "kind": "oracle"}
        P2 = I.poisson2d(64)
        b2 = oracle.spmv_csr(P2, np.ones(P2.n))
        for th in (1, nt):
            oracle.use_threads(th)
            t0 = time.perf_counter()
            nrep = 0
            while time.perf_counter() - t0 < 1.0:
                rc = oracle.cg(P2, b2, tol=1e-10)
                nrep += 1
            t_ = (time.perf_counter() - t0) / nrep
            co[f"cg_poisson2d_64_{th}t"] = {"iters": rc.iters, "s_per_solve": round(t_, 5),
                                            "solves_per_s": round(1.0 / t_, 1)}
        CD = I.convdiff3d(N)
        P3 = I.poisson3d(N)
        for th in (1, nt):
            oracle.use_threads(th)
            for label, Q, fn, its in (("cg_poisson3d", P3, oracle.cg, 4),
                                      ("bicgstab_convdiff3d", CD, oracle.bicgstab, 3),
                                      ("gmres30_convdiff3d_first_steps", CD, oracle.gmres, 8)):
                bq = oracle.spmv_csr(Q, I.uniform_vector(Q.n, I.VECTOR_SEED))
                t0 = time.perf_counter()
                rq = fn(Q, bq, tol=1e-10, maxit=its)
                tq = time.perf_counter() - t0
                co[f"{label}_{N}_{th}t"] = {"iters_timed": rq.iters,
                                            "s_per_iter": round(tq / max(rq.iters, 1), 4)}
        # serving: the first 100 requests by the oracle's CG, one system per
        # thread (the single-thread build; ctypes releases the interpreter
        # lock during each solve)
        oracle.use_threads(1)
        reqs = I.serving_stream(100, rate=0.0)
        sysm = [(I.serving_system(int(r.m), r.seed), I.serving_rhs(r.m * r.m, r.seed))
                for r in reqs]
        for th in (1, nt):
            t0 = time.perf_counter()
            with ThreadPoolExecutor(th) as ex:
                list(ex.map(lambda ab: oracle.cg(ab[0], ab[1], tol=1e-10), sysm))
            ts = time.perf_counter() - t0
            co[f"serving_cg_first_100_{th}t"] = {"solves_per_s": round(len(sysm) / ts, 1)}
        extra["cpu_oracle"] = co
        log("cpu oracle", json.dumps(co))
        # every solver row against the oracle's own solution of its system
        oracle.use_threads(nt)
        refs = attach_oracle_errors(sols, extra, N)
        oracle.use_threads(1)
        extra["oracle_reference_solutions"] = refs
        log("oracle references", json.dumps(refs))
    out["extra"] = extra
    print(json.dumps(out), flush=True)
    M.close()
    ctx.close()


def attach_oracle_errors(sols, extra, N):
    """Adds err_vs_oracle = ||x - x_oracle|| / ||x_oracle|| to every solver
    row whose solution is in `sols` ({system: {(section, row): x}}).  The
    oracle forms b from the same x* itself and solves to 1e-12: CG for the
    SPD Poisson matrices, BiCGSTAB for the convection-diffusion matrix,
    Jacobi-preconditioned CG for the random SPD matrix.  Returns what each
    reference solve took."""
    import oracle
    from paper_2103_10116_amd import inputs as I
    refs = {}
    for system, rows in sols.items():
        if system == "poisson2d_64":
            Q = I.poisson2d(64)
            ref = oracle.cg(Q, oracle.spmv_csr(Q, np.ones(Q.n)), tol=1e-12)
            kind = "cg"
        else:
            if system.startswith("poisson3d"):
                Q, kind = I.poisson3d(N), "cg"
            elif system.startswith("convdiff3d"):
                Q, kind = I.convdiff3d(N), "bicgstab"
            else:
                Q, kind = I.random_spd(2 ** 20), "pcg_jacobi"
            bq = oracle.spmv_csr(Q, I.uniform_vector(Q.n, I.VECTOR_SEED))
            if kind == "cg":
                ref = oracle.cg(Q, bq, tol=1e-12)
            elif kind == "bicgstab":
                ref = oracle.bicgstab(Q, bq, tol=1e-12)
            else:
                _, Mj = oracle.jacobi(Q)
                ref = oracle.pcg(Q, bq, Mj, tol=1e-12)
        nx = float(np.linalg.norm(ref.x))
        refs[system] = {"solver": kind, "iters": ref.iters, "relres_true": ref.relres_true}
        for (sec, row), xg in rows.items():
            tgt = extra[sec][system] if sec == "iterative_refinement" else extra[sec]
            tgt[row]["err_vs_oracle"] = float(np.linalg.norm(xg - ref.x)) / nx
    return refs


def _cpu_info():
    """CPU model, physical cores and logical CPUs this process may run on,
    and the threads the all-core baseline uses (OMP_NUM_THREADS if set,
    else the physical cores available)."""
    model, cores = "unknown", set()
    allowed = os.sched_getaffinity(0)
    try:
        cpu = phys = core = None
        for line in list(open("/proc/cpuinfo")) + [""]:
            if ":" in line:
                k, v = (t.strip() for t in line.split(":", 1))
                if k == "processor":
                    cpu = int(v)
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif k == "model name" and model == "unknown":
                    model = v
            elif cpu is not None:
                if cpu in allowed:
                    cores.add((phys, core))
                cpu = phys = core = None
    except OSError:
        pass
    physical = len(cores) or len(allowed)
    threads = int(os.environ.get("OMP_NUM_THREADS", physical))
    return {"model": model, "physical_cores": physical, "logical_cpus": len(allowed),
            "threads_used": max(1, min(threads, len(allowed)))}


if __name__ == "__main__":
    main()

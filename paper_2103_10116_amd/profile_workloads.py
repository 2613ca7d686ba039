"""Runs named SpMV workloads a few times each, for rocprofv3 counter runs.

  python -m paper_2103_10116_amd.profile_workloads <workload>[,<workload>...] [--reps R]

Workloads (each product is launched R times; "cold" ones evict the 256 MB
Infinity Cache with a 1 GiB read-modify-write pass before every launch, so
each dispatch of the product kernel starts with nothing of the matrix or x
cached beyond L2 residue):

  powerlaw   n = 2^20 power-law matrices, s = 1.79 (mean 16) and s = 2.0:
             CSR FP64 / FP32 / row-scaled FP16 and COO FP64 / FP32, cold
  spd        the random SPD matrix of n = 2^20: CSR FP64 / FP32 / FP16, cold
  stencil27  the 27-point 128^3 matrix: CSR, COO, ELL FP64 and the 7-point
             128^3 CSR FP64 (warm: the 27-point matrix is larger than the cache)
  cold7      the 7-point Poisson and convection-diffusion 128^3 CSR FP64,
             cold and then warm (the cache's share of in-solver products)
  panels     the s = 1.79 power-law matrix, merge-path CSR FP64 and FP32 with
             1, 2 and 4 column panels, cold
  coopanels  both power-law matrices, COO FP64 and FP32 with 1, 2, 4 and 8
             column panels, cold
  probe      the HBM probe (read, copy, triad on 1 GiB arrays): the streaming
             kernels' counters beside the products'
  cg7        CG iterations without a stopping test (tolerance 0, 200 steps)
             on the 7-point Poisson 128^3 in FP64, then the same count as the
             FP32 inner solve of one refinement step
  cgspd      the same FP64 CG iterations on the n = 2^20 random SPD matrix

Prints one line per product (per solve for `cg`) with the mean event-timed
duration, so a counter run's per-dispatch figures can be matched to launches.
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _time(torch, fn, reps, flush=None):
    ts = []
    for _ in range(reps):
        if flush:
            flush()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e3)
    return sum(ts) / len(ts)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workloads")
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    import torch

    from paper_2103_10116_amd import inputs as I
    from paper_2103_10116_amd import mxs

    dev = torch.device("cuda:0")
    ctx = mxs.Context(0)
    flush = lambda: mxs.flush_cache(ctx, 1 << 30)  # noqa: E731

    def run(label, M, variants, cold, **opts):
        x64 = torch.from_numpy(I.uniform_vector(M.n, I.VECTOR_SEED)).to(dev)
        for fmt, dt in variants:
            B = M if (fmt, dt) == ("csr", "f64") and not opts else M.convert(fmt, dt, **opts)
            x = x64 if dt == "f64" else x64.float()
            y = torch.zeros_like(x)
            fn = lambda B=B, x=x, y=y: mxs.spmv(ctx, B, x, y)  # noqa: E731
            fn()
            torch.cuda.synchronize()
            us = _time(torch, fn, args.reps, flush if cold else None)
            print(f"{label} {fmt} {dt} {'cold' if cold else 'warm'}: {us:.1f} us "
                  f"(csr_kernel {B.info()['csr_kernel']}, panels {B.info()['col_panels']})",
                  flush=True)
            if B is not M:
                B.close()

    for w in args.workloads.split(","):
        if w == "powerlaw":
            for s in (1.79, 2.0):
                Z = mxs.Matrix.from_host(ctx, I.zipf_random(2 ** 20, s, 4096))
                run(f"powerlaw_s{s}", Z, [("csr", "f64"), ("csr", "f32"), ("csr", "f16"),
                                          ("coo", "f64"), ("coo", "f32")], True)
                Z.close()
        elif w == "spd":
            S = mxs.Matrix.from_host(ctx, I.random_spd(2 ** 20))
            run("random_spd", S, [("csr", "f64"), ("csr", "f32"), ("csr", "f16")], True)
            S.close()
        elif w == "stencil27":
            T = mxs.Matrix.from_host(ctx, I.stencil27(128))
            run("stencil27_128", T, [("csr", "f64"), ("coo", "f64"), ("ell", "f64")], False)
            T.close()
            P = mxs.Matrix.from_host(ctx, I.poisson3d(128))
            run("poisson3d_128", P, [("csr", "f64")], False)
            P.close()
        elif w == "cold7":
            for label, gen in (("poisson3d_128", I.poisson3d), ("convdiff3d_128", I.convdiff3d)):
                P = mxs.Matrix.from_host(ctx, gen(128))
                run(label, P, [("csr", "f64")], True)
                run(label, P, [("csr", "f64")], False)
                P.close()
        elif w in ("cg7", "cgspd"):
            steps = 200
            label = "poisson3d_128" if w == "cg7" else "random_spd"
            P = mxs.Matrix.from_host(ctx, I.poisson3d(128) if w == "cg7"
                                     else I.random_spd(2 ** 20))
            b = torch.from_numpy(I.uniform_vector(P.n, I.VECTOR_SEED)).to(dev)
            x = torch.zeros_like(b)
            solve = lambda: mxs.solve(ctx, "cg", P, b, x.zero_(), tol=0.0,  # noqa: E731
                                      max_iters=steps, raise_on_error=False)
            solve()
            torch.cuda.synchronize()
            us = _time(torch, solve, args.reps)
            print(f"{label} cg f64: {us / steps:.2f} us per iteration", flush=True)
            if w == "cg7":
                L = P.convert("csr", "f32")
                # one outer step whose inner FP32 CG runs all its steps (an
                # inner tolerance it cannot reach)
                ir = lambda: mxs.solve_ir(ctx, P, L, b, x.zero_(), tol=1e-30,  # noqa: E731
                                          outer_max=1, inner_tol=1e-30, inner_max=steps,
                                          raise_on_error=False)
                ir()
                torch.cuda.synchronize()
                us = _time(torch, ir, args.reps)
                print(f"{label} refinement f32 inner: {us / steps:.2f} us per inner "
                      f"iteration (with one outer step)", flush=True)
                L.close()
            P.close()
        elif w == "probe":
            bw = mxs.hbm_probe(ctx, 1 << 30, 2)
            print("probe", {k: round(v, 1) for k, v in bw.items()}, flush=True)
        elif w == "coopanels":
            for sv in (1.79, 2.0):
                Z = mxs.Matrix.from_host(ctx, I.zipf_random(2 ** 20, sv, 4096))
                for p in (1, 2, 4, 8):
                    run(f"powerlaw_s{sv}_coo_panels{p}", Z, [("coo", "f64"), ("coo", "f32")], True,
                        col_panels=p)
                Z.close()
        elif w == "panels":
            Z = mxs.Matrix.from_host(ctx, I.zipf_random(2 ** 20, 1.79, 4096))
            for p in (1, 2, 4):
                run(f"powerlaw_s1.79_panels{p}", Z, [("csr", "f64"), ("csr", "f32")], True,
                    csr_kernel="merge", col_panels=p)
            Z.close()
        else:
            raise SystemExit(f"unknown workload {w!r}")
    ctx.close()


if __name__ == "__main__":
    main()

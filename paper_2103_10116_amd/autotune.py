"""Autotuner: picks launch shapes by timing candidates on the GPU.

* Batched CG: for each size class, the threads per system (128 ... 1024)
  that solves a batch of systems of that class fastest.
* SpMV: for a CSR matrix, the kernel (row-block stream, lanes-per-row
  vector, thread per row, rows from LDS or products through LDS) and its
  work-unit shape with the shortest product.

Results are cached as JSON keyed by the device name and the problem
signature, so a configuration depends only on the inputs' sizes, never on
what else is running (the batched results stay bitwise reproducible).
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import inputs as I

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "mxs", "autotune.json")
CLASS_BOUNDS = (1024, 2304, 4096, 8192, 10240)
BLOCKS = (128, 256, 512, 1024)


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path, data):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _device_name():
    import torch
    return torch.cuda.get_device_name(0)


def tune_batch_classes(ctx, bounds=CLASS_BOUNDS, per_class=128, tol=1e-10, cache=DEFAULT_CACHE,
                       refresh=False, log=None):
    """Returns [(max_n, block, 0), ...] for mxs.Batch(classes=...)."""
    from . import mxs
    key = f"batch|{_device_name()}|{','.join(map(str, bounds))}|{per_class}"
    data = _load(cache)
    if not refresh and key in data:
        return [tuple(c) for c in data[key]["classes"]]
    chosen = []
    timings = {}
    lo = 0
    for mx in bounds:
        side_hi = int(np.floor(np.sqrt(mx)))
        side_lo = max(2, int(np.floor(np.sqrt(lo))) + 1)
        sides = np.linspace(side_lo, side_hi, per_class).astype(int)
        systems = [I.serving_system(int(m), 1000 + i) for i, m in enumerate(sides)]
        rhs = [I.serving_rhs(A.n, 1000 + i) for i, A in enumerate(systems)]
        best = None
        for blk in BLOCKS:
            if (mx + blk - 1) // blk > 16:
                continue
            # the other classes get one slot each, on the fewest threads
            # that keep their rows per thread within the engine's 16
            classes = [(b_, blk if b_ == mx else next(k for k in BLOCKS if -(-b_ // k) <= 16),
                        per_class if b_ == mx else 1) for b_ in bounds]
            B = mxs.Batch(ctx, 1 << 30, sum(c[2] for c in classes), 32, classes,
                          staging_bytes=64 << 20)
            for A, b in zip(systems, rhs):
                B.submit(A, b, tol)
            t0 = time.perf_counter()
            while True:
                st = B.step()
                if st["active"] == 0 and st["pending"] == 0:
                    break
            t = time.perf_counter() - t0
            B.close()
            timings[f"{mx}:{blk}"] = t
            if log:
                log(f"autotune batch class n<={mx}: {blk} threads/system {t*1e3:.2f} ms")
            if best is None or t < best[1]:
                best = (blk, t)
        chosen.append((mx, best[0], 0))
        lo = mx
    data[key] = {"classes": chosen, "timings_s": timings}
    _save(cache, data)
    return chosen


CSR_CANDIDATES = ([dict(csr_kernel="stream", block_nnz=b) for b in (256, 512, 1024)] +
                  [dict(csr_kernel="vector", lanes_per_row=g, rows_per_group=r)
                   for g in (4, 8, 16, 32) for r in (4, 8)] +
                  [dict(csr_kernel="vector", lanes_per_row=1)] +
                  [dict(csr_kernel="rows_lds", block_nnz=b, lanes_per_row=g)
                   for b in (512, 1024) for g in (1, 2)] +
                  [dict(csr_kernel="products", block_nnz=b) for b in (512, 1024)] +
                  [dict(csr_kernel="merge", block_nnz=b) for b in (256, 512)])

COO_CANDIDATES = [dict(coo_kernel=k, block_nnz=b, waves_per_group=w)
                  for k in ("lds", "runs") for b in (256, 512, 1024) for w in (1, 4)]
CANDIDATES = {"csr": CSR_CANDIDATES, "coo": COO_CANDIDATES}


def tune_spmv(ctx, M, dtype="f64", reps=20, cache=DEFAULT_CACHE, signature=None, refresh=False,
              log=None, fmt="csr"):
    """Best convert options for the product of F64 CSR matrix M stored in
    format `fmt` ("csr": kernel, block and lanes; "coo": kernel, chunk and
    work-group shape), timed on this device and cached by matrix signature."""
    import torch
    from . import mxs
    d = M.info()
    sig = signature or f"{d['nrows']}x{d['ncols']}:{d['nnz']}"
    key = f"spmv|{_device_name()}|{sig}|{dtype}" + ("" if fmt == "csr" else f"|{fmt}")
    data = _load(cache)
    if not refresh and key in data:
        return data[key]["opts"]
    tdt = torch.float64 if dtype == "f64" else torch.float32
    x = torch.rand(d["ncols"], dtype=tdt, device="cuda")
    y = torch.zeros(d["nrows"], dtype=tdt, device="cuda")
    best = None
    timings = {}
    for opts in CANDIDATES[fmt]:
        B = M.convert(fmt, dtype, **opts)
        for _ in range(3):
            mxs.spmv(ctx, B, x, y)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            mxs.spmv(ctx, B, x, y)
        e1.record()
        e1.synchronize()
        t = e0.elapsed_time(e1) / reps
        B.close()
        name = json.dumps(opts, sort_keys=True)
        timings[name] = t
        if log:
            log(f"autotune spmv {sig} {dtype} {name}: {t*1e3:.1f} us")
        if best is None or t < best[1]:
            best = (opts, t)
    data[key] = {"opts": best[0], "ms": best[1], "timings_ms": timings}
    _save(cache, data)
    return best[0]

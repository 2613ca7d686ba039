"""bench.py's command-line contract, checked without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_summary_parses():
    """The committed PMC summary parses into (kernel, grid) -> bytes and holds
    the probe's copy kernel, whose scaled traffic is its 2 GiB."""
    sys.path.insert(0, ROOT)
    from paper_2103_10116_amd import profile_summary
    path = os.path.join(ROOT, "profiles", "spmv_stencil27_128_traffic.txt")
    rows = {}
    for ln in open(path).read().splitlines():
        p = ln.split()
        if ln and not ln.startswith("#") and len(p) == 5:
            rows[(p[0], int(p[1]))] = float(p[4])
    assert rows
    copy = [v for (k, _), v in rows.items() if k == "k_probe_copy1"]
    assert copy and abs(copy[0] - 2.0 * (1 << 30)) / (1 << 30) < 1e-3
    assert callable(profile_summary.load_traffic)


def test_traffic_lookup_finds_the_step_kernels():
    """bench.py's traffic lookup finds, in the committed summary, every kernel
    the default step runs on the 27-point matrix (with the shapes AUTO picks
    there), so a renamed kernel shows up here rather than as a null figure."""
    sys.path.insert(0, ROOT)
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    n, nnz = 128 ** 3, 55742968
    coo = {"block_nnz": 512, "waves_per_group": 4, "blocks": -(-nnz // 512), "coo_kernel": 1,
           "csr_kernel": 0, "lanes_per_row": 0, "nrows": n, "ell_width": 0, "ell_stride": n,
           "coo_nnz": nnz}
    ell = dict(coo, ell_width=27, coo_nnz=0, coo_kernel=0)
    for dt in ("f64", "f32"):
        assert bench.measured_traffic("coo", dt, coo, 27), dt
        assert bench.measured_traffic("ell", dt, ell, 27), dt

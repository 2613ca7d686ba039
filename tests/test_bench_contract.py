"""bench.py's command-line contract, checked without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402  (importing it runs nothing: main() is guarded)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_summary_parses():
    """The committed PMC summary parses into (kernel, grid) -> bytes and holds
    the probe's copy kernel, whose scaled traffic is the 4 GiB it reads plus
    the 4 GiB it writes."""
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
    assert copy and abs(copy[0] - 8.0 * (1 << 30)) / (1 << 30) < 1e-3
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
    coo = {"block_nnz": 256, "waves_per_group": 4, "blocks": -(-nnz // 256), "coo_kernel": 1,
           "csr_kernel": 0, "lanes_per_row": 0, "nrows": n, "nnz": nnz, "ell_width": 0,
           "ell_stride": n, "coo_nnz": nnz}
    ell = dict(coo, ell_width=27, coo_nnz=0, coo_kernel=0)
    for dt in ("f64", "f32"):
        assert bench.measured_traffic("coo", dt, coo, 27), dt
        assert bench.measured_traffic("ell", dt, ell, 27), dt


def test_oracle_errors_attach_to_every_solver_row():
    """The CPU leg's err_vs_oracle: each stored GPU solution gets its
    distance to the oracle's solution of the same system (here a small grid,
    with the oracle's own 1e-10 solutions standing in for GPU results)."""
    import numpy as np
    import oracle
    from paper_2103_10116_amd import inputs as I
    N = 10
    P = I.poisson3d(N)
    b = oracle.spmv_csr(P, I.uniform_vector(P.n, I.VECTOR_SEED))
    x_cg = oracle.cg(P, b, tol=1e-10).x
    C = I.convdiff3d(N)
    bc = oracle.spmv_csr(C, I.uniform_vector(C.n, I.VECTOR_SEED))
    x_bi = oracle.bicgstab(C, bc, tol=1e-10).x
    sols = {f"poisson3d_{N}": {("krylov", "cg_poisson3d"): x_cg,
                               ("iterative_refinement", "plain_f64_cg"): x_cg + 1e-3},
            f"convdiff3d_{N}": {("krylov", "bicgstab_convdiff3d"): x_bi}}
    extra = {"krylov": {"cg_poisson3d": {}, "bicgstab_convdiff3d": {}},
             "iterative_refinement": {f"poisson3d_{N}": {"plain_f64_cg": {}}}}
    refs = bench.attach_oracle_errors(sols, extra, N)
    assert refs[f"poisson3d_{N}"]["solver"] == "cg"
    assert refs[f"convdiff3d_{N}"]["relres_true"] <= 1e-12 * (1 + 1e-6)
    assert extra["krylov"]["cg_poisson3d"]["err_vs_oracle"] < 1e-7
    assert extra["krylov"]["bicgstab_convdiff3d"]["err_vs_oracle"] < 1e-7
    e = extra["iterative_refinement"][f"poisson3d_{N}"]["plain_f64_cg"]["err_vs_oracle"]
    assert abs(e - 1e-3 * np.sqrt(P.n) / np.linalg.norm(x_cg)) < 1e-6


def test_cpu_info():
    info = bench._cpu_info()
    assert info["physical_cores"] >= 1 and 1 <= info["threads_used"] <= info["logical_cpus"]
    assert isinstance(info["model"], str)


def test_fastest_refinement_ignores_preconditioned_and_failed_rows():
    rows = {"plain_f64_cg": {"time_s": 1.0, "status": 0},
            "ir_f32_jacobi_inner": {"time_s": 0.01, "speedup_vs_plain": 100.0, "status": 0},
            "ir_f32": {"time_s": 1.1, "speedup_vs_plain": 0.91, "status": 0},
            "ir_f32_carry": {"time_s": 0.9, "speedup_vs_plain": 1.11, "status": 0},
            "ir_f16_carry": {"time_s": 0.5, "speedup_vs_plain": 2.0, "status": 6}}
    best = bench.fastest_refinement(rows)
    assert best == {"variant": "ir_f32_carry", "speedup_vs_plain": 1.11,
                    "literal_ir_f32_speedup_vs_plain": 0.91}
    assert bench.fastest_refinement({"plain_f64_cg": {"time_s": 1.0}}) is None

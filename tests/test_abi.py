"""The C-ABI library loads on the CPU and exports every function the header
declares; the binding declares exactly those names.  No GPU call is made."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "mxs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mxs_\w+)\s*\(", text)))


def test_library_exports_every_declared_function():
    from paper_2103_10116_amd import mxs
    lib = ctypes.CDLL(mxs.LIB_PATH)
    names = header_functions()
    assert len(names) >= 17
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(mxs.exported_symbols()) == names


def test_host_only_functions():
    from paper_2103_10116_amd import mxs
    assert mxs.version().startswith("mxs")
    assert mxs.status_string(mxs.OK) == "MXS_OK"
    assert mxs.status_string(mxs.NOT_CONVERGED) == "MXS_NOT_CONVERGED"
    assert mxs.status_string(99) == "MXS_UNKNOWN"


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import importlib.util
    import pytest
    src = os.path.join(ROOT, "paper_2103_10116_amd", "mxs.py")
    dst = tmp_path / "mxs.py"
    dst.write_text(open(src).read())
    spec = importlib.util.spec_from_file_location("mxs_copy", str(dst))
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError):
        spec.loader.exec_module(mod)


def test_binding_structs_match_header(tmp_path):
    """Every struct the binding passes by pointer has the header's size and
    field offsets (a C program built from the header prints them)."""
    import subprocess
    import numpy as np
    from paper_2103_10116_amd import mxs
    pairs = {"mxs_allocator": mxs.Allocator, "mxs_convert_opts": mxs.ConvertOpts,
             "mxs_matrix_desc": mxs.MatrixDesc, "mxs_stop": mxs.Stop,
             "mxs_solver_opts": mxs.SolverOpts, "mxs_solve_info": mxs.SolveInfo,
             "mxs_ir_info": mxs.IRInfo, "mxs_batch_opts": mxs.BatchOpts,
             "mxs_batch_stats": mxs.BatchStats, "mxs_bw_result": mxs.BwResult}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mxs.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    req = mxs.Batch._REQ
    lines.append('  printf("mxs_batch_request size %zu\\n", sizeof(mxs_batch_request));')
    for f in req.names:
        lines.append(f'  printf("mxs_batch_request {f} %zu\\n", offsetof(mxs_batch_request, {f}));')
    for macro in ("MXS_IR_LAST_STEP", "MXS_IR_CARRY_DIRECTION"):
        lines.append(f'  printf("define {macro} %d\\n", {macro});')
    lines.append("  return 0;\n}")
    src = tmp_path / "sizes.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(ln.split()[:2]): int(ln.split()[2]) for ln in out if ln}
    for cname, py in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
    assert got[("define", "MXS_IR_LAST_STEP")] == mxs.IR_LAST_STEP
    assert got[("define", "MXS_IR_CARRY_DIRECTION")] == mxs.IR_CARRY_DIRECTION
    assert got[("mxs_batch_request", "size")] == req.itemsize
    for f in req.names:
        assert got[("mxs_batch_request", f)] == req.fields[f][1], f

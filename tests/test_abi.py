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

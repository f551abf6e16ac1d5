"""The C-ABI library loads and exports every symbol its headers declare
(no compute calls: these run without a GPU)."""
import ctypes

import pytest

import paper_2506_08355_amd as L


def test_library_exports_declared_symbols():
    lib = L.lib()
    names = L.declared_symbols()
    assert "lrep_solve" in names and "lrep_submit" in names and "lrep_poll" in names
    assert "lrep_create_dense" in names and "lrep_create_lowrank" in names
    for name in names:
        assert hasattr(lib, name), name


def test_strerror_and_version():
    assert L.lrep_version() == 100
    for code in range(0, -10, -1):
        assert L.lrep_strerror(code)
    assert L.lrep_strerror(-123) == "unknown error"


def test_invalid_arguments_are_rejected_without_device_work():
    lib = L.lib()
    h = ctypes.c_void_p()
    assert lib.lrep_init(None, 0, 0, None) == L.LREP_EINVAL
    assert lib.lrep_init(ctypes.byref(h), -1, 0, None) == L.LREP_EINVAL
    assert lib.lrep_finalize(None) == L.LREP_EINVAL
    assert lib.lrep_solve(None, 1, 1, 1, 1e-8, None, None, None, None, 1, None) == L.LREP_EINVAL
    assert lib.lrep_poll(None, 1, None) == L.LREP_EINVAL
    assert lib.lrep_destroy_op(None) == L.LREP_EINVAL
    assert lib.lrep_create_callback(None, 10, None, None, 0, None) == L.LREP_EINVAL
    assert lib.lrep_set_metric(None, 10, None, 0) == L.LREP_EINVAL
    assert lib.lrep_find_nullspace(None, 4, 1e-10, 0, None, None) == L.LREP_EINVAL
    assert lib.lrep_set_metric_dense(None, 10, None, 10, 0) == L.LREP_EINVAL
    assert lib.lrep_xy_to_uv(None, 10, 1, None, None, 10, None, None, 10) == L.LREP_EINVAL


def test_binding_layout_checks():
    import numpy as np
    with pytest.raises(ValueError):
        L.colmajor(np.zeros((4, 3)))          # C order
    p, ld, dev = L.colmajor(np.zeros((4, 3), order="F"))
    assert ld == 4 and not dev
    torch = pytest.importorskip("torch")
    t = torch.zeros(3, 5, dtype=torch.float64).T
    p, ld, dev = L.colmajor(t)
    assert ld == 5 and not dev


def test_headers_are_c99_and_layouts_match_the_binding(tmp_path):
    """tests/abi_check.c includes both headers as plain C99 (-pedantic, no
    warnings), links the library and prints the struct layouts, which must
    match the ctypes mirrors."""
    import os
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    libdir = os.path.dirname(L.LIB_PATH)
    exe = str(tmp_path / "abi_check")
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                        "-I" + os.path.join(root, "include"), os.path.join(root, "tests", "abi_check.c"),
                        "-o", exe, "-L" + libdir, "-llrep", "-Wl,-rpath," + libdir,
                        "-Wl,--allow-shlib-undefined"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, (r.returncode, r.stderr)
    f = r.stdout.split()
    vals = dict(zip(f[0::2], (int(v) for v in f[1::2])))
    assert vals["opts"] == ctypes.sizeof(L.lrep_solve_opts_t)
    assert vals["stats"] == ctypes.sizeof(L.lrep_stats_t)
    assert vals["request"] == ctypes.sizeof(L.lrep_request_t)
    assert vals["graphs"] == L.lrep_solve_opts_t.graphs.offset
    assert vals["precision"] == L.lrep_solve_opts_t.precision.offset
    assert vals["init_U"] == L.lrep_solve_opts_t.init_U.offset

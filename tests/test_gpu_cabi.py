"""A whole solve driven from plain C through the ABI (tests/abi_solve.c),
with host arrays and no Python binding in between, checked against the
oracle: eigenvalues of the dense n = 256 workload within 1e-10, residual
<= 1e-8 and max |X^T Y - I| <= 1e-12."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import gen
import paper_2506_08355_amd as L
from oracle import exact
from gpu_util import h_residual

pytestmark = pytest.mark.gpu


def test_c_driver_solves_config1(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    libdir = os.path.dirname(L.LIB_PATH)
    exe = str(tmp_path / "abi_solve")
    r = subprocess.run([gcc, "-std=c99", "-O2", "-I" + os.path.join(root, "include"),
                        os.path.join(root, "tests", "abi_solve.c"), "-o", exe, "-L" + libdir, "-llrep",
                        "-Wl,-rpath," + libdir, "-Wl,--allow-shlib-undefined"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    n, nev, block, tol = 256, 8, 16, 1e-10
    K, M, f = gen.dense_operator(n, 1001)
    U, _ = gen.init_block(n, 3 * block, 7)
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(fin, "wb") as fh:
        np.array([n, nev, block, U.shape[1]], dtype=np.int64).tofile(fh)
        np.array([tol], dtype=np.float64).tofile(fh)
        for a in (K, M, U):
            np.asfortranarray(a).ravel(order="F").tofile(fh)
    print("[cabi] running the C driver", flush=True)
    r = subprocess.run([exe, str(fin), str(fout)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    out = np.fromfile(fout, dtype=np.float64)
    lam = out[:nev]
    X = out[nev:nev + n * nev].reshape((n, nev), order="F")
    Y = out[nev + n * nev:].reshape((n, nev), order="F")
    np.testing.assert_allclose(lam, exact.dense_spectrum(f.q1, f.k, f.q2, f.m, nev), rtol=1e-10)
    assert h_residual(lambda v: K @ v, lambda v: M @ v, X, Y, lam, f.norm_H()).max() <= 1e-8
    assert np.abs(X.T @ Y - np.eye(nev)).max() <= 1e-12

"""Host check of the standard form of a real 2x2 Schur block (csrc/std2x2.h, used by the
host Schur code and by the batched restart's device Schur code): M = G M' G^T with G a
rotation, M' upper triangular for real eigenvalues or with equal diagonal and b' c' < 0
for a complex pair, and M' with M's eigenvalues (against numpy)."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2104_01253_amd", "csrc")


@pytest.fixture(scope="module")
def std2x2(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("std2x2")
    src = d / "w.cpp"
    src.write_text('#include "std2x2.h"\n'
                   'extern "C" void std2x2_c(double* v) {\n'
                   '  dcgs2::std2x2(v[0], v[1], v[2], v[3], v[4], v[5]);\n}\n')
    so = d / "w.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC, str(src), "-o",
                    str(so)], check=True)
    lib = ctypes.CDLL(str(so))
    lib.std2x2_c.argtypes = [ctypes.POINTER(ctypes.c_double)]

    def run(M):
        v = (ctypes.c_double * 6)(M[0, 0], M[0, 1], M[1, 0], M[1, 1], 0.0, 0.0)
        lib.std2x2_c(v)
        a, b, c, dd, cs, sn = list(v)
        return np.array([[a, b], [c, dd]]), cs, sn
    return run


def blocks():
    rng = np.random.default_rng(11)
    fixed = [[[1, 2], [3, 4]], [[1, 0], [3, 4]], [[2, -1], [1, 2]], [[2, 1], [-1e-17, 2]],
             [[0, 1], [1e-300, 0]], [[5, 0], [0, 5]], [[1, 1e-12], [-1e-12, 1]],
             [[3, 0], [0, -2]], [[0, -4], [1, 0]], [[1e8, 1], [-1, 1e8]]]
    out = [np.array(b, dtype=float) for b in fixed]
    for _ in range(3000):
        out.append(rng.standard_normal((2, 2)) * 10.0 ** rng.integers(-5, 6))
    return out


def test_standard_form_backward_stable_and_spectrum(std2x2):
    eps = np.finfo(float).eps
    for M in blocks():
        Mp, cs, sn = std2x2(M)
        G = np.array([[cs, -sn], [sn, cs]])
        scale = max(np.linalg.norm(M), 1e-300)
        assert abs(cs * cs + sn * sn - 1.0) <= 4 * eps
        assert np.linalg.norm(G @ Mp @ G.T - M) <= 8 * eps * scale, M
        real = Mp[1, 0] == 0.0
        assert real or (Mp[0, 0] == Mp[1, 1] and Mp[0, 1] * Mp[1, 0] < 0.0), (M, Mp)
        ev = np.sort_complex(np.linalg.eigvals(M))
        evp = np.sort_complex(np.linalg.eigvals(Mp))
        # eigenvalues of a 2x2 block move by at most about sqrt(eps ||M||) near a double one
        tol = 1e-6 * scale + 1e3 * eps * scale
        assert np.max(np.abs(ev - evp)) <= tol, (M, ev, evp)

"""Host real Schur form + reordering used by the Krylov-Schur driver (CPU only).

Pins: eigenvalues against LAPACK (numpy.linalg.eigvals), Z orthogonal,
A = Z T Z^T, T quasi-triangular with standard 2x2 blocks, and the leading
block after reordering holding the largest-magnitude eigenvalues.
"""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2104_01253_amd", "csrc")


@pytest.fixture(scope="module")
def shim():
    d = tempfile.mkdtemp()
    so = os.path.join(d, "schur_shim.so")
    cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", f"-I{CSRC}",
           os.path.join(CSRC, "schur.cpp"), os.path.join(ROOT, "tests", "_schur_shim.cpp"), "-o", so]
    subprocess.run(cmd, check=True)
    lib = ctypes.CDLL(so)
    P = ctypes.c_void_p
    lib.shim_real_schur.argtypes = [ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int]
    lib.shim_reorder.argtypes = [ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_double]
    lib.shim_eigs.argtypes = [ctypes.c_int, P, ctypes.c_int, P, P]
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _schur(lib, A):
    p = A.shape[0]
    T = np.asfortranarray(A.copy())
    Z = np.zeros((p, p), order="F")
    assert lib.shim_real_schur(p, _ptr(T), p, _ptr(Z), p) == 0
    return T, Z


def _check_form(T, Z, A):
    p = A.shape[0]
    assert np.linalg.norm(Z.T @ Z - np.eye(p)) <= 1e-13 * p
    assert np.linalg.norm(Z @ T @ Z.T - A) <= 1e-13 * p * np.linalg.norm(A)
    assert np.all(np.tril(T, -2) == 0.0)
    for i in range(p - 1):
        if T[i + 1, i] != 0.0:                       # standard complex block
            assert T[i, i] == T[i + 1, i + 1]
            assert T[i, i + 1] * T[i + 1, i] < 0
            assert i + 2 >= p or T[i + 2, i + 1] == 0.0


def _eigs(lib, T):
    p = T.shape[0]
    re, im = np.zeros(p), np.zeros(p)
    lib.shim_eigs(p, _ptr(T), p, _ptr(re), _ptr(im))
    return re + 1j * im


def _match(a, b, tol):
    b = list(b)
    for x in a:
        k = int(np.argmin(np.abs(np.array(b) - x)))
        assert abs(b[k] - x) <= tol, (x, b[k])
        b.pop(k)


@pytest.mark.parametrize("p,seed", [(1, 0), (2, 1), (5, 2), (30, 3), (61, 4), (120, 5)])
def test_real_schur_random(shim, p, seed):
    A = np.random.default_rng(seed).standard_normal((p, p))
    T, Z = _schur(shim, A)
    _check_form(T, Z, A)
    scale = max(1.0, np.max(np.abs(np.linalg.eigvals(A))))
    _match(_eigs(shim, T), np.linalg.eigvals(A), 1e-10 * scale)


def test_real_schur_hessenberg_with_full_row(shim):
    """The Krylov-Schur shape: [T_k; b^T] block then Hessenberg columns."""
    g = np.random.default_rng(9)
    p, k = 40, 12
    A = np.triu(g.standard_normal((p, p)), -1)
    A[k, :k] = g.standard_normal(k)
    A[:k, :k] = np.triu(g.standard_normal((k, k)))
    T, Z = _schur(shim, A)
    _check_form(T, Z, A)
    _match(_eigs(shim, T), np.linalg.eigvals(A), 1e-10 * np.max(np.abs(np.linalg.eigvals(A))))


@pytest.mark.parametrize("p,count,seed", [(30, 5, 11), (60, 20, 12), (60, 10, 13), (8, 8, 14)])
def test_reorder_by_magnitude(shim, p, count, seed):
    A = np.random.default_rng(seed).standard_normal((p, p))
    T, Z = _schur(shim, A)
    k = shim.shim_reorder(p, _ptr(T), p, _ptr(Z), p, count, 1e-8)
    assert k >= count
    _check_form(T, Z, A)
    ev = _eigs(shim, T)
    mags = np.abs(ev)
    assert np.min(mags[:k]) >= np.max(mags[k:], initial=0.0) - 1e-12
    assert np.all(np.diff(mags[:k]) <= 1e-10 * mags[0])      # decreasing in the lead block
    # the leading k Schur vectors span an invariant subspace
    Zk = Z[:, :k]
    assert np.linalg.norm(A @ Zk - Zk @ T[:k, :k]) <= 1e-12 * p * np.linalg.norm(A)


def test_reorder_keeps_equal_magnitudes_together(shim):
    # a symmetric-grid style spectrum with exact double eigenvalues
    g = np.random.default_rng(5)
    D = np.diag([9.0, 7.0, 7.0, 5.0, 3.0, 3.0, 1.0])
    V = np.linalg.qr(g.standard_normal((7, 7)))[0]
    A = V @ D @ V.T
    T, Z = _schur(shim, A)
    k = shim.shim_reorder(7, _ptr(T), 7, _ptr(Z), 7, 2, 1e-8)
    assert k == 3

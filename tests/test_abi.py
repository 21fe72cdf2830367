"""The C-ABI library: loads, exports every declared symbol, and validates
arguments before any device work (CPU only; no compute calls)."""
import ctypes
import os
import re

import numpy as np

import pytest

from paper_2104_01253_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dcgs2.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "sizeof")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("dcgs2_qr", "dcgs2_arnoldi", "gmres_solve", "krylov_schur_eigs"):
        assert n in names
    assert set(names) == set(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    for n in declared_functions():
        assert hasattr(lib, n), n


@pytest.fixture()
def ctx():
    lib = binding.load()
    h = ctypes.c_void_p()
    assert lib.dcgs2_create(ctypes.byref(h), 0, None) == binding.OK   # lazy: no device call
    yield lib, h
    lib.dcgs2_destroy(h)


FAKE = 4096          # never dereferenced: validation fails first


def test_qr_argument_validation(ctx):
    lib, h = ctx
    st = binding.Stats()
    E = binding.EINVAL
    assert lib.dcgs2_qr(None, 100, 10, FAKE, 100, FAKE, 100, FAKE, 10, None) == E
    assert lib.dcgs2_qr(h, 10, 20, FAKE, 10, FAKE, 10, FAKE, 20, None) == E      # n > m
    assert lib.dcgs2_qr(h, 100, 0, FAKE, 100, FAKE, 100, FAKE, 10, None) == E    # n < 1
    assert lib.dcgs2_qr(h, 100, 10, FAKE, 99, FAKE, 100, FAKE, 10, None) == E    # ldb < m
    assert lib.dcgs2_qr(h, 100, 10, FAKE, 100, FAKE, 99, FAKE, 10, None) == E    # ldq < m
    assert lib.dcgs2_qr(h, 100, 10, FAKE, 100, FAKE, 100, FAKE, 9, None) == E    # ldr < n
    assert lib.dcgs2_qr(h, 100, 10, None, 100, FAKE, 100, FAKE, 10, None) == E   # null B
    assert lib.dcgs2_qr(h, 5000, 2000, FAKE, 5000, FAKE, 5000, FAKE, 2000, ctypes.byref(st)) == E


def test_arnoldi_gmres_ks_argument_validation(ctx):
    lib, h = ctx
    E = binding.EINVAL
    op = binding.stencil_op((8, 8), 1.0, (1.0, 1.0))
    bad = binding.stencil_op((8, 8), 1.0, (1.0, 1.0))
    bad.m = 63                                                    # nx*ny != m
    H = (ctypes.c_double * 100)()
    assert lib.dcgs2_arnoldi(h, ctypes.byref(bad), FAKE, 5, FAKE, 64, H, 6, None) == E
    assert lib.dcgs2_arnoldi(h, ctypes.byref(op), FAKE, 64, FAKE, 64, H, 65, None) == E  # n >= m
    assert lib.dcgs2_arnoldi(h, ctypes.byref(op), FAKE, 5, FAKE, 64, H, 5, None) == E    # ldh
    assert lib.dcgs2_arnoldi(h, None, FAKE, 5, FAKE, 64, H, 6, None) == E
    assert lib.gmres_solve(h, ctypes.byref(op), FAKE, FAKE, 0, 1e-8, 10, None) == E      # restart
    assert lib.gmres_solve(h, ctypes.byref(op), FAKE, FAKE, 10, 0.0, 10, None) == E      # rtol
    assert lib.gmres_solve(h, ctypes.byref(op), FAKE, FAKE, 10, 1e-8, -1, None) == E
    re_, im_ = (ctypes.c_double * 10)(), (ctypes.c_double * 10)()
    assert lib.krylov_schur_eigs(h, ctypes.byref(op), 10, 30, 10, 1e-8, 5, FAKE, re_, im_, None) == E
    assert lib.krylov_schur_eigs(h, ctypes.byref(op), 5, 64, 10, 1e-8, 5, FAKE, re_, im_, None) == E
    assert lib.krylov_schur_eigs(h, ctypes.byref(op), 5, 30, 10, -1.0, 5, FAKE, re_, im_, None) == E
    ops = (binding.Stencil2d * 2)(binding.stencil2d((8, 8)), binding.stencil2d((6, 5)))
    re2, im2 = (ctypes.c_double * 20)(), (ctypes.c_double * 20)()
    infos = (binding.KsInfo * 2)()
    ksb = lib.krylov_schur_batched
    assert ksb(h, 2, ops, 2, 30, 8, 1e-8, 5, FAKE, re2, im2, infos, 1) == E     # ncv >= 6*5
    assert ksb(h, 0, ops, 2, 20, 8, 1e-8, 5, FAKE, re2, im2, infos, 1) == E     # count < 1
    assert ksb(h, 1, ops, 2, 20, 2, 1e-8, 5, FAKE, re2, im2, infos, 1) == E     # keep <= nev
    assert ksb(h, 1, ops, 2, 20, 8, 0.0, 5, FAKE, re2, im2, infos, 1) == E      # tol
    assert ksb(h, 1, None, 2, 20, 8, 1e-8, 5, FAKE, re2, im2, infos, 1) == E
    csr = binding.Op()
    csr.kind = binding.OP_CSR
    csr.m = 10
    assert lib.dcgs2_apply(h, ctypes.byref(csr), FAKE, FAKE) == E                     # null arrays


def test_tuning_knobs(ctx):
    lib, h = ctx
    v = ctypes.c_int32()
    E = binding.EINVAL
    for key, good, bad in [(binding.TUNE_FUSED_WAVES, (8, 16), (4, 32)),
                           (binding.TUNE_REDUCE_GRID, (0, 1, 1024), (-1, 1025)),
                           (binding.TUNE_FUSED_MIN_J, (0, 16, 1024), (-1, 1025)),
                           (binding.TUNE_BATCH_REDUCE_ROWS, (512, 8192, 65536), (256, 3000, 131072)),
                           (binding.TUNE_FUSED_PAIR_SLOTS, (0, 5, 16), (-1, 17)),
                           (binding.TUNE_BATCH_DENSE, (1, 0), (-1, 2)),
                           (binding.TUNE_MATVEC_FOLD, (0, 1), (-1, 2)),
                           (binding.TUNE_UPDATE_GRID, (0, 1, 512, 65536), (-1, 65537))]:
        for g in good:
            assert lib.dcgs2_set_tuning(h, key, g) == binding.OK
            assert lib.dcgs2_get_tuning(h, key, ctypes.byref(v)) == binding.OK and v.value == g
        for b in bad:
            assert lib.dcgs2_set_tuning(h, key, b) == E
    assert lib.dcgs2_set_tuning(h, 8, 0) == E
    assert lib.dcgs2_get_tuning(h, 8, ctypes.byref(v)) == E


def test_tolerance_validation_and_status_strings(ctx):
    lib, h = ctx
    assert lib.dcgs2_set_tolerances(h, 1e-8, 1e-12) == binding.OK
    assert lib.dcgs2_set_tolerances(h, -1.0, 1e-12) == binding.EINVAL
    assert lib.dcgs2_set_tolerances(h, 1e-8, 1.0) == binding.EINVAL
    assert lib.dcgs2_set_tolerances(None, 1e-8, 1e-12) == binding.EINVAL
    for code in (0, -1, -2, -3, 1, 2, 3):
        assert binding.status_str(code) != "unknown status"
    assert lib.dcgs2_destroy(None) == binding.OK


def test_stencil_coefficients_match_definition():
    c0, lo, hi = binding.stencil_coefficients((32, 32), 1.0, (10.0, 10.0))
    h = 1 / 33
    assert c0 == pytest.approx(4 / h**2)
    assert lo[0] == pytest.approx(-1 / h**2 - 10 / (2 * h))
    assert hi[1] == pytest.approx(-1 / h**2 + 10 / (2 * h))


def test_guess_argument_validation(ctx):
    lib, h = ctx
    E = binding.EINVAL
    out = ctypes.c_void_p()
    w = (ctypes.c_int32 * 3)(8, 0, 4)
    assert lib.dcgs2_mlp_create(h, 2, w, 16, ctypes.byref(out)) == E            # width 0
    w = (ctypes.c_int32 * 3)(8, 5, 4)
    assert lib.dcgs2_mlp_create(h, 2, w, 0, ctypes.byref(out)) == E             # max_batch
    assert lib.dcgs2_mlp_create(None, 2, w, 16, ctypes.byref(out)) == E
    assert lib.dcgs2_mlp_create(h, 0, w, 16, ctypes.byref(out)) == E            # no layer
    assert lib.dcgs2_mlp_forward(None, 1, FAKE, FAKE) == E
    assert lib.dcgs2_mlp_adam(None, 1e-3, 0.9, 0.999, 1e-8) == E
    assert lib.dcgs2_guess_features(h, 1, 30, 4, FAKE, FAKE, 2, 18, FAKE, FAKE) == E   # 30 % 4
    assert lib.dcgs2_guess_features(h, 1, 32, 4, FAKE, FAKE, 2, 17, FAKE, FAKE) == E   # fdim
    assert lib.dcgs2_guess_targets(h, 0, 32, 4, FAKE, FAKE, 1.0, FAKE) == E            # count
    assert lib.dcgs2_guess_targets(h, 1, 32, 4, FAKE, FAKE, 0.0, FAKE) == E            # gain
    assert lib.dcgs2_guess_prolong(h, 1, 32, 1, FAKE, FAKE, 1.0, FAKE) == E            # nc < 2
    assert lib.dcgs2_guess_prolong(h, 1, 32, 4, FAKE, FAKE, -2.0, FAKE) == E           # gain
    op = binding.stencil_op((8, 8), 1.0, (1.0, 1.0))
    kept = ctypes.c_int32()
    assert lib.dcgs2_guess_guard(h, ctypes.byref(op), FAKE, FAKE, 0.0, ctypes.byref(kept),
                                 None) == E                                       # max_ratio


def test_varcoef_csr_matches_the_oracle_assembly():
    import scipy.sparse as sp
    from oracle.operators import varcoef_matrix
    from paper_2104_01253_amd import guess, synth
    for seed, n in [(3, 24), (4, 17)]:
        p = synth.varcoef_instances(1, n=n, seed=seed, vel=(10.0, -4.0))[0]
        rp, ci, va = guess.varcoef_csr(p)
        A = sp.csr_matrix((va, ci, rp), shape=(p.m, p.m))
        B = varcoef_matrix(p)
        assert abs(A - B).max() <= 1e-15 * abs(B).max()
        assert np.all(np.diff(ci.reshape(-1)[rp[0]:rp[1]]) > 0)


def test_steps_argument_validation(ctx):
    """dcgs2_arnoldi_steps / dcgs2_qr_steps reject bad step ranges and layouts."""
    lib, h = ctx
    E = binding.EINVAL
    op = binding.stencil_op((8, 8), 1.0, (1.0, 1.0))
    H = (ctypes.c_double * 4096)()
    K = (ctypes.c_double * 4096)()
    ok = (h, ctypes.byref(op), 3, 5, FAKE, 64, FAKE, H, K, 5, 1.0, None, None)

    def arn(**kw):
        a = list(ok)
        for i, v in kw.items():
            a[int(i[1:])] = v
        return lib.dcgs2_arnoldi_steps(*a)
    assert arn(a2=1) == E                        # j0 < 2
    assert arn(a3=2) == E                        # j1 < j0
    assert arn(a3=65) == E                       # j1 > m
    assert arn(a5=63) == E                       # ldq < m
    assert arn(a9=4) == E                        # ldh < j1
    assert arn(a10=float("nan")) == E            # rho
    assert arn(a10=-1.0) == E
    assert arn(a6=None) == E                     # w
    assert arn(a0=None) == E
    S = (ctypes.c_double * 64)()
    R = (ctypes.c_double * 4096)()
    okq = [h, 100, 3, 5, FAKE, 100, FAKE, 100, FAKE, R, 4, S, 1.0, None, None]

    def qr(**kw):
        a = list(okq)
        for i, v in kw.items():
            a[int(i[1:])] = v
        return lib.dcgs2_qr_steps(*a)
    assert qr(a1=1) == E                         # m < 2
    assert qr(a2=1) == E                         # j0 < 2
    assert qr(a3=101) == E                       # j1 > m
    assert qr(a5=99) == E                        # ldb < m
    assert qr(a7=99) == E                        # ldq < m
    assert qr(a10=3) == E                        # ldr < j1 - 1
    assert qr(a11=None) == E                     # S
    assert qr(a12=float("inf")) == E             # rho


def test_qr_noalloc_argument_validation(ctx):
    """The allocation-free QR rejects sizes beyond its fixed scratch before any device
    call, as well as everything dcgs2_qr rejects."""
    lib, h = ctx
    E = binding.EINVAL
    f = lib.dcgs2_qr_noalloc
    assert f(h, 2 ** 21 + 1, 10, FAKE, 2 ** 21 + 1, FAKE, 2 ** 21 + 1, FAKE, 10, None) == E
    assert f(h, 1000, 129, FAKE, 1000, FAKE, 1000, FAKE, 129, None) == E
    assert f(h, 10, 20, FAKE, 10, FAKE, 10, FAKE, 20, None) == E                  # n > m
    assert f(h, 100, 10, FAKE, 99, FAKE, 100, FAKE, 10, None) == E                # ldb < m
    assert f(None, 100, 10, FAKE, 100, FAKE, 100, FAKE, 10, None) == E

"""Pins for the FP32-stored-basis variant of the oracle (CPU only).

The FP64 oracle (itself pinned) is the reference: storing each basis column in
single precision perturbs the factorisation by O(eps_32) = 6e-8 relative, the
loss of orthogonality sits at the eps_32 level instead of eps_64, and R / H stay
FP64 quantities close to the FP64 ones.  The columns must be exactly representable
in FP32 and the iteration counts of GMRES must not change at these tolerances.
"""
import numpy as np

from oracle import arnoldi as ar
from oracle import gram_schmidt as gs
from oracle import operators as ops
from oracle.gmres import gmres_dcgs2
from oracle.metrics import loss_of_orthogonality, qr_error, representation_error
from paper_2104_01253_amd import synth

EPS32 = np.finfo(np.float32).eps


def test_qr_fp32_basis_against_fp64():
    for ce in (2, 8):
        B = synth.tall_skinny(20000, 60, ce)
        a = gs.dcgs2_qr(B)
        b = gs.dcgs2_qr(B, qdtype=np.float32)
        assert b["Q"].dtype == np.float32 and b["status"] == 0
        Q = b["Q"].astype(np.float64)
        loo = loss_of_orthogonality(Q)
        assert EPS32 / 100 <= loo <= 60 * EPS32, loo          # eps_32 level, not eps_64
        assert np.linalg.norm(b["R"] - a["R"]) / np.linalg.norm(a["R"]) <= 10 * EPS32
        assert qr_error(B, Q, b["R"]) <= 10 * EPS32


def test_arnoldi_fp32_basis_against_fp64():
    prob, r0, n = synth.arnoldi_cd2d_32()
    A = ops.convection_diffusion(prob.grid, prob.D, prob.vel)
    a = ar.dcgs2_arnoldi(lambda x: A @ x, r0, n)
    b = ar.dcgs2_arnoldi(lambda x: A @ x, r0, n, qdtype=np.float32)
    Q = b["Q"].astype(np.float64)
    assert loss_of_orthogonality(Q) <= 60 * EPS32
    assert np.linalg.norm(b["H"] - a["H"]) / np.linalg.norm(a["H"]) <= 10 * EPS32
    assert representation_error(A, Q, b["H"], n) <= EPS32


def test_gmres_fp32_basis_same_convergence():
    prob, bb = synth.gmres_cd3d(16)
    A = ops.convection_diffusion(prob.grid, prob.D, prob.vel)
    x64, i64 = gmres_dcgs2(A, bb)
    x32, i32 = gmres_dcgs2(A, bb, qdtype=np.float32)
    assert i32["relres_true"] <= 1e-8
    assert abs(i32["iters"] - i64["iters"]) <= 2

"""Pins for the QR oracle (CPU only).

What fixes the oracle independently of itself:
  * the unique thin QR with positive R diagonal -- LAPACK Householder (numpy) and
    a 50-digit mpmath Gram-Schmidt on tiny inputs;
  * the loss-of-orthogonality orders of Table loss_of_orth (CGS2 / DCGS2 O(eps),
    MGS O(eps) kappa, CGS O(eps) kappa^2), with one-pass CGS as negative control;
  * the reduction counts of Tables iteration / full (one per column for DCGS2,
    three for CGS2);
  * the readings for the guard, breakdown and non-finite input.
"""
import numpy as np
import pytest

from oracle import gram_schmidt as gs
from oracle.metrics import loss_of_orthogonality, qr_error
from paper_2104_01253_amd import synth
from tests import _brute


def householder_qr(B):
    Qh, Rh = np.linalg.qr(B)
    d = np.sign(np.diag(Rh))
    return Qh * d[None, :], Rh * d[:, None]


@pytest.mark.parametrize("cond_exp", [2, 8])
def test_dcgs2_qr_matches_householder_R(cond_exp):
    B = synth.tall_skinny(20000, 60, cond_exp)
    out = gs.dcgs2_qr(B)
    assert out["status"] == gs.OK and out["k"] == 60
    Qh, Rh = householder_qr(B)
    relR = np.linalg.norm(out["R"] - Rh) / np.linalg.norm(Rh)
    assert relR <= 1e-12, relR
    # (Q - Qh) R: the column space error weighted by R; meaningful at any kappa
    relQR = np.linalg.norm((out["Q"] - Qh) @ Rh) / np.linalg.norm(B)
    assert relQR <= 1e-12, relQR
    if cond_exp <= 2:
        assert np.linalg.norm(out["Q"] - Qh) / np.sqrt(60) <= 1e-12
    assert qr_error(B, out["Q"], out["R"]) <= 1e-14
    assert np.all(np.diag(out["R"]) > 0)


def test_dcgs2_qr_tiny_against_50_digit_gram_schmidt():
    B = synth.tall_skinny(9, 6, 3, seed_g=11, seed_v=12)
    Qx, Rx = _brute.qr_exact(B)
    out = gs.dcgs2_qr(B)
    assert np.max(np.abs(out["Q"] - Qx)) <= 1e-13
    assert np.max(np.abs(out["R"] - Rx)) / np.max(np.abs(Rx)) <= 1e-14
    for f in (gs.cgs2_qr, gs.mgs_qr):
        Q, R, _ = f(B)
        assert np.max(np.abs(Q - Qx)) <= 1e-12


def test_loss_of_orthogonality_orders_kappa_1e8():
    """Table loss_of_orth at kappa(B) ~ 1e8: CGS2 and DCGS2 at O(eps), MGS ~ eps kappa, CGS lost."""
    B = synth.tall_skinny(20000, 100, 8)
    loo = {}
    out = gs.dcgs2_qr(B)
    loo["dcgs2"] = loss_of_orthogonality(out["Q"])
    loo["cgs2"] = loss_of_orthogonality(gs.cgs2_qr(B)[0])
    loo["mgs"] = loss_of_orthogonality(gs.mgs_qr(B)[0])
    loo["cgs"] = loss_of_orthogonality(gs.cgs_qr(B)[0])
    assert loo["dcgs2"] <= 1e-13, loo
    assert loo["cgs2"] <= 1e-13, loo
    assert 1e-11 <= loo["mgs"] <= 1e-6, loo          # ~ eps * kappa
    assert loo["cgs"] >= 1e-3, loo                   # ~ eps * kappa^2: orthogonality lost


def test_dcgs2_matches_cgs2_R():
    B = synth.tall_skinny(20000, 100, 8)
    out = gs.dcgs2_qr(B)
    _, R2, _ = gs.cgs2_qr(B)
    assert np.linalg.norm(out["R"] - R2) / np.linalg.norm(R2) <= 1e-13


def test_reduction_counts():
    """One reduction per column for DCGS2 (n-1 steps + 2 for the last column); 3 for CGS2."""
    n = 30
    B = synth.tall_skinny(3000, n, 4)
    assert gs.dcgs2_qr(B)["reductions"] == n + 1
    assert gs.cgs2_qr(B)[2] == 3 * (n - 1) + 1
    assert gs.mgs_qr(B)[2] == n * (n + 1) // 2
    # one column: the last-column finish has nothing to project out, only a norm
    assert gs.dcgs2_qr(B[:, :1])["reductions"] == 1


def test_forced_pythagorean_fallback_gives_same_factorization():
    """tau >= 1 forces the explicit-norm branch at every step; same QR to rounding."""
    B = synth.tall_skinny(5000, 40, 4)
    a = gs.dcgs2_qr(B)
    b = gs.dcgs2_qr(B, tau=1.0)
    assert b["fallbacks"] == 39 and a["fallbacks"] == 0
    assert b["reductions"] == a["reductions"] + 39
    assert np.linalg.norm(a["R"] - b["R"]) / np.linalg.norm(a["R"]) <= 1e-14
    assert np.linalg.norm(a["Q"] - b["Q"]) <= 1e-12


def test_breakdown_on_dependent_column():
    B = synth.tall_skinny(2000, 8, 2)
    B[:, 3] = B[:, 0] - 2.0 * B[:, 2]
    out = gs.dcgs2_qr(B)
    assert out["status"] == gs.BREAKDOWN
    assert out["k"] == 3
    Qk = out["Q"][:, :3]
    assert loss_of_orthogonality(Qk) <= 1e-14
    # the dependent column is represented in the valid prefix
    assert np.linalg.norm(B[:, 3] - Qk @ out["R"][:3, 3]) <= 1e-12 * np.linalg.norm(B[:, 3])


def test_nonfinite_input():
    B = synth.tall_skinny(500, 6, 2)
    B[17, 4] = np.nan
    out = gs.dcgs2_qr(B)
    assert out["status"] == gs.NONFINITE
    assert out["k"] == 3


def test_single_column():
    B = synth.tall_skinny(100, 1, 0)
    out = gs.dcgs2_qr(B)
    assert out["status"] == gs.OK
    assert np.isclose(out["R"][0, 0], np.linalg.norm(B[:, 0]), rtol=1e-15)

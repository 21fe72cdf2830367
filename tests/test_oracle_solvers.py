"""Pins for the GMRES and Krylov-Schur oracles (CPU only).

GMRES is pinned by a direct sparse solve (scipy spsolve, SuperLU) and by the
true residual; its iteration count is compared with SciPy's own restarted
GMRES, an independent implementation.  Krylov-Schur is pinned by the closed-form
spectrum of the convection-diffusion operator (low cell Peclet, well-conditioned
eigenvalues) and by LAPACK eigvals on a dense random matrix.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import operators as ops
from oracle.gmres import gmres_dcgs2
from oracle.krylov_schur import krylov_schur
from paper_2104_01253_amd import synth


def _scipy_gmres_iters(A, b, restart, rtol):
    count = [0]

    def cb(_):
        count[0] += 1
    spla.gmres(A, b, rtol=rtol, atol=0.0, restart=restart, maxiter=200,
               callback=cb, callback_type="pr_norm")
    return count[0]


def test_gmres_matches_direct_solve_16cube():
    prob, b = synth.gmres_cd3d(16)
    A = ops.convection_diffusion(prob.grid, prob.D, prob.vel)
    x, info = gmres_dcgs2(A, b, restart=50, rtol=1e-8)
    assert info["status"] == 0
    relres = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert relres <= 1e-8
    xs = spla.spsolve(A.tocsc(), b)
    # forward error bounded by cond * residual; cond(A) here is O(1e2)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-5
    it_scipy = _scipy_gmres_iters(A, b, 50, 1e-8)
    assert abs(info["iters"] - it_scipy) <= max(3, 0.05 * it_scipy), (info["iters"], it_scipy)


def test_gmres_zero_rhs_and_warm_start():
    prob, b = synth.gmres_cd3d(8)
    A = ops.convection_diffusion(prob.grid, prob.D, prob.vel)
    x, info = gmres_dcgs2(A, np.zeros_like(b), restart=10)
    assert np.all(x == 0) and info["status"] == 0 and info["iters"] == 0
    xs = spla.spsolve(A.tocsc(), b)
    x, info = gmres_dcgs2(A, b, x0=xs, restart=10)
    assert info["iters"] == 0 and info["status"] == 0


def test_gmres_max_iters_not_converged():
    prob, b = synth.gmres_cd3d(16)
    A = ops.convection_diffusion(prob.grid, prob.D, prob.vel)
    x, info = gmres_dcgs2(A, b, restart=20, rtol=1e-12, max_iters=30)
    assert info["status"] == 2 and info["iters"] == 30 and info["cycles"] == 2


def test_krylov_schur_closed_form_2d():
    """Largest eigenvalues of a low-Peclet 2-D operator (well-conditioned spectrum)."""
    prob = synth.cd2d(24, vel=(4.0, 6.0))
    A = ops.convection_diffusion(prob.grid, prob.D, prob.vel)
    ref = ops.closed_form_eigenvalues(prob.grid, prob.D, prob.vel)[::-1][:10]
    v0 = synth.normal_vector(prob.m, 5)
    ev, info = krylov_schur(A, v0, nev=10, ncv=40, keep=16, tol=1e-10, max_restarts=300)
    assert info["status"] == 0, info
    got = np.sort(ev.real)[::-1]
    assert np.max(np.abs(ev.imag)) <= 1e-6 * np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) / np.max(ref) <= 1e-8, (got, ref)
    assert info["restarts"] >= 1


def test_krylov_schur_dense_random_vs_lapack():
    g = synth.rng(7)
    m = 300
    A = g.standard_normal((m, m)) / np.sqrt(m)
    A[:10, :10] += np.diag(np.linspace(3.0, 5.0, 10))   # separated dominant part
    ev, info = krylov_schur(A, synth.normal_vector(m, 8), nev=6, ncv=30, keep=12, tol=1e-10)
    assert info["status"] == 0
    ref = np.linalg.eigvals(A)
    ref = ref[np.argsort(-np.abs(ref))][:6]
    for lam in ev:
        assert np.min(np.abs(ref - lam)) <= 1e-8 * np.abs(lam)

"""Pins for the Arnoldi oracle and the test operators (CPU only).

What fixes them independently of themselves:
  * Table stab_manteuffel (golden fixture) and eq. eigs_manteuffel evaluated by
    hand (golden fixture) -- pin the operator builder and the closed form;
  * closed-form eigenvalues against LAPACK eigvals -- pin the stencil signs;
  * the exact Arnoldi decomposition by 50-digit Gram-Schmidt on tiny inputs;
  * DCGS2 agreeing with CGS2 (Alg. cgs2_arnoldi) to rounding, O(eps) loss of
    orthogonality and representation error (Sec. 6.1), MGS at O(eps) kappa;
  * eq. (41) on the recorded step quantities (the projection algebra);
  * reduction counts (one per step plus two for the last column);
  * an invariant subspace of dimension 3 giving breakdown with exact Ritz values.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import arnoldi as ar
from oracle import operators as ops
from oracle.metrics import loss_of_orthogonality, representation_error
from paper_2104_01253_amd import synth
from tests import _brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_table(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


def _golden_values(name):
    return np.array([float(l) for l in open(os.path.join(GOLDEN, name))
                     if l.strip() and not l.startswith("#")])


def test_manteuffel_table_values():
    """Table stab_manteuffel: ||A||_2, Cond(A), normality for k=50, beta=0.5, h=1."""
    ref = _golden_table("manteuffel_k50.txt")
    A = ops.manteuffel(50, 0.5).toarray()
    s = np.linalg.svd(A, compute_uv=False)
    assert f"{s[0]:.2e}" == f"{ref['norm2_A']:.2e}"
    assert f"{s[0] / s[-1]:.2e}" == f"{ref['cond_A']:.2e}"
    normality = np.linalg.norm(A.T @ A - A @ A.T) / np.linalg.norm(A) ** 2
    assert f"{normality:.2e}" == f"{ref['normality']:.2e}"


def test_manteuffel_formula_hand_values():
    ref = _golden_values("manteuffel_eigs_k3.txt")
    assert np.allclose(ops.manteuffel_eigenvalues(3, 0.5), ref, rtol=0, atol=1e-14)
    ev = np.sort(np.linalg.eigvals(ops.manteuffel(3, 0.5).toarray()).real)
    assert np.allclose(ev, ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("grid,vel", [((32, 32), (10.0, 10.0)), ((6, 5, 4), (3.0, 7.0, 9.0)),
                                      ((12,), (5.0,))])
def test_closed_form_eigenvalues(grid, vel):
    A = ops.convection_diffusion(grid, 1.0, vel)
    ev = np.linalg.eigvals(A.toarray())
    assert np.max(np.abs(ev.imag)) <= 1e-8 * np.max(np.abs(ev))
    ref = ops.closed_form_eigenvalues(grid, 1.0, vel)
    assert np.max(np.abs(np.sort(ev.real) - ref)) / np.max(ref) <= 1e-11


def test_stencil_row_layout():
    """x fastest: row (ix,iy) couples to ix+-1 with the x coefficients, to iy+-1 with y's."""
    nx, ny, D, vx, vy = 4, 3, 1.0, 2.0, 5.0
    A = ops.convection_diffusion((nx, ny), D, (vx, vy)).toarray()
    hx, hy = 1 / (nx + 1), 1 / (ny + 1)
    i = 1 + nx * 1                      # interior point (1, 1)
    assert np.isclose(A[i, i], 2 * D / hx**2 + 2 * D / hy**2)
    assert np.isclose(A[i, i - 1], -D / hx**2 - vx / (2 * hx))
    assert np.isclose(A[i, i + 1], -D / hx**2 + vx / (2 * hx))
    assert np.isclose(A[i, i - nx], -D / hy**2 - vy / (2 * hy))
    assert np.isclose(A[i, i + nx], -D / hy**2 + vy / (2 * hy))
    assert A[nx - 1, nx] == 0.0          # no wrap-around across the x boundary


def test_dcgs2_arnoldi_tiny_against_50_digit():
    A = synth.rng(21).standard_normal((10, 10)) + 3 * np.eye(10)
    r0 = synth.normal_vector(10, 22)
    n = 6
    Qx, Hx = _brute.arnoldi_exact(A, r0, n)
    out = ar.dcgs2_arnoldi(lambda x: A @ x, r0, n)
    assert out["status"] == ar.OK
    assert np.max(np.abs(out["H"] - Hx)) / np.max(np.abs(Hx)) <= 1e-13
    assert np.max(np.abs(out["Q"] - Qx)) <= 1e-12


def test_config1_dcgs2_vs_cgs2_mgs():
    prob, r0, n = synth.arnoldi_cd2d_32()
    A = ops.convection_diffusion(prob.grid, prob.D, prob.vel)
    mv = lambda x: A @ x
    d = ar.dcgs2_arnoldi(mv, r0, n)
    Q2, H2, red2 = ar.cgs2_arnoldi(mv, r0, n)
    Qm, Hm, _ = ar.mgs_arnoldi(mv, r0, n)
    assert d["status"] == ar.OK and d["k"] == n
    assert np.linalg.norm(d["H"] - H2) / np.linalg.norm(H2) <= 1e-13
    assert np.linalg.norm(d["Q"] - Q2) / np.linalg.norm(Q2) <= 1e-12
    loo_d = loss_of_orthogonality(d["Q"])
    assert loo_d <= 1e-13
    assert loss_of_orthogonality(Q2) <= 1e-13
    assert loss_of_orthogonality(Qm) >= 10 * loo_d      # MGS: O(eps) kappa
    assert representation_error(A, d["Q"], d["H"], n) <= 1e-15
    assert representation_error(A, Q2, H2, n) <= 1e-15
    assert d["reductions"] == n + 2
    assert red2 == 3 * n + 1


def test_eq41_projection_identity():
    """eq. (41): A w_{j-1} = Q_{1:j-2} S + (1/alpha) q_{j-1} (sigma - C^T S) + alpha w_j."""
    prob, r0, n = synth.arnoldi_cd2d_32()
    A = ops.convection_diffusion(prob.grid, prob.D, prob.vel)
    arn = ar.DCGS2Arnoldi(lambda x: A @ x, r0, 20)
    arn.trace = []
    w_prev = r0.copy()
    for _ in range(20):
        arn.step()
        t = arn.trace[-1]
        J = t["j"] - 2
        Aw = A @ w_prev
        rhs = (arn.Q[:, :J] @ t["S"] + arn.Q[:, J] * (t["sigma"] - t["C"] @ t["S"]) / t["alpha"]
               + t["alpha"] * t["w"])
        assert np.linalg.norm(Aw - rhs) <= 1e-13 * np.linalg.norm(Aw)
        w_prev = t["w"]


def test_forced_fallback_same_decomposition():
    prob, r0, n = synth.arnoldi_cd2d_32()
    A = ops.convection_diffusion(prob.grid, prob.D, prob.vel)
    a = ar.dcgs2_arnoldi(lambda x: A @ x, r0, 30)
    b = ar.dcgs2_arnoldi(lambda x: A @ x, r0, 30, tau=1.0)
    assert b["fallbacks"] == 30 and a["fallbacks"] == 0
    assert np.linalg.norm(a["H"] - b["H"]) / np.linalg.norm(a["H"]) <= 1e-14
    assert np.linalg.norm(a["Q"] - b["Q"]) <= 1e-12


def test_breakdown_on_invariant_subspace():
    """r0 in a 3-dimensional invariant subspace: breakdown with k = 3, exact Ritz values."""
    lam = np.arange(1.0, 201.0)
    A = sp.diags(lam).tocsr()
    r0 = np.zeros(200)
    r0[[4, 50, 120]] = [1.0, -2.0, 0.5]
    out = ar.dcgs2_arnoldi(lambda x: A @ x, r0, 10)
    assert out["status"] == ar.BREAKDOWN
    assert out["k"] == 3
    ritz = np.sort(np.linalg.eigvals(out["H"][:3, :3]).real)
    assert np.allclose(ritz, [5.0, 51.0, 121.0], rtol=1e-12)
    assert abs(out["H"][3, 2]) <= 1e-12 * np.linalg.norm(out["H"][:3, :3])


def test_nonfinite_start():
    A = ops.convection_diffusion((8, 8), 1.0, (1.0, 1.0))
    r0 = np.ones(64)
    r0[5] = np.inf
    with np.errstate(invalid="ignore"):      # inf - inf in the products is the point here
        out = ar.dcgs2_arnoldi(lambda x: A @ x, r0, 5)
    assert out["status"] == ar.NONFINITE and out["k"] == 0


def test_krylov_schur_continuation_keeps_arnoldi_relation():
    """After a truncation-style restart, the resumed expansion keeps A Q_p = Q_{p+1} H."""
    prob, r0, _ = synth.arnoldi_cd2d_32()
    A = ops.convection_diffusion(prob.grid, prob.D, prob.vel)
    mv = lambda x: A @ x
    p, k = 30, 10
    a = ar.DCGS2Arnoldi(mv, r0, p).run()
    import scipy.linalg as sla
    T, Z = sla.schur(a.H[:p, :p], output="real")
    if T[k, k - 1] != 0.0:
        k += 1
    Qn = np.zeros_like(a.Q)
    Qn[:, :k] = a.Q[:, :p] @ Z[:, :k]
    Qn[:, k] = a.Q[:, p]
    Hn = np.zeros_like(a.H)
    Hn[:k, :k] = T[:k, :k]
    Hn[k, :k] = a.H[p, p - 1] * Z[p - 1, :k]
    b = ar.DCGS2Arnoldi.resume(mv, Qn, Hn, k, p).run()
    assert b.status == ar.OK
    assert representation_error(A, b.Q, b.H, p) <= 1e-14
    assert loss_of_orthogonality(b.Q) <= 1e-13
    assert b.matvecs == p - k


def test_mgs_arnoldi_tiny_against_50_digit():
    """MGS Arnoldi (Sec. 2) against the exact decomposition by 50-digit Gram-Schmidt:
    a wrong index, sign or dropped projection in H or Q fails it."""
    A = synth.rng(23).standard_normal((10, 10)) + 3 * np.eye(10)
    r0 = synth.normal_vector(10, 24)
    n = 7
    Qx, Hx = _brute.arnoldi_exact(A, r0, n)
    Qm, Hm, red = ar.mgs_arnoldi(lambda x: A @ x, r0, n)
    assert np.max(np.abs(Hm - Hx)) / np.max(np.abs(Hx)) <= 1e-13
    assert np.max(np.abs(Qm - Qx)) <= 1e-12
    assert red == 1 + n * (n + 1) // 2 + n      # j projections + one norm at step j


def test_mgs_arnoldi_relation_and_structure_config1():
    """MGS Arnoldi on the 2-D 32x32 workload: the Arnoldi relation to O(eps) (it holds
    for MGS whatever its orthogonality, Sec. 6.1), H upper Hessenberg with a positive
    subdiagonal, and H equal to the CGS2 Hessenberg matrix to O(eps kappa)."""
    prob, r0, n = synth.arnoldi_cd2d_32()
    A = ops.convection_diffusion(prob.grid, prob.D, prob.vel)
    mv = lambda x: A @ x
    Qm, Hm, _ = ar.mgs_arnoldi(mv, r0, n)
    Q2, H2, _ = ar.cgs2_arnoldi(mv, r0, n)
    assert representation_error(A, Qm, Hm, n) <= 1e-15
    assert np.all(np.tril(Hm, -2) == 0.0)
    assert np.all(np.diag(Hm, -1) > 0.0)
    assert np.allclose(Qm[:, 0], r0 / np.linalg.norm(r0), rtol=0, atol=1e-15)
    colnorm = np.linalg.norm(H2, axis=0)
    assert np.max(np.abs(Hm - H2) / colnorm[None, :]) <= 1e-9
    # loss of orthogonality at the MGS rate O(eps) kappa, far above CGS2's O(eps)
    assert 1e-13 < loss_of_orthogonality(Qm) < 1e-8


def test_varcoef_constant_diffusion_is_the_kronecker_operator():
    """xi = 0 gives D = 1: the flux-form assembly must equal the Kronecker-sum
    convection-diffusion operator built independently (same grid, h and velocity)."""
    from oracle.operators import varcoef_matrix
    for n, vel in [(9, (10.0, 10.0)), (16, (3.0, -7.0))]:
        p = synth.VarCoefProblem(n, (0.0,) * len(synth.KL_MODES), ((0.5, 0.5, 0.1, 1.0),) * 4,
                                 vel)
        A = varcoef_matrix(p)
        B = ops.convection_diffusion((n, n), 1.0, vel)
        assert abs(A - B).max() <= 1e-12 * abs(B).max()


def test_varcoef_symmetric_without_convection():
    """With v = 0 the face-centred diffusion stencil is symmetric for any D(x, y)."""
    from oracle.operators import varcoef_matrix
    p = synth.varcoef_instances(1, n=14, seed=9, vel=(0.0, 0.0))[0]
    A = varcoef_matrix(p)
    assert abs(A - A.T).max() <= 1e-13 * abs(A).max()
    d = A.diagonal()
    off = np.asarray(abs(A).sum(axis=1)).ravel() - np.abs(d)
    assert np.all(d >= off * (1 - 1e-14))         # weakly diagonally dominant (M-matrix)


def test_varcoef_second_order_manufactured_solution():
    """The assembly approximates -div(D grad u) + v.grad u to second order: with
    u = sin(pi x) sin(pi y) (zero on the boundary) the error of A u against the
    analytic operator at the grid points falls by about 4 when h halves.  A misplaced
    face, a swapped axis or a wrong sign leaves an O(1) error instead."""
    from oracle.operators import varcoef_matrix
    xi = synth.rng(31).standard_normal(len(synth.KL_MODES))
    vel = (10.0, -4.0)
    errs = []
    for n in (15, 31, 63):
        p = synth.VarCoefProblem(n, tuple(float(v) for v in xi), ((0.5, 0.5, 0.1, 1.0),) * 4,
                                 vel)
        h = 1.0 / (n + 1)
        t = np.arange(1, n + 1) * h
        X, Y = np.meshgrid(t, t, indexing="xy")       # x fastest
        X, Y = X.ravel(), Y.ravel()
        pi = np.pi
        s = np.zeros_like(X)
        sx = np.zeros_like(X)
        sy = np.zeros_like(X)
        for (pp, qq), z in zip(synth.KL_MODES, xi):
            a = z / (pp * pp + qq * qq) * 2.0
            s += a * np.sin(pp * pi * X) * np.sin(qq * pi * Y)
            sx += a * pp * pi * np.cos(pp * pi * X) * np.sin(qq * pi * Y)
            sy += a * qq * pi * np.sin(pp * pi * X) * np.cos(qq * pi * Y)
        D = np.exp(s)
        u = np.sin(pi * X) * np.sin(pi * Y)
        ux = pi * np.cos(pi * X) * np.sin(pi * Y)
        uy = pi * np.sin(pi * X) * np.cos(pi * Y)
        lap = -2.0 * pi * pi * u
        exact = -(D * sx * ux + D * sy * uy + D * lap) + vel[0] * ux + vel[1] * uy
        Au = varcoef_matrix(p) @ u
        errs.append(np.max(np.abs(Au - exact)) / np.max(np.abs(exact)))
    assert errs[0] < 0.05
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs

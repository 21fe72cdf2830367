"""Krylov-Schur eigensolver on the DCGS2 basis, FP64 (test infrastructure only).

Paper Sec. 6.1: Krylov-Schur relies on the Schur decomposition of the
Hessenberg matrix H_n from the Arnoldi expansion; a Ritz pair is accepted by the
Arnoldi residual ||(A - lambda I) z|| = |H_{n+1,n}| |e_n^T y| (eq. ArnoldiRes).
Stewart's Krylov-Schur restart keeps the wanted part of the Schur form.

Readings (the GPU path implements the same):
  * which = largest magnitude.  A cut never separates two Ritz values whose
    magnitudes differ by less than 1e-8 |theta_1| (so a complex-conjugate pair,
    or an exactly double eigenvalue of a symmetric grid, is never split): the cut
    moves further down until that gap exists.
  * Convergence: with H_p = Z T Z^T (wanted eigenvalues leading) and
    b = h_{p+1,p} Z_{p,:}, the leading nev Schur vectors are converged when
    ||b_{1:nev}||_2 <= tol * min_{i<=nev} |theta_i| -- the backward error of the
    partial Schur form A (Q Z_1) - (Q Z_1) T_11 = q_{p+1} b_1^T, relative to the
    smallest wanted Ritz value (the paper's absolute 1e-7 made relative because
    the workloads have ||A|| up to 1e5).
  * Truncation to k = keep: Q_k <- Q_p Z_{:,1:k}; q_{k+1} <- q_{p+1};
    H_{1:k,1:k} = T_11; H_{k+1,1:k} = b_{1:k}^T; then the DCGS2 expansion resumes
    (DCGS2Arnoldi.resume).
  * The Schur form and its reordering use scipy.linalg.schur with a selection
    function (LAPACK gees/trsen), a library primitive.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .arnoldi import DCGS2Arnoldi, OK, BREAKDOWN, NONFINITE

NOT_CONVERGED = 2
CUT_GAP = 1e-8      # relative magnitude gap required at a truncation / convergence cut


def _block_starts(T):
    """Start indices of the 1x1 / 2x2 diagonal blocks of a real quasi-triangular T."""
    p = T.shape[0]
    starts, i = [], 0
    while i < p:
        starts.append(i)
        i += 2 if (i + 1 < p and T[i + 1, i] != 0.0) else 1
    return starts


def _ordered_schur(Hp, count):
    """Real Schur form with (at least) the `count` largest-|theta| eigenvalues leading.

    Returns (T, Z, kk) where kk >= count is the size of the selected leading
    block (count + 1 when a conjugate pair straddles the cut).
    """
    ev = np.linalg.eigvals(Hp)
    mags = np.sort(np.abs(ev))[::-1]
    # never cut between Ritz values of (nearly) equal magnitude: conjugate pairs
    # and the exact double eigenvalues of symmetric grids
    while count < len(mags) and mags[count - 1] - mags[count] <= CUT_GAP * mags[0]:
        count += 1
    if count >= len(mags):
        T, Z = sla.schur(Hp, output="real")
        return T, Z, len(mags)
    thr = 0.5 * (mags[count - 1] + mags[count])
    T, Z, sdim = sla.schur(Hp, output="real", sort=lambda re, im: np.hypot(re, im) > thr)
    return T, Z, int(sdim)


def krylov_schur(A, v0, nev=10, ncv=60, keep=20, tol=1e-8, max_restarts=200,
                 tau=1e-8, eta=1e-12):
    """Largest-magnitude eigenvalues of A by Krylov-Schur with DCGS2 expansion.

    Returns (eigenvalues (complex, nev of them, by decreasing magnitude), info).
    """
    matvec = A if callable(A) else (lambda x: A @ x)
    p = ncv
    arn = DCGS2Arnoldi(matvec, v0, p, tau, eta).run()
    info = dict(restarts=0, matvecs=arn.matvecs, status=OK, nconv=0, resid=np.inf)
    while True:
        if arn.status != OK:
            info["status"] = arn.status
            return None, info
        Q, H = arn.Q, arn.H
        Hp = H[:p, :p]
        h = H[p, p - 1]
        # convergence test on the leading nev Schur vectors
        T1, Z1, kn = _ordered_schur(Hp, nev)
        b1 = h * Z1[p - 1, :kn]
        theta = np.linalg.eigvals(T1[:kn, :kn])
        resid = np.linalg.norm(b1) / np.min(np.abs(theta))
        info["resid"] = resid
        if resid <= tol:
            info["nconv"] = kn
            order = np.argsort(-np.abs(theta), kind="stable")
            return theta[order][:nev], info
        if info["restarts"] >= max_restarts:
            info["status"] = NOT_CONVERGED
            order = np.argsort(-np.abs(theta), kind="stable")
            return theta[order][:nev], info
        # truncation to the leading `keep` Schur vectors
        T, Z, k = _ordered_schur(Hp, keep)
        Qn = np.zeros_like(Q)
        Qn[:, :k] = Q[:, :p] @ Z[:, :k]
        Qn[:, k] = Q[:, p]
        Hn = np.zeros_like(H)
        Hn[:k, :k] = T[:k, :k]
        Hn[k, :k] = h * Z[p - 1, :k]
        info["restarts"] += 1
        arn = DCGS2Arnoldi.resume(matvec, Qn, Hn, k, p, tau, eta).run()
        info["matvecs"] += arn.matvecs

"""Restarted GMRES on the DCGS2 Arnoldi basis, FP64 (test infrastructure only).

GMRES (Saad & Schultz, cited in Sec. 1) minimises ||b - A x|| over x0 + K_k:
x = x0 + Q_k y with y = argmin || beta e_1 - H_{1:k+1,1:k} y ||, beta = ||r0||.
The small least-squares problem is solved here with numpy.linalg.lstsq (a
library primitive) -- the plain definition -- rather than Givens rotations.

Readings (the GPU path implements the same):
  * x0 = 0 unless given; convergence is judged on the TRUE relative residual
    ||b - A x|| / ||b|| <= rtol; the least-squares residual only ends a cycle early.
  * With DCGS2, H column j-2 is complete after step j, so the estimate for k
    columns is available one matvec after the k-th basis vector.
  * A cycle runs min(restart, max_iters - iters) steps, then the CGS2 last-column
    finish; ``iters`` counts Arnoldi matvecs.
  * b = 0 gives x = 0 and status OK.
  * qdtype=np.float32 stores the basis in single precision; x, r, H, the
    least-squares solve and every reduction stay FP64.
"""
from __future__ import annotations

import numpy as np

from .arnoldi import DCGS2Arnoldi, OK, BREAKDOWN, NONFINITE

NOT_CONVERGED = 2


def _lsq(H, k, beta):
    rhs = np.zeros(k + 1)
    rhs[0] = beta
    y, *_ = np.linalg.lstsq(H[:k + 1, :k], rhs, rcond=None)
    est = np.linalg.norm(rhs - H[:k + 1, :k] @ y)
    return y, est


def gmres_dcgs2(A, b, x0=None, restart=50, rtol=1e-8, max_iters=10000,
                tau=1e-8, eta=1e-12, qdtype=np.float64):
    """Restarted GMRES(restart) with DCGS2 Arnoldi.  A: scipy sparse matrix or callable."""
    matvec = A if callable(A) else (lambda x: A @ x)
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    info = dict(iters=0, cycles=0, status=OK, relres_true=0.0, relres_est=0.0, history=[])
    if bnorm == 0.0:
        x[:] = 0.0
        return x, info
    while True:
        r = b - matvec(x)
        relres = np.linalg.norm(r) / bnorm
        info["relres_true"] = relres
        info["history"].append(relres)
        if relres <= rtol:
            info["status"] = OK
            return x, info
        if info["iters"] >= max_iters:
            info["status"] = NOT_CONVERGED
            return x, info
        n = min(restart, max_iters - info["iters"])
        arn = DCGS2Arnoldi(matvec, r, n, tau, eta, qdtype)
        info["cycles"] += 1
        k = None
        while arn.j <= n + 1:
            st = arn.step()
            info["iters"] += 1
            if st != OK:
                break
            if arn.k >= 1:                      # column arn.k just completed
                y, est = _lsq(arn.H, arn.k, arn.alphas[0])
                if est <= rtol * bnorm:
                    k = arn.k
                    break
        if arn.status == NONFINITE:
            info["status"] = NONFINITE
            return x, info
        if k is None:
            if arn.status == OK:
                arn.finish()
            k = arn.k
        if k == 0:
            info["status"] = NONFINITE if arn.status == NONFINITE else BREAKDOWN
            return x, info
        y, est = _lsq(arn.H, k, arn.alphas[0])
        info["relres_est"] = est / bnorm
        x = x + np.asarray(arn.Q[:, :k], dtype=np.float64) @ y

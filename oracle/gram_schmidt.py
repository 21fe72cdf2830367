"""Left-looking Gram-Schmidt QR variants, FP64 (test infrastructure only).

Paper: Sec. 3 (Alg. cgs2 and Alg. qr), Sec. 2 (MGS), Tables iteration / full
(reduction counts).  Every "reduction" counted here is one global reduction in
the paper's sense: one batch of inner products that would need one
MPI_Allreduce across a row partition.

Inner products use BLAS through NumPy (a library primitive).  No blocking or
reordering beyond what each algorithm states.
"""
from __future__ import annotations

import numpy as np

OK, BREAKDOWN, NONFINITE = 0, 1, 3


def cgs_qr(B):
    """One-pass classical Gram-Schmidt (Sec. 1): project once, then normalise.

    Two reductions per column; loss of orthogonality O(eps) kappa^2 (Table
    loss_of_orth).  Used only as a negative control.
    """
    m, n = B.shape
    Q = np.zeros((m, n), order="F")
    R = np.zeros((n, n))
    red = 0
    for j in range(n):
        a = B[:, j]
        s = Q[:, :j].T @ a                      # reduction 1
        w = a - Q[:, :j] @ s
        alpha = np.linalg.norm(w)               # reduction 2
        red += 2 if j > 0 else 1
        Q[:, j] = w / alpha
        R[:j, j] = s
        R[j, j] = alpha
    return Q, R, red


def cgs2_qr(B):
    """CGS2, Alg. cgs2: two projections then a normalisation (3 reductions/column)."""
    m, n = B.shape
    Q = np.zeros((m, n), order="F")
    R = np.zeros((n, n))
    red = 0
    for j in range(n):
        a = B[:, j]
        Qj = Q[:, :j]
        S = Qj.T @ a                            # first projection   (reduction)
        w = a - Qj @ S
        C = Qj.T @ w                            # second projection  (reduction)
        u = w - Qj @ C
        alpha = np.linalg.norm(u)               # normalisation      (reduction)
        red += 3 if j > 0 else 1
        Q[:, j] = u / alpha
        R[:j, j] = S + C
        R[j, j] = alpha
    return Q, R, red


def mgs_qr(B):
    """Modified Gram-Schmidt (Sec. 2): sequential rank-1 projections, j reductions at column j."""
    m, n = B.shape
    Q = np.zeros((m, n), order="F")
    R = np.zeros((n, n))
    red = 0
    for j in range(n):
        w = B[:, j].copy()
        for i in range(j):
            R[i, j] = Q[:, i] @ w               # one reduction per projection
            w -= R[i, j] * Q[:, i]
            red += 1
        R[j, j] = np.linalg.norm(w)
        red += 1
        Q[:, j] = w / R[j, j]
    return Q, R, red


def _f64(x):
    """FP64 view of stored basis columns (exact widening when Q is stored in FP32)."""
    return np.asarray(x, dtype=np.float64)


def dcgs2_qr(B, tau=1e-8, eta=1e-12, qdtype=np.float64):
    """Delayed CGS2 QR, Alg. qr, with the last column finished by CGS2 (end of Sec. 3).

    Step j (paper's 1-based j = 2..n) finalises q_{j-1} and forms w_j with ONE
    reduction [Q_{1:j-2}, w_{j-1}]^T [w_{j-1}, a_j]:
      C = Q^T w_{j-1}, beta = w^T w, S = Q^T a_j, sigma = w^T a_j  (and a_j^T a_j,
      kept only as the breakdown scale of the next step),
      alpha = sqrt(beta - C^T C)                   (Pythagorean trick, Sec. 3)
      q_{j-1} = (w_{j-1} - Q C) / alpha           (delayed reorthogonalisation)
      S_{j-1,j} = (sigma - C^T S) / alpha         (Stephen's trick, Sec. 3)
      w_j = a_j - Q_{1:j-1} S_{1:j-1,j}
      R_{1:j-2,j-1} = S_{1:j-2,j-1} + C,  R_{j-1,j-1} = alpha.
    Last column: c = Q^T w_n; u = w_n - Q c; alpha = ||u||; two reductions.

    Readings where the paper is silent (both sides implement the same):
    * Pythagorean guard: if not (beta - C^T C > tau*beta), or it is not finite,
      alpha is recomputed explicitly as ||w - Q C|| (one extra reduction).
    * Breakdown: alpha_{j-1} <= eta * ||a_{j-1}||  ->  status BREAKDOWN and the
      first k = j-2 columns of Q and R are the valid prefix.
    * Any non-finite reduced scalar -> status NONFINITE.

    qdtype=np.float32 stores Q in single precision (each q_j rounded once when it
    is written); every product with Q, every reduction, R and the scalars stay
    FP64, and the update uses the stored (rounded) column.

    Returns dict(Q, R, status, k, reductions, fallbacks).
    """
    B = np.asarray(B, dtype=np.float64)
    m, n = B.shape
    Q = np.zeros((m, n), order="F", dtype=qdtype)
    R = np.zeros((n, n))
    red = 0
    fallbacks = 0
    w = B[:, 0].copy()                      # w_1 = a_1
    S_prev = np.zeros(0)                    # S_{1:j-2, j-1}
    gamma_prev = None                       # ||a_{j-1}||^2

    def result(status, k):
        return dict(Q=Q, R=R, status=status, k=k, reductions=red, fallbacks=fallbacks)

    for j in range(2, n + 1):
        J = j - 2                           # columns q_1..q_{j-2} are final
        a = B[:, j - 1]                     # a_j
        Qk = _f64(Q[:, :J])
        # --- the one global reduction of step j
        C = Qk.T @ w
        beta = w @ w
        S = Qk.T @ a
        sigma = w @ a
        gamma = a @ a
        red += 1
        if not (np.all(np.isfinite(C)) and np.all(np.isfinite(S))
                and np.isfinite(beta) and np.isfinite(sigma) and np.isfinite(gamma)):
            return result(NONFINITE, J)
        rho = np.sqrt(beta) if j == 2 else np.sqrt(gamma_prev)   # ||a_{j-1}||
        # --- delayed normalisation (Pythagorean trick) with the explicit fallback
        d = beta - C @ C
        if np.isfinite(d) and d > tau * beta:
            alpha = np.sqrt(d)
        else:
            alpha = np.linalg.norm(w - Qk @ C)
            red += 1
            fallbacks += 1
        if not np.isfinite(alpha):
            return result(NONFINITE, J)
        if alpha <= eta * rho:
            R[:J, J] = S_prev + C
            R[J, J] = alpha
            return result(BREAKDOWN, J)
        # --- delayed reorthogonalisation of column j-1
        Q[:, J] = (w - Qk @ C) / alpha
        # --- projection of a_j, with Stephen's trick for q_{j-1}^T a_j
        s_last = (sigma - C @ S) / alpha
        S_full = np.concatenate([S, [s_last]])
        w = a - _f64(Q[:, :J + 1]) @ S_full
        # --- representation R_{:, j-1}
        R[:J, J] = S_prev + C
        R[J, J] = alpha
        S_prev = S_full
        gamma_prev = gamma

    # --- last column: CGS2 finish, two reductions (end of Sec. 3)
    J = n - 1
    Qk = _f64(Q[:, :J])
    c = Qk.T @ w
    u = w - Qk @ c
    alpha = np.linalg.norm(u)
    red += 2 if J > 0 else 1
    if not (np.all(np.isfinite(c)) and np.isfinite(alpha)):
        return result(NONFINITE, J)
    rho = np.linalg.norm(w) if n == 1 else np.sqrt(gamma_prev)
    if alpha <= eta * rho:
        R[:J, J] = S_prev + c
        R[J, J] = alpha
        return result(BREAKDOWN, J)
    Q[:, J] = u / alpha
    R[:J, J] = S_prev + c
    R[J, J] = alpha
    return result(OK, n)

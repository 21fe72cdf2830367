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


def dcgs2_qr_step(Q, J, w, a, S_prev, rho, tau=1e-8, eta=1e-12):
    """Step j = J + 2 of Alg. qr from a given state (test infrastructure only).

    State: the final columns q_1..q_J in Q[:, :J] (stored values; q_{J+1} is written
    into Q[:, J]), w = w_{j-1}, a = a_j, S_prev = S_{1:J, j-1}, rho = ||a_{j-1}||
    (None at j = 2, where the breakdown scale is ||w_1|| = ||a_1||).  The one global
    reduction of the step is [Q_{1:j-2}, w_{j-1}]^T [w_{j-1}, a_j]:
      C = Q^T w, beta = w^T w, S = Q^T a, sigma = w^T a  (and gamma = a^T a, the
      breakdown scale of the next step),
      alpha = sqrt(beta - C^T C)                   (Pythagorean trick, Sec. 3)
      q_{j-1} = (w_{j-1} - Q C) / alpha           (delayed reorthogonalisation)
      S_{j-1,j} = (sigma - C^T S) / alpha         (Stephen's trick, Sec. 3)
      w_j = a_j - Q_{1:j-1} S_{1:j-1,j}
      R_{1:j-2,j-1} = S_{1:j-2,j-1} + C,  R_{j-1,j-1} = alpha.
    Returns dict(status, C, beta, S, sigma, gamma, alpha, fallback, s_full, w, rcol);
    on OK q_{j-1} is in Q[:, J].
    """
    Qk = _f64(Q[:, :J])
    C = Qk.T @ w
    beta = w @ w
    S = Qk.T @ a
    sigma = w @ a
    gamma = a @ a
    out = dict(status=OK, C=C, beta=beta, S=S, sigma=sigma, gamma=gamma, alpha=None,
               fallback=False, s_full=None, w=None, rcol=None)
    if not (np.all(np.isfinite(C)) and np.all(np.isfinite(S))
            and np.isfinite(beta) and np.isfinite(sigma) and np.isfinite(gamma)):
        out["status"] = NONFINITE
        return out
    if rho is None:
        rho = np.sqrt(beta)                 # j = 2: ||a_1||
    # --- delayed normalisation (Pythagorean trick) with the explicit fallback
    d = beta - C @ C
    if np.isfinite(d) and d > tau * beta:
        alpha = np.sqrt(d)
    else:
        alpha = np.linalg.norm(w - Qk @ C)
        out["fallback"] = True
    out["alpha"] = alpha
    if not np.isfinite(alpha):
        out["status"] = NONFINITE
        return out
    out["rcol"] = np.concatenate([S_prev + C, [alpha]])
    if alpha <= eta * rho:
        out["status"] = BREAKDOWN
        return out
    # --- delayed reorthogonalisation of column j-1
    Q[:, J] = (w - Qk @ C) / alpha
    # --- projection of a_j, with Stephen's trick for q_{j-1}^T a_j
    s_last = (sigma - C @ S) / alpha
    out["s_full"] = np.concatenate([S, [s_last]])
    out["w"] = a - _f64(Q[:, :J + 1]) @ out["s_full"]
    return out


def dcgs2_qr(B, tau=1e-8, eta=1e-12, qdtype=np.float64):
    """Delayed CGS2 QR, Alg. qr, with the last column finished by CGS2 (end of Sec. 3).

    Steps j = 2..n follow ``dcgs2_qr_step`` (one reduction each); the last column
    is finished by CGS2: c = Q^T w_n; u = w_n - Q c; alpha = ||u||; two reductions.

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
        rho = None if j == 2 else np.sqrt(gamma_prev)
        o = dcgs2_qr_step(Q, J, w, B[:, j - 1], S_prev, rho, tau, eta)
        red += 2 if o["fallback"] else 1
        fallbacks += 1 if o["fallback"] else 0
        if o["rcol"] is not None:
            R[:J + 1, J] = o["rcol"]
        if o["status"] != OK:
            return result(o["status"], J)
        w = o["w"]
        S_prev = o["s_full"]
        gamma_prev = o["gamma"]

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

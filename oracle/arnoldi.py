"""Arnoldi-QR expansions, FP64 (test infrastructure only).

Paper: Sec. 4 -- Alg. cgs2_arnoldi (CGS2), the derivation eqs. (08)-(52) and
Alg. arnoldi (DCGS2); Sec. 2 for MGS; the Arnoldi relation eq. (eq:arnoldi)
A Q_{1:k} = Q_{1:k+1} H_{1:k+1,1:k}.

``matvec`` is any callable x -> A x (a scipy.sparse matrix's ``@``).
"""
from __future__ import annotations

import numpy as np

OK, BREAKDOWN, NONFINITE = 0, 1, 3


def _f64(x):
    """FP64 view of stored basis columns (exact widening when Q is stored in FP32)."""
    return np.asarray(x, dtype=np.float64)


def cgs2_arnoldi(matvec, r0, n):
    """Alg. cgs2_arnoldi: v = A q_{j-1}; two projections; normalisation (3 reductions/step)."""
    m = r0.size
    Q = np.zeros((m, n + 1), order="F")
    H = np.zeros((n + 1, n))
    Q[:, 0] = r0 / np.linalg.norm(r0)
    red = 1
    for j in range(1, n + 1):                   # builds q_{j+1} (1-based) from A q_j
        v = matvec(Q[:, j - 1])
        Qj = Q[:, :j]
        S = Qj.T @ v
        w = v - Qj @ S
        C = Qj.T @ w
        u = w - Qj @ C
        alpha = np.linalg.norm(u)
        red += 3
        H[:j, j - 1] = S + C
        H[j, j - 1] = alpha
        Q[:, j] = u / alpha
    return Q, H, red


def mgs_arnoldi(matvec, r0, n):
    """Arnoldi with modified Gram-Schmidt (Sec. 2): one reduction per rank-1 projection."""
    m = r0.size
    Q = np.zeros((m, n + 1), order="F")
    H = np.zeros((n + 1, n))
    Q[:, 0] = r0 / np.linalg.norm(r0)
    red = 1
    for j in range(1, n + 1):
        w = matvec(Q[:, j - 1])
        for i in range(j):
            H[i, j - 1] = Q[:, i] @ w
            w = w - H[i, j - 1] * Q[:, i]
            red += 1
        H[j, j - 1] = np.linalg.norm(w)
        red += 1
        Q[:, j] = w / H[j, j - 1]
    return Q, H, red


class DCGS2Arnoldi:
    """Step-exact DCGS2 Arnoldi-QR expansion (Alg. arnoldi), one reduction per step.

    State after the call to ``step`` for the paper's step j (j = 2..n+1):
      * q_1..q_{j-1} final in Q[:, :j-1];
      * H columns 1..j-2 final (H_{1:j-1, 1:j-2}); K column j-1 partial;
      * w holds w_j (unnormalised, once projected).

    Step j, following the algorithm in the paper's order of operations:
      v = A w_{j-1}                                        (matvec on w, eq. (11))
      C = Q_{1:j-2}^T w,  beta = w^T w,                    } the one reduction
      S = Q_{1:j-2}^T v,  sigma = w^T v,  gamma = v^T v    }
      alpha = sqrt(beta - C^T C)                           (delayed normalisation)
      T_{j-1} = (sigma - C^T S) / alpha^2,  T_{1:j-2} = S / alpha
      q_{j-1} = (w - Q_{1:j-2} C) / alpha                  (delayed reorthogonalisation)
      w_j = v/alpha - Q_{1:j-1} T                          (projection, eq. (32))
      H_{1:j-2, j-2} = K_{1:j-2, j-2} + C ;  H_{j-1, j-2} = alpha     (j >= 3)
      K_{1:j-1, j-1} = T - (1/alpha) H_{1:j-1, 1:j-2} C    (representation, eq. (52))
    The listing sets H_{j-1,j-2} after forming K, but the derivation's
    H_{j-1,j-1} contains -(1/alpha) H_{j-1,j-2} C_{j-2,j-1}, so H_{j-1,j-2} is set
    first.  H C is a dense product: after a Krylov-Schur restart row k+1 of H is full.

    ``finish()`` completes column n with CGS2 (two reductions, end of Sec. 3):
      c = Q_{1:n}^T w_{n+1};  u = w - Q c;  alpha = ||u||;  q_{n+1} = u/alpha;
      H_{1:n,n} = K_{1:n,n} + c;  H_{n+1,n} = alpha.

    Readings where the paper is silent (the GPU implements the same):
      * Pythagorean guard: if not (beta - C^T C > tau*beta) (or non-finite),
        alpha = ||w - Q C|| explicitly (one extra reduction, counted in fallbacks).
      * Breakdown: alpha_{j-1} <= eta * rho_{j-1}, rho = norm of the vector that
        w_{j-1} was projected from: ||r0|| for j-1 = 1, else sqrt(gamma_{j-1})/alpha_{j-2}.
        Then H column j-2 is completed, k = j-2, status BREAKDOWN.
      * Any non-finite reduced scalar: status NONFINITE.

    qdtype=np.float32 stores the basis in single precision (each column rounded
    once when written); all products with Q, reductions, H, K and scalars stay
    FP64 and the projections use the stored columns.
    """

    def __init__(self, matvec, r0, n, tau=1e-8, eta=1e-12, qdtype=np.float64):
        r0 = np.asarray(r0, dtype=np.float64)
        self.matvec = matvec
        self.m = r0.size
        self.n = n
        self.tau, self.eta = tau, eta
        self.Q = np.zeros((self.m, n + 1), order="F", dtype=qdtype)
        self.H = np.zeros((n + 1, n))
        self.K = np.zeros((n + 1, n + 1))
        self.w = r0.copy()                      # w_1 = r0 (unnormalised)
        self.j = 2                              # next step to run
        self.rho_next = None                    # rho for the vector held in w
        self.alphas = []                        # alpha_1, alpha_2, ...
        self.reductions = 0
        self.fallbacks = 0
        self.matvecs = 0
        self.status = OK
        self.k = 0                              # number of final H columns
        self.restart_step = False               # first step after a KS truncation
        self.trace = None                       # optional per-step record (tests)

    # -- Krylov-Schur continuation -------------------------------------------------
    @classmethod
    def resume(cls, matvec, Q, H, k, n, tau=1e-8, eta=1e-12, qdtype=np.float64):
        """Continue an expansion from a truncated Krylov-Schur decomposition.

        Given orthonormal Q_{1:k+1} and H_{1:k+1,1:k} = [S_k; b^T] with
        A Q_k = Q_{k+1} H_{1:k+1,1:k}, extend to n columns.  The first step
        (j = k+2) has w_{k+1} = q_{k+1} already normalised, so C = 0 and alpha = 1:
        it reduces only S = Q_{1:k+1}^T v, sets T = S, w_{k+2} = v - Q_{1:k+1} T,
        K_{:,k+1} = T, and leaves H column k alone (it is already final).
        """
        self = cls(matvec, _f64(Q[:, k]), n, tau, eta, qdtype)
        self.Q[:, :k + 1] = Q[:, :k + 1]
        self.H[:k + 1, :k] = H[:k + 1, :k]
        self.w = _f64(Q[:, k]).copy()
        self.j = k + 2
        self.k = k
        self.restart_step = True
        return self

    # ------------------------------------------------------------------------------
    def step(self):
        """Run the paper's step j = self.j.  Returns the status."""
        j = self.j
        J = j - 2
        Q, H, K = self.Q, self.H, self.K
        w = self.w
        v = self.matvec(w)
        self.matvecs += 1
        Qk = _f64(Q[:, :J])
        if self.restart_step:
            # Krylov-Schur continuation: q_{k+1} is final; one reduction of Q_{1:k+1}^T v
            T = _f64(Q[:, :J + 1]).T @ v
            gamma = v @ v
            self.reductions += 1
            if not (np.all(np.isfinite(T)) and np.isfinite(gamma)):
                self.status = NONFINITE
                return self.status
            self.w = v - _f64(Q[:, :J + 1]) @ T
            K[:J + 1, J] = T
            self.alphas.append(1.0)
            self.rho_next = np.sqrt(gamma)
            self.restart_step = False
            self.j += 1
            return self.status
        # --- the one global reduction: [Q_{1:j-2}, w]^T [w, v]
        C = Qk.T @ w
        beta = w @ w
        S = Qk.T @ v
        sigma = w @ v
        gamma = v @ v
        self.reductions += 1
        if not (np.all(np.isfinite(C)) and np.all(np.isfinite(S)) and np.isfinite(beta)
                and np.isfinite(sigma) and np.isfinite(gamma)):
            self.status = NONFINITE
            return self.status
        rho = np.sqrt(beta) if j == 2 else self.rho_next
        # --- delayed normalisation
        d = beta - C @ C
        if np.isfinite(d) and d > self.tau * beta:
            alpha = np.sqrt(d)
        else:
            alpha = np.linalg.norm(w - Qk @ C)
            self.reductions += 1
            self.fallbacks += 1
        if not np.isfinite(alpha):
            self.status = NONFINITE
            return self.status
        if alpha <= self.eta * rho:
            if j >= 3:
                H[:J, J - 1] = K[:J, J - 1] + C
                H[J, J - 1] = alpha
                self.k = J
            self.status = BREAKDOWN
            return self.status
        T = np.empty(J + 1)
        T[J] = (sigma - C @ S) / (alpha * alpha)
        T[:J] = S / alpha
        # --- projection
        Q[:, J] = (w - Qk @ C) / alpha
        self.w = v / alpha - _f64(Q[:, :J + 1]) @ T
        # --- representation: complete H column j-2, then the partial column K_{:, j-1}
        if j >= 3:
            H[:J, J - 1] = K[:J, J - 1] + C
            H[J, J - 1] = alpha
            self.k = J
        K[:J + 1, J] = T - (H[:J + 1, :J] @ C) / alpha
        self.alphas.append(alpha)
        self.rho_next = np.sqrt(gamma) / alpha
        if self.trace is not None:
            self.trace.append(dict(j=j, C=C.copy(), beta=beta, S=S.copy(), sigma=sigma,
                                   gamma=gamma, alpha=alpha, T=T.copy(), w=self.w.copy(),
                                   rho_next=self.rho_next, fallback=not (np.isfinite(d) and
                                                                          d > self.tau * beta)))
        self.j += 1
        return self.status

    def finish(self):
        """Last column by CGS2 (two reductions): completes H column n and q_{n+1}."""
        n = self.n
        Q, H, K = self.Q, self.H, self.K
        w = self.w
        Qk = _f64(Q[:, :n])
        c = Qk.T @ w
        u = w - Qk @ c
        alpha = np.linalg.norm(u)
        self.reductions += 2
        if not (np.all(np.isfinite(c)) and np.isfinite(alpha)):
            self.status = NONFINITE
            return self.status
        H[:n, n - 1] = K[:n, n - 1] + c
        H[n, n - 1] = alpha
        self.k = n
        if alpha <= self.eta * self.rho_next:
            self.status = BREAKDOWN
            return self.status
        Q[:, n] = u / alpha
        self.alphas.append(alpha)
        if self.trace is not None:
            self.trace.append(dict(j=n + 2, C=c.copy(), alpha=alpha))
        return self.status

    def run(self):
        while self.j <= self.n + 1 and self.status == OK:
            self.step()
        if self.status == OK:
            self.finish()
        return self


def dcgs2_arnoldi(matvec, r0, n, tau=1e-8, eta=1e-12, qdtype=np.float64):
    """Full DCGS2 Arnoldi-QR expansion of n steps: returns dict(Q, H, status, k, ...)."""
    a = DCGS2Arnoldi(matvec, r0, n, tau, eta, qdtype).run()
    return dict(Q=a.Q, H=a.H, status=a.status, k=a.k, reductions=a.reductions,
                fallbacks=a.fallbacks, matvecs=a.matvecs)

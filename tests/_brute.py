"""High-precision brute force for tiny problems (mpmath, 50 digits).

The exact thin QR (R_jj > 0) and the exact Arnoldi decomposition
(q_1 = r0/||r0||, H_{j+1,j} > 0) are unique; at 50 digits plain Gram-Schmidt
(applied twice) computes them to far below double precision, independently of
any float64 code in the repository.
"""
import mpmath as mp
import numpy as np

mp.mp.dps = 50


def _col(M, j):
    return [M[i, j] for i in range(M.rows)]


def _dot(a, b):
    return mp.fsum(x * y for x, y in zip(a, b))


def qr_exact(B):
    m, n = B.shape
    A = mp.matrix(B.tolist())
    Q = mp.matrix(m, n)
    R = mp.matrix(n, n)
    for j in range(n):
        w = _col(A, j)
        for _ in range(2):
            for i in range(j):
                qi = _col(Q, i)
                c = _dot(qi, w)
                R[i, j] += c
                w = [x - c * y for x, y in zip(w, qi)]
        nrm = mp.sqrt(_dot(w, w))
        R[j, j] = nrm
        for i in range(m):
            Q[i, j] = w[i] / nrm
    return (np.array(Q.tolist(), dtype=float), np.array(R.tolist(), dtype=float))


def arnoldi_exact(A, r0, n):
    m = A.shape[0]
    Am = mp.matrix(np.asarray(A).tolist())
    Q = mp.matrix(m, n + 1)
    H = mp.matrix(n + 1, n)
    r = [mp.mpf(float(x)) for x in r0]
    nr = mp.sqrt(_dot(r, r))
    for i in range(m):
        Q[i, 0] = r[i] / nr
    for j in range(n):
        qj = _col(Q, j)
        w = [mp.fsum(Am[i, k] * qj[k] for k in range(m)) for i in range(m)]
        for _ in range(2):
            for i in range(j + 1):
                qi = _col(Q, i)
                c = _dot(qi, w)
                H[i, j] += c
                w = [x - c * y for x, y in zip(w, qi)]
        nrm = mp.sqrt(_dot(w, w))
        H[j + 1, j] = nrm
        for i in range(m):
            Q[i, j + 1] = w[i] / nrm
    return (np.array(Q.tolist(), dtype=float), np.array(H.tolist(), dtype=float))

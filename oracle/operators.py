"""Test operators for the oracle (test infrastructure only; see oracle/__init__).

The paper's stability experiments (Sec. 6.1) use Manteuffel's central-difference
convection-diffusion matrix, A = M/h^2 + (beta/2h) N, whose eigenvalues are known
in closed form (eq. eigs_manteuffel).  The formula, with L = k+1 and h = 1, fixes
A = I (x) T + T (x) I with T = tridiag(-1 - beta/2, 2, -1 + beta/2).

The workloads use the same discretisation of -D Lap(u) + v . grad(u) on the unit
cube with homogeneous Dirichlet conditions, h = 1/(n+1) per axis, central
differences and lexicographic ordering (x fastest).  In one dimension the row of
grid point i reads

    (-D/h^2 - v/(2h)) u[i-1] + (2D/h^2) u[i] + (-D/h^2 + v/(2h)) u[i+1].

This module builds those matrices from that definition with scipy.sparse; it is
independent of the GPU stencil kernels, which receive only the coefficients.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def tridiag_1d(n: int, D: float, v: float, h: float) -> sp.csr_matrix:
    """1-D central-difference convection-diffusion matrix (Sec. 6.1 discretisation)."""
    lower = -D / h**2 - v / (2.0 * h)   # coefficient of u[i-1]
    diag = 2.0 * D / h**2
    upper = -D / h**2 + v / (2.0 * h)   # coefficient of u[i+1]
    return sp.diags([np.full(n - 1, lower), np.full(n, diag), np.full(n - 1, upper)],
                    [-1, 0, 1], format="csr")


def convection_diffusion(grid, D=1.0, vel=None, h=None) -> sp.csr_matrix:
    """Kronecker-sum matrix of -D Lap + v.grad on a tensor grid.

    grid: (nx,) / (nx, ny) / (nx, ny, nz); lexicographic order with x fastest, so
    the x operator acts on the last Kronecker factor.
    h: mesh width per axis (default 1/(n_i + 1)); Manteuffel's case uses h = 1.
    """
    grid = tuple(int(g) for g in grid)
    d = len(grid)
    vel = (0.0,) * d if vel is None else tuple(float(v) for v in vel)
    hs = tuple(1.0 / (g + 1) for g in grid) if h is None else (
        (float(h),) * d if np.isscalar(h) else tuple(float(x) for x in h))
    A = None
    for axis in range(d):
        T = tridiag_1d(grid[axis], D, vel[axis], hs[axis])
        # identity factors: axes after `axis` are slower (outer), before are faster (inner)
        left = sp.identity(int(np.prod(grid[axis + 1:])) if axis + 1 < d else 1, format="csr")
        right = sp.identity(int(np.prod(grid[:axis])) if axis > 0 else 1, format="csr")
        term = sp.kron(sp.kron(left, T), right, format="csr")
        A = term if A is None else A + term
    return A.tocsr()


def manteuffel(k: int, beta: float) -> sp.csr_matrix:
    """Manteuffel matrix of Sec. 6.1 with L = k+1 (so h = 1): A = I(x)T + T(x)I."""
    return convection_diffusion((k, k), D=1.0, vel=(beta, beta), h=1.0)


def closed_form_eigenvalues(grid, D=1.0, vel=None, h=None) -> np.ndarray:
    """Eigenvalues of ``convection_diffusion`` in closed form (real when |v h / 2D| < 1).

    A tridiagonal Toeplitz matrix tridiag(a, d, c) with a*c > 0 has eigenvalues
    d - 2 sqrt(a c) cos(l pi/(n+1)); a Kronecker sum adds them over the axes.  With
    h = 1, D = 1, v = beta this is eq. eigs_manteuffel of the paper.
    """
    grid = tuple(int(g) for g in grid)
    d = len(grid)
    vel = (0.0,) * d if vel is None else tuple(float(v) for v in vel)
    hs = tuple(1.0 / (g + 1) for g in grid) if h is None else (
        (float(h),) * d if np.isscalar(h) else tuple(float(x) for x in h))
    per_axis = []
    for n, v, hh in zip(grid, vel, hs):
        a = -D / hh**2 - v / (2 * hh)
        c = -D / hh**2 + v / (2 * hh)
        if a * c <= 0:
            raise ValueError("closed form needs cell Peclet |v h / 2D| < 1")
        l = np.arange(1, n + 1)
        per_axis.append(2 * D / hh**2 - 2 * np.sqrt(a * c) * np.cos(l * np.pi / (n + 1)))
    lam = per_axis[0]
    for ev in per_axis[1:]:
        lam = (lam[:, None] + ev[None, :]).ravel()
    return np.sort(lam)


def manteuffel_eigenvalues(k: int, beta: float) -> np.ndarray:
    """eq. eigs_manteuffel: 2[2 - sqrt(1-(beta/2)^2)(cos(l pi/L) + cos(j pi/L))], L = k+1."""
    L = k + 1
    c = np.cos(np.arange(1, k + 1) * np.pi / L)
    lam = 2.0 * (2.0 - np.sqrt(1.0 - (beta / 2.0) ** 2) * (c[:, None] + c[None, :]))
    return np.sort(lam.ravel())


def varcoef_matrix(prob) -> sp.csr_matrix:
    """Variable-diffusion convection-diffusion (the learned-guess family), assembled.

    -div(D grad u) + v.grad u on (0,1)^2, Dirichlet, h = 1/(n+1), x fastest.
    Diffusion uses D at the cell faces (midpoints between grid points), the
    convection central differences:
      row(i,j): (1/h^2)[(D_e + D_w + D_n + D_s) u_ij - D_e u_{i+1,j} - D_w u_{i-1,j}
                - D_n u_{i,j+1} - D_s u_{i,j-1}] + vx (u_{i+1,j} - u_{i-1,j})/(2h)
                + vy (u_{i,j+1} - u_{i,j-1})/(2h)
    log D(x,y) = sum_k xi_k a_k phi_k, phi_{p,q} = 2 sin(p pi x) sin(q pi y),
    a_{p,q} = 1/(p^2+q^2) (modes and amplitudes as stated in synth.VarCoefProblem).
    """
    n = prob.n
    h = 1.0 / (n + 1)
    modes = ((1, 1), (1, 2), (2, 1), (2, 2), (1, 3), (3, 1), (2, 3), (3, 2))

    def D(x, y):
        s = np.zeros_like(x)
        for (p, q), xi in zip(modes, prob.xi):
            s += xi / (p * p + q * q) * 2.0 * np.sin(p * np.pi * x) * np.sin(q * np.pi * y)
        return np.exp(s)

    vx, vy = prob.vel
    rows, cols, vals = [], [], []
    for j in range(n):            # y index
        for i in range(n):        # x index
            x, y = (i + 1) * h, (j + 1) * h
            De, Dw = D(np.array(x + h / 2), np.array(y)), D(np.array(x - h / 2), np.array(y))
            Dn, Ds = D(np.array(x), np.array(y + h / 2)), D(np.array(x), np.array(y - h / 2))
            r = i + n * j
            rows.append(r); cols.append(r); vals.append(float(De + Dw + Dn + Ds) / h**2)
            if i + 1 < n:
                rows.append(r); cols.append(r + 1); vals.append(float(-De / h**2 + vx / (2 * h)))
            if i > 0:
                rows.append(r); cols.append(r - 1); vals.append(float(-Dw / h**2 - vx / (2 * h)))
            if j + 1 < n:
                rows.append(r); cols.append(r + n); vals.append(float(-Dn / h**2 + vy / (2 * h)))
            if j > 0:
                rows.append(r); cols.append(r - n); vals.append(float(-Ds / h**2 - vy / (2 * h)))
    return sp.csr_matrix((vals, (rows, cols)), shape=(n * n, n * n))

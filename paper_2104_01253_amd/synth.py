"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module draws random numbers and assembles the workload parameters; it holds
none of the orthogonalisation, Krylov or operator arithmetic.  All generators
use NumPy's PCG64 (``numpy.random.default_rng(seed)``).

Workloads (the paper's experiments run on synthetic tall-skinny matrices and on
convection-diffusion operators; the sizes below are the project's workloads):

* ``tall_skinny``: B = G diag(logspace(0, -e, n)) V with G ~ N(0,1) (m x n) and V
  Haar-orthogonal (QR of an n x n N(0,1) matrix, columns sign-fixed), so that
  kappa(B) ~ 10^e.  Returned column-major.
* ``cd2d`` / ``cd3d``: grid and coefficients of -D Lap + v.grad on the unit
  square / cube (Dirichlet, central differences) plus seeded vectors.
* ``ks_instances``: a family of 2-D convection-diffusion instances with
  n_x ~ U[48, 256] and v ~ U(0, 50)^2.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def haar_orthogonal(n: int, seed: int) -> np.ndarray:
    """Haar-distributed orthogonal n x n matrix (QR of a Gaussian, columns sign-fixed)."""
    X = rng(seed).standard_normal((n, n))
    Qh, Rh = np.linalg.qr(X)
    return Qh * np.sign(np.diag(Rh))[None, :]


def tall_skinny(m: int, n: int, cond_exp: float = 8.0, seed_g: int = 1, seed_v: int = 2,
                dtype=np.float64) -> np.ndarray:
    """B = G diag(logspace(0, -cond_exp, n)) V, column-major (Fortran order), m x n."""
    Gt = rng(seed_g).standard_normal((n, m))           # G^T, row-major n x m
    V = haar_orthogonal(n, seed_v)
    M = np.logspace(0.0, -cond_exp, n)[:, None] * V    # diag(s) V
    B = (M.T @ Gt).T                                    # = G M, Fortran-ordered m x n
    return B.astype(dtype, copy=False)


def normal_vector(m: int, seed: int) -> np.ndarray:
    return rng(seed).standard_normal(m)


def uniform_vector(m: int, seed: int) -> np.ndarray:
    return rng(seed).uniform(0.0, 1.0, m)


@dataclass(frozen=True)
class CDProblem:
    """-D Lap(u) + v.grad(u) on (0,1)^d, Dirichlet, h_i = 1/(n_i+1)."""
    grid: tuple
    D: float
    vel: tuple

    @property
    def m(self) -> int:
        return int(np.prod(self.grid))


def cd2d(nx: int = 32, ny: int | None = None, D: float = 1.0, vel=(10.0, 10.0)) -> CDProblem:
    return CDProblem((nx, nx if ny is None else ny), float(D), tuple(float(v) for v in vel))


def cd3d(n: int = 128, D: float = 1.0, vel=(10.0, 10.0, 10.0)) -> CDProblem:
    return CDProblem((n, n, n), float(D), tuple(float(v) for v in vel))


def ks_instances(count: int, seed: int = 4, nmin: int = 48, nmax: int = 256, vmax: float = 50.0):
    """Batched Krylov-Schur family: n_x ~ U{nmin..nmax} (square grids), v ~ U(0, vmax)^2."""
    g = rng(seed)
    nx = g.integers(nmin, nmax + 1, size=count)
    vel = g.uniform(0.0, vmax, size=(count, 2))
    return [CDProblem((int(n), int(n)), 1.0, (float(v[0]), float(v[1]))) for n, v in zip(nx, vel)]


def gmres_batched_instances(count: int, seed: int = 6, nmin: int = 32, nmax: int = 128,
                            vmax: float = 30.0, rmin: int = 20, rmax: int = 60):
    """Batched GMRES family: 2-D grids n_x, n_y ~ U{nmin..nmax} (independently, so grids
    are rectangular), v ~ U(0, vmax)^2, restart lengths ~ U{rmin..rmax}, b ~ U(0,1)
    with seed 5000 + i.  Returns [(CDProblem, restart, b)]."""
    g = rng(seed)
    nx = g.integers(nmin, nmax + 1, size=count)
    ny = g.integers(nmin, nmax + 1, size=count)
    vel = g.uniform(0.0, vmax, size=(count, 2))
    rs = g.integers(rmin, rmax + 1, size=count)
    out = []
    for i in range(count):
        p = CDProblem((int(nx[i]), int(ny[i])), 1.0, (float(vel[i, 0]), float(vel[i, 1])))
        out.append((p, int(rs[i]), uniform_vector(p.m, 5000 + i)))
    return out


# Named workloads ------------------------------------------------------------------
def arnoldi_cd2d_32():
    """FP64 DCGS2 Arnoldi, 50 steps, 2-D convection-diffusion 32x32, v=(10,10), r0 ~ N(0,1) seed 0."""
    prob = cd2d(32, vel=(10.0, 10.0))
    return prob, normal_vector(prob.m, 0), 50


def gmres_cd3d(n: int = 128):
    """GMRES(50) on 3-D convection-diffusion n^3, v=(10,10,10), b ~ U(0,1) seed 3, rtol 1e-8."""
    prob = cd3d(n, vel=(10.0, 10.0, 10.0))
    return prob, uniform_vector(prob.m, 3)


# Learned-initial-guess family ---------------------------------------------------------
KL_MODES = ((1, 1), (1, 2), (2, 1), (2, 2), (1, 3), (3, 1), (2, 3), (3, 2))


@dataclass(frozen=True)
class VarCoefProblem:
    """-div(D grad u) + v.grad u = b on (0,1)^2, Dirichlet, n x n interior grid.

    log D(x, y) = sum_k xi_k a_k phi_k(x, y) with phi_{p,q} = 2 sin(p pi x) sin(q pi y),
    a_{p,q} = 1 / (p^2 + q^2) (eight modes, KL_MODES); b is a sum of four Gaussian
    bumps with centres, widths and amplitudes in `bumps` (rows: cx, cy, width, amp).
    """
    n: int
    xi: tuple
    bumps: tuple
    vel: tuple = (10.0, 10.0)

    @property
    def m(self) -> int:
        return self.n * self.n


def varcoef_instances(count: int, seed: int = 5, n: int = 256, vel=(10.0, 10.0)):
    g = rng(seed)
    out = []
    for _ in range(count):
        xi = g.standard_normal(len(KL_MODES))
        cxy = g.uniform(0.2, 0.8, size=(4, 2))
        width = g.uniform(0.03, 0.1, size=(4, 1))
        amp = g.uniform(-1.0, 1.0, size=(4, 1))
        bumps = np.hstack([cxy, width, amp])
        out.append(VarCoefProblem(n, tuple(float(v) for v in xi),
                                  tuple(tuple(float(v) for v in r) for r in bumps),
                                  tuple(float(v) for v in vel)))
    return out


def varcoef_rhs(prob: VarCoefProblem) -> np.ndarray:
    """b at the interior grid points (x fastest), the four Gaussian bumps."""
    h = 1.0 / (prob.n + 1)
    t = np.arange(1, prob.n + 1) * h
    X, Y = np.meshgrid(t, t, indexing="xy")          # rows = y, columns = x -> x fastest
    b = np.zeros_like(X)
    for cx, cy, wd, amp in prob.bumps:
        b += amp * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * wd * wd))
    return b.ravel()

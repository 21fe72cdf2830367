"""Learned initial guess for GMRES: CPU reference (test infrastructure only).

The paper's solvers start from a given x0 (GMRES minimises over x0 + K_k,
Sec. 1); this module defines a data-driven x0 for the variable-coefficient
convection-diffusion family.  Nothing here comes from the paper; every piece is
a plain textbook definition, written in float64 so that the FP32 GPU kernels can
be checked against it:

* grid transfers between the fine n x n interior grid (h = 1/(n+1), x fastest)
  and a coarse nc x nc grid (r = n / nc fine points per coarse cell and axis):
  - restriction R: the mean of each r x r block;
  - prolongation P: tensor-product piecewise-linear interpolation of the values
    at the coarse block centres, extended by zero at the Dirichlet boundary;
* features of an instance: R(b) / s with s = RMS of R(b), then the operator
  parameters, zero-padded to the input width;
* a multilayer perceptron: Z_l = X_l W_l + b_l, X_{l+1} = ReLU(Z_l) for the
  hidden layers, the last layer linear; row-major, one sample per row;
* its mean-squared-error loss and the gradients by the chain rule;
* the Adam update (Kingma & Ba, 2015, Algorithm 1, with the bias corrections).

The guess is x0 = s * P(MLP(features)); the MLP is trained on targets R(x)/s of
solved instances.
"""
from __future__ import annotations

import numpy as np


# ---- grid transfers ---------------------------------------------------------------
def restrict(x: np.ndarray, n: int, nc: int) -> np.ndarray:
    """Mean over each r x r block of the fine grid (x fastest in both layouts)."""
    r = n // nc
    assert r * nc == n
    X = np.asarray(x, dtype=np.float64).reshape(n, n)        # [y, x]
    return X.reshape(nc, r, nc, r).mean(axis=(1, 3)).ravel()


def coarse_centres(n: int, nc: int) -> np.ndarray:
    """Physical coordinates of the coarse block centres along one axis."""
    r = n // nc
    h = 1.0 / (n + 1)
    return (np.arange(nc) * r + (r - 1) / 2.0 + 1.0) * h


def interp_matrix_1d(n: int, nc: int) -> np.ndarray:
    """n x nc matrix of the 1-D piecewise-linear interpolation from the coarse
    centres (plus zero at 0 and 1) to the fine points (i+1) h."""
    h = 1.0 / (n + 1)
    nodes = np.concatenate([[0.0], coarse_centres(n, nc), [1.0]])
    M = np.zeros((n, nc + 2))
    for i in range(n):
        x = (i + 1) * h
        k = np.searchsorted(nodes, x, side="right") - 1      # nodes[k] <= x < nodes[k+1]
        k = min(k, nc)
        t = (x - nodes[k]) / (nodes[k + 1] - nodes[k])
        M[i, k] += 1.0 - t
        M[i, k + 1] += t
    return M[:, 1:nc + 1]                                     # boundary nodes carry zero


def prolong(xc: np.ndarray, n: int, nc: int) -> np.ndarray:
    """Tensor-product linear interpolation of coarse values to the fine grid."""
    M = interp_matrix_1d(n, nc)
    Xc = np.asarray(xc, dtype=np.float64).reshape(nc, nc)    # [y, x]
    return (M @ Xc @ M.T).ravel()


def features(b: np.ndarray, params, n: int, nc: int, fdim: int):
    """(feature vector of length fdim, scale s); s = 0 gives zero features."""
    bc = restrict(b, n, nc)
    s = float(np.sqrt(np.mean(bc * bc)))
    f = np.zeros(fdim)
    if s > 0.0:
        f[:nc * nc] = bc / s
    p = np.asarray(params, dtype=np.float64)
    f[nc * nc:nc * nc + p.size] = p
    return f, s


# ---- multilayer perceptron ----------------------------------------------------------
def forward(params, X):
    """params: list of (W (K x N), b (N,)); returns the list of pre-activations Z_l
    and the output (= Z of the last layer)."""
    A = np.asarray(X, dtype=np.float64)
    Zs = []
    for l, (W, b) in enumerate(params):
        Z = A @ W + b[None, :]
        Zs.append(Z)
        A = np.maximum(Z, 0.0) if l + 1 < len(params) else Z
    return Zs, A


def mse(Y, T) -> float:
    D = np.asarray(Y, dtype=np.float64) - np.asarray(T, dtype=np.float64)
    return float(np.mean(D * D))


def gradients(params, X, T):
    """Loss and the gradients [(dW, db), ...] of the mean squared error."""
    X = np.asarray(X, dtype=np.float64)
    Zs, Y = forward(params, X)
    loss = mse(Y, T)
    dZ = 2.0 * (Y - T) / Y.size                    # d loss / d output
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        Ain = X if l == 0 else np.maximum(Zs[l - 1], 0.0)
        W, _ = params[l]
        grads[l] = (Ain.T @ dZ, dZ.sum(axis=0))
        if l > 0:
            dA = dZ @ W.T
            dZ = dA * (Zs[l - 1] > 0.0)
    return loss, grads


class Adam:
    """Kingma & Ba (2015), Algorithm 1, applied to a list of arrays."""

    def __init__(self, shapes, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = [np.zeros(s) for s in shapes]
        self.v = [np.zeros(s) for s in shapes]
        self.t = 0

    def step(self, theta, grads):
        self.t += 1
        out = []
        for i, (p, g) in enumerate(zip(theta, grads)):
            self.m[i] = self.b1 * self.m[i] + (1.0 - self.b1) * g
            self.v[i] = self.b2 * self.v[i] + (1.0 - self.b2) * g * g
            mhat = self.m[i] / (1.0 - self.b1 ** self.t)
            vhat = self.v[i] / (1.0 - self.b2 ** self.t)
            out.append(p - self.lr * mhat / (np.sqrt(vhat) + self.eps))
        return out

"""Stability metrics of Sec. 6 (test infrastructure only)."""
from __future__ import annotations

import numpy as np


def loss_of_orthogonality(Q):
    """||I - Q^T Q||_F over all columns given (Sec. 6.1)."""
    k = Q.shape[1]
    return np.linalg.norm(np.eye(k) - Q.T @ Q, "fro")


def representation_error(A, Q, H, k):
    """RRE = ||A Q_{1:k} - Q_{1:k+1} H_{1:k+1,1:k}||_F / ||A||_F (Sec. 6.1)."""
    AQ = A @ Q[:, :k]
    normA = np.sqrt((A.multiply(A)).sum()) if hasattr(A, "multiply") else np.linalg.norm(A, "fro")
    return np.linalg.norm(AQ - Q[:, :k + 1] @ H[:k + 1, :k], "fro") / normA


def qr_error(B, Q, R):
    """||B - Q R||_F / ||B||_F."""
    return np.linalg.norm(B - Q @ R, "fro") / np.linalg.norm(B, "fro")

"""Oracle: FP64 Lanczos ground energy with full re-orthogonalisation.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper uses a matrix-free Lanczos to reach ground states (Sec. 2.1, App. D)
but gives no details.  The textbook iteration taken here:

    v_0 = x / |x|,  beta_{-1} = 0
    for j = 0 .. m-1:
        w = H v_j - beta_{j-1} v_{j-1}
        alpha_j = v_j . w
        w = w - alpha_j v_j
        w = w - V (V^T w), twice (classical Gram-Schmidt against v_0..v_j)
        beta_j = |w|;  stop if beta_j <= tol * max_i(|alpha_i|, beta_i) or j+1 = dim
        v_{j+1} = w / beta_j
    Ritz values: eigenvalues of the tridiagonal T (LAPACK via scipy).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def lanczos(apply, v0: np.ndarray, steps: int, dim: int | None = None,
            reorth: bool = True, tol: float = 1e-12):
    """Returns (alpha, beta, V) with V[:, j] = v_j for the steps taken."""
    v = np.asarray(v0, dtype=np.float64)
    dim = dim if dim is not None else len(v)
    m = max(1, min(steps, dim))
    V = np.zeros((len(v), m))
    V[:, 0] = v / np.linalg.norm(v)
    alpha, beta = [], []
    scale = 0.0
    for j in range(m):
        w = apply(V[:, j])
        if j > 0:
            w = w - beta[j - 1] * V[:, j - 1]
        a = float(V[:, j] @ w)
        w = w - a * V[:, j]
        if reorth:
            B = V[:, :j + 1]
            for _ in range(2):
                w = w - B @ (B.T @ w)
        alpha.append(a)
        b = float(np.linalg.norm(w))
        scale = max(scale, abs(a), b)
        if j + 1 == m or b <= tol * scale:
            break
        beta.append(b)
        V[:, j + 1] = w / b
    alpha = np.array(alpha)
    beta = np.array(beta[:len(alpha) - 1])
    return alpha, beta, V[:, :len(alpha)]


def ritz(alpha: np.ndarray, beta: np.ndarray, vectors: bool = False):
    if len(alpha) == 1:
        return (alpha.copy(), np.ones((1, 1))) if vectors else alpha.copy()
    if vectors:
        return scipy.linalg.eigh_tridiagonal(alpha, beta)
    return scipy.linalg.eigh_tridiagonal(alpha, beta, eigvals_only=True)


def ground_state(apply, v0, steps, dim=None):
    """(E0, psi0, alpha, beta) from a fully re-orthogonalised Lanczos run."""
    alpha, beta, V = lanczos(apply, v0, steps, dim)
    evals, evecs = ritz(alpha, beta, vectors=True)
    s0 = evecs[:, 0]
    psi = V @ s0
    psi /= np.linalg.norm(psi)
    return float(evals[0]), psi, alpha, beta

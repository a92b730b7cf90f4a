"""Block Lanczos of the oracle: several lowest eigenvalues at once.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The block form of the Lanczos recurrence (the method the paper builds on,
Secs. 1 and 4), in FP64 with numpy, one oracle H x per column:

    V_0 R_0 = X0
    W   = H V_k - V_{k-1} B_{k-1}^T
    A_k = V_k^T W;   W = W - V_k A_k
    twice: W = W - V (V^T W)            (V = all blocks so far)
    V_{k+1} B_k = W                      (QR, B_k upper triangular)

QR is Cholesky QR applied twice.  The run stops when what is left of W is at
the rounding level of the recurrence (largest squared column norm at most
(1e-12 max |A, B entries|)^2) or rank deficient.  The eigenvalues of the block
tridiagonal matrix approximate the lowest eigenvalues of H on H(M).
"""
import numpy as np
import scipy.linalg

from .core import Subspace


def cholqr2(W, tol: float = 1e-12):
    """Q R = W with Q^T Q = I (Cholesky QR twice), or None if W is rank deficient."""
    Rs = []
    for pass_ in range(2):
        G = W.T @ W
        G = 0.5 * (G + G.T)
        dmax = float(np.max(np.diag(G)))
        if not dmax > 0.0:
            return None
        try:
            L = np.linalg.cholesky(G)
        except np.linalg.LinAlgError:
            return None
        if np.min(np.diag(L)) ** 2 <= (tol if pass_ == 0 else 1e-14) * dmax:
            return None
        R = L.T
        W = scipy.linalg.solve_triangular(R, W.T, trans="T", lower=False).T
        Rs.append(R)
    return W, Rs[1] @ Rs[0]


def block_lanczos(sub: Subspace, J, X0, steps: int):
    """Diagonal blocks A (n x p x p), sub-diagonal blocks B (n-1 x p x p)."""
    X0 = np.asarray(X0, dtype=np.float64)
    if X0.shape[0] != sub.dim:
        X0 = X0.T
    p = X0.shape[1]
    qr = cholqr2(X0)
    if qr is None:
        raise ValueError("start block is rank deficient")
    V = [qr[0]]
    A, B = [], []
    scale = 0.0
    for k in range(steps):
        W = np.column_stack([sub.apply(J, V[k][:, q]) for q in range(p)])
        if k > 0:
            W -= V[k - 1] @ B[k - 1].T
        Ak = V[k].T @ W
        W -= V[k] @ Ak
        A.append(0.5 * (Ak + Ak.T))
        scale = max(scale, float(np.abs(A[-1]).max()))
        Vall = np.hstack(V)
        for _ in range(2):
            W -= Vall @ (Vall.T @ W)
        if k + 1 == steps:
            break
        if float(np.max(np.sum(W * W, axis=0))) <= (1e-12 * scale) ** 2:
            break
        qr = cholqr2(W)
        if qr is None:
            break
        V.append(qr[0])
        B.append(qr[1])
        scale = max(scale, float(np.abs(qr[1]).max()))
    return np.array(A), np.array(B).reshape(-1, p, p), np.hstack(V)


def block_tridiagonal(A, B) -> np.ndarray:
    n, p = len(A), A[0].shape[0]
    T = np.zeros((n * p, n * p))
    for k in range(n):
        T[k * p:(k + 1) * p, k * p:(k + 1) * p] = A[k]
        if k + 1 < n:
            T[(k + 1) * p:(k + 2) * p, k * p:(k + 1) * p] = B[k]
            T[k * p:(k + 1) * p, (k + 1) * p:(k + 2) * p] = B[k].T
    return T


def lowest_levels(sub: Subspace, J, X0, steps: int, count: int) -> np.ndarray:
    A, B, _ = block_lanczos(sub, J, X0, steps)
    return np.linalg.eigvalsh(block_tridiagonal(A, B))[:count]

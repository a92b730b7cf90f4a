"""Lanczos iteration, ground state and bond correlations of the oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper cites the Lanczos method (Sec. 1, Sec. 4: its basic step is the
repeated application of H to a vector, Eq. (E-4-a)) but does not write the
recurrence out.  The oracle uses the textbook three-term recurrence in
Paige's ordering, in FP64:

    v_1 = v0 / |v0|,  v_0 = 0,  beta_0 = 0
    for k = 1, 2, ...:
        w       = H v_k - beta_{k-1} v_{k-1}
        alpha_k = <w, v_k>
        w       = w - alpha_k v_k
        [full reorthogonalization: twice  w = w - V_k (V_k^T w)]
        beta_k  = |w|
        stop if beta_k <= tol * max_{j<=k}(|alpha_j|, beta_j)
        v_{k+1} = w / beta_k

E0 is the smallest eigenvalue of the k x k tridiagonal matrix with diagonal
alpha_1..alpha_k and off-diagonal beta_1..beta_{k-1}; the library routine
scipy.linalg.eigh_tridiagonal (LAPACK's implicit QL/QR driver stev, which
also copes with the near-repeated Ritz values of runs continued past
convergence) serves as that step.  The ground-state
vector is the Ritz vector V_k c from the *stored* Krylov basis, and bond
correlations <psi| s(u).s(v) |psi> come from the oracle's own H x with a
coupling matrix that has a single entry J_uv = -1 (then H = s(u).s(v) by
Eq. (E-2-1)).  By Hellmann-Feynman, dE0/dJ_uv = -<s(u).s(v)>.
"""
import numpy as np
import scipy.linalg

from .core import Subspace


def lanczos(sub: Subspace, J, v0, steps: int, full_reorth: bool = False,
            tol: float = 1e-12, keep_basis: bool = False):
    """Run the recurrence above.

    Returns dict(alpha, beta, steps_done, E0, basis) where alpha and beta have
    length steps_done and basis is the (steps_done, dim) array of v_k (only if
    keep_basis or full_reorth).
    """
    J = np.asarray(J, dtype=np.float64)
    v = np.asarray(v0, dtype=np.float64).copy()
    if v.shape != (sub.dim,):
        raise ValueError("v0 must have length dim")
    v /= np.linalg.norm(v)
    v_prev = np.zeros_like(v)
    beta_prev = 0.0
    alphas, betas, basis = [], [], []
    scale = 0.0
    store = keep_basis or full_reorth
    for _ in range(steps):
        if store:
            basis.append(v.copy())
        w = sub.apply(J, v) - beta_prev * v_prev
        alpha = float(np.dot(w, v))
        w -= alpha * v
        if full_reorth:
            V = np.asarray(basis)
            for _rep in range(2):
                w -= V.T @ (V @ w)
        beta = float(np.linalg.norm(w))
        alphas.append(alpha)
        betas.append(beta)
        scale = max(scale, abs(alpha), beta)
        if beta <= tol * scale:
            break
        v_prev, v = v, w / beta
        beta_prev = beta
    alpha = np.array(alphas)
    beta = np.array(betas)
    E0, _ = ritz(alpha, beta)
    return dict(alpha=alpha, beta=beta, steps_done=len(alphas), E0=E0,
                basis=np.asarray(basis) if store else None)


def ritz(alpha, beta, which: int = 0):
    """Eigenpair `which` (0 = lowest) of tridiag(alpha; beta[:-1])."""
    alpha = np.asarray(alpha, dtype=np.float64)
    k = alpha.shape[0]
    off = np.asarray(beta, dtype=np.float64)[: k - 1]
    if k == 1:
        return float(alpha[0]), np.ones(1)
    w, z = scipy.linalg.eigh_tridiagonal(alpha, off, lapack_driver="stev")
    return float(w[which]), z[:, which].copy()


def ritz_all(alpha, beta):
    """All Ritz values and first components of the eigenvectors of T_k."""
    alpha = np.asarray(alpha, dtype=np.float64)
    k = alpha.shape[0]
    if k == 1:
        return alpha.copy(), np.ones(1)
    w, z = scipy.linalg.eigh_tridiagonal(
        alpha, np.asarray(beta, dtype=np.float64)[: k - 1], lapack_driver="stev")
    return w, z[0, :] ** 2


def ground_state(sub: Subspace, J, v0, steps: int, full_reorth: bool = False,
                 tol: float = 1e-12):
    """E0 and the normalized Ritz vector psi0 = V c from the stored basis."""
    res = lanczos(sub, J, v0, steps, full_reorth=full_reorth, tol=tol,
                  keep_basis=True)
    E0, c = ritz(res["alpha"], res["beta"])
    psi = res["basis"].T @ c
    psi /= np.linalg.norm(psi)
    res["psi"] = psi
    res["c"] = c
    return res


def bond_correlations(sub: Subspace, psi, bonds) -> np.ndarray:
    """<psi| s(u).s(v) |psi> for each bond (u, v), 0-based sites, u != v."""
    psi = np.asarray(psi, dtype=np.float64)
    out = np.empty(len(bonds))
    for b, (u, v) in enumerate(bonds):
        Jb = np.zeros((sub.N, sub.N))
        lo, hi = min(u, v), max(u, v)
        Jb[lo, hi] = Jb[hi, lo] = -1.0
        out[b] = float(np.dot(psi, sub.apply(Jb, psi)))
    return out

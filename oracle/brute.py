"""Brute-force references for tiny systems (numpy / scipy.sparse).

TEST INFRASTRUCTURE ONLY.  These helpers share nothing with oracle/oracle.c:
they build the full (2s+1)^N Hilbert space (Sec. 2) directly and are used to
pin the oracle.

  * the product basis |a_1..a_N> is numbered by the base-(2s+1) number
    sum_u a_u (2s+1)^(u-1), site 1 least significant, Eq. (E-3-a);
  * the basis of H(M) is found by scanning all those numbers and keeping the
    ones whose digit sum is A (the "generate all and sort out" route of
    Sec. 3.1), in ascending order;
  * the Hamiltonian of Eq. (E-2-1) is assembled from Kronecker products of the
    textbook spin-s matrices and restricted to H(M) by selecting rows and
    columns.
"""
import itertools

import numpy as np
import scipy.sparse as sp


def enumerate_subspace(N: int, two_s: int, A: int):
    """Digits (n_states, N) and full-space indices of H(M = N s - A)."""
    base = two_s + 1
    full = base ** N
    idx = np.arange(full, dtype=np.int64)
    digits = np.empty((full, N), dtype=np.int64)
    rest = idx.copy()
    for u in range(N):
        digits[:, u] = rest % base
        rest //= base
    keep = digits.sum(axis=1) == A
    return digits[keep], idx[keep]


def count_by_enumeration(N: int, two_s: int, A: int) -> int:
    """Number of N-digit strings over {0..2s} with digit sum A, by scanning."""
    if A < 0 or A > N * two_s:
        return 0
    total = 0
    for digits in itertools.product(range(two_s + 1), repeat=N):
        if sum(digits) == A:
            total += 1
    return total


def spin_matrices(two_s: int):
    """s_z, s_+ and s_- in the basis ordered by a = s - m = 0..2s."""
    s = two_s / 2.0
    m = s - np.arange(two_s + 1)           # m for a = 0, 1, ..., 2s
    sz = np.diag(m)
    sp_ = np.zeros((two_s + 1, two_s + 1))
    for a in range(1, two_s + 1):
        # s+ |s, m> = sqrt(s(s+1) - m(m+1)) |s, m+1>;  m+1 has digit a-1
        mm = m[a]
        sp_[a - 1, a] = np.sqrt(s * (s + 1) - mm * (mm + 1))
    return sz, sp_, sp_.T.copy()


def site_operator(op, u: int, N: int, two_s: int):
    """op acting on site u (0-based) of the full space; site 0 least significant."""
    dim = two_s + 1
    out = sp.identity(1, format="csr")
    # kron(X, Y): the index of Y varies fastest, so build from site N-1 down to 0
    for site in range(N - 1, -1, -1):
        factor = sp.csr_matrix(op) if site == u else sp.identity(dim, format="csr")
        out = sp.kron(out, factor, format="csr")
    return out


def full_hamiltonian(N: int, two_s: int, J):
    """H = - sum_{u<v} J_uv s(u).s(v) on the full (2s+1)^N space (sparse)."""
    J = np.asarray(J, dtype=np.float64)
    sz, spl, smi = spin_matrices(two_s)
    Sz = [site_operator(sz, u, N, two_s) for u in range(N)]
    Sp = [site_operator(spl, u, N, two_s) for u in range(N)]
    Sm = [site_operator(smi, u, N, two_s) for u in range(N)]
    full = (two_s + 1) ** N
    H = sp.csr_matrix((full, full))
    for u in range(N):
        for v in range(u + 1, N):
            if J[u, v] == 0.0:
                continue
            dot = Sz[u] @ Sz[v] + 0.5 * (Sp[u] @ Sm[v] + Sm[u] @ Sp[v])
            H = H - J[u, v] * dot
    return H.tocsr()


def bond_operator(N: int, two_s: int, u: int, v: int):
    """s(u).s(v) on the full space (sparse)."""
    sz, spl, smi = spin_matrices(two_s)
    return (site_operator(sz, u, N, two_s) @ site_operator(sz, v, N, two_s)
            + 0.5 * (site_operator(spl, u, N, two_s) @ site_operator(smi, v, N, two_s)
                     + site_operator(smi, u, N, two_s) @ site_operator(spl, v, N, two_s)))


def subspace_hamiltonian(N: int, two_s: int, A: int, J) -> np.ndarray:
    """Dense block of H on H(M), rows/columns in ascending base-(2s+1) order."""
    _, idx = enumerate_subspace(N, two_s, A)
    H = full_hamiltonian(N, two_s, J)
    return H[idx][:, idx].toarray()


def subspace_bond_operator(N: int, two_s: int, A: int, u: int, v: int):
    _, idx = enumerate_subspace(N, two_s, A)
    return bond_operator(N, two_s, u, v)[idx][:, idx].toarray()

"""Pins of the oracle's Lanczos recurrence, ground state and bond correlations.

References: dense diagonalization of the Kronecker-built block (oracle/brute.py),
closed forms (dimer, Majumdar-Ghosh ring), the Marshall sign rule, central
finite differences, Euler's identity for a Hamiltonian linear in J, and the
total-spin sum rule.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_0706_3293_amd import inputs


def dense_block(N, two_s, A, J):
    return brute.subspace_hamiltonian(N, two_s, A, J)


def test_ring12_energy_matches_dense():
    """N=12 s=1/2 ring, M=0, 120 steps with full reorthogonalization."""
    N = 12
    J = inputs.ring_couplings(N, -1.0)
    sub = oracle.Subspace(N, 1, 6)
    res = oracle.lanczos(sub, J, inputs.start_vector(sub.dim, 0), 120,
                         full_reorth=True)
    Hb = dense_block(N, 1, 6, J)
    exact = np.linalg.eigvalsh(Hb)[0]
    assert res["steps_done"] == 120
    assert abs(res["E0"] - exact) < 1e-12
    v1 = inputs.start_vector(sub.dim, 0)
    v1 /= np.linalg.norm(v1)
    assert abs(res["alpha"][0] - v1 @ Hb @ v1) < 1e-13


def test_majumdar_ghosh_point():
    """J2 = J1/2 < 0 on an even ring: E0 = -3N/8, twice degenerate."""
    for N in (8, 10, 12):
        J = inputs.ring_couplings(N, -1.0, -0.5)
        sub = oracle.Subspace(N, 1, N // 2)
        res = oracle.lanczos(sub, J, inputs.start_vector(sub.dim, 1), 80,
                             full_reorth=True)
        assert abs(res["E0"] + 3 * N / 8) < 1e-11
        ev = np.linalg.eigvalsh(dense_block(N, 1, N // 2, J))
        assert abs(ev[0] + 3 * N / 8) < 1e-11 and abs(ev[1] + 3 * N / 8) < 1e-11


def test_lanczos_general_spin_matches_dense():
    rng = np.random.default_rng(4)
    for N, two_s, A in ((7, 2, 7), (5, 3, 7), (4, 4, 8)):
        J = rng.normal(size=(N, N))
        J = np.triu(J, 1)
        J = J + J.T
        sub = oracle.Subspace(N, two_s, A)
        res = oracle.lanczos(sub, J, rng.uniform(-1, 1, sub.dim), min(sub.dim, 150),
                             full_reorth=True)
        exact = np.linalg.eigvalsh(dense_block(N, two_s, A, J))[0]
        assert abs(res["E0"] - exact) < 1e-10


def test_breakdown_on_exact_eigenvector():
    """The dimer singlet is an eigenvector: beta_1 = 0 stops the recurrence
    after one step with E0 = alpha_1 = J s(s+1) = -3/4 for J = -1."""
    J = np.array([[0.0, -1.0], [-1.0, 0.0]])
    sub = oracle.Subspace(2, 1, 1)
    singlet = np.array([1.0, -1.0])
    res = oracle.lanczos(sub, J, singlet, 10)
    assert res["steps_done"] == 1
    assert abs(res["E0"] + 0.75) < 1e-15
    # a 2-dimensional space is exhausted after two steps
    res = oracle.lanczos(sub, J, np.array([0.3, 0.9]), 10)
    assert res["steps_done"] == 2
    assert abs(res["E0"] + 0.75) < 1e-14


def test_ground_state_vector_and_marshall_sign():
    N = 12
    J = inputs.ring_couplings(N, -1.0)
    sub = oracle.Subspace(N, 1, 6)
    res = oracle.ground_state(sub, J, inputs.start_vector(sub.dim, 0), 120,
                              full_reorth=True)
    w, z = np.linalg.eigh(dense_block(N, 1, 6, J))
    assert abs(abs(res["psi"] @ z[:, 0]) - 1.0) < 1e-10
    # Marshall: sign(psi_i) = (-1)^(number of a_u = 1 on odd sites), up to a global sign
    signs = np.array([(-1) ** int(sub.unrank(i)[1::2].sum()) for i in range(sub.dim)])
    prod = np.sign(res["psi"]) * signs
    assert np.all(prod == prod[0])
    # ring translation invariance: every bond carries E0 / N
    C = oracle.bond_correlations(sub, res["psi"], [(u, (u + 1) % N) for u in range(N)])
    assert np.allclose(C, res["E0"] / N, atol=1e-10)


def _all_to_all(N, seed):
    J, bonds, vals = inputs.all_to_all_couplings(N, seed)
    return J, bonds, vals


def test_gradient_matches_dense_and_finite_differences():
    """dE0/dJ_uv = -<s(u).s(v)> (Hellmann-Feynman) on an N=8 all-to-all system."""
    N, A = 8, 4
    J, bonds, vals = _all_to_all(N, 0)
    sub = oracle.Subspace(N, 1, A)
    res = oracle.ground_state(sub, J, inputs.start_vector(sub.dim, 0), sub.dim,
                              full_reorth=True)
    C = oracle.bond_correlations(sub, res["psi"], bonds)
    grad = -C
    # dense gradient from the exact eigenvector
    Hb = dense_block(N, 1, A, J)
    w, z = np.linalg.eigh(Hb)
    assert w[1] - w[0] > 1e-3  # non-degenerate ground state
    dense_grad = np.array([-(z[:, 0] @ brute.subspace_bond_operator(N, 1, A, u, v) @ z[:, 0])
                           for u, v in bonds])
    assert np.abs(grad - dense_grad).max() < 1e-9
    # central finite differences of the dense E0, h = 1e-5
    h = 1e-5
    fd = []
    for b in range(len(bonds)):
        e = []
        for sgn in (+1, -1):
            vv = vals.copy()
            vv[b] += sgn * h
            Jb = inputs.bond_vector_to_matrix(N, bonds, vv)
            e.append(np.linalg.eigvalsh(dense_block(N, 1, A, Jb))[0])
        fd.append((e[0] - e[1]) / (2 * h))
    assert np.abs(grad - np.array(fd)).max() < 1e-8
    # Euler: H is linear in J, so sum_b J_b dE0/dJ_b = E0
    assert abs(np.dot(vals, grad) - res["E0"]) < 1e-10
    # all pairs covered: sum_b s(u).s(v) = (S^2 - N s(s+1)) / 2 with integer S
    S2 = 2 * C.sum() + N * 0.75
    S = (-1 + math.sqrt(1 + 4 * S2)) / 2
    assert abs(S - round(S)) < 1e-8


def test_bond_correlation_general_spin():
    N, two_s, A = 5, 2, 5
    rng = np.random.default_rng(9)
    J = rng.normal(size=(N, N))
    J = np.triu(J, 1)
    J = J + J.T
    sub = oracle.Subspace(N, two_s, A)
    w, z = np.linalg.eigh(dense_block(N, two_s, A, J))
    psi = z[:, 0]
    bonds = [(0, 1), (1, 3), (2, 4), (0, 4)]
    C = oracle.bond_correlations(sub, psi, bonds)
    for (u, v), c in zip(bonds, C):
        assert abs(c - psi @ brute.subspace_bond_operator(N, two_s, A, u, v) @ psi) < 1e-12


@pytest.mark.parametrize("two_s", [1, 2])
def test_spin_flip_symmetry(two_s):
    """E0(M) = E0(-M): sector A and sector 2Ns - A have the same spectrum."""
    N = 8 if two_s == 1 else 6
    rng = np.random.default_rng(1)
    J = rng.normal(size=(N, N))
    J = np.triu(J, 1)
    J = J + J.T
    for A in range(N * two_s + 1):
        a = oracle.Subspace(N, two_s, A)
        b = oracle.Subspace(N, two_s, N * two_s - A)
        ea = oracle.lanczos(a, J, rng.uniform(-1, 1, a.dim), a.dim, full_reorth=True)["E0"]
        eb = oracle.lanczos(b, J, rng.uniform(-1, 1, b.dim), b.dim, full_reorth=True)["E0"]
        assert abs(ea - eb) < 1e-10

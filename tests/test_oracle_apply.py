"""Pins of the oracle's row-gather H x (Sec. 4, Eq. (E-4-b)) and its spectrum.

The reference is the Hamiltonian of Eq. (E-2-1) assembled from Kronecker
products of the textbook spin-s matrices on the full (2s+1)^N space and
restricted to H(M) (oracle/brute.py), which shares nothing with the oracle's
digit arithmetic.
"""
import numpy as np
import pytest

import oracle
from oracle import brute
from paper_0706_3293_amd import inputs


def random_J(N, rng, density=1.0):
    J = rng.normal(size=(N, N))
    J = np.triu(J, 1)
    J *= rng.uniform(size=J.shape) < density
    return J + J.T


APPLY_CASES = [(6, 1), (9, 1), (12, 1), (5, 2), (7, 2), (4, 3), (5, 3), (4, 4), (3, 5)]


@pytest.mark.parametrize("N,two_s", APPLY_CASES)
def test_apply_matches_dense_kronecker(N, two_s):
    rng = np.random.default_rng(N * 10 + two_s)
    J = random_J(N, rng, density=0.7)
    H = brute.full_hamiltonian(N, two_s, J)
    for A in range(N * two_s + 1):
        digits, idx = brute.enumerate_subspace(N, two_s, A)
        block = H[idx][:, idx].toarray()
        sub = oracle.Subspace(N, two_s, A)
        x = rng.uniform(-1, 1, sub.dim)
        y = sub.apply(J, x)
        scale = np.abs(block).sum(axis=1).max() * np.abs(x).max() + 1e-300
        assert np.abs(y - block @ x).max() <= 1e-13 * scale, (A,)


@pytest.mark.parametrize("N,two_s", [(8, 1), (5, 2), (4, 3)])
def test_magnetization_blocks_cover_the_spectrum(N, two_s):
    """Rotation about z splits H into the H(M) blocks (Sec. 1, Sec. 3): the
    union of the block spectra is the full spectrum, and Tr H = 0."""
    rng = np.random.default_rng(3)
    J = random_J(N, rng)
    full = np.linalg.eigvalsh(brute.full_hamiltonian(N, two_s, J).toarray())
    parts, trace = [], 0.0
    for A in range(N * two_s + 1):
        sub = oracle.Subspace(N, two_s, A)
        cols = np.stack([sub.apply(J, e) for e in np.eye(sub.dim)], axis=1)
        assert np.allclose(cols, cols.T, atol=1e-13)   # H is real symmetric
        parts.append(np.linalg.eigvalsh(cols))
        trace += np.trace(cols)
    assert np.allclose(np.sort(np.concatenate(parts)), full, atol=1e-12)
    assert abs(trace) < 1e-11


def test_apply_rows_matches_apply():
    rng = np.random.default_rng(11)
    sub = oracle.Subspace(16, 1, 8)
    J = inputs.ring_couplings(16, -1.0, -0.3)
    x = rng.uniform(-1, 1, sub.dim)
    y = sub.apply(J, x)
    rows = rng.integers(0, sub.dim, 500)
    assert np.array_equal(sub.apply_rows(J, x, rows), y[rows])


def test_hashed_input_rows_match_apply():
    # the counter-based input: its values are exact multiples of 2^-24 in
    # [-1/2, 1/2), and rows computed from it equal H x with x materialized
    from oracle.core import hashed_input
    sub = oracle.Subspace(14, 2, 14)
    J = inputs.chain_couplings(np.linspace(-1.0, -0.5, 13))
    x = hashed_input(np.arange(sub.dim))
    assert x.min() >= -0.5 and x.max() < 0.5
    assert np.all(x * 2 ** 24 == np.round(x * 2 ** 24))
    assert hashed_input([0, 1])[0] == -0.5 and abs(hashed_input([1])[0] - 0.1180338) < 1e-6
    rows = np.random.default_rng(3).integers(0, sub.dim, 300)
    assert np.array_equal(sub.apply_rows_hashed(J, rows), sub.apply(J, x)[rows])


def test_dimer_closed_form():
    """Two spins: H = -J s1.s2 has E = -(J/2)[S(S+1) - 2 s(s+1)]."""
    for two_s in (1, 2, 3, 4):
        s = two_s / 2
        Jc = -1.3
        J = np.array([[0.0, Jc], [Jc, 0.0]])
        evals = []
        for A in range(2 * two_s + 1):
            sub = oracle.Subspace(2, two_s, A)
            Hb = np.stack([sub.apply(J, e) for e in np.eye(sub.dim)], axis=1)
            evals.extend(np.linalg.eigvalsh(Hb))
        expect = []
        for twoS in range(0, 2 * two_s + 1, 2):
            S = twoS / 2
            expect += [-(Jc / 2) * (S * (S + 1) - 2 * s * (s + 1))] * (twoS + 1)
        assert np.allclose(sorted(evals), sorted(expect), atol=1e-12)
        # M = 0 ground state for an antiferromagnetic coupling: J s(s+1)
        sub = oracle.Subspace(2, two_s, two_s)
        Hb = np.stack([sub.apply(J, e) for e in np.eye(sub.dim)], axis=1)
        assert np.isclose(np.linalg.eigvalsh(Hb)[0], Jc * s * (s + 1))


def test_ferromagnet_ground_state_in_every_sector():
    """All J >= 0 (ferromagnetic under the minus sign): E0 = -s^2 sum_{u<v} J."""
    rng = np.random.default_rng(2)
    for N, two_s in ((6, 2), (8, 1), (5, 3)):
        J = np.abs(random_J(N, rng))
        s = two_s / 2
        expect = -s * s * np.triu(J, 1).sum()
        for A in range(N * two_s + 1):
            sub = oracle.Subspace(N, two_s, A)
            Hb = np.stack([sub.apply(J, e) for e in np.eye(sub.dim)], axis=1)
            assert np.isclose(np.linalg.eigvalsh(Hb)[0], expect, atol=1e-10)


def test_uniform_complete_graph_closed_form():
    """H = -J sum_{u<v} s.s = -(J/2)(S^2 - N s(s+1)); for J < 0 the lowest
    state of sector M has total spin S = |M|."""
    Jc = -0.7
    for N, two_s in ((7, 1), (6, 2), (4, 3)):
        s = two_s / 2
        J = np.full((N, N), Jc)
        np.fill_diagonal(J, 0.0)
        for A in range(N * two_s + 1):
            M = N * s - A
            sub = oracle.Subspace(N, two_s, A)
            Hb = np.stack([sub.apply(J, e) for e in np.eye(sub.dim)], axis=1)
            S = abs(M)
            expect = -(Jc / 2) * (S * (S + 1) - N * s * (s + 1))
            assert np.isclose(np.linalg.eigvalsh(Hb)[0], expect, atol=1e-10)

"""Pins of the oracle's block Lanczos (CPU only): the p = 1 case is the scalar
recurrence, the lowest levels (degenerate ones included) are the dense
spectrum's, and the block basis is orthonormal with V^T H V = T."""
import numpy as np
import pytest

import oracle
from oracle import block, sectors


def _ring(N, J1, J2):
    from paper_0706_3293_amd import inputs
    return inputs.ring_couplings(N, J1, J2)


def test_single_column_is_the_scalar_recurrence():
    N, A = 10, 5
    sub = oracle.Subspace(N, 1, A)
    J = _ring(N, -1.0, -0.3)
    v0 = np.random.default_rng(0).uniform(-1, 1, sub.dim)
    Ab, Bb, _ = block.block_lanczos(sub, J, v0[:, None], 20)
    ref = oracle.lanczos(sub, J, v0, 20, full_reorth=True)
    assert np.allclose(Ab[:, 0, 0], ref["alpha"][:20], rtol=0, atol=1e-11)
    # R factors have positive diagonals: B_k = beta_k
    assert np.allclose(Bb[:, 0, 0], ref["beta"][:19], rtol=0, atol=1e-11)


@pytest.mark.parametrize("N,two_s,A,p", [(12, 1, 6, 4), (10, 1, 4, 2), (6, 2, 6, 4)])
def test_lowest_levels_match_dense_with_degeneracies(N, two_s, A, p):
    # a translation-invariant ring has +-k degenerate pairs in every sector;
    # the block recurrence resolves them
    sub = oracle.Subspace(N, two_s, A)
    J = _ring(N, -1.0, -0.3)
    exact = sectors.sector_spectrum(N, two_s, A, J)
    X0 = np.random.default_rng(p).uniform(-1, 1, (sub.dim, p))
    got = block.lowest_levels(sub, J, X0, 80, p)
    assert np.abs(got - exact[:p]).max() < 1e-10 * np.abs(exact).max()
    # the dense spectrum does have a degenerate pair among the lowest levels
    # for the s = 1/2 rings used here
    if two_s == 1:
        gaps = np.diff(exact[:p + 1])
        assert np.min(gaps) < 1e-10


def test_block_basis_orthonormal_and_projection():
    N, A, p = 10, 5, 4
    sub = oracle.Subspace(N, 1, A)
    J = _ring(N, -1.0, -0.2)
    X0 = np.random.default_rng(1).uniform(-1, 1, (sub.dim, p))
    Ab, Bb, V = block.block_lanczos(sub, J, X0, 6)
    assert np.abs(V.T @ V - np.eye(V.shape[1])).max() < 1e-12
    HV = np.column_stack([sub.apply(J, V[:, q]) for q in range(V.shape[1])])
    T = block.block_tridiagonal(Ab, Bb)
    assert np.abs(V.T @ HV - T).max() < 1e-11


def test_exhausted_space_and_rank_deficient_start():
    # dim 10 with p = 2: the block Krylov space is exhausted after 5 blocks
    # (no deflation: a fixed p stops at the first rank-deficient block); the
    # levels are then the full spectrum
    N, A = 5, 2
    sub = oracle.Subspace(N, 1, A)
    J = _ring(N, -1.0, 0.0) + _ring(N, 0.0, -0.4)
    X0 = np.random.default_rng(2).uniform(-1, 1, (sub.dim, 2))
    Ab, Bb, V = block.block_lanczos(sub, J, X0, 10)
    assert len(Ab) == 5
    got = np.linalg.eigvalsh(block.block_tridiagonal(Ab, Bb))
    exact = sectors.sector_spectrum(N, 1, A, J)
    for e in exact:
        assert np.abs(got - e).min() < 1e-10
    with pytest.raises(ValueError):
        block.block_lanczos(sub, J, np.column_stack([X0[:, 0], 2 * X0[:, 0]]), 3)

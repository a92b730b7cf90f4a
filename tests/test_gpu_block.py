"""GPU checks of block Lanczos (hm_block_lanczos) against the oracle's block
recurrence and the dense spectrum, including degenerate lowest levels."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _ring(N, J1, J2):
    from paper_0706_3293_amd import inputs
    return inputs.ring_couplings(N, J1, J2)


@pytest.mark.parametrize("N,two_s,A,p", [(12, 1, 6, 4), (12, 1, 5, 8), (10, 1, 5, 2),
                                         (12, 1, 6, 1), (7, 2, 7, 4), (14, 1, 7, 16)])
def test_block_coefficients_match_oracle(N, two_s, A, p):
    import oracle
    from oracle import block
    from paper_0706_3293_amd import Basis
    print("block lanczos", N, two_s, A, p, flush=True)
    b = Basis(N, two_s=two_s, two_M=N * two_s - 2 * A)
    sub = oracle.Subspace(N, two_s, A)
    J = _ring(N, -1.0, -0.3)
    X0 = np.random.default_rng(N + p).uniform(-1, 1, (b.dim, p))
    steps = 6
    Ag, Bg, k = b.block_lanczos(J, torch.tensor(X0, device="cuda"), steps)
    Ao, Bo, _ = block.block_lanczos(sub, J, X0, steps)
    assert k == steps
    scale = np.abs(Ao).max()
    assert np.abs(Ag - Ao).max() <= 1e-10 * scale
    assert np.abs(Bg - Bo[: steps - 1]).max() <= 1e-10 * scale


@pytest.mark.parametrize("N,two_s,A,p", [(12, 1, 6, 4), (7, 2, 7, 4), (16, 1, 8, 4)])
def test_lowest_levels_with_degeneracies_match_dense(N, two_s, A, p):
    from oracle import sectors
    from paper_0706_3293_amd import Basis
    b = Basis(N, two_s=two_s, two_M=N * two_s - 2 * A)
    J = _ring(N, -1.0, -0.3)
    exact = sectors.sector_spectrum(N, two_s, A, J) if b.dim <= 2000 else None
    got = b.lowest_levels(J, p, steps=100, p=p, seed=3)
    if exact is None:
        import oracle
        from oracle import block
        sub = oracle.Subspace(N, two_s, A)
        X0 = np.random.default_rng(5).uniform(-1, 1, (b.dim, p))
        exact = block.lowest_levels(sub, J, X0, 100, p)
    assert np.abs(got - exact[:p]).max() <= 1e-9 * np.abs(exact[:p]).max()


def test_block_lanczos_errors():
    from paper_0706_3293_amd import Basis, _lib
    b = Basis(10, two_s=1, two_M=0)
    J = _ring(10, -1.0, 0.0)
    x = torch.tensor(np.random.default_rng(0).uniform(-1, 1, (b.dim, 1)), device="cuda")
    with pytest.raises(_lib.HMError):          # rank-deficient start block
        b.block_lanczos(J, torch.cat([x, 2 * x], dim=1), 4)
    with pytest.raises(_lib.HMError):          # p not a power of two up to 16
        b.block_lanczos(J, x.repeat(1, 3) + torch.rand(b.dim, 3, dtype=torch.float64,
                                                       device="cuda"), 4)

"""GPU checks of the ablation kernels of hm_apply_kernel: the successor sweep
(kernel 3, against the oracle and bitwise equal to the generic kernel) and the column scatter with
atomic adds (kernel 4, equal up to the order of the additions)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _J(N, seed):
    rng = np.random.default_rng(seed)
    J = np.triu(rng.normal(size=(N, N)) * (rng.uniform(size=(N, N)) < 0.5), 1)
    return J + J.T


CASES = [
    # N, two_s, A: ragged run tails (dim not a multiple of 16), s = 1/2 .. 7/2,
    # the one-state sectors and a sector with a single ball
    (12, 1, 6), (13, 1, 5), (7, 2, 7), (6, 2, 1), (5, 3, 7), (4, 4, 8), (3, 7, 10),
    (9, 1, 0), (9, 1, 9), (16, 1, 8), (10, 2, 10),
]


@pytest.mark.parametrize("N,two_s,A", CASES)
def test_successor_sweep_matches_oracle_and_generic(N, two_s, A):
    """Kernel 3 against the oracle's row gather (FP64 and FP32 tolerances),
    and bitwise against the generic kernel (same per-row arithmetic)."""
    import oracle
    from paper_0706_3293_amd import Basis
    print("successor sweep", N, two_s, A, flush=True)
    b = Basis(N, two_s=two_s, two_M=N * two_s - 2 * A)
    sub = oracle.Subspace(N, two_s, A)
    J = _J(N, N + A)
    xh = np.random.default_rng(A).uniform(-1, 1, b.dim)
    scale = float(np.abs(sub.apply(np.abs(J), np.abs(xh))).max()) + 1e-300
    x = torch.tensor(xh, device="cuda")
    y3 = b.apply(J, x, kernel=3)
    assert np.abs(y3.cpu().numpy() - sub.apply(J, xh)).max() <= 1e-13 * scale
    x32 = x.float()
    y3f = b.apply(J, x32, kernel=3)
    ref32 = sub.apply(J, x32.double().cpu().numpy())
    assert np.abs(y3f.double().cpu().numpy() - ref32).max() <= 2e-6 * scale
    for xd, yd in ((x, y3), (x32, y3f)):
        assert torch.equal(b.apply(J, xd, kernel=1), yd)


@pytest.mark.parametrize("N,two_s,A", CASES)
def test_column_scatter_matches_oracle(N, two_s, A):
    import oracle
    from paper_0706_3293_amd import Basis
    print("column scatter", N, two_s, A, flush=True)
    b = Basis(N, two_s=two_s, two_M=N * two_s - 2 * A)
    sub = oracle.Subspace(N, two_s, A)
    J = _J(N, 2 * N + A)
    x = np.random.default_rng(A + 1).uniform(-1, 1, b.dim)
    ref = sub.apply(J, x)
    scale = float(np.abs(sub.apply(np.abs(J), np.abs(x))).max()) + 1e-300
    y = b.apply(J, torch.tensor(x, device="cuda"), kernel=4).cpu().numpy()
    assert np.abs(y - ref).max() <= 1e-13 * scale
    y32 = b.apply(J, torch.tensor(x, device="cuda").float(), kernel=4).double().cpu().numpy()
    ref32 = sub.apply(J, x.astype(np.float32).astype(np.float64))
    assert np.abs(y32 - ref32).max() <= 2e-6 * scale


def test_ablation_kernels_reject_wide_digits():
    from paper_0706_3293_amd import Basis, _lib
    b = Basis(3, two_s=17, two_M=3)           # 5 bits per digit
    J = _J(3, 0)
    x = torch.zeros(b.dim, dtype=torch.float64, device="cuda")
    for k in (3, 4):
        with pytest.raises(_lib.HMError):
            b.apply(J, x, kernel=k)
    with pytest.raises(_lib.HMError):
        b.apply(J, x, kernel=5)

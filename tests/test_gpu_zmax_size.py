"""Maximum-size checks: N=36, s=1/2, M=0 (dim 9,075,135,300 > 2^32), where
the kernels run with 64-bit indices.  The input x_j is the counter-based
value both sides compute from j (Knuth's multiplicative hash), so the oracle
checks sampled rows without holding the 36-72 GB vector."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

N = 36
GOLDEN = 0x9E3779B97F4A7C15 - (1 << 64)   # the hash constant as int64


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _hashed_x(dim, dtype):
    x = torch.empty(dim, dtype=dtype, device="cuda")
    chunk = 1 << 28
    for s in range(0, dim, chunk):
        n = min(chunk, dim - s)
        h = torch.arange(s, s + n, dtype=torch.int64, device="cuda") * GOLDEN
        x[s:s + n] = (((h >> 40) & 0xFFFFFF).to(torch.float64) / 16777216.0 - 0.5).to(dtype)
        del h
    return x


def _rows(dim):
    rng = np.random.default_rng(36)
    rows = np.sort(rng.integers(0, dim, 3000))
    return np.concatenate([[0, 1, dim // 2, dim - 2, dim - 1], rows])


@pytest.mark.parametrize("kernel,dtype", [(2, "f32"), (1, "f32"), (2, "f64")])
def test_n36_sampled_rows_with_64bit_indices(kernel, dtype):
    import oracle
    from oracle.core import hashed_input
    from paper_0706_3293_amd import Basis, inputs
    print("N=36 sampled rows", kernel, dtype, flush=True)
    b = Basis(N, two_s=1, two_M=0)
    assert b.dim == 9075135300 and b.dim > 2 ** 32
    tdt = torch.float32 if dtype == "f32" else torch.float64
    need = 2 * b.dim * (4 if dtype == "f32" else 8) + (8 << 30)
    if torch.cuda.mem_get_info()[0] < need:
        pytest.skip("not enough free device memory")
    J = inputs.ring_couplings(N, -1.0, -0.25)
    x = _hashed_x(b.dim, tdt)
    probe = np.array([0, 1, 12345, b.dim - 1])
    assert np.array_equal(x[torch.tensor(probe, device="cuda")].double().cpu().numpy(),
                          hashed_input(probe))
    y = b.apply(J, x, kernel=kernel)
    del x
    rows = _rows(b.dim)
    got = y[torch.tensor(rows, device="cuda")].double().cpu().numpy()
    del y
    torch.cuda.empty_cache()
    ref = oracle.Subspace(N, 1, N // 2).apply_rows_hashed(J, rows)
    scale = 0.5 * float(np.abs(np.triu(J, 1)).sum())     # |x| <= 1/2, |H| row sum bound
    tol = 2e-6 if dtype == "f32" else 1e-13
    assert np.abs(got - ref).max() <= tol * scale

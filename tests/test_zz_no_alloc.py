"""The bond correlations through the entry point that allocates nothing
(hm_bond_corr_noalloc), against hm_bond_corr on the same inputs: two calls
in a row on one GPU, the second with a smaller input, each bitwise equal to
hm_bond_corr (same kernels, same fixed-order sums) and within 1e-12 of the
oracle's correlations."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _noalloc(b, bonds, psi):
    from paper_0706_3293_amd import _lib
    from paper_0706_3293_amd.api import _stream
    uv = np.ascontiguousarray(np.asarray(bonds, dtype=np.int32).reshape(-1, 2))
    out = np.full(uv.shape[0], np.nan)
    _lib.check(_lib.lib().hm_bond_corr_noalloc(
        b.handle, uv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), uv.shape[0],
        ctypes.c_void_p(psi.data_ptr()), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        _stream()))
    return out


def test_noalloc_bond_corr_matches_allocating_entry_point():
    import oracle
    from paper_0706_3293_amd import Basis, inputs
    cases = [
        # larger input first: N=20 all-to-all (190 bonds, 184,756 rows)
        (20, 1, 10, inputs.all_to_all_couplings(20, 0)[1]),
        # then a smaller one: N=12 spin-1 chain, a few bonds, another basis
        (12, 2, 12, [(0, 1), (3, 7), (11, 2), (5, 6)]),
    ]
    for N, two_s, A, bonds in cases:
        b = Basis(N, two_s=two_s, two_M=N * two_s - 2 * A)
        sub = oracle.Subspace(N, two_s, A)
        psi_h = np.random.default_rng(N).uniform(-1, 1, b.dim)
        psi_h /= np.linalg.norm(psi_h)
        psi = torch.tensor(psi_h, device="cuda")
        got = _noalloc(b, bonds, psi)
        ref = b.bond_corr(bonds, psi)
        print(f"N={N} 2s={two_s} bonds={len(bonds)} max|noalloc - alloc| "
              f"{np.abs(got - ref).max():.1e}", flush=True)
        assert np.array_equal(got, ref)
        want = oracle.bond_correlations(sub, psi_h, bonds)
        assert np.abs(got - want).max() <= 1e-12


def test_noalloc_rejects_bad_and_oversized_input():
    from paper_0706_3293_amd import Basis, _lib
    b = Basis(24, two_s=1, two_M=0)
    psi = torch.zeros(b.dim, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.HMError):
        _noalloc(b, [(0, 0)], psi)
    many = [(u, v) for u in range(24) for v in range(u + 1, 24)]
    many = (many * 4)[:1000]            # 1000 bonds on 2.7e6 rows: > 4 MiB of partials
    with pytest.raises(_lib.HMError):
        _noalloc(b, many, psi)

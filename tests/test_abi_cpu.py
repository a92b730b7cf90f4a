"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and its host-side codec and argument checks behave as the
header documents (compared bit for bit with the oracle)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hm.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_0706_3293_amd import _lib
    return _lib.lib()


def test_header_symbols_are_exported(L):
    names = declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), f"{n} declared in hm.h but not exported"
    from paper_0706_3293_amd import _lib
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


def test_host_codec_matches_oracle():
    import oracle
    from paper_0706_3293_amd import Basis
    for N, two_s in ((10, 1), (6, 2), (5, 3), (4, 4), (3, 7)):
        for A in range(N * two_s + 1):
            b = Basis(N, two_s=two_s, two_M=N * two_s - 2 * A)
            sub = oracle.Subspace(N, two_s, A)
            assert b.dim == sub.dim and b.A == A
            for i in range(sub.dim):
                d = b.unrank(i)
                assert np.array_equal(d, sub.unrank(i))
                assert b.rank(d) == i


def test_host_codec_large_sampled():
    import oracle
    from paper_0706_3293_amd import Basis
    for N, two_s, two_M in ((32, 1, 0), (40, 1, 4), (20, 2, 0), (21, 3, 1)):
        b = Basis(N, two_s=two_s, two_M=two_M)
        sub = oracle.Subspace(N, two_s, (N * two_s - two_M) // 2)
        assert b.dim == sub.dim
        for i in np.random.default_rng(0).integers(0, b.dim, 200):
            d = b.unrank(int(i))
            assert np.array_equal(d, sub.unrank(int(i)))
            assert b.rank(d) == int(i)
        assert b.rank(b.unrank(b.dim - 1)) == b.dim - 1


def test_count_matches_oracle():
    import oracle
    from paper_0706_3293_amd import count
    for two_s in (1, 2, 3, 5):
        for n in range(0, 13):
            for A in range(-1, n * two_s + 2):
                assert count(n, two_s, A) == oracle.count(n, two_s, A)


def test_error_paths(L):
    from paper_0706_3293_amd import Basis, _lib
    with pytest.raises(_lib.HMError) as e:
        Basis(5, two_s=1, two_M=2)            # N*two_s - two_M odd
    assert e.value.code == _lib.HM_EINVAL
    with pytest.raises(_lib.HMError) as e:
        Basis(4, two_s=1, two_M=10)           # |M| > N s
    assert e.value.code == _lib.HM_EINVAL
    with pytest.raises(_lib.HMError) as e:
        Basis(0, two_s=1, two_M=0)
    assert e.value.code == _lib.HM_EINVAL
    with pytest.raises(_lib.HMError) as e:
        Basis(33, two_s=2, two_M=0)           # 33 * 2 bits > 64
    assert e.value.code == _lib.HM_ERANGE
    b = Basis(6, two_s=2, two_M=0)
    with pytest.raises(_lib.HMError):
        b.unrank(b.dim)
    with pytest.raises(_lib.HMError):
        b.unrank(-1)
    with pytest.raises(_lib.HMError):
        b.rank([3, 0, 0, 0, 0, 3])            # digit > 2s
    with pytest.raises(_lib.HMError):
        b.rank([1, 0, 0, 0, 0, 0])            # wrong digit sum
    # schedule and work-split arguments are checked on the host
    h = Basis(16, two_s=1, two_M=0)
    for args in ((15, 0, 0), (0, 96, 0), (0, 0, 3), (9, 0, 0)):
        if args == (9, 0, 0):
            h.set_schedule(*args)                # valid: K = 9
            continue
        with pytest.raises(_lib.HMError):
            h.set_schedule(*args)
    for mode in (-1, 3):
        assert L.hm_basis_set_staging(h.handle, mode) == _lib.HM_EINVAL
    assert L.hm_basis_set_staging(None, 1) == _lib.HM_EINVAL
    for mode in (0, 1, 2):
        assert L.hm_basis_set_staging(h.handle, mode) == _lib.HM_OK
    for ipw in (-1, 65537):
        assert L.hm_basis_set_items_per_wave(h.handle, ipw) == _lib.HM_EINVAL
    assert L.hm_basis_set_items_per_wave(None, 4) == _lib.HM_EINVAL
    for ipw in (0, 1, 64, 65536):
        assert L.hm_basis_set_items_per_wave(h.handle, ipw) == _lib.HM_OK
    out = ctypes.c_int64()
    assert L.hm_count(3, 0, 0, ctypes.byref(out)) == _lib.HM_EINVAL
    assert L.hm_count(3, 1, 0, None) == _lib.HM_EINVAL
    assert b"null" in L.hm_last_error()
    # host tridiagonal solver vs scipy on a random matrix
    import scipy.linalg
    from paper_0706_3293_amd import tridiag_lowest
    rng = np.random.default_rng(0)
    a, bb = rng.normal(size=50), rng.uniform(0.1, 1, 50)
    ev, vec = tridiag_lowest(a, bb)
    w, z = scipy.linalg.eigh_tridiagonal(a, bb[:49])
    assert abs(ev - w[0]) < 1e-12
    assert abs(abs(vec @ z[:, 0]) - 1) < 1e-10


@pytest.mark.parametrize("k", [1, 2, 5, 40, 300])
def test_tridiag_ritz_matches_lapack(k):
    # all Ritz values and Gauss weights vs LAPACK's tridiagonal eigensolver
    import scipy.linalg
    from paper_0706_3293_amd import tridiag_ritz
    rng = np.random.default_rng(k)
    a, b = rng.normal(size=k), rng.uniform(0.05, 1, max(k - 1, 0))
    vals, wts = tridiag_ritz(a, b)
    if k == 1:
        assert vals[0] == a[0] and wts[0] == 1.0
        return
    w, z = scipy.linalg.eigh_tridiagonal(a, b, lapack_driver="stev")
    scale = np.abs(a).max() + 2 * b.max()
    assert np.abs(vals - w).max() <= 1e-13 * k * scale
    assert np.abs(wts - z[0] ** 2).max() <= 1e-12
    assert abs(wts.sum() - 1.0) < 1e-13


def test_tridiag_ritz_decoupled_and_degenerate_blocks(L):
    # beta = 0 splits T; the start vector only sees the first block, so the
    # other blocks' eigenvalues get weight 0; repeated eigenvalues stay finite
    from paper_0706_3293_amd import tridiag_ritz
    a = np.array([2.0, 2.0, -1.0, 3.0, 3.0])
    b = np.array([1.0, 0.0, 0.5, 0.0])
    vals, wts = tridiag_ritz(a, b)
    want = np.sort(np.concatenate([[1.0, 3.0], np.linalg.eigvalsh([[-1.0, 0.5], [0.5, 3.0]]),
                                   [3.0]]))
    assert np.abs(vals - want).max() < 1e-14
    w_first = {1.0: 0.5, 3.0: 0.5}
    assert abs(wts.sum() - 1.0) < 1e-15
    assert abs(wts[np.argmin(np.abs(vals - 1.0))] - w_first[1.0]) < 1e-14
    assert L.hm_tridiag_ritz(0, None, None, None, None) == -1
    nan = np.array([np.nan, 1.0])
    p = nan.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.hm_tridiag_ritz(2, p, p, p, p) == -1


def test_half_integer_arguments():
    from fractions import Fraction
    from paper_0706_3293_amd import Basis
    b = Basis(3, Fraction(3, 2), Fraction(1, 2))
    assert (b.two_s, b.two_M, b.A) == (3, 1, 4)
    b = Basis(4, 0.5, 0)
    assert b.dim == 6

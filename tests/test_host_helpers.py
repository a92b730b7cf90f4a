"""Host-side helpers of the package that need no GPU, against the oracle's
independent versions."""
import numpy as np

from oracle import block, sectors


def test_thermo_sums_match_oracle():
    from paper_0706_3293_amd.sectors import thermo_sums
    rng = np.random.default_rng(0)
    lev = rng.normal(size=200) * 3
    w = rng.uniform(0, 2, 200)
    T = np.array([0.05, 0.3, 1.0, 7.0])
    got = thermo_sums(lev, w, T)
    want = sectors.thermo_from_levels(lev, w, T)
    for k in ("Z", "E", "C"):
        assert np.allclose(got[k], want[k], rtol=1e-12, atol=1e-14)
    assert got["E_min"] == want["E_min"]


def test_block_tridiagonal_assembly_matches_oracle():
    from paper_0706_3293_amd import block_tridiag_eigenvalues
    rng = np.random.default_rng(1)
    p, n = 3, 5
    A = rng.normal(size=(n, p, p))
    A = 0.5 * (A + A.transpose(0, 2, 1))
    B = np.triu(rng.normal(size=(n - 1, p, p)))
    got = block_tridiag_eigenvalues(A, B)
    want = np.linalg.eigvalsh(block.block_tridiagonal(A, B))
    assert np.allclose(got, want, rtol=0, atol=1e-12)


def test_sector_enumeration_and_multiplicity():
    from paper_0706_3293_amd import count
    from paper_0706_3293_amd.sectors import multiplicity, sector_two_M
    for N, two_s in ((7, 1), (6, 2), (5, 3)):
        tms = sector_two_M(N, two_s)
        assert tms[0] == N * two_s and min(tms) in (0, 1) and all(t >= 0 for t in tms)
        total = sum(multiplicity(t) * count(N, two_s, (N * two_s - t) // 2) for t in tms)
        assert total == (two_s + 1) ** N
        assert [(N * two_s - t) // 2 for t in tms] == sectors.sector_lowerings(N, two_s)

"""Host-side helpers of the package that need no GPU, against the oracle's
independent versions."""
import numpy as np
import pytest

from oracle import block, sectors


def test_thermo_sums_match_oracle():
    from paper_0706_3293_amd.sectors import thermo_sums
    rng = np.random.default_rng(0)
    lev = rng.normal(size=200) * 3
    w = rng.uniform(0, 2, 200)
    T = np.array([0.05, 0.3, 1.0, 7.0])
    got = thermo_sums(lev, w, T)
    want = sectors.thermo_from_levels(lev, w, T)
    for k in ("Z", "E"):
        assert np.allclose(got[k], want[k], rtol=1e-12, atol=1e-14)
    # C = (<H^2> - <H>^2) / T^2 cancels <H^2> against <H>^2: the library's
    # compensated sums are good to about an ulp of <H^2>, numpy's pairwise
    # sums of n terms to about log2(n) ulps, so |dC| <= (log2(n) + 4) ulps of
    # <H^2>, divided by T^2
    h2 = want["C"] * T ** 2 + want["E"] ** 2
    ulps = np.log2(len(lev)) + 4
    assert np.all(np.abs(got["C"] - want["C"]) <= ulps * np.finfo(float).eps * h2 / T ** 2)
    assert got["E_min"] == want["E_min"]


def test_ftl_sums_run_scales_and_errors():
    """Per-run weight scales equal pre-scaled weights of one run; bad input
    (T <= 0, non-finite levels, zero total weight) is rejected."""
    from paper_0706_3293_amd import _lib
    from paper_0706_3293_amd.sectors import ftl_sums, thermo_sums
    rng = np.random.default_rng(3)
    runs = [rng.normal(size=n) for n in (5, 1, 12)]
    wts = [rng.uniform(0, 1, len(r)) for r in runs]
    scales = [3.0, 0.5, 7.0]
    T = np.array([0.2, 1.5])
    got = ftl_sums(runs, wts, scales, T)
    want = thermo_sums(np.concatenate(runs), np.concatenate([w * s for w, s in zip(wts, scales)]), T)
    for k in ("Z", "E", "C"):
        assert np.allclose(got[k], want[k], rtol=1e-13, atol=0)
    with pytest.raises(_lib.HMError):
        ftl_sums(runs, wts, scales, np.array([0.0]))
    with pytest.raises(_lib.HMError):
        ftl_sums([np.array([np.nan])], [np.ones(1)], [1.0], T)
    with pytest.raises(_lib.HMError):
        ftl_sums([np.ones(3)], [np.zeros(3)], [1.0], T)


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


@pytest.mark.parametrize("p,n", [(1, 1), (1, 30), (2, 17), (4, 40), (8, 12), (16, 9)])
def test_block_tridiagonal_eigensolve_matches_lapack(p, n):
    """The library's host block eigensolve (Householder + implicit QR) against
    LAPACK's dense symmetric eigensolver, including a split (zero sub-diagonal
    block) and a repeated eigenvalue."""
    from paper_0706_3293_amd import block_tridiag_eigenvalues
    rng = np.random.default_rng(10 * p + n)
    A = rng.normal(size=(n, p, p))
    A = 0.5 * (A + A.transpose(0, 2, 1))
    B = np.triu(rng.normal(size=(max(n - 1, 1), p, p)))[: n - 1]
    if n > 4:
        B[n // 2] = 0.0                          # splits into two blocks
        A[-1] = np.eye(p) * A[0, 0, 0]           # a repeated eigenvalue
    T = block.block_tridiagonal(A, B)
    got = block_tridiag_eigenvalues(A, B)
    want = np.linalg.eigvalsh(T)
    assert np.abs(got - want).max() <= 1e-12 * max(1.0, np.abs(want).max())


def test_block_tridiagonal_eigensolve_rejects_bad_input():
    from paper_0706_3293_amd import _lib, block_tridiag_eigenvalues
    A = np.ones((2, 2, 2))
    B = np.ones((1, 2, 2))
    A[1, 0, 0] = np.nan
    with pytest.raises(_lib.HMError):
        block_tridiag_eigenvalues(A, B)


def test_sector_enumeration_and_multiplicity():
    from paper_0706_3293_amd import count
    from paper_0706_3293_amd.sectors import multiplicity, sector_two_M
    for N, two_s in ((7, 1), (6, 2), (5, 3)):
        tms = sector_two_M(N, two_s)
        assert tms[0] == N * two_s and min(tms) in (0, 1) and all(t >= 0 for t in tms)
        total = sum(multiplicity(t) * count(N, two_s, (N * two_s - t) // 2) for t in tms)
        assert total == (two_s + 1) ** N
        assert [(N * two_s - t) // 2 for t in tms] == sectors.sector_lowerings(N, two_s)


def test_autotune_candidates_and_bench_schedule_lookup(tmp_path, monkeypatch):
    """Host logic around the block kernel's schedules: the candidate list
    (staged splits only where the blocks fit and indices are 32-bit) and the
    benchmark's use of the schedule stored with the committed counters (only
    while the kernel source is unchanged, and traffic only for that schedule)."""
    import json
    import importlib.util
    import os
    from paper_0706_3293_amd import autotune
    c28 = autotune.candidates(28)
    assert all(len(s) == 4 and s[3] in (1, 2) for s in c28)
    staged = [s for s in c28 if s[3] == 2]
    assert staged and all(s[0] <= 11 and (s[2] <= 2 if s[0] == 11 else s[2] <= 4) for s in staged)
    assert all(28 - s[0] <= 24 for s in c28)
    assert not [s for s in autotune.candidates(36) if s[3] == 2]      # dim >= 2^32
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    path = tmp_path / "traffic.json"
    entry = {"schedule": [13, 256, 8, 1], "bytes_per_launch": 123.0}
    path.write_text(json.dumps({"kernel_sha1": bench.kernel_hash(),
                                "entries": {"w/f32_mixed": entry}}))
    monkeypatch.setattr(bench, "TRAFFIC", str(path))
    assert bench.stored_schedule("w", "f32_mixed") == (13, 256, 8, 1)
    assert bench.stored_schedule("w", "f64") is None
    assert bench.measured_traffic("w", "f32_mixed", (13, 256, 8, 1)) == 123.0
    assert bench.measured_traffic("w", "f32_mixed", (12, 256, 4, 1)) is None
    path.write_text(json.dumps({"kernel_sha1": "0" * 40, "entries": {"w/f32_mixed": entry}}))
    assert bench.stored_schedule("w", "f32_mixed") is None
    assert bench.measured_traffic("w", "f32_mixed", (13, 256, 8, 1)) is None

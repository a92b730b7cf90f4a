"""Pins of the oracle's count table, encoding, decoding and successor (Sec. 3).

Everything here is checked against something other than the oracle itself:
brute-force enumeration of all (2s+1)^N digit strings, closed forms for the
subspace dimensions, and the paper's own worked examples (tests/golden).
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import brute


def closed_form_count(N, two_s, A):
    """Coefficient of x^A in (1 + x + ... + x^{2s})^N by inclusion-exclusion."""
    if A < 0 or A > N * two_s:
        return 0
    if N == 0:
        return 1
    total = 0
    for j in range(0, N + 1):
        top = A - j * (two_s + 1) + N - 1
        if top < N - 1:
            break
        total += (-1) ** j * math.comb(N, j) * math.comb(top, N - 1)
    return total


@pytest.mark.parametrize("two_s", [1, 2, 3, 4, 5])
def test_count_table_matches_closed_form(two_s):
    N = 16 if two_s == 1 else 10
    D = oracle.count_table(N, two_s)
    for n in range(N + 1):
        for A in range(N * two_s + 1):
            assert D[n, A] == closed_form_count(n, two_s, A), (n, A)


@pytest.mark.parametrize("N,two_s", [(3, 1), (4, 2), (3, 3), (2, 4), (5, 2)])
def test_count_table_matches_enumeration(N, two_s):
    D = oracle.count_table(N, two_s)
    for A in range(N * two_s + 1):
        assert D[N, A] == brute.count_by_enumeration(N, two_s, A)


@pytest.mark.parametrize("two_s", [1, 2, 3])
def test_count_table_invariants(two_s):
    """Sum over A is (2s+1)^N (Sec. 2); D(N,A) = D(N, 2Ns - A) (s_z -> -s_z)."""
    N = 12
    D = oracle.count_table(N, two_s)
    for n in range(1, N + 1):
        assert D[n, : n * two_s + 1].sum() == (two_s + 1) ** n
        for A in range(n * two_s + 1):
            assert D[n, A] == D[n, n * two_s - A]


def test_count_boundaries_from_paper(golden):
    """Seed values stated with Eq. (E-3-c)."""
    for two_s in (1, 2, 3, 4):
        N = 7
        D = oracle.count_table(N, two_s)
        assert all(D[1, A] == 1 for A in range(two_s + 1))
        for n in range(1, N + 1):
            assert D[n, 0] == 1
            assert D[n, 1] == n
        assert oracle.count(N, two_s, -1) == 0
        assert oracle.count(N, two_s, N * two_s + 1) == 0


def test_spin_half_is_binomial():
    D = oracle.count_table(40, 1)
    for n in range(41):
        for A in range(n + 1):
            assert D[n, A] == math.comb(n, A)


def test_workload_dimensions():
    """Dimensions of the measured workloads from independent closed forms."""
    assert oracle.count(12, 1, 6) == math.comb(12, 6) == 924
    assert oracle.count(28, 1, 14) == math.comb(28, 14) == 40116600
    assert oracle.count(20, 1, 10) == math.comb(20, 10) == 184756
    assert oracle.count(32, 1, 16) == math.comb(32, 16) == 601080390

    def central_trinomial(n):
        return sum(math.comb(n, 2 * k) * math.comb(2 * k, k) for k in range(n // 2 + 1))

    for n, expect in ((8, 1107), (10, 8953), (12, 73789), (14, 616227)):
        assert oracle.count(n, 2, n) == central_trinomial(n) == expect


def test_full_basis_order_matches_paper_listing(golden):
    """Eq. (E-3-a): the full basis is ordered as base-(2s+1) numbers, a_1 lowest."""
    g = golden["full_basis_order"]
    N, two_s = g["N"], g["two_s"]
    digits, idx = brute.enumerate_subspace(N, two_s, 0)  # A=0: only |0..0>
    assert list(digits[0]) == g["first_states"][0]
    full = list(itertools.product(range(two_s + 1), repeat=N))
    # itertools varies the last position fastest; reverse so a_1 varies fastest
    ordered = [tuple(reversed(t)) for t in full]
    assert [list(t) for t in ordered[:4]] == g["first_states"]
    assert list(ordered[-1]) == g["last_state"]


CODEC_CASES = [(8, 1), (12, 1), (6, 2), (7, 2), (4, 3), (5, 4), (4, 5), (3, 7)]


@pytest.mark.parametrize("N,two_s", CODEC_CASES)
def test_rank_unrank_exhaustive_vs_enumeration(N, two_s):
    """Decoding i gives the i-th state of the filtered, ascending full basis;
    encoding inverts it (Sec. 3.1, 3.2), for every subspace A."""
    for A in range(N * two_s + 1):
        digits, _ = brute.enumerate_subspace(N, two_s, A)
        sub = oracle.Subspace(N, two_s, A)
        assert sub.dim == digits.shape[0]
        for i in range(sub.dim):
            a = sub.unrank(i)
            assert np.array_equal(a, digits[i]), (A, i)
            assert sub.rank(digits[i]) == i


@pytest.mark.parametrize("N,two_s", CODEC_CASES)
def test_successor_walks_the_whole_subspace(N, two_s):
    for A in range(N * two_s + 1):
        digits, _ = brute.enumerate_subspace(N, two_s, A)
        sub = oracle.Subspace(N, two_s, A)
        cur = digits[0]
        for i in range(1, digits.shape[0]):
            cur = sub.successor(cur)
            assert cur is not None and np.array_equal(cur, digits[i]), (A, i)
        assert sub.successor(cur) is None


def test_successor_worked_example(golden):
    g = golden["successor_example"]
    sub = oracle.Subspace(g["N"], g["two_s"], g["A"])
    assert list(sub.successor(g["state"])) == g["successor"]
    # the position named in the example is the first k with a_k > 0, a_{k+1} < 2s
    st = g["state"]
    k = next(u for u in range(g["N"] - 1) if st[u] > 0 and st[u + 1] < g["two_s"])
    assert k + 1 == g["first_position_1based"]


def test_rank_worked_example(golden):
    """Sec. 3.2: the position is one plus the listed subspace dimensions.

    The dimensions are counted by brute-force enumeration, and the position of
    the example state is found by scanning the ordered subspace."""
    g = golden["rank_example"]
    N, two_s, A = g["N"], g["two_s"], g["A"]
    terms = sum(brute.count_by_enumeration(n, two_s, a) for n, a in g["terms_D_n_A"])
    digits, _ = brute.enumerate_subspace(N, two_s, A)
    scanned = next(i for i in range(digits.shape[0])
                   if list(digits[i]) == g["state"])
    assert scanned == terms  # 0-based position = sum of the terms
    assert oracle.Subspace(N, two_s, A).rank(g["state"]) == terms
    assert terms + 1 == 42


def test_rank_unrank_large_sampled():
    """N=32, s=1/2: the index equals the colex rank sum_t C(c_t, t) of the set
    positions (combinatorial number system), an independent closed form."""
    sub = oracle.Subspace(32, 1, 16)
    rng = np.random.default_rng(5)
    for i in rng.integers(0, sub.dim, 300):
        a = sub.unrank(int(i))
        pos = np.nonzero(a)[0]
        colex = sum(math.comb(int(c), t + 1) for t, c in enumerate(pos))
        assert colex == i
        assert sub.rank(a) == i


def test_codec_rejects_bad_input():
    sub = oracle.Subspace(6, 2, 5)
    with pytest.raises(IndexError):
        sub.unrank(sub.dim)
    with pytest.raises(IndexError):
        sub.unrank(-1)
    with pytest.raises(ValueError):
        sub.rank([3, 0, 0, 2, 0, 0])      # digit above 2s
    with pytest.raises(ValueError):
        sub.rank([1, 0, 0, 0, 0, 0])      # wrong digit sum


def test_single_site_and_extreme_subspaces():
    for two_s in (1, 2, 3):
        for A in range(two_s + 1):
            sub = oracle.Subspace(1, two_s, A)
            assert sub.dim == 1
            assert list(sub.unrank(0)) == [A]
        sub = oracle.Subspace(9, two_s, 0)
        assert sub.dim == 1 and not sub.unrank(0).any()
        sub = oracle.Subspace(9, two_s, 9 * two_s)
        assert sub.dim == 1 and (sub.unrank(0) == two_s).all()


@pytest.mark.parametrize("N,two_s", [(8, 1), (6, 2), (4, 3), (3, 7)])
def test_unrank_range_matches_enumeration(N, two_s):
    """The batch decoder returns the filtered, ascending full basis."""
    for A in range(N * two_s + 1):
        digits, _ = brute.enumerate_subspace(N, two_s, A)
        sub = oracle.Subspace(N, two_s, A)
        assert np.array_equal(sub.unrank_range(0, sub.dim), digits.astype(np.uint8)), A
        if sub.dim > 2:
            assert np.array_equal(sub.unrank_range(1, sub.dim - 2),
                                  digits[1:-1].astype(np.uint8))


def test_unrank_range_colex_closed_form():
    """s=1/2, N=20, M=0: every decoded state's colex rank sum_t C(c_t, t)
    equals its index (combinatorial number system)."""
    sub = oracle.Subspace(20, 1, 10)
    d = sub.unrank_range(0, sub.dim).astype(np.int64)
    assert (d.sum(axis=1) == 10).all()
    C = np.array([[math.comb(n, k) for k in range(21)] for n in range(21)], dtype=np.int64)
    t = np.cumsum(d, axis=1)                      # ordinal of each set bit
    pos = np.arange(20)[None, :]
    colex = (d * C[pos, t]).sum(axis=1)
    assert np.array_equal(colex, np.arange(sub.dim))
    with pytest.raises(IndexError):
        sub.unrank_range(sub.dim - 1, 2)

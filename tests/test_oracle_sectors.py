"""Pins of the oracle's magnetization sectors and thermodynamic sums against
closed forms, brute force and exact identities (CPU only)."""
import numpy as np
import pytest

import oracle
from oracle import brute, sectors


def _random_J(N, seed):
    rng = np.random.default_rng(seed)
    J = np.triu(rng.normal(size=(N, N)), 1)
    return J + J.T


@pytest.mark.parametrize("N,two_s", [(7, 1), (5, 2), (4, 3)])
def test_saturated_sector_closed_form(N, two_s):
    # A = 0: all sites at m = s, a single state with E = -s^2 sum_{u<v} J_uv
    J = _random_J(N, 1)
    s = two_s / 2
    E = sectors.sector_spectrum(N, two_s, 0, J)
    assert E.shape == (1,)
    assert abs(E[0] + s * s * np.triu(J, 1).sum()) < 1e-12


@pytest.mark.parametrize("N,two_s", [(8, 1), (6, 2), (5, 3)])
def test_one_magnon_sector_is_laplacian_spectrum(N, two_s):
    # A = 1: states |u> with site u lowered once; H = E_sat + s L(J) with the
    # graph Laplacian L = diag(sum_v J_uv) - J (diagonal: bonds at u lose
    # J_uv s; hop u -> v: -(J_uv/2) sqrt(2s) sqrt(2s) = -s J_uv)
    J = _random_J(N, 2)
    s = two_s / 2
    E_sat = -s * s * np.triu(J, 1).sum()
    L = np.diag(J.sum(axis=1)) - J
    want = np.sort(E_sat + s * np.linalg.eigvalsh(L))
    got = sectors.sector_spectrum(N, two_s, 1, J)
    assert np.abs(got - want).max() < 1e-11


def test_ring_one_magnon_dispersion():
    # ring with J1, J2: E(k) = E_sat + sum_d 2 J_d s (1 - cos(d k)), k = 2 pi n / N
    from paper_0706_3293_amd import inputs
    N, J1, J2, s = 10, -1.0, -0.3, 0.5
    J = inputs.ring_couplings(N, J1, J2)
    k = 2 * np.pi * np.arange(N) / N
    E_sat = -s * s * np.triu(J, 1).sum()
    want = np.sort(E_sat + 2 * s * (J1 * (1 - np.cos(k)) + J2 * (1 - np.cos(2 * k))))
    assert np.abs(sectors.sector_spectrum(N, 1, 1, J) - want).max() < 1e-12


@pytest.mark.parametrize("N,two_s", [(8, 1), (5, 2)])
def test_su2_nesting_of_sector_spectra(N, two_s):
    # H commutes with total S^2: every level of sector M + 1 also lies in M
    # (for M >= 0), so E0(M) is non-decreasing in M >= 0
    J = _random_J(N, 3)
    specs = [sectors.sector_spectrum(N, two_s, A, J) for A in sectors.sector_lowerings(N, two_s)]
    for lo, hi in zip(specs[:-1], specs[1:]):      # A, A + 1: hi has the smaller M
        for e in lo:
            assert np.abs(hi - e).min() < 1e-9
    E0 = [sp[0] for sp in specs]
    assert all(E0[i] >= E0[i + 1] - 1e-12 for i in range(len(E0) - 1))


@pytest.mark.parametrize("N,two_s", [(7, 1), (4, 2), (3, 3)])
def test_sector_dimensions_cover_the_space(N, two_s):
    total = sum(sectors.multiplicity(N, two_s, A) * oracle.count(N, two_s, A)
                for A in sectors.sector_lowerings(N, two_s))
    assert total == (two_s + 1) ** N


def test_sector_energies_match_kronecker_spectrum():
    # lowest level of each sector = lowest eigenvalue of the Kronecker H on the
    # states with that M (brute force)
    N, two_s = 6, 1
    J = _random_J(N, 4)
    E0 = sectors.sector_energies(N, two_s, J)
    for A, e in zip(sectors.sector_lowerings(N, two_s), E0):
        Hs = brute.subspace_hamiltonian(N, two_s, A, J)
        assert abs(np.linalg.eigvalsh(Hs)[0] - e) < 1e-12


def test_exact_thermodynamics_two_sites():
    # two spins 1/2, H = -J s1.s2: triplet -J/4 (x3), singlet 3J/4
    Jv = 0.8
    J = np.array([[0.0, Jv], [Jv, 0.0]])
    T = np.array([0.1, 0.5, 1.0, 3.0])
    got = sectors.exact_thermodynamics(2, 1, J, T)
    lev = np.array([-Jv / 4] * 3 + [3 * Jv / 4])
    b = np.exp(-lev[None, :] / T[:, None])
    Z = b.sum(axis=1)
    E = (b * lev).sum(axis=1) / Z
    C = ((b * lev ** 2).sum(axis=1) / Z - E ** 2) / T ** 2
    assert np.allclose(got["E"], E, rtol=0, atol=1e-14)
    assert np.allclose(got["C"], C, rtol=1e-12, atol=1e-14)
    assert np.allclose(got["Z"] * np.exp(-got["E_min"] / T), Z, rtol=1e-13)


def test_exact_thermodynamics_matches_full_kronecker_spectrum():
    N, two_s = 6, 1
    J = _random_J(N, 5)
    T = np.array([0.2, 1.0, 4.0])
    got = sectors.exact_thermodynamics(N, two_s, J, T)
    lev = np.linalg.eigvalsh(brute.full_hamiltonian(N, two_s, J).toarray())
    want = sectors.thermo_from_levels(lev, np.ones_like(lev), T)
    for key in ("Z", "E", "C"):
        assert np.allclose(got[key], want[key], rtol=1e-11, atol=1e-12)
    # H is traceless: <H> -> 0 as T -> infinity
    assert abs(sectors.exact_thermodynamics(N, two_s, J, [1e8])["E"][0]) < 1e-6


def test_ftl_exact_with_canonical_start_vectors():
    # start vectors e_1..e_D of each sector and runs to breakdown (full
    # reorthogonalization, so the run stops when the Krylov space is exhausted):
    # the Gauss
    # quadrature sum_j |<e_i|y_j>|^2 f(theta_j) = <e_i|f(H)|e_i> is exact, and
    # the sum over i with weight D / R = 1 is the trace
    N, two_s = 6, 1
    J = _random_J(N, 6)
    T = np.array([0.3, 1.0, 2.5])
    V0s = [np.eye(oracle.count(N, two_s, A)) for A in sectors.sector_lowerings(N, two_s)]
    got = sectors.ftl_thermodynamics(N, two_s, J, V0s, steps=64, temps=T, full_reorth=True)
    want = sectors.exact_thermodynamics(N, two_s, J, T)
    for key in ("E", "C"):
        assert np.allclose(got[key], want[key], rtol=1e-9, atol=1e-11)
    assert np.allclose(got["Z"] * np.exp(-got["E_min"] / T),
                       want["Z"] * np.exp(-want["E_min"] / T), rtol=1e-9)


def test_ftl_sum_rule_and_low_temperature_limit():
    # each run's Gauss weights sum to 1, so Z(T -> infinity) = sum_M mult D_M;
    # as T -> 0, <H> -> the lowest level over all sectors
    from paper_0706_3293_amd import inputs
    N, two_s = 8, 1
    J = inputs.ring_couplings(N, -1.0, -0.2)
    rng = np.random.default_rng(7)
    V0s = [rng.uniform(-1, 1, (4, oracle.count(N, two_s, A)))
           for A in sectors.sector_lowerings(N, two_s)]
    lev, w = sectors.ftl_levels(N, two_s, J, V0s, steps=40)
    assert abs(w.sum() - 2 ** N) < 1e-9 * 2 ** N
    E0 = sectors.sector_energies(N, two_s, J).min()
    lowT = sectors.thermo_from_levels(lev, w, [1e-3])
    assert abs(lowT["E"][0] - E0) < 1e-8

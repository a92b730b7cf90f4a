"""GPU checks of the magnetization curve E0(M) and the finite-temperature
Lanczos sums (all sectors in one batched launch) against the oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _random_chain(N, seed):
    rng = np.random.default_rng(seed)
    J = np.zeros((N, N))
    for u in range(N - 1):
        J[u, u + 1] = J[u + 1, u] = rng.normal(-1.0, 0.3)
    return J


@pytest.mark.parametrize("N,two_s,kind,method", [
    (12, 1, "ring", "batched"), (12, 1, "ring", "single"), (8, 2, "chain", "auto"),
    (5, 3, "chain", "auto"), (6, 2, "chain", "single")])
def test_magnetization_curve_matches_oracle(N, two_s, kind, method):
    from oracle import sectors as osec
    from paper_0706_3293_amd import inputs, magnetization_curve
    print("magnetization curve", N, two_s, kind, method, flush=True)
    J = inputs.ring_couplings(N, -1.0, -0.3) if kind == "ring" else _random_chain(N, N)
    curve = magnetization_curve(N, two_s, J, steps=150, nvec=2, seed=1, method=method)
    want = osec.sector_energies(N, two_s, J)
    assert list(curve.two_M) == [N * two_s - 2 * A for A in osec.sector_lowerings(N, two_s)]
    s = two_s / 2
    scale = s * s * np.abs(np.triu(J, 1)).sum()
    # FP32 vectors, FP64 coefficients: relative 1e-6 of the energy scale
    assert np.abs(curve.E0 - want).max() <= 1e-6 * scale
    # the saturated sector is one state, E = -s^2 sum_{u<v} J_uv, reached in one step
    assert abs(curve.E0[0] + s * s * np.triu(J, 1).sum()) <= 1e-6 * scale
    assert curve.steps_done[0].max() == 1


def test_magnetization_curve_closed_forms():
    # saturated sector and one-magnon dispersion of a J1-J2 ring
    from paper_0706_3293_amd import inputs, magnetization_curve
    N, J1, J2, s = 16, -1.0, -0.25, 0.5
    J = inputs.ring_couplings(N, J1, J2)
    curve = magnetization_curve(N, 1, J, steps=200, nvec=1, seed=3)
    E_sat = -s * s * np.triu(J, 1).sum()
    k = 2 * np.pi * np.arange(N) / N
    E1 = E_sat + (2 * s * (J1 * (1 - np.cos(k)) + J2 * (1 - np.cos(2 * k)))).min()
    assert abs(curve.E0[0] - E_sat) < 1e-6
    assert abs(curve.E0[1] - E1) < 1e-5
    # antiferromagnetic couplings: E0(M) non-decreasing in M >= 0 (SU(2) nesting)
    assert np.all(np.diff(curve.E0) <= 1e-5)


def test_ftl_matches_oracle_with_same_start_vectors():
    import oracle
    from oracle import sectors as osec
    from paper_0706_3293_amd import ftl_thermodynamics, inputs
    N, two_s, R, steps = 10, 1, 4, 40
    J = inputs.ring_couplings(N, -1.0, -0.4)
    T = np.array([0.25, 0.5, 1.0, 2.0, 5.0])
    rng = np.random.default_rng(11)
    V0s = [rng.uniform(-1, 1, (R, oracle.count(N, two_s, A)))
           for A in osec.sector_lowerings(N, two_s)]
    got = ftl_thermodynamics(N, two_s, J, T, steps=steps, nvec=R, V0s=V0s)
    want = osec.ftl_thermodynamics(N, two_s, J, V0s, steps, T)
    # every run's Gauss weights sum to 1: Z(T -> infinity) = 2^N
    assert abs(got["weights"].sum() - 2 ** N) < 1e-9 * 2 ** N
    assert got["total_dim"] == 2 ** N
    assert np.allclose(got["E"], want["E"], rtol=2e-5, atol=1e-6)
    assert np.allclose(got["C"], want["C"], rtol=2e-4, atol=1e-5)
    zg = got["Z"] * np.exp(-got["E_min"] / T)
    zw = want["Z"] * np.exp(-want["E_min"] / T)
    assert np.allclose(zg, zw, rtol=2e-5)


def test_ftl_random_vectors_approach_exact_thermodynamics():
    # an estimator, not an identity: 16 random vectors per sector bring E(T)
    # within a few percent of the exact value at moderate T and the lowest
    # level at low T
    from oracle import sectors as osec
    from paper_0706_3293_amd import ftl_thermodynamics, inputs
    N, two_s = 12, 1
    J = inputs.ring_couplings(N, -1.0, -0.2)
    T = np.array([0.5, 1.0, 2.0])
    got = ftl_thermodynamics(N, two_s, J, T, steps=60, nvec=16, seed=5)
    ex = osec.exact_thermodynamics(N, two_s, J, T)
    assert np.allclose(got["E"], ex["E"], rtol=0.05, atol=0.05)
    low = ftl_thermodynamics(N, two_s, J, [1e-3], steps=60, nvec=2, seed=6)
    assert abs(low["E"][0] - ex["E_min"]) < 1e-5 * abs(ex["E_min"])

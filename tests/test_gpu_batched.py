"""GPU checks of the batched persistent Lanczos (hm_lanczos_batched).

Each (instance, start vector) pair must reproduce the single-instance path on
the same inputs (FP32-mixed, tolerance for the different FP32 summation
order), the oracle's FP64 energies, and the per-pair breakdown handling.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rand_J(N, rng):
    J = np.triu(rng.normal(size=(N, N)), 1)
    return J + J.T


@pytest.mark.parametrize("nvec", [3, 7, 12])
def test_batched_heterogeneous_spin_half_vs_single_and_oracle(nvec):
    """nvec 3, 7, 12 run 4, 8 and 16 columns: one lane per row, and rows
    shared by 2 and 4 lanes."""
    import oracle
    from paper_0706_3293_amd import Basis, lanczos_batched
    print("batched vs single and oracle, nvec", nvec, flush=True)
    rng = np.random.default_rng(nvec)
    specs = [(8, 4), (10, 5), (12, 6), (10, 3), (14, 7), (6, 3), (9, 4)]
    bases, Js, V0s = [], [], []
    for N, A in specs:
        b = Basis(N, two_s=1, two_M=N - 2 * A)
        bases.append(b)
        Js.append(_rand_J(N, rng))
        V0s.append(rng.uniform(-1, 1, (nvec, b.dim)))
    steps = 40
    res = lanczos_batched(bases, Js, V0s, steps)
    for k, (N, A) in enumerate(specs):
        sub = oracle.Subspace(N, 1, A)
        for r in range(nvec):
            v0 = torch.tensor(V0s[k][r], device="cuda")
            single = bases[k].lanczos(Js[k], v0, steps, precision="f32_mixed")
            ref = oracle.lanczos(sub, Js[k], V0s[k][r], steps)
            assert res.steps_done[k, r] == single.steps_done == ref["steps_done"], (k, r)
            n = min(10, single.steps_done)
            assert np.abs(res.alpha[k, r, :n] - single.alpha[:n]).max() < 1e-5
            assert abs(res.E0[k, r] - ref["E0"]) <= 1e-6 * abs(ref["E0"])


def test_batched_spin_one_chains_subset():
    """The spin-1 chain workload (a subset of its instances), 16 vectors."""
    from paper_0706_3293_amd import Basis, inputs, lanczos_batched
    inst = inputs.batched_instances(lambda n: Basis(n, two_s=2, two_M=0).dim, count=64)[:8]
    bases = [Basis(d["N"], two_s=2, two_M=0) for d in inst]
    res = lanczos_batched(bases, [d["J"] for d in inst], [d["V0"] for d in inst], 80)
    for k, d in enumerate(inst):
        e = res.E0[k]
        ref = bases[k].lanczos(d["J"], torch.tensor(d["V0"][0], device="cuda"), 200)
        print(f"instance {k}: N={d['N']} E0 spread {e.max() - e.min():.2e} "
              f"vs f64 {e.min() - ref.E0:.2e}", flush=True)
        assert np.all(np.isfinite(e))
        assert e.min() >= ref.E0 - 1e-6 * abs(ref.E0)        # variational bound
        assert abs(np.median(e) - ref.E0) <= 1e-5 * abs(ref.E0)


def test_batched_breakdown_and_padding():
    """nvec = 5 (padded to 8 columns); one start vector is an exact eigenvector."""
    from paper_0706_3293_amd import Basis, lanczos_batched
    b = Basis(2, two_s=1, two_M=0)
    J = np.array([[0.0, -1.0], [-1.0, 0.0]])
    V = np.array([[1.0, -1.0], [0.3, 0.9], [1.0, 1.0], [0.2, -0.7], [2.0, 0.5]])
    res = lanczos_batched([b], [J], [V], 10)
    assert res.steps_done[0, 0] == 1 and abs(res.E0[0, 0] + 0.75) < 1e-6
    assert res.steps_done[0, 2] == 1 and abs(res.E0[0, 2] - 0.25) < 1e-6   # triplet
    for r in (1, 3, 4):
        assert res.steps_done[0, r] == 2 and abs(res.E0[0, r] + 0.75) < 1e-6


def test_batched_rejects_bad_input():
    from paper_0706_3293_amd import Basis, _lib, lanczos_batched
    b1 = Basis(4, two_s=1, two_M=0)
    b2 = Basis(3, two_s=2, two_M=0)
    J4, J3 = np.zeros((4, 4)), np.zeros((3, 3))
    J4[0, 1] = J4[1, 0] = 1.0
    J3[0, 1] = J3[1, 0] = 1.0
    with pytest.raises(_lib.HMError):
        lanczos_batched([b1, b2], [J4, J3], [np.ones((2, b1.dim)), np.ones((2, b2.dim))], 5)
    with pytest.raises(_lib.HMError):
        lanczos_batched([b1], [J4], [np.zeros((2, b1.dim))], 5)


def test_batched_full_workload_runs():
    """64 spin-1 chains x 16 vectors x 80 steps in one launch."""
    import time
    from paper_0706_3293_amd import Basis, inputs, lanczos_batched
    inst = inputs.batched_instances(lambda n: Basis(n, two_s=2, two_M=0).dim, count=64)
    bases = [Basis(d["N"], two_s=2, two_M=0) for d in inst]
    t = time.perf_counter()
    res = lanczos_batched(bases, [d["J"] for d in inst], [d["V0"] for d in inst], 80)
    print(f"batched 64x16x80: {time.perf_counter() - t:.3f} s, "
          f"rows {sum(b.dim for b in bases)}", flush=True)
    assert np.all(np.isfinite(res.E0))
    for k in range(64):
        assert np.ptp(res.E0[k]) <= 1e-4 * abs(res.E0[k].mean())


@pytest.mark.parametrize("nvec", [8, 16])
def test_batched_spin_one_and_three_halves_vs_oracle(nvec):
    """General spin in the shared-row layout: s = 1 and s = 3/2 chains with
    8 and 16 columns against the oracle's FP64 recurrence."""
    import oracle
    from paper_0706_3293_amd import Basis, lanczos_batched
    rng = np.random.default_rng(100 + nvec)
    # one launch per spin (the instances of a launch share it); (N, 2s, A)
    for specs in ([(8, 2, 8), (7, 2, 5), (9, 2, 7)], [(6, 3, 9), (5, 3, 6)]):
        bases, Js, V0s = [], [], []
        for N, two_s, A in specs:
            b = Basis(N, two_s=two_s, two_M=N * two_s - 2 * A)
            bases.append(b)
            Js.append(_rand_J(N, rng))
            V0s.append(rng.uniform(-1, 1, (nvec, b.dim)))
        steps = 30
        res = lanczos_batched(bases, Js, V0s, steps)
        for k, (N, two_s, A) in enumerate(specs):
            sub = oracle.Subspace(N, two_s, A)
            for r in range(nvec):
                ref = oracle.lanczos(sub, Js[k], V0s[k][r], steps)
                assert res.steps_done[k, r] == ref["steps_done"], (k, r)
                assert np.abs(res.alpha[k, r, :5] - ref["alpha"][:5]).max() <= \
                    2e-6 * np.abs(ref["alpha"][:5]).max()
                assert abs(res.E0[k, r] - ref["E0"]) <= 1e-6 * abs(ref["E0"])

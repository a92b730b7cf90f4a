"""GPU checks of the batched persistent Lanczos (hm_lanczos_batched).

Each (instance, start vector) pair must reproduce the single-instance path on
the same inputs (FP32-mixed, tolerance for the different FP32 summation
order), the oracle's FP64 energies, and the per-pair breakdown handling.
Energies of converged runs are gated at 1e-7 relative to the oracle (the
FP32-mixed target); the short 40-step runs compare coefficients, whose
digits FP32 vectors limit to about 1e-6.
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
            m = min(5, n)                # the first coefficients (later ones drift, FP32)
            assert np.abs(res.alpha[k, r, :m] - ref["alpha"][:m]).max() <= \
                2e-6 * np.abs(ref["alpha"][:m]).max()


@pytest.mark.parametrize("nvec", [4, 16])
def test_batched_converged_energy_within_1e7_of_oracle(nvec):
    """Runs long enough to converge (150 steps on subspaces of 252..3432
    states): every pair's E0 within 1e-7 relative of the oracle's FP64
    recurrence from the same start vector and step count."""
    import oracle
    from paper_0706_3293_amd import Basis, lanczos_batched
    rng = np.random.default_rng(200 + nvec)
    specs = [(10, 5), (12, 6), (14, 7), (13, 4), (11, 5)]
    bases, Js, V0s = [], [], []
    for N, A in specs:
        b = Basis(N, two_s=1, two_M=N - 2 * A)
        bases.append(b)
        Js.append(_rand_J(N, rng))
        V0s.append(rng.uniform(-1, 1, (nvec, b.dim)))
    steps = 150
    res = lanczos_batched(bases, Js, V0s, steps)
    worst = 0.0
    for k, (N, A) in enumerate(specs):
        sub = oracle.Subspace(N, 1, A)
        for r in range(nvec):
            ref = oracle.lanczos(sub, Js[k], V0s[k][r], steps)
            rel = abs(res.E0[k, r] - ref["E0"]) / abs(ref["E0"])
            worst = max(worst, rel)
            assert rel <= 1e-7, (k, r, rel)
    print(f"batched converged, nvec {nvec}: worst relative E0 error {worst:.2e}", flush=True)


def test_batched_spin_one_chains_subset_vs_oracle():
    """The spin-1 chain workload at its own step count (80): the instances
    of the seeded workload with N <= 12 run in one launch with all 16 start
    vectors, and 4 vectors of each are checked against the oracle's FP64
    recurrence (E0 within 1e-7 relative, same steps, first coefficients)."""
    import oracle
    from paper_0706_3293_amd import Basis, inputs, lanczos_batched
    inst = inputs.batched_instances(lambda n: Basis(n, two_s=2, two_M=0).dim, count=64)
    inst = [d for d in inst if d["N"] <= 12][:8]
    bases = [Basis(d["N"], two_s=2, two_M=0) for d in inst]
    res = lanczos_batched(bases, [d["J"] for d in inst], [d["V0"] for d in inst], 80)
    worst = 0.0
    for k, d in enumerate(inst):
        sub = oracle.Subspace(d["N"], 2, d["N"])
        for r in range(4):
            ref = oracle.lanczos(sub, d["J"], d["V0"][r], 80)
            assert res.steps_done[k, r] == ref["steps_done"], (k, r)
            rel = abs(res.E0[k, r] - ref["E0"]) / abs(ref["E0"])
            worst = max(worst, rel)
            assert rel <= 1e-7, (k, d["N"], r, rel)
            assert np.abs(res.alpha[k, r, :5] - ref["alpha"][:5]).max() <= \
                2e-6 * np.abs(ref["alpha"][:5]).max()
    print(f"spin-1 chains subset ({len(inst)} instances, N <= 12): worst relative "
          f"E0 error {worst:.2e}", flush=True)


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
    J4 = np.zeros((4, 4))
    J4[0, 1] = J4[1, 0] = 1.0
    with pytest.raises(_lib.HMError):
        lanczos_batched([b1], [J4], [np.zeros((2, b1.dim))], 5)
    # 40 sites of spin 1/2 fit one 64-bit word alone, but not at the 2 bits
    # per digit that a spin-1 instance in the same batch needs
    b40 = Basis(40, two_s=1, two_M=36)
    b3 = Basis(3, two_s=2, two_M=0)
    J40 = np.zeros((40, 40))
    J40[0, 1] = J40[1, 0] = 1.0
    J3 = np.zeros((3, 3))
    J3[0, 1] = J3[1, 0] = 1.0
    with pytest.raises(_lib.HMError, match="64 bits"):
        lanczos_batched([b40, b3], [J40, J3], [np.ones((2, b40.dim)), np.ones((2, b3.dim))], 5)


def test_batched_mixed_spins_vs_oracle():
    """Instances of spin 1/2, 1, 3/2 and 7/2 in one launch (digits packed at
    the widest spin's 3 bits) against the oracle's FP64 recurrence: E0 within
    1e-7 relative on converged runs, first coefficients at the FP32 level."""
    import oracle
    from paper_0706_3293_amd import Basis, lanczos_batched
    rng = np.random.default_rng(7)
    specs = [(12, 1, 6), (8, 2, 8), (6, 3, 9), (4, 7, 14), (11, 1, 4)]   # (N, 2s, A)
    bases, Js, V0s = [], [], []
    for N, two_s, A in specs:
        b = Basis(N, two_s=two_s, two_M=N * two_s - 2 * A)
        bases.append(b)
        Js.append(_rand_J(N, rng))
        V0s.append(rng.uniform(-1, 1, (4, b.dim)))
    steps = 120
    res = lanczos_batched(bases, Js, V0s, steps)
    for k, (N, two_s, A) in enumerate(specs):
        sub = oracle.Subspace(N, two_s, A)
        for r in range(4):
            ref = oracle.lanczos(sub, Js[k], V0s[k][r], steps)
            assert res.steps_done[k, r] == ref["steps_done"], (k, r)
            assert np.abs(res.alpha[k, r, :5] - ref["alpha"][:5]).max() <= \
                2e-6 * np.abs(ref["alpha"][:5]).max()
            assert abs(res.E0[k, r] - ref["E0"]) <= 1e-7 * abs(ref["E0"]), (k, r)


def test_batched_full_workload_vs_f64():
    """64 spin-1 chains x 16 vectors x 80 steps in one launch; every pair's
    E0 within 1e-7 relative of the instance's FP64 single-path ground state
    (200 steps, converged)."""
    import time
    from paper_0706_3293_amd import Basis, inputs, lanczos_batched
    inst = inputs.batched_instances(lambda n: Basis(n, two_s=2, two_M=0).dim, count=64)
    bases = [Basis(d["N"], two_s=2, two_M=0) for d in inst]
    t = time.perf_counter()
    res = lanczos_batched(bases, [d["J"] for d in inst], [d["V0"] for d in inst], 80)
    print(f"batched 64x16x80: {time.perf_counter() - t:.3f} s, "
          f"rows {sum(b.dim for b in bases)}", flush=True)
    assert np.all(np.isfinite(res.E0))
    worst = 0.0
    for k, d in enumerate(inst):
        ref = bases[k].lanczos(d["J"], torch.tensor(d["V0"][0], device="cuda"), 200)
        rel = np.abs(res.E0[k] - ref.E0).max() / abs(ref.E0)
        worst = max(worst, rel)
        assert rel <= 1e-7, (k, d["N"], rel)
    print(f"full workload: worst relative E0 error vs FP64 {worst:.2e}", flush=True)


@pytest.mark.parametrize("nvec", [8, 16])
def test_batched_spin_one_and_three_halves_vs_oracle(nvec):
    """General spin in the shared-row layout: s = 1 and s = 3/2 chains with
    8 and 16 columns against the oracle's FP64 recurrence."""
    import oracle
    from paper_0706_3293_amd import Basis, lanczos_batched
    rng = np.random.default_rng(100 + nvec)
    # one launch per spin; (N, 2s, A)
    for specs in ([(8, 2, 8), (7, 2, 5), (9, 2, 7)], [(6, 3, 9), (5, 3, 6)]):
        bases, Js, V0s = [], [], []
        for N, two_s, A in specs:
            b = Basis(N, two_s=two_s, two_M=N * two_s - 2 * A)
            bases.append(b)
            Js.append(_rand_J(N, rng))
            V0s.append(rng.uniform(-1, 1, (nvec, b.dim)))
        steps = 120                      # long enough to converge E0
        res = lanczos_batched(bases, Js, V0s, steps)
        for k, (N, two_s, A) in enumerate(specs):
            sub = oracle.Subspace(N, two_s, A)
            for r in range(nvec):
                ref = oracle.lanczos(sub, Js[k], V0s[k][r], steps)
                assert res.steps_done[k, r] == ref["steps_done"], (k, r)
                assert np.abs(res.alpha[k, r, :5] - ref["alpha"][:5]).max() <= \
                    2e-6 * np.abs(ref["alpha"][:5]).max()
                assert abs(res.E0[k, r] - ref["E0"]) <= 1e-7 * abs(ref["E0"])


def test_batched_schedules_and_autotuner(tmp_path):
    """The batched launch under other schedules (items per chunk, workgroups
    per compute unit) gives the same steps and energies within the FP32-mixed
    tolerance; the autotuner's choice is a candidate, is cached, and its run
    matches the oracle at 1e-7 on converged runs (80 steps of the spin-1
    chain workload's instances with N <= 12)."""
    import oracle
    from paper_0706_3293_amd import Basis, autotune, inputs, lanczos_batched
    inst = inputs.batched_instances(lambda n: Basis(n, two_s=2, two_M=0).dim, count=64)
    inst = [d for d in inst if d["N"] <= 12][:6]
    bases = [Basis(d["N"], two_s=2, two_M=0) for d in inst]
    Js = [d["J"] for d in inst]
    V0s = [d["V0"][:4] for d in inst]
    ref = lanczos_batched(bases, Js, V0s, 80)
    for sched in ((1, 1), (16, 2), (2, 8)):
        r = lanczos_batched(bases, Js, V0s, 80, schedule=sched)
        assert np.array_equal(r.steps_done, ref.steps_done), sched
        assert np.abs(r.E0 - ref.E0).max() <= 1e-7 * np.abs(ref.E0).max(), sched
    cache = str(tmp_path / "tune.json")
    best = autotune.tune_batched(bases, Js, V0s, 80, reps=1, cache=cache)
    assert best in autotune.BATCH_CANDIDATES
    assert autotune.tune_batched(bases, Js, V0s, 80, cache=cache) == best     # cached
    r = lanczos_batched(bases, Js, V0s, 80, schedule=best)
    for k, d in enumerate(inst):
        sub = oracle.Subspace(d["N"], 2, d["N"])
        for q in range(4):
            o = oracle.lanczos(sub, d["J"], d["V0"][q], 80)
            assert r.steps_done[k, q] == o["steps_done"]
            assert abs(r.E0[k, q] - o["E0"]) <= 1e-7 * abs(o["E0"]), (k, q)
    from paper_0706_3293_amd import _lib
    with pytest.raises(_lib.HMError):
        lanczos_batched(bases, Js, V0s, 5, schedule=(0, 9))
    with pytest.raises(_lib.HMError):
        lanczos_batched(bases, Js, V0s, 5, schedule=(65, 4))

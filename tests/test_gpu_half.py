"""GPU parity of the spin-1/2 block kernel (hm_apply_kernel kernel=2) against
the oracle and against the generic digit kernel, across schedules (low bits
K, workgroup size), precisions, ragged block tails and edge subspaces."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _basis(N, A, K=0, block=0, R=0, staging=0):
    from paper_0706_3293_amd import Basis
    b = Basis(N, two_s=1, two_M=N - 2 * A)
    if K or block or R or staging:
        b.set_schedule(K, block, R, staging)
    return b


def _scale(sub, J, x):
    return float(np.abs(sub.apply(np.abs(J), np.abs(x))).max()) + 1e-300


CASES = [
    # N, A, K, block, rows per lane, couplings
    (16, 8, 12, 256, 1, "j1j2"), (16, 8, 10, 64, 2, "j1j2"), (16, 5, 9, 128, 4, "ring"),
    (20, 10, 12, 256, 4, "a2a"), (20, 10, 14, 256, 1, "a2a"), (20, 7, 8, 64, 8, "a2a"),
    (12, 6, 12, 256, 4, "ring"), (9, 3, 4, 64, 2, "j1j2"), (22, 11, 11, 256, 4, "j1j2"),
    (18, 2, 6, 128, 8, "random"), (18, 16, 10, 256, 2, "random"), (6, 0, 4, 64, 4, "ring"),
    (6, 6, 4, 64, 1, "ring"), (5, 1, 5, 64, 8, "ring"), (24, 12, 13, 256, 8, "j1j2"),
    (22, 11, 10, 128, 8, "random"),
]


def _J(kind, N, rng):
    from paper_0706_3293_amd import inputs
    if kind == "ring":
        return inputs.ring_couplings(N, -1.0)
    if kind == "j1j2":
        return inputs.ring_couplings(N, -1.0, -0.41)
    if kind == "a2a":
        return inputs.all_to_all_couplings(N, 1)[0]
    J = rng.normal(size=(N, N)) * (rng.uniform(size=(N, N)) < 0.4)
    J = np.triu(J, 1)
    return J + J.T


@pytest.mark.parametrize("N,A,K,block,R,kind", CASES)
def test_block_kernel_matches_oracle(N, A, K, block, R, kind):
    import oracle
    print("block kernel", N, A, K, block, R, kind, flush=True)
    rng = np.random.default_rng(N * 100 + A)
    J = _J(kind, N, rng)
    b = _basis(N, A, K, block, R)
    sub = oracle.Subspace(N, 1, A)
    x = rng.uniform(-1, 1, sub.dim)
    scale = _scale(sub, J, x)
    xd = torch.tensor(x, device="cuda")
    y = b.apply(J, xd, kernel=2).cpu().numpy()
    assert np.abs(y - sub.apply(J, x)).max() <= 1e-13 * scale
    y_gen = b.apply(J, xd, kernel=1).cpu().numpy()
    assert np.abs(y - y_gen).max() <= 1e-13 * scale
    x32 = xd.float()
    y32 = b.apply(J, x32, kernel=2).double().cpu().numpy()
    ref32 = sub.apply(J, x32.double().cpu().numpy())
    assert np.abs(y32 - ref32).max() <= 2e-6 * scale


STAGED = [
    # N, A, K, rows per lane, couplings: staged blocks (work split 2)
    (16, 8, 10, 4, "j1j2"), (16, 5, 9, 2, "ring"), (20, 10, 11, 2, "a2a"),
    (20, 7, 9, 4, "a2a"), (18, 2, 10, 1, "random"), (18, 16, 10, 2, "random"),
    (12, 6, 9, 4, "ring"), (22, 11, 11, 1, "j1j2"), (24, 12, 10, 2, "j1j2"),
    (9, 3, 4, 2, "j1j2"), (6, 0, 4, 4, "ring"), (6, 6, 4, 1, "ring"), (5, 1, 5, 4, "ring"),
]


@pytest.mark.parametrize("N,A,K,R,kind", STAGED)
def test_staged_blocks_match_oracle_and_chunked_bitwise(N, A, K, R, kind):
    """The staged work split gives the chunked split's result bit for bit
    (same per-row arithmetic in the same bond order) and the oracle's."""
    import oracle
    print("staged blocks", N, A, K, R, kind, flush=True)
    rng = np.random.default_rng(N * 100 + A + 7)
    J = _J(kind, N, rng)
    b1 = _basis(N, A, K, 256, R, 1)
    b2 = _basis(N, A, K, 256, R, 2)
    sub = oracle.Subspace(N, 1, A)
    x = rng.uniform(-1, 1, sub.dim)
    scale = _scale(sub, J, x)
    xd = torch.tensor(x, device="cuda")
    y2 = b2.apply(J, xd, kernel=2)
    assert torch.equal(y2, b1.apply(J, xd, kernel=2))
    assert np.abs(y2.cpu().numpy() - sub.apply(J, x)).max() <= 1e-13 * scale
    x32 = xd.float()
    y32 = b2.apply(J, x32, kernel=2)
    assert torch.equal(y32, b1.apply(J, x32, kernel=2))
    ref32 = sub.apply(J, x32.double().cpu().numpy())
    assert np.abs(y32.double().cpu().numpy() - ref32).max() <= 2e-6 * scale


@pytest.mark.parametrize("precision", ["f64", "f32_mixed"])
def test_staged_blocks_lanczos_with_reorthogonalization(precision):
    """Both fused variants of the staged kernel (with the alpha partials, and
    with the stored Krylov vectors of full reorthogonalization): the exact
    Majumdar-Ghosh energy, and coefficients equal to the chunked split's up to
    the grouping of the partial sums."""
    from paper_0706_3293_amd import inputs
    N = 20
    J = inputs.ring_couplings(N, -1.0, -0.5)
    b1 = _basis(N, N // 2, 10, 256, 2, 1)
    b2 = _basis(N, N // 2, 10, 256, 2, 2)
    v0 = torch.tensor(inputs.start_vector(b1.dim, 0), device="cuda")
    tol = 1e-10 if precision == "f64" else 1e-7
    for reorth in (False, True):
        r2 = b2.lanczos(J, v0, 120, precision=precision, full_reorth=reorth, kernel=2)
        assert abs(r2.E0 + 3 * N / 8) <= tol * 3 * N / 8
        r1 = b1.lanczos(J, v0, 120, precision=precision, full_reorth=reorth, kernel=2)
        ctol = 1e-11 if precision == "f64" else 1e-5
        assert np.abs(r1.alpha[:20] - r2.alpha[:20]).max() < ctol


def test_staged_blocks_rejected_where_blocks_do_not_fit():
    from paper_0706_3293_amd import _lib, inputs
    J = inputs.ring_couplings(16, -1.0)
    x = torch.zeros(12870, dtype=torch.float64, device="cuda")
    for K, R in ((12, 1), (11, 4), (10, 8)):
        b = _basis(16, 8, K, 256, R, 2)
        with pytest.raises(_lib.HMError):
            b.apply(J, x, kernel=2)
    with pytest.raises(_lib.HMError):
        _basis(16, 8, 10, 256, 1, 3)


@pytest.mark.parametrize("N,schedule", [(28, None), (32, None), (32, (10, 256, 2, 2))])
def test_block_kernel_full_size_sampled_rows(N, schedule):
    """Workload sizes: 2^20 sampled rows against the oracle, FP64 and FP32 (the
    default schedule, and at N=32 the staged schedule the autotuner picks
    for FP32 on MI355X)."""
    import oracle
    from paper_0706_3293_amd import inputs
    print("full size", N, schedule, flush=True)
    J = inputs.ring_couplings(N, -1.0, -0.5 if N == 28 else -0.25)
    b = _basis(N, N // 2, *(schedule or ()))
    sub = oracle.Subspace(N, 1, N // 2)
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, b.dim)
    rows = np.sort(rng.integers(0, b.dim, 1 << 20))
    rows = np.concatenate([rows, [0, 1, b.dim - 2, b.dim - 1]])
    scale = float(np.abs(J).sum() / 2) * 1.0
    ref = sub.apply_rows(J, x, rows)
    xd = torch.tensor(x, device="cuda")
    y = b.apply(J, xd, kernel=2)
    got = y[torch.tensor(rows, device="cuda")].cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-13 * scale
    del y
    x32 = xd.float()
    del xd
    y32 = b.apply(J, x32, kernel=2)
    got32 = y32[torch.tensor(rows, device="cuda")].double().cpu().numpy()
    ref32 = sub.apply_rows(J, x32.double().cpu().numpy(), rows)
    assert np.abs(got32 - ref32).max() <= 2e-6 * scale


@pytest.mark.parametrize("precision,schedule", [("f32_mixed", (13, 256, 8, 1)),
                                                ("f64", (13, 256, 4, 1)),
                                                ("f64", (13, 256, 2, 1)),
                                                ("f32_mixed", (9, 256, 4, 2))])
def test_bench_configuration_lanczos_n28(precision, schedule):
    """The timed workload in the launch configuration the benchmark uses (the
    autotuner's schedules on MI355X): 200 steps reach the exact Majumdar-Ghosh
    energy, and the first coefficients equal the oracle's."""
    import oracle
    from paper_0706_3293_amd import inputs
    N = 28
    print("bench configuration", precision, schedule, flush=True)
    b = _basis(N, N // 2, *schedule)
    J = inputs.ring_couplings(N, -1.0, -0.5)
    v0h = inputs.start_vector(b.dim, 0)
    v0 = torch.tensor(v0h, device="cuda")
    res = b.lanczos(J, v0, 200, precision=precision)
    tol = 1e-10 if precision == "f64" else 1e-7
    assert abs(res.E0 + 3 * N / 8) <= tol * 3 * N / 8
    ref = oracle.lanczos(oracle.Subspace(N, 1, N // 2), J, v0h, 2)
    ctol = 1e-12 if precision == "f64" else 1e-6
    assert np.abs(res.alpha[:2] - ref["alpha"]).max() <= ctol * np.abs(ref["alpha"]).max()
    assert abs(res.beta[0] - ref["beta"][0]) <= ctol * ref["beta"][0]


@pytest.mark.parametrize("precision", ["f64", "f32_mixed"])
def test_block_kernel_lanczos_majumdar_ghosh(precision):
    from paper_0706_3293_amd import inputs
    N = 20
    b = _basis(N, N // 2)
    J = inputs.ring_couplings(N, -1.0, -0.5)
    v0 = torch.tensor(inputs.start_vector(b.dim, 0), device="cuda")
    res = b.lanczos(J, v0, 200, precision=precision, kernel=2)
    tol = 1e-10 if precision == "f64" else 1e-7
    assert abs(res.E0 + 3 * N / 8) <= tol * 3 * N / 8
    res1 = b.lanczos(J, v0, 30, precision=precision, kernel=1)
    res2 = b.lanczos(J, v0, 30, precision=precision, kernel=2)
    assert np.abs(res1.alpha[:20] - res2.alpha[:20]).max() < (1e-11 if precision == "f64" else 1e-5)


def test_block_kernel_lanczos_matches_golden_all_to_all():
    import json
    import os
    from paper_0706_3293_amd import inputs
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "all_to_all20_oracle.json")))
    b = _basis(20, 10)
    J = inputs.all_to_all_couplings(20, 0)[0]
    v0 = torch.tensor(inputs.start_vector(b.dim, 0), device="cuda")
    res = b.lanczos(J, v0, 300, kernel=2)
    assert abs(res.E0 - g["E0"]) <= 1e-10 * abs(g["E0"])
    assert np.abs(res.alpha[:30] - g["alpha"][:30]).max() < 1e-10


def test_schedule_rejected_after_first_use():
    from paper_0706_3293_amd import _lib, inputs
    b = _basis(12, 6)
    b.apply(inputs.ring_couplings(12, -1.0), torch.zeros(b.dim, dtype=torch.float64,
                                                         device="cuda"), kernel=2)
    with pytest.raises(_lib.HMError):
        b.set_schedule(8, 64)
    with pytest.raises(_lib.HMError):
        _basis(12, 6).set_schedule(15, 64)
    with pytest.raises(_lib.HMError):
        _basis(12, 6).set_schedule(8, 96)
    with pytest.raises(_lib.HMError):
        _basis(12, 6).set_schedule(8, 64, 3)


def test_autotuner_picks_a_valid_schedule(tmp_path):
    import oracle
    from paper_0706_3293_amd import autotune, inputs
    N = 18
    J = inputs.ring_couplings(N, -1.0, -0.3)
    cache = str(tmp_path / "tune.json")
    b, sched = autotune.tuned_basis(N, J, reps=2, cache=cache)
    assert len(sched) == 5 and sched[4] in autotune.IPW_CANDIDATES
    assert sched[:4] in [tuple(c) for c in autotune.candidates(N)]
    assert autotune.tune(N, J, reps=2, cache=cache) == sched      # cached
    sub = oracle.Subspace(N, 1, N // 2)
    x = np.random.default_rng(0).uniform(-1, 1, b.dim)
    y = b.apply(J, torch.tensor(x, device="cuda"), kernel=2).cpu().numpy()
    assert np.abs(y - sub.apply(J, x)).max() < 1e-12

"""GPU parity at the largest single-GPU workload: the s=1/2 J1-J2 ring with
N=32, J1=-1, J2=-0.25, M=0 (dim 601,080,390), in the launch configuration the
benchmark times (its stored schedule for each precision).

Pins:
  - the first two Lanczos coefficients against the oracle's (two full oracle
    H x applications, Sec. 4 Eq. (E-4-b), stored by
    tests/golden/make_oracle_golden.py): FP64 within 1e-12 relative,
    FP32-mixed within 1e-6 relative (FP32 vectors and matrix elements);
  - 150 steps without reorthogonalization in both precisions: E0 of the
    FP32-mixed path within 1e-7 relative of the FP64 path's.
"""
import json
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden", "j1j2_ring32_oracle.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def problem():
    from paper_0706_3293_amd import inputs
    J = inputs.workload_couplings("j1j2_ring32")
    with open(GOLDEN) as f:
        g = json.load(f)
    v0 = torch.tensor(inputs.start_vector(g["dim"], 0), device="cuda")
    yield J, g, v0
    del v0
    torch.cuda.empty_cache()


def _bench_basis(prec):
    """Basis with the schedule bench.py runs for this precision."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_0706_3293_amd import Basis
    b = Basis(32, two_s=1, two_M=0)
    sched = bench.stored_schedule("j1j2_ring32", prec)
    if sched is not None:
        b.set_schedule(*sched)
    return b, sched


_E0 = {}


@pytest.mark.parametrize("prec", ["f64", "f32_mixed"])
def test_ring32_lanczos_vs_oracle(problem, prec):
    J, g, v0 = problem
    b, sched = _bench_basis(prec)
    print("ring32 lanczos", prec, "schedule", sched, flush=True)
    assert b.dim == g["dim"] == 601080390
    res = b.lanczos(J, v0, 150, precision=prec)
    assert res.steps_done == 150
    tol = 1e-12 if prec == "f64" else 1e-6
    a_ref, b_ref = np.array(g["alpha"]), np.array(g["beta"])
    print(f"alpha {res.alpha[:2]} oracle {a_ref}; beta {res.beta[:2]} oracle {b_ref}; "
          f"E0 {res.E0:.15f}", flush=True)
    assert np.abs(res.alpha[:2] - a_ref).max() <= tol * np.abs(a_ref).max()
    assert np.abs(res.beta[:2] - b_ref).max() <= tol * np.abs(b_ref).max()
    _E0[prec] = res.E0


def test_ring32_mixed_energy_within_1e7_of_f64():
    if len(_E0) < 2:
        pytest.skip("needs both Lanczos runs of this module")
    rel = abs(_E0["f32_mixed"] - _E0["f64"]) / abs(_E0["f64"])
    print(f"E0 f64 {_E0['f64']:.15f} mixed {_E0['f32_mixed']:.15f} rel {rel:.2e}", flush=True)
    assert rel <= 1e-7

"""Benchmark of the Lanczos hot path on one MI355X.

Workload (default): the s=1/2 J1-J2 ring with N=28, J1=-1, J2=-0.5 in the
M=0 subspace (dim 40,116,600), uniform[-1,1] start vector from seed 0.  One
"step" is one Lanczos step: the fused H x pass (decode, diagonal, ladder
flips, encode, gather), the alpha/beta reductions and the vector update.
K steps are timed for the FP32-mixed path (vectors and matrix elements in
FP32, dots/norms in FP64) and, separately, for the FP64 path; E0 of both is
compared with the exact Majumdar-Ghosh value -3N/8 of this workload.

Prints one JSON line (rank 0, one GPU).  `value` is the whole-job
throughput of the FP32-mixed path in rows/s (dim x K / time, inputs already
resident in HBM); the FP64 throughput, the mixed/FP64 step ratio and the H x
kernel measurements travel in extra fields.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H·x rows/s + HBM GB/s; Lanczos steps/s, FP32-mixed vs FP64 at |ΔE0|<1e-7"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="j1j2_ring28",
                    choices=["j1j2_ring28", "j1j2_ring32"])
    ap.add_argument("--kernel", type=int, default=0, help="0 auto, 1 generic, 2 spin-1/2 block")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=1 << 23)
    ap.add_argument("--hx-repeats", type=int, default=20)
    return ap.parse_args()


def cpu_baseline(N, J, x, rows):
    """The oracle's row-gather H x on a random sample of rows (host cores)."""
    import oracle
    sub = oracle.Subspace(N, 1, N // 2)
    rng = np.random.default_rng(1)
    sample = np.sort(rng.integers(0, sub.dim, rows))
    t0 = time.perf_counter()
    sub.apply_rows(J, x, sample)
    dt = time.perf_counter() - t0
    return dict(value=rows / dt, unit="rows/s", cores=oracle.max_threads(), kind="oracle",
                sample=f"oracle FP64 H x on {rows} random rows of the same workload "
                       f"({dt:.1f} s)")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the "
              "multi-GPU sharding of this path is described, not built.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_0706_3293_amd import Basis, api, inputs

    torch.cuda.set_device(0)
    w = inputs.WORKLOADS[args.workload]
    N = w["N"]
    J = inputs.workload_couplings(args.workload)
    b = Basis(N, two_s=1, two_M=0)
    D = b.dim
    exact = {"j1j2_ring28": -3 * N / 8}.get(args.workload)
    print(f"[bench] workload {args.workload} dim {D}", file=sys.stderr, flush=True)
    v0_host = inputs.start_vector(D, w["seed"])
    v0 = torch.tensor(v0_host, device="cuda")

    results = {}
    for prec in ("f32_mixed", "f64"):
        # warmup: a short run builds tables, uploads couplings, fills caches
        b.lanczos(J, v0, max(args.warmup, 1), precision=prec, kernel=args.kernel)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = b.lanczos(J, v0, args.steps, precision=prec, kernel=args.kernel)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        results[prec] = dict(ms_per_step=1e3 * dt / args.steps, E0=res.E0,
                             steps_done=res.steps_done)
        print(f"[bench] {prec}: {1e3 * dt / args.steps:.3f} ms/step E0={res.E0:.12f}",
              file=sys.stderr, flush=True)

    # H x kernel time inside the Lanczos step, by HIP events on the call's stream
    hx = {}
    for prec, es in (("f32_mixed", 4), ("f64", 8)):
        api.set_timing(True)
        b.lanczos(J, v0, args.hx_repeats, precision=prec, kernel=args.kernel, use_graph=False)
        api.set_timing(False)
        t = api.last_timing()
        avg_ms = t["hx_ms"] / max(t["hx_launches"], 1)
        alg_bytes = 3 * es * D          # read x and previous vector, write w
        hx[prec] = dict(avg_ms=avg_ms, alg_bytes=alg_bytes,
                        gbs=alg_bytes / (avg_ms * 1e-3) / 1e9,
                        rows_per_s=D / (avg_ms * 1e-3))
        print(f"[bench] H x pass ({prec}): {avg_ms:.3f} ms, {hx[prec]['gbs']:.0f} GB/s "
              "algorithmic", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(N, J, v0_host, args.cpu_rows)
        print(f"[bench] cpu baseline {cpu['value']:.3g} rows/s on {cpu['cores']} threads",
              file=sys.stderr, flush=True)

    mixed, f64 = results["f32_mixed"], results["f64"]
    dE = {p: (abs(r["E0"] - exact) if exact is not None else None) for p, r in results.items()}
    line = {
        "metric": METRIC,
        "value": D / (mixed["ms_per_step"] * 1e-3),
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: s=1/2 J1-J2 ring N={N}, M=0, dim {D}, "
                               f"{args.steps} Lanczos steps, FP32-mixed",
                   "dim": D, "parallelism": "single GPU"},
        "lanczos_steps_per_s": {"f32_mixed": 1e3 / mixed["ms_per_step"],
                                "f64": 1e3 / f64["ms_per_step"]},
        "mixed_over_f64_step_speedup": f64["ms_per_step"] / mixed["ms_per_step"],
        "f64_rows_per_s": D / (f64["ms_per_step"] * 1e-3),
        "E0": {"f32_mixed": mixed["E0"], "f64": f64["E0"], "exact": exact},
        "abs_dE0": dE,
        "rel_dE0": {p: (v / abs(exact) if v is not None else None) for p, v in dE.items()},
        "hx_pass": hx,
        "roofline": {"bound": "hbm", "achieved": hx["f32_mixed"]["gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": hx["f32_mixed"]["gbs"] / HBM_PEAK_GBS,
                     "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

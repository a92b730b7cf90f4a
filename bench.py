"""Benchmark of the Lanczos hot path on one MI355X.

Workload (default): the s=1/2 J1-J2 ring with N=32, J1=-1, J2=-0.25 in the
M=0 subspace (dim 601,080,390, 2.4 GB per FP32 vector), uniform[-1,1] start
vector from seed 0: the largest configuration of the measurement plan that
fits one GPU.  One "step" is one Lanczos step: the H x pass (decode,
diagonal, ladder flips, encode, gather), the alpha/beta reductions and the
vector update.  K steps are timed for the FP32-mixed path (vectors and matrix
elements in FP32, dots/norms in FP64) and, separately, for the FP64 path.

Accuracy is measured outside the timed region on a full run of the
workload's own length (150 steps at N=32, 200 at N=28) in both precisions:
|E0(FP32-mixed) - E0(FP64)| absolute and relative, the first coefficients of
the FP64 run against the oracle's stored values (two full oracle H x
applications, tests/golden/), and at N=28 the exact energy -3N/8.
--workload j1j2_ring28 runs the N=28, J2=-0.5 ring (dim 40,116,600).

Prints one JSON line (one GPU).  `value` is the whole-job throughput of the
FP32-mixed path in rows/s (dim x K / time, inputs already resident in HBM);
the FP64 throughput, the mixed/FP64 step ratio, the H x kernel measurements,
the roofline of the dominant kernel and the oracle's CPU rate travel in extra
fields.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H·x rows/s + HBM GB/s; Lanczos steps/s, FP32-mixed vs FP64 at |ΔE0|<1e-7"
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_0706_3293_amd", "csrc", "hx_half.hip")
TRAFFIC = os.path.join(ROOT, "profiles", "hx_half_traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="j1j2_ring32", choices=["j1j2_ring28", "j1j2_ring32"])
    ap.add_argument("--kernel", type=int, default=0, help="0 auto, 1 generic, 2 spin-1/2 block")
    ap.add_argument("--no-tune", action="store_true", help="default schedule, no autotuning")
    ap.add_argument("--tune", action="store_true",
                    help="autotune even where a schedule is stored beside the counters")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=1 << 27,
                    help="rows of the oracle's timed H x sample (about 15 s on 16 host threads)")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the full-length accuracy runs")
    ap.add_argument("--oracle-full", action="store_true",
                    help="also time three full oracle H x and one full oracle Lanczos step "
                         "of the workload on the host (minutes at N=32)")
    ap.add_argument("--hx-repeats", type=int, default=20)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also time a 1 GiB device copy (profiling reference)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the timings of the other workloads")
    ap.add_argument("--extras-only", action="store_true",
                    help="only time the other workloads (a profiling mode: prints "
                         "{\"other_workloads\": ...}, not the benchmark line)")
    ap.add_argument("--extras-select", default=None,
                    help="comma-separated names of the other workloads to run "
                         "(j1j2_ring28, ring12, all_to_all20, spin1_chains_batched, "
                         "sectors, hx_design_ablations, block_lanczos_ring24, "
                         "paper_vector_length_484500, hx_ring36_f32); default all")
    return ap.parse_args()


def kernel_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()


def stored_schedule(workload, prec):
    """The schedule the autotuner picked when the committed counters were
    taken (stored with them), if the kernel source is unchanged since."""
    try:
        with open(TRAFFIC) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha1") != kernel_hash():
        return None
    e = t.get("entries", {}).get(f"{workload}/{prec}")
    return tuple(e["schedule"]) if e and e.get("schedule") else None


def measured_traffic(workload, prec, schedule):
    """HBM bytes per launch from the committed counter summary, or None if
    the kernel source changed since the counters were taken or they were
    taken with another schedule."""
    try:
        with open(TRAFFIC) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha1") != kernel_hash():
        return None
    e = t.get("entries", {}).get(f"{workload}/{prec}")
    if e is None or e.get("schedule") != (list(schedule) if schedule else None):
        return None
    return e.get("bytes_per_launch")


# The oracle timed in a child process (no GPU), so that OMP_NUM_THREADS can be
# set per run: rows/s of its H x on a row sample of the main workload, a full
# N=12 Lanczos run and one full N=20 all-to-all H x.
_ORACLE_CHILD = r"""
import json, sys, time
import numpy as np
cfg = json.load(sys.stdin)
sys.path.insert(0, cfg["root"])
import oracle
out = {"threads": oracle.max_threads()}
J = np.array(cfg["J"])
sub = oracle.Subspace(cfg["N"], 1, cfg["N"] // 2)
x = np.random.default_rng(0).uniform(-1.0, 1.0, sub.dim)
rows = np.sort(np.random.default_rng(1).integers(0, sub.dim, cfg["rows"]))
t0 = time.perf_counter(); sub.apply_rows(J, x, rows); dt = time.perf_counter() - t0
out["hx_rows_per_s"] = cfg["rows"] / dt
out["hx_sample_rows"] = cfg["rows"]
if cfg["full_runs"]:
    J12 = np.array(cfg["J12"]); s12 = oracle.Subspace(12, 1, 6)
    v12 = np.random.default_rng(0).uniform(-1.0, 1.0, s12.dim)
    t0 = time.perf_counter(); r = oracle.lanczos(s12, J12, v12, 120, full_reorth=True)
    out["ring12_120_steps_s"] = time.perf_counter() - t0; out["ring12_E0"] = r["E0"]
    J20 = np.array(cfg["J20"]); s20 = oracle.Subspace(20, 1, 10)
    v20 = np.random.default_rng(0).uniform(-1.0, 1.0, s20.dim)
    t0 = time.perf_counter(); s20.apply(J20, v20)
    out["all_to_all20_hx_s"] = time.perf_counter() - t0
    t0 = time.perf_counter(); oracle.lanczos(s20, J20, v20, 3)
    out["all_to_all20_s_per_step"] = (time.perf_counter() - t0) / 3
    Jp = np.array(cfg["Jp"]); sp = oracle.Subspace(20, 2, 7)
    vp = np.random.default_rng(0).uniform(-1.0, 1.0, sp.dim)
    t0 = time.perf_counter(); oracle.lanczos(sp, Jp, vp, 10)
    out["paper_vector_length_s_per_step"] = (time.perf_counter() - t0) / 10
    # the N=28 J1-J2 ring (dim 40,116,600): one full H x and one step
    J28 = np.array(cfg["J28"]); s28 = oracle.Subspace(28, 1, 14)
    v28 = np.random.default_rng(0).uniform(-1.0, 1.0, s28.dim)
    t0 = time.perf_counter(); s28.apply(J28, v28)
    out["j1j2_ring28_hx_s"] = time.perf_counter() - t0
    t0 = time.perf_counter(); oracle.lanczos(s28, J28, v28, 1)
    out["j1j2_ring28_step_s"] = time.perf_counter() - t0
print(json.dumps(out))
"""


def oracle_child(N, J, rows, threads, full_runs):
    import subprocess
    from paper_0706_3293_amd import inputs
    cfg = dict(root=ROOT, N=N, J=np.asarray(J).tolist(), rows=rows, full_runs=full_runs,
               J12=inputs.ring_couplings(12, -1.0).tolist(),
               J20=inputs.all_to_all_couplings(20, 0)[0].tolist(),
               Jp=inputs.ring_couplings(20, -1.0).tolist(),
               J28=inputs.workload_couplings("j1j2_ring28").tolist())
    env = dict(os.environ)
    if threads:
        env["OMP_NUM_THREADS"] = str(threads)
    res = subprocess.run([sys.executable, "-c", _ORACLE_CHILD], input=json.dumps(cfg),
                         capture_output=True, text=True, env=env, timeout=300)
    if res.returncode != 0:
        return {"error": res.stderr[-500:]}
    return json.loads(res.stdout.strip().splitlines()[-1])


def host_info():
    info = {"nproc": os.cpu_count()}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu"] = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                info["mem_gib"] = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    return info


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _extra_j1j2_ring28(out):
    import torch

    from paper_0706_3293_amd import Basis, inputs
    # the N=28 J1-J2 ring at the Majumdar-Ghosh point (dim 40,116,600): 200
    # Lanczos steps in each precision with the schedules stored for it, E0
    # against the exact -3N/8
    J28 = inputs.workload_couplings("j1j2_ring28")
    r28 = {}
    for prec in ("f32_mixed", "f64"):
        b = Basis(28, two_s=1, two_M=0)
        sched = stored_schedule("j1j2_ring28", prec)
        if sched is not None:
            b.set_schedule(*sched)
        v0 = torch.tensor(inputs.start_vector(b.dim, 0), device="cuda")
        b.lanczos(J28, v0, 3, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = b.lanczos(J28, v0, 200, precision=prec)
        dt = time.perf_counter() - t0
        r28[prec] = dict(ms_per_step=1e3 * dt / 200, E0=res.E0, schedule=sched,
                         rel_dE0_vs_exact=abs(res.E0 + 10.5) / 10.5)
        del v0, b
    r28["mixed_over_f64_step_speedup"] = r28["f64"]["ms_per_step"] / r28["f32_mixed"]["ms_per_step"]
    out["j1j2_ring28"] = r28
    torch.cuda.empty_cache()


def _extra_ring12(out):
    import torch

    from paper_0706_3293_amd import Basis, inputs
    # N=12 ring, 120 steps with full reorthogonalization, FP64
    b = Basis(12, two_s=1, two_M=0)
    J = inputs.ring_couplings(12, -1.0)
    v0 = torch.tensor(inputs.start_vector(b.dim, 0), device="cuda")
    out["ring12"] = dict(steps=120)
    # kernel 3: every step in one launch of one workgroup; kernel 1: the
    # multi-kernel step (what the automatic choice runs with reorthogonalization)
    for name, kern in (("one_workgroup", 3), ("multi_kernel", 1)):
        b.lanczos(J, v0, 120, full_reorth=True, kernel=kern)
        best = float("inf")
        for _ in range(3):                      # best of three (short run)
            t0 = time.perf_counter()
            res = b.lanczos(J, v0, 120, full_reorth=True, kernel=kern)
            best = min(best, time.perf_counter() - t0)
        out["ring12"][name + "_ms"] = 1e3 * best
        out["ring12"][name + "_E0"] = res.E0


def _extra_all_to_all20(out):
    import torch

    from paper_0706_3293_amd import Basis, autotune, ground_state_energy, inputs
    # N=20 all-to-all: E0(J) forward (300 steps FP64) and gradient of 190
    # bonds, on the block kernel in its default schedule and in the one the
    # autotuner picks for these couplings (FP64; kept in the tuner's cache, so
    # that profiled runs after the first take the same schedule)
    J, bonds, vals = inputs.all_to_all_couplings(20, 0)
    tuned = autotune.tune(20, J, dtype=torch.float64, reps=20)
    runs = {}
    for label, sched in (("default", None), ("tuned", tuned)):
        b = Basis(20, two_s=1, two_M=0)
        if sched is not None:
            b.set_schedule(*sched)
        v0 = torch.tensor(inputs.start_vector(b.dim, 0), device="cuda")
        Jv = torch.tensor(vals, dtype=torch.float64, requires_grad=True)
        ground_state_energy(Jv, b, bonds, v0, 300).backward()      # warm
        best = None
        for _ in range(3):                      # best of three (short runs)
            Jv = torch.tensor(vals, dtype=torch.float64, requires_grad=True)
            t0 = time.perf_counter()
            E0 = ground_state_energy(Jv, b, bonds, v0, 300)
            t1 = time.perf_counter()
            E0.backward()
            t2 = time.perf_counter()
            if best is None or t2 - t0 < best[2] - best[0]:
                best = (t0, t1, t2, E0, Jv)
        runs[label] = best
        dim = b.dim
    t0, t1, t2, E0, Jv = runs["tuned"]
    d0, d1, d2 = runs["default"][:3]
    # bond evaluations: every row tests every bond once per H x (300 forward
    # steps; the backward repeats them and adds one pass over all bonds)
    bond_evals = 300 * dim * len(bonds)
    out["all_to_all20"] = dict(forward_ms=1e3 * (t1 - t0), backward_ms=1e3 * (t2 - t1),
                               schedule=list(tuned), forward_ms_default_schedule=1e3 * (d1 - d0),
                               backward_ms_default_schedule=1e3 * (d2 - d1),
                               steps=300, bonds=len(bonds), E0=float(E0.detach()),
                               forward_bond_evals_per_s=bond_evals / (t1 - t0),
                               euler_residual=abs(float(np.dot(vals, Jv.grad.numpy())) - float(E0)))


def _extra_spin1_chains_batched(out):
    import torch

    from paper_0706_3293_amd import Basis, BatchedProblem, inputs
    # 64 spin-1 chains x 16 start vectors x 80 steps, one persistent launch,
    # in the default schedule and in the one the autotuner picks
    from paper_0706_3293_amd import autotune
    inst = inputs.batched_instances(lambda n: Basis(n, two_s=2, two_M=0).dim, count=64)
    bases = [Basis(d["N"], two_s=2, two_M=0) for d in inst]
    Js, V0s = [d["J"] for d in inst], [d["V0"] for d in inst]
    prob = BatchedProblem(bases, Js, V0s, 80)
    tuned = autotune.tune_batched(bases, Js, V0s, 80, cache=None)
    runs = {}
    for label, sched in (("default", (0, 0)), ("tuned", tuned)):
        prob.schedule = sched
        prob.run()
        torch.cuda.synchronize()
        dt = float("inf")
        for _ in range(3):                      # best of three
            t0 = time.perf_counter()
            r = prob.run()
            dt = min(dt, time.perf_counter() - t0)
        runs[label] = (dt, r)
    dt, r = runs["tuned"]
    # compulsory bytes per (row, vector, step): pass A reads r_k and r_{k-1}
    # and writes w, pass B reads w and r_k and writes w: 6 x 4 B in FP32
    alg = prob.rows * 16 * 80 * 24
    out["spin1_chains_batched"] = dict(
        ms=1e3 * dt, ms_default_schedule=1e3 * runs["default"][0], schedule=list(tuned),
        instances=64, vectors=16, steps=80, rows=prob.rows,
        row_vector_steps_per_s=prob.rows * 16 * 80 / dt,
        alg_gbs=alg / dt / 1e9, hbm_frac=alg / dt / 1e9 / HBM_PEAK_GBS,
        hbm_frac_default_schedule=alg / runs["default"][0] / 1e9 / HBM_PEAK_GBS,
        E0_spread_max=float(np.max(np.ptp(r.E0, axis=1))))
    del prob


def _extra_sectors(out):
    import torch

    from paper_0706_3293_amd import inputs
    # magnetization curve of the N=24 J1-J2 ring: 13 sectors M >= 0, 2 start
    # vectors each, 150 steps (one Lanczos run per sector and vector on the
    # block kernel, and the batched path for comparison); then finite-
    # temperature Lanczos of the N=20 ring, 11 sectors x 16 vectors x 60 steps
    from paper_0706_3293_amd import ftl_thermodynamics, magnetization_curve
    J24 = inputs.ring_couplings(24, -1.0, -0.25)
    curve = {}
    for method in ("single", "batched"):
        magnetization_curve(24, 1, J24, 150, nvec=2, seed=0, method=method)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c = magnetization_curve(24, 1, J24, 150, nvec=2, seed=0, method=method)
        curve[method] = (1e3 * (time.perf_counter() - t0), c)
    c = curve["single"][1]
    out["magnetization_curve_ring24"] = dict(
        ms=curve["single"][0], ms_batched_path=curve["batched"][0], sectors=len(c.two_M),
        rows=int(c.dim.sum()), vectors=2, steps=150, E0=[float(e) for e in c.E0],
        max_abs_diff_paths=float(np.abs(c.E0 - curve["batched"][1].E0).max()))
    J20 = inputs.ring_couplings(20, -1.0, -0.25)
    temps = [0.1, 0.25, 0.5, 1.0, 2.0, 4.0]
    ftl_thermodynamics(20, 1, J20, temps, 60, nvec=16, seed=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th = ftl_thermodynamics(20, 1, J20, temps, 60, nvec=16, seed=0)
    dt = time.perf_counter() - t0
    out["ftl_ring20"] = dict(ms=1e3 * dt, sectors=11, vectors=16, steps=60, T=temps,
                             E=[float(e) for e in th["E"]], C=[float(x) for x in th["C"]])


def _extra_hx_design_ablations(out):
    import torch

    from paper_0706_3293_amd import Basis, inputs
    # the paper's design alternatives for H x, FP32, ms per apply: 1 generic
    # row gather (decode every row), 2 spin-1/2 block kernel, 3 successor
    # sweep (decode one row in 16), 4 column scatter with atomic adds
    abl = {}
    cases = (("s1/2 N=28 J1-J2 ring M=0", 28, 1, inputs.ring_couplings(28, -1.0, -0.5), (1, 2, 3, 4)),
             ("s1 N=16 chain M=0", 16, 2, inputs.chain_couplings(-np.ones(15)), (1, 3, 4)))
    for name, N, two_s, Jc, kernels in cases:
        b = Basis(N, two_s=two_s, two_M=0)
        x = torch.rand(b.dim, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        t = {"dim": b.dim}
        for k in kernels:
            b.apply(Jc, x, out=y, kernel=k)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                b.apply(Jc, x, out=y, kernel=k)
            e1.record()
            torch.cuda.synchronize()
            t[f"kernel{k}_ms"] = e0.elapsed_time(e1) / 5
        abl[name] = t
        del x, y
    out["hx_design_ablations"] = abl


def _extra_block_lanczos_ring24(out):
    import torch

    from paper_0706_3293_amd import Basis, inputs
    # block Lanczos: the 4 lowest levels of the N=24 J1-J2 ring at M=0 (dim
    # 2,704,156), p = 4, 60 block steps with full reorthogonalization, FP64
    b = Basis(24, two_s=1, two_M=0)
    J24 = inputs.ring_couplings(24, -1.0, -0.25)
    b.lowest_levels(J24, 4, steps=4, p=4, seed=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lev = b.lowest_levels(J24, 4, steps=60, p=4, seed=0)
    dt = time.perf_counter() - t0
    out["block_lanczos_ring24"] = dict(ms=1e3 * dt, dim=b.dim, p=4, steps=60,
                                       levels=[float(e) for e in lev])


def _extra_paper_vector_length_484500(out):
    import torch

    from paper_0706_3293_amd import Basis, inputs
    # the vector length of the paper's only timing experiment (200 Lanczos
    # iterations, length 484,500 = D(N=20, s=1, M=13); the system is not
    # named, so an N=20 spin-1 ring stands in), FP64
    b = Basis(20, two_s=2, two_M=26)
    Jp = inputs.ring_couplings(20, -1.0)
    v0 = torch.tensor(inputs.start_vector(b.dim, 0), device="cuda")
    b.lanczos(Jp, v0, 200)
    torch.cuda.synchronize()
    dt = float("inf")
    for _ in range(3):                          # best of three (short run)
        t0 = time.perf_counter()
        res = b.lanczos(Jp, v0, 200)
        dt = min(dt, time.perf_counter() - t0)
    out["paper_vector_length_484500"] = dict(ms=1e3 * dt, dim=b.dim, steps=200,
                                             ms_per_step=1e3 * dt / 200, E0=res.E0)


def _extra_hx_ring36_f32(out):
    import torch

    from paper_0706_3293_amd import Basis, inputs
    # the largest size: N=36 J1-J2 ring at M=0 (dim 9,075,135,300 > 2^32, 64-bit
    # indices), one FP32 H x on the block kernel, 36 GB per vector
    b = Basis(36, two_s=1, two_M=0)
    J36 = inputs.ring_couplings(36, -1.0, -0.25)
    x = torch.empty(b.dim, dtype=torch.float32, device="cuda")
    for s0 in range(0, b.dim, 1 << 28):        # any values; filled chunk by chunk
        x[s0:s0 + (1 << 28)].uniform_(-1.0, 1.0)
    y = torch.empty_like(x)
    b.apply(J36, x, out=y, kernel=2)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        b.apply(J36, x, out=y, kernel=2)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 3
    # algorithmic bytes of a plain H x: read x once, write y once (8 B per row)
    out["hx_ring36_f32"] = dict(ms=ms, dim=b.dim, rows_per_s=b.dim / (ms * 1e-3),
                                alg_gbs=8 * b.dim / (ms * 1e-3) / 1e9)
    del x, y
    torch.cuda.empty_cache()


EXTRAS = (
    ("j1j2_ring28", _extra_j1j2_ring28),
    ("ring12", _extra_ring12),
    ("all_to_all20", _extra_all_to_all20),
    ("spin1_chains_batched", _extra_spin1_chains_batched),
    ("sectors", _extra_sectors),
    ("hx_design_ablations", _extra_hx_design_ablations),
    ("block_lanczos_ring24", _extra_block_lanczos_ring24),
    ("paper_vector_length_484500", _extra_paper_vector_length_484500),
    ("hx_ring36_f32", _extra_hx_ring36_f32),
)


def extras(select=None):
    """Timings of the other measured workloads (one GPU, inputs resident);
    select: names of EXTRAS to run (all when None)."""
    import torch
    out = {}
    for name, fn in EXTRAS:
        if select is None or name in select:
            fn(out)
            torch.cuda.empty_cache()
    return out


def oracle_full_size(N, J, x):
    """The oracle on the whole workload, on all host threads: three full H x
    applications and one full Lanczos step (minutes at N=32), each phase
    reported as it ends."""
    import oracle
    sub = oracle.Subspace(N, 1, N // 2)
    out = {"threads": oracle.max_threads(), "dim": sub.dim, "hx_s": []}
    for k in range(3):
        t0 = time.perf_counter()
        sub.apply(J, x)
        out["hx_s"].append(time.perf_counter() - t0)
        log(f"oracle full H x {k + 1}/3: {out['hx_s'][-1]:.1f} s")
    t0 = time.perf_counter()
    oracle.lanczos(sub, J, x, 1)
    out["lanczos_step_s"] = time.perf_counter() - t0
    log(f"oracle full Lanczos step: {out['lanczos_step_s']:.1f} s")
    out["hx_rows_per_s"] = sub.dim / min(out["hx_s"])
    return out


def load_golden(workload):
    """The oracle's stored first Lanczos coefficients of the workload (written
    by tests/golden/make_oracle_golden.py, which calls only the oracle)."""
    path = os.path.join(ROOT, "tests", "golden", f"{workload}_oracle.json")
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return None


def main():
    args = parse()
    select = set(args.extras_select.split(",")) if args.extras_select else None
    if select is not None and not select <= {n for n, _ in EXTRAS}:
        print(f"unknown --extras-select names: {sorted(select - {n for n, _ in EXTRAS})}",
              file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the "
              "multi-GPU sharding of this path is described, not built.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_0706_3293_amd import Basis, api, autotune, inputs

    torch.cuda.set_device(0)
    if args.extras_only:
        print(json.dumps({"other_workloads": extras(select)}), flush=True)
        return
    w = inputs.WORKLOADS[args.workload]
    N = w["N"]
    J = inputs.workload_couplings(args.workload)
    exact = -3 * N / 8 if args.workload == "j1j2_ring28" else None
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        bb = torch.empty_like(a)
        for _ in range(3):
            bb.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 1 GiB device copies done")
        del a, bb

    bases, schedules = {}, {}
    for prec, dt in (("f32_mixed", torch.float32), ("f64", torch.float64)):
        stored = None if (args.tune or args.no_tune) else stored_schedule(args.workload, prec)
        if args.no_tune or args.kernel == 1:
            bases[prec] = Basis(N, two_s=1, two_M=0)
            schedules[prec] = None
        elif stored is not None:
            # the autotuner's choice recorded with the committed counters, so
            # the timed kernel is the profiled one (near-ties between
            # schedules would otherwise flip from run to run)
            bases[prec] = Basis(N, two_s=1, two_M=0)
            bases[prec].set_schedule(*stored)
            schedules[prec] = stored
            log(f"schedule {prec} (stored with the counters): {stored}")
        else:
            t0 = time.perf_counter()
            bases[prec], schedules[prec] = autotune.tuned_basis(N, J, dtype=dt)
            log(f"autotune {prec}: schedule (K, block, rows/lane, work split) = {schedules[prec]} "
                f"in {time.perf_counter() - t0:.1f} s")
    D = bases["f64"].dim
    log(f"workload {args.workload} dim {D}")
    v0_host = inputs.start_vector(D, w["seed"])
    v0 = torch.tensor(v0_host, device="cuda")

    # the timed region: K steps of each precision, inputs resident in HBM
    results = {}
    for prec in ("f32_mixed", "f64"):
        b = bases[prec]
        b.lanczos(J, v0, max(args.warmup, 1), precision=prec, kernel=args.kernel)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = b.lanczos(J, v0, args.steps, precision=prec, kernel=args.kernel)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        results[prec] = dict(ms_per_step=1e3 * dt / args.steps, steps_done=res.steps_done)
        log(f"{prec}: {1e3 * dt / args.steps:.3f} ms/step ({args.steps} steps timed)")

    # accuracy, outside the timed region: the workload's full run length in
    # both precisions, FP32-mixed against FP64, and FP64 against the oracle
    acc = None
    if not args.no_accuracy:
        full = {}
        for prec in ("f32_mixed", "f64"):
            res = bases[prec].lanczos(J, v0, w["steps"], precision=prec, kernel=args.kernel)
            full[prec] = res
            log(f"{prec}: {w['steps']} steps, E0 = {res.E0:.15f}")
        e32, e64 = full["f32_mixed"].E0, full["f64"].E0
        acc = {"steps": w["steps"], "E0": {"f32_mixed": e32, "f64": e64},
               "abs_dE0_mixed_vs_f64": abs(e32 - e64),
               "rel_dE0_mixed_vs_f64": abs(e32 - e64) / abs(e64)}
        if exact is not None:
            acc["exact"] = exact
            acc["abs_dE0_vs_exact"] = {p: abs(r.E0 - exact) for p, r in full.items()}
            acc["rel_dE0_vs_exact"] = {p: abs(r.E0 - exact) / abs(exact)
                                       for p, r in full.items()}
        g = load_golden(args.workload)
        if g is not None:
            n = len(g["alpha"])
            ra, rb = np.array(g["alpha"]), np.array(g["beta"])
            acc["oracle_coefficients"] = {
                p: {"steps": n,
                    "rel_alpha": float(np.abs(r.alpha[:n] - ra).max() / np.abs(ra).max()),
                    "rel_beta": float(np.abs(r.beta[:n] - rb).max() / np.abs(rb).max())}
                for p, r in full.items()}
        log(f"accuracy: {json.dumps(acc)}")

    # H x pass inside the Lanczos step, timed by HIP events on the call's stream
    hx = {}
    for prec, es in (("f32_mixed", 4), ("f64", 8)):
        api.set_timing(True)
        bases[prec].lanczos(J, v0, args.hx_repeats, precision=prec, kernel=args.kernel,
                            use_graph=False)
        api.set_timing(False)
        t = api.last_timing()
        avg_ms = t["hx_ms"] / max(t["hx_launches"], 1)
        alg_bytes = 3 * es * D          # read x and the previous vector, write w
        traffic = measured_traffic(args.workload, prec, schedules[prec])
        hx[prec] = dict(avg_ms=avg_ms, launches=t["hx_launches"], alg_bytes=alg_bytes,
                        alg_gbs=alg_bytes / (avg_ms * 1e-3) / 1e9,
                        rows_per_s=D / (avg_ms * 1e-3), traffic_bytes=traffic,
                        traffic_gbs=(traffic / (avg_ms * 1e-3) / 1e9) if traffic else None)
        log(f"H x pass ({prec}): {avg_ms:.3f} ms, {hx[prec]['alg_gbs']:.0f} GB/s algorithmic")

    other = None
    if not args.no_extras:
        other = extras(select)
        log(f"other workloads: {json.dumps(other)}")

    cpu = cpu_detail = None
    if not args.no_cpu_baseline:
        # the oracle on a bounded sample of the same workload's rows, and the
        # GPU's FP64 H x of the same vector checked on those rows
        import oracle
        sub = oracle.Subspace(N, 1, N // 2)
        sample = np.sort(np.random.default_rng(1).integers(0, D, args.cpu_rows))
        t0 = time.perf_counter()
        y_ref = sub.apply_rows(J, v0_host, sample)
        dt = time.perf_counter() - t0
        cpu = dict(value=args.cpu_rows / dt, unit="rows/s", cores=oracle.max_threads(),
                   kind="oracle",
                   sample=f"oracle FP64 H x of {args.cpu_rows} random rows of the same workload "
                          f"(N={N}, dim {D}; {dt:.1f} s on the host)")
        y = bases["f64"].apply(J, v0)
        got = y[torch.tensor(sample, device="cuda")].cpu().numpy()
        del y
        cpu["gpu_f64_rows_max_abs_diff"] = float(np.abs(got - y_ref).max())
        del got, y_ref, sample
        log(f"cpu baseline {cpu['value']:.3g} rows/s on {cpu['cores']} threads; "
            f"GPU FP64 H x on the sampled rows: max |diff| {cpu['gpu_f64_rows_max_abs_diff']:.2e}")
        cpu_detail = {"host": host_info(),
                      "one_thread": oracle_child(N, J, 1 << 18, 1, False),
                      "all_threads": oracle_child(N, J, 1 << 22, 0, True)}
        if args.oracle_full:
            cpu_detail["full_size"] = oracle_full_size(N, J, v0_host)
        log(f"cpu baseline detail: {json.dumps(cpu_detail)}")

    mixed, f64 = results["f32_mixed"], results["f64"]
    h32 = hx["f32_mixed"]
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
        "config": {"workload": f"{args.workload}: s=1/2 J1-J2 ring N={N} M=0 (dim {D}), "
                               f"Lanczos steps, FP32-mixed (FP64 dots)",
                   "dim": D, "steps": args.steps, "parallelism": "single GPU",
                   "schedule": {p: s for p, s in schedules.items()}},
        "lanczos_steps_per_s": {"f32_mixed": 1e3 / mixed["ms_per_step"],
                                "f64": 1e3 / f64["ms_per_step"]},
        "mixed_over_f64_step_speedup": f64["ms_per_step"] / mixed["ms_per_step"],
        "f64_rows_per_s": D / (f64["ms_per_step"] * 1e-3),
        "accuracy": acc,
        "hx_pass": hx,
        "roofline": {"bound": "hbm", "achieved": h32["alg_gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": h32["alg_gbs"] / HBM_PEAK_GBS,
                     "traffic": h32["traffic_bytes"],
                     "kernel": kernel_name(schedules["f32_mixed"]),
                     "schedule": schedules["f32_mixed"],
                     "alg_bytes_per_launch": h32["alg_bytes"]},
        "cpu_baseline": cpu,
        "cpu_baseline_detail": cpu_detail,
        "other_workloads": other,
    }
    print(json.dumps(line), flush=True)


def kernel_name(schedule):
    """The FP32 H x kernel(s) a schedule runs (pass A of the Lanczos step)."""
    split = (schedule or (0, 0, 0, 1))[3]
    if split == 2:
        return "hx_half_staged_kernel<float, uint32, R, C, DOT=true>"
    return "hx_half_kernel<float, uint32, R, DOT=true>"


if __name__ == "__main__":
    main()

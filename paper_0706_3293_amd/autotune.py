"""Autotuners for the spin-1/2 block kernel's schedule and the batched
persistent Lanczos launch.

For a given problem (N, M, couplings, element type) every candidate schedule
(low bits K, workgroup size, rows per lane, work split) is built on a fresh basis handle
and timed with HIP events over the H x pass of a few Lanczos steps (the kernel
variant the steps run: with the previous vector and the FP64 dot, whose
register needs differ from the bare H x); then the grid of the fastest is
tuned (work items per wave, 0 for the default grid).  The result, a 5-tuple, is remembered in a JSON cache keyed by the
problem.
A chosen schedule is fixed for the lifetime of its basis handle, so the two
Lanczos passes of the gradient (which must agree bit for bit) always run the
same kernel configuration.
"""
import hashlib
import json
import os

import numpy as np
import torch

from . import api
from .api import Basis

DEFAULT_CACHE = os.environ.get(
    "HM_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "hm_autotune.json"))


TIE = 0.01      # relative timing difference treated as a tie
# work items per wave tried for the grid of the fastest schedule (0: the
# default grid, listed first so that near-ties keep it)
IPW_CANDIDATES = (0, 4, 8, 16, 32, 64)


def candidates(N):
    """Schedules worth trying for N sites: (K, block threads, rows per lane,
    staging), staging 1 = chunked items, 2 = staged blocks."""
    out = []
    for K in sorted({max(1, min(N, k)) for k in (10, 11, 12, 13, 14)}):
        if N - K > 24:
            continue
        for R in (1, 2, 4, 8):
            out.append((K, 256, R, 1))
    out.append((min(N, 12), 128, 4, 1))
    # staged blocks need C(K, K/2) <= 512 and 32-bit indices (dim < 2^32)
    if _indices_fit_32(N):
        for K, rows in ((9, (1, 2, 4)), (10, (1, 2, 4)), (11, (1, 2))):
            if K <= N and N - K <= 24:
                for R in rows:
                    out.append((K, 256, R, 2))
    return out


def _indices_fit_32(N):
    """Whether the M = 0 (or nearest) subspace of N spins 1/2 has fewer than
    2^32 states, the condition for 32-bit indices."""
    from math import comb
    return comb(N, N // 2) < (1 << 32)


def _key(N, two_M, J, dtype):
    h = hashlib.sha1(np.ascontiguousarray(np.asarray(J, dtype=np.float64)).tobytes()).hexdigest()
    # "passA": timed on the Lanczos H x pass (entries timed on the bare H x
    # have keys without it and are tuned again)
    return f"passA:N={N},2M={two_M},dtype={dtype},J={h[:16]}"


def time_apply(b, J, x, y, reps):
    """Average ms of one H x application (block kernel) by HIP events."""
    b.apply(J, x, out=y, kernel=2)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(reps):
        b.apply(J, x, out=y, kernel=2)
    stop.record()
    stop.synchronize()
    return start.elapsed_time(stop) / reps


def time_pass_a(b, J, v0, precision, reps):
    """Average ms of the H x pass of Lanczos steps (the library's HIP events
    around every pass), over reps + 1 steps after a two-step warm-up."""
    b.lanczos(J, v0, 2, precision=precision, kernel=2)
    api.set_timing(True)
    try:
        b.lanczos(J, v0, reps + 1, precision=precision, kernel=2)
    finally:
        api.set_timing(False)
    t = api.last_timing()
    return t["hx_ms"] / max(t["hx_launches"], 1)


def tune(N, J, two_M=0, dtype=torch.float32, reps=5, cache=DEFAULT_CACHE, verbose=False):
    """Best (K, block, R, staging, items per wave) for the Lanczos H x pass
    with these couplings; results are cached (entries of older formats are
    tuned again).  The trials run Lanczos steps, so they hold an FP64 start
    vector and the Lanczos workspace (three vectors of dtype) on the device:
    20 B per row in FP32 and 32 B per row in FP64 beyond the tables (12 GB
    and 19 GB at N=32)."""
    key = _key(N, two_M, J, str(dtype))
    table = {}
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
    if key in table and len(table[key]["schedule"]) == 5:
        return tuple(table[key]["schedule"])
    probe = Basis(N, two_s=1, two_M=two_M)
    gen = torch.Generator(device="cuda").manual_seed(0)
    v0 = torch.rand(probe.dim, dtype=torch.float64, device="cuda", generator=gen) - 0.5
    del probe
    precision = "f64" if dtype == torch.float64 else "f32_mixed"
    trials = []
    for sched in candidates(N):
        b = Basis(N, two_s=1, two_M=two_M)
        b.set_schedule(*sched)
        ms = time_pass_a(b, J, v0, precision, reps)
        trials.append((sched, ms))
        if verbose:
            print(f"[autotune] K={sched[0]} block={sched[1]} R={sched[2]} "
                  f"staging={sched[3]}: {ms:.3f} ms", flush=True)
        del b
    # the first candidate (in the order above) within TIE of the fastest, so
    # that near-ties do not flip the choice from one run to the next
    fastest = min(ms for _, ms in trials)
    best4 = next(s for s, ms in trials if ms <= (1.0 + TIE) * fastest)
    # second stage: the grid of that schedule
    for ipw in IPW_CANDIDATES:
        sched = tuple(best4) + (ipw,)
        b = Basis(N, two_s=1, two_M=two_M)
        b.set_schedule(*sched)
        ms = time_pass_a(b, J, v0, precision, reps)
        trials.append((sched, ms))
        if verbose:
            print(f"[autotune] {best4} items/wave={ipw}: {ms:.3f} ms", flush=True)
        del b
    staged2 = [(s, ms) for s, ms in trials if len(s) == 5]
    fastest = min(ms for _, ms in staged2)
    best, best_ms = next((s, ms) for s, ms in staged2 if ms <= (1.0 + TIE) * fastest)
    if cache:
        table[key] = {"schedule": list(best), "ms": best_ms,
                      "trials": [[list(s), m] for s, m in trials]}
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            with open(cache, "w") as f:
                json.dump(table, f, indent=1)
        except OSError:
            pass
    return best


def tuned_basis(N, J, two_M=0, dtype=torch.float32, **kw):
    """A spin-1/2 basis whose block kernel runs the tuned schedule."""
    sched = tune(N, J, two_M=two_M, dtype=dtype, **kw)
    b = Basis(N, two_s=1, two_M=two_M)
    b.set_schedule(*sched)
    return b, sched


# --- batched persistent Lanczos -------------------------------------------
# (items per chunk, workgroups per compute unit): the first is the default
BATCH_CANDIDATES = [(4, 4)] + [(c, w) for w in (4, 2, 8, 1) for c in (1, 2, 4, 8, 16)
                               if (c, w) != (4, 4)]


def _batch_key(bases, nvec, steps):
    shapes = ";".join(f"{b.N}/{b.two_s}/{b.two_M}" for b in bases)
    h = hashlib.sha1(shapes.encode()).hexdigest()[:16]
    return f"batched:n={len(bases)},nvec={nvec},steps={steps},shapes={h}"


def tune_batched(bases, Js, V0s, steps, reps=2, cache=DEFAULT_CACHE, verbose=False):
    """Best (chunk, workgroups per CU) of the batched persistent Lanczos for
    this set of instances (their shapes, the number of start vectors and
    steps), timed over whole runs; cached like the block kernel's schedules."""
    import time
    from .batched import BatchedProblem
    nvec = int(V0s[0].shape[0])
    key = _batch_key(bases, nvec, steps)
    table = {}
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
    if key in table:
        return tuple(table[key]["schedule"])
    prob = BatchedProblem(bases, Js, V0s, steps)
    trials = []
    for sched in BATCH_CANDIDATES:
        prob.schedule = sched
        prob.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            prob.run()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        trials.append((sched, ms))
        if verbose:
            print(f"[autotune batched] chunk={sched[0]} wg/CU={sched[1]}: {ms:.2f} ms", flush=True)
    fastest = min(ms for _, ms in trials)
    best, best_ms = next((s, ms) for s, ms in trials if ms <= (1.0 + TIE) * fastest)
    if cache:
        table[key] = {"schedule": list(best), "ms": best_ms,
                      "trials": [[list(s), m] for s, m in trials]}
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            with open(cache, "w") as f:
                json.dump(table, f, indent=1)
        except OSError:
            pass
    return best

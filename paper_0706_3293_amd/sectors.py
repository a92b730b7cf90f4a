"""Magnetization curve E0(M) and finite-temperature Lanczos thermodynamics.

H conserves the total S^z = M, which is why the paper works in the sectors
H(M) (Sec. 2); a magnetization curve needs the lowest energy of each one.  By
the spin-flip symmetry a_u -> 2s - a_u the sectors M and -M share their
spectrum, so only M >= 0 (A = Ns - M = 0 .. floor(Ns)) is computed.

Every sector of one coupling matrix is one instance of the batched persistent
Lanczos (hm_lanczos_batched): all sectors and start vectors run in a single
launch.  For finite temperature, each (sector, start vector) run gives Ritz
values theta_j and Gauss weights |<r|y_j>|^2 (hm_tridiag_ritz), and

    Z_M ~ (D_M / R) sum_r sum_j |<r|y_j>|^2 exp(-theta_j / T)

(likewise for <H> and <H^2>) with R random unit start vectors per sector;
sectors M > 0 count twice.  The Boltzmann sums run in libhm (hm_ftl_sums).
"""
import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from ._lib import check, lib
from .api import Basis
from .batched import BatchedProblem


def sector_two_M(N: int, two_s: int):
    """2M of every sector with M >= 0, from the saturated one down."""
    top = N * two_s
    return list(range(top, -1, -2))


def sector_bases(N: int, two_s: int):
    return [Basis(N, two_s=two_s, two_M=tm) for tm in sector_two_M(N, two_s)]


def multiplicity(two_M: int) -> int:
    return 1 if two_M == 0 else 2


def random_start_vectors(bases, nvec: int, seed: int = 0):
    """uniform[-1, 1) FP64 start vectors (nvec x dim) per basis, on the device.

    Sector k draws from torch's CUDA generator seeded with seed + k.
    """
    out = []
    for k, b in enumerate(bases):
        g = torch.Generator(device="cuda")
        g.manual_seed(int(seed) + k)
        v = torch.rand((nvec, b.dim), generator=g, dtype=torch.float64, device="cuda")
        out.append(v.mul_(2.0).sub_(1.0))
    return out


@dataclass
class MagnetizationCurve:
    two_M: np.ndarray        # [sectors], descending
    dim: np.ndarray          # [sectors]
    E0: np.ndarray           # [sectors]: lowest over the start vectors
    E0_runs: np.ndarray      # [sectors][nvec]
    steps_done: np.ndarray   # [sectors][nvec]


def _run(N, two_s, J, steps, nvec, seed, V0s, tol):
    bases = sector_bases(N, two_s)
    if V0s is None:
        V0s = random_start_vectors(bases, nvec, seed)
    if len(V0s) != len(bases):
        raise ValueError(f"need start vectors for {len(bases)} sectors")
    J = np.asarray(J, dtype=np.float64)
    res = BatchedProblem(bases, [J] * len(bases), V0s, steps, tol).run()
    return bases, res


def magnetization_curve(N: int, two_s: int, J, steps: int, nvec: int = 1, seed: int = 0,
                        V0s=None, tol: float = 0.0, method: str = "auto") -> MagnetizationCurve:
    """E0 of every sector M >= 0 (FP32 vectors, FP64 coefficients and sums).

    method "batched": all sectors and start vectors in one persistent launch
    (hm_lanczos_batched); "single": one hm_lanczos run per sector and start
    vector, which for s = 1/2 runs the block H x kernel; "auto": single for
    s = 1/2, batched otherwise.  V0s: optional list of (nvec, dim) start
    vectors per sector in the order of sector_two_M."""
    if method == "auto":
        method = "single" if two_s == 1 else "batched"
    if method == "batched":
        bases, res = _run(N, two_s, J, steps, nvec, seed, V0s, tol)
        E0_runs, done = res.E0, res.steps_done
    elif method == "single":
        bases = sector_bases(N, two_s)
        if V0s is None:
            V0s = random_start_vectors(bases, nvec, seed)
        E0_runs = np.zeros((len(bases), nvec))
        done = np.zeros((len(bases), nvec), dtype=np.int32)
        for k, (b, V) in enumerate(zip(bases, V0s)):
            V = V if torch.is_tensor(V) else torch.as_tensor(np.asarray(V))
            V = V.to("cuda", torch.float64)
            for r in range(nvec):
                res = b.lanczos(J, V[r].contiguous(), steps, precision="f32_mixed", tol=tol)
                E0_runs[k, r] = res.E0
                done[k, r] = res.steps_done
    else:
        raise ValueError(f"unknown method {method!r}")
    return MagnetizationCurve(
        two_M=np.array(sector_two_M(N, two_s)),
        dim=np.array([b.dim for b in bases], dtype=np.int64),
        E0=E0_runs.min(axis=1), E0_runs=E0_runs, steps_done=done)


def ftl_sums(levels, weights, scales, temps):
    """Boltzmann sums of finite-temperature Lanczos (libhm's hm_ftl_sums):
    levels[r] and weights[r] are the Ritz values and Gauss weights of run r,
    scales[r] the factor of its weights.  Returns Z (relative to
    exp(-E_min / T)), <H> and C = (<H^2> - <H>^2) / T^2 per temperature."""
    lens = np.array([len(l) for l in levels], dtype=np.int32)
    lv = np.ascontiguousarray(np.concatenate([np.asarray(l, dtype=np.float64) for l in levels]))
    wt = np.ascontiguousarray(np.concatenate([np.asarray(w, dtype=np.float64) for w in weights]))
    sc = np.ascontiguousarray(np.asarray(scales, dtype=np.float64))
    T = np.ascontiguousarray(np.asarray(temps, dtype=np.float64).ravel())
    Z, E, C = (np.empty(len(T)) for _ in range(3))
    emin = ctypes.c_double()
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib().hm_ftl_sums(len(lens), lens.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                            lv.ctypes.data_as(dp), wt.ctypes.data_as(dp), sc.ctypes.data_as(dp),
                            len(T), T.ctypes.data_as(dp), Z.ctypes.data_as(dp),
                            E.ctypes.data_as(dp), C.ctypes.data_as(dp), ctypes.byref(emin)))
    return {"T": T, "E_min": emin.value, "Z": Z, "E": E, "C": C}


def thermo_sums(levels, weights, temps):
    """Z (relative to exp(-E_min / T)), <H> and C = (<H^2> - <H>^2) / T^2 of
    one list of levels with weights."""
    return ftl_sums([levels], [weights], [1.0], temps)


def ftl_thermodynamics(N: int, two_s: int, J, temps, steps: int, nvec: int = 16,
                       seed: int = 0, V0s=None, tol: float = 0.0):
    """Finite-temperature Lanczos Z(T), E(T), C(T) over all sectors (k_B = 1).

    Returns the sums of thermo_sums plus the levels and weights they came
    from and the dimension the weights add up to at T -> infinity."""
    bases, res = _run(N, two_s, J, steps, nvec, seed, V0s, tol)
    levels, weights, scales = [], [], []
    for k, (b, tm) in enumerate(zip(bases, sector_two_M(N, two_s))):
        for r in range(nvec):
            th, w = res.ritz(k, r)
            levels.append(th)
            weights.append(w)
            scales.append(multiplicity(tm) * b.dim / nvec)
    out = ftl_sums(levels, weights, scales, temps)
    out.update(levels=np.concatenate(levels),
               weights=np.concatenate([w * s for w, s in zip(weights, scales)]),
               total_dim=sum(multiplicity(tm) * b.dim
                             for b, tm in zip(bases, sector_two_M(N, two_s))))
    return out

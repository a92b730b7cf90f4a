"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the method: it only draws random numbers
and lays out coupling matrices.  Dimensions are passed in by the caller, so
each side (the HIP library or the oracle) supplies its own D(N, A).

Couplings follow H = -sum_{u<v} J_uv s(u).s(v) (Eq. (E-2-1)); J is returned
as a dense symmetric N x N float64 matrix with a zero diagonal.
"""
import numpy as np


def ring_couplings(N: int, J1: float, J2: float = 0.0) -> np.ndarray:
    """Periodic ring with nearest (J1) and next-nearest (J2) neighbour bonds.

    Bond (u, u+d mod N) adds J_d to both J[u, u+d] and J[u+d, u]; for N <= 2d
    the same pair is reached twice and the contributions add up.
    """
    J = np.zeros((N, N))
    for d, Jd in ((1, J1), (2, J2)):
        if Jd == 0.0 or N <= d:
            continue
        for u in range(N):
            v = (u + d) % N
            if u == v:
                continue
            J[u, v] += Jd
            J[v, u] += Jd
    return J


def chain_couplings(Js) -> np.ndarray:
    """Open chain with bond (u, u+1) carrying Js[u], u = 0..N-2."""
    Js = np.asarray(Js, dtype=np.float64)
    N = Js.shape[0] + 1
    J = np.zeros((N, N))
    for u in range(N - 1):
        J[u, u + 1] = J[u + 1, u] = Js[u]
    return J


def upper_bonds(N: int):
    """All pairs (u, v), u < v, in row-major upper-triangle order."""
    return [(u, v) for u in range(N) for v in range(u + 1, N)]


def bond_vector_to_matrix(N: int, bonds, values) -> np.ndarray:
    J = np.zeros((N, N))
    for (u, v), val in zip(bonds, values):
        J[u, v] += val
        J[v, u] += val
    return J


def all_to_all_couplings(N: int, seed: int = 0):
    """Random symmetric J_uv ~ N(0, 1) / sqrt(N) on every pair u < v.

    Returns (J matrix, bond list, bond values); the values are drawn with
    numpy's PCG64 from `seed`, in row-major upper-triangle order.
    """
    bonds = upper_bonds(N)
    vals = np.random.default_rng(seed).normal(0.0, 1.0, len(bonds)) / np.sqrt(N)
    return bond_vector_to_matrix(N, bonds, vals), bonds, vals


def start_vector(dim: int, seed: int = 0) -> np.ndarray:
    """Uniform[-1, 1] start vector of length dim, numpy PCG64 from `seed`."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, dim)


def batched_instances(dim_of, count: int = 64, nvec: int = 16, seed: int = 0,
                      sizes=(8, 10, 12, 14), mean: float = -1.0,
                      sigma: float = 0.2):
    """Instances of the batched workload: spin-1 open chains at M = 0.

    For instance k a generator is spawned from SeedSequence(seed); it draws
    N_k uniformly from `sizes`, the chain couplings J_{u,u+1} ~ N(mean,
    sigma^2), and `nvec` uniform[-1, 1] start vectors of length
    dim_of(N_k) (the caller's D(N_k, A = N_k) for two_s = 2).
    Returns a list of dicts with keys N, J, V0 (nvec x dim).
    """
    out = []
    for child in np.random.SeedSequence(seed).spawn(count):
        rng = np.random.default_rng(child)
        N = int(rng.choice(np.asarray(sizes)))
        Js = rng.normal(mean, sigma, N - 1)
        dim = int(dim_of(N))
        V0 = rng.uniform(-1.0, 1.0, (nvec, dim))
        out.append(dict(N=N, J=chain_couplings(Js), V0=V0))
    return out


# Named workloads (the five configurations the path is measured on).
WORKLOADS = {
    "ring12": dict(N=12, two_s=1, two_M=0, J=("ring", -1.0, 0.0), steps=120,
                   full_reorth=True, seed=0),
    "j1j2_ring28": dict(N=28, two_s=1, two_M=0, J=("ring", -1.0, -0.5),
                        steps=200, full_reorth=False, seed=0),
    "spin1_chains_batched": dict(two_s=2, count=64, nvec=16, steps=80, seed=0),
    "all_to_all20": dict(N=20, two_s=1, two_M=0, J=("all_to_all", 0), steps=300,
                         full_reorth=False, seed=0),
    "j1j2_ring32": dict(N=32, two_s=1, two_M=0, J=("ring", -1.0, -0.25),
                        steps=150, full_reorth=False, seed=0),
}


def workload_couplings(name: str) -> np.ndarray:
    w = WORKLOADS[name]
    kind = w["J"][0]
    if kind == "ring":
        return ring_couplings(w["N"], w["J"][1], w["J"][2])
    if kind == "all_to_all":
        return all_to_all_couplings(w["N"], w["J"][1])[0]
    raise KeyError(name)

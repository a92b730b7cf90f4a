"""Magnetization sectors, E0(M) and finite-temperature sums of the oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper splits the Hilbert space into the sectors H(M) of fixed total
S^z = M (Sec. 2) because H conserves M; a magnetization curve needs the
lowest energy of every sector.  By the spin-flip symmetry a_u -> 2s - a_u
(M -> -M) the sectors M and -M have the same spectrum, so only M >= 0 is
computed (A = Ns - M = 0, 1, ..., floor(Ns)).

Plain definitions used here:
  * E0(M): the smallest eigenvalue of H restricted to H(M), the matrix being
    built column by column from the oracle's own H x (Eq. (E-4-b)) and
    diagonalized densely (numpy eigvalsh as a library step);
  * exact thermodynamics: Z(T) = sum_n exp(-E_n / T) over the full spectrum
    (every sector with its multiplicity: 1 for M = 0, 2 for M > 0),
    E = <H>, C = (<H^2> - <H>^2) / T^2, with k_B = 1;
  * finite-temperature Lanczos (FTL) sums: for R unit start vectors r in a
    sector of dimension D, Z_M ~ (D / R) sum_r sum_j |<r|y_j>|^2 exp(-theta_j / T)
    with the Ritz values theta_j and Gauss weights of each run (the
    Krylov quadrature of <r| exp(-H/T) |r>), likewise for <H> and <H^2>.
"""
import numpy as np

from .core import Subspace
from .lanczos import lanczos, ritz_all


def sector_lowerings(N: int, two_s: int):
    """A = Ns - M for every sector with M >= 0: A = 0 .. floor(N two_s / 2)."""
    return list(range(0, N * two_s // 2 + 1))


def multiplicity(N: int, two_s: int, A: int) -> int:
    """1 for the sector M = 0, else 2 (the sector -M has the same spectrum)."""
    return 1 if 2 * A == N * two_s else 2


def sector_matrix(sub: Subspace, J) -> np.ndarray:
    """Dense H restricted to H(M), column j = H e_j from the oracle's H x."""
    H = np.empty((sub.dim, sub.dim))
    e = np.zeros(sub.dim)
    for j in range(sub.dim):
        e[j] = 1.0
        H[:, j] = sub.apply(J, e)
        e[j] = 0.0
    return H


def sector_spectrum(N: int, two_s: int, A: int, J) -> np.ndarray:
    return np.linalg.eigvalsh(sector_matrix(Subspace(N, two_s, A), J))


def sector_energies(N: int, two_s: int, J) -> np.ndarray:
    """E0 of every sector M >= 0, in the order of sector_lowerings."""
    return np.array([sector_spectrum(N, two_s, A, J)[0]
                     for A in sector_lowerings(N, two_s)])


def thermo_from_levels(levels, weights, temps):
    """Z, <H>, C from energy levels with weights (Boltzmann sums, k_B = 1).

    Z is returned relative to exp(-E_min / T) to stay finite at low T:
    Z(T) = sum_n w_n exp(-(E_n - E_min) / T).
    """
    levels = np.asarray(levels, dtype=np.float64)
    weights = np.asarray(weights, dtype=np.float64)
    e_min = levels.min()
    out = {"T": np.asarray(temps, dtype=np.float64), "E_min": e_min}
    Z, E, C = [], [], []
    for T in out["T"]:
        b = np.exp(-(levels - e_min) / T) * weights
        z = b.sum()
        e1 = (b * levels).sum() / z
        e2 = (b * levels ** 2).sum() / z
        Z.append(z)
        E.append(e1)
        C.append((e2 - e1 * e1) / T ** 2)
    out.update(Z=np.array(Z), E=np.array(E), C=np.array(C))
    return out


def exact_thermodynamics(N: int, two_s: int, J, temps):
    """Thermodynamics from the full spectrum (every sector, with multiplicity)."""
    levels, weights = [], []
    for A in sector_lowerings(N, two_s):
        ev = sector_spectrum(N, two_s, A, J)
        levels.append(ev)
        weights.append(np.full(ev.shape, float(multiplicity(N, two_s, A))))
    return thermo_from_levels(np.concatenate(levels), np.concatenate(weights), temps)


def ftl_levels(N: int, two_s: int, J, start_vectors, steps: int, full_reorth: bool = False):
    """Ritz values and FTL weights of every (sector, start vector) run.

    start_vectors[i] is an (R, D_A) array for sector A = sector_lowerings[i].
    Each run is the oracle's Lanczos from r / |r| (optionally with full
    reorthogonalization); a level theta_j gets the weight mult_M (D / R) |z_1j|^2.
    """
    levels, weights = [], []
    for A, V in zip(sector_lowerings(N, two_s), start_vectors):
        sub = Subspace(N, two_s, A)
        V = np.atleast_2d(np.asarray(V, dtype=np.float64))
        R = V.shape[0]
        for r in range(R):
            res = lanczos(sub, J, V[r], steps, full_reorth=full_reorth)
            th, w = ritz_all(res["alpha"], res["beta"])
            levels.append(th)
            weights.append(w * multiplicity(N, two_s, A) * sub.dim / R)
    return np.concatenate(levels), np.concatenate(weights)


def ftl_thermodynamics(N: int, two_s: int, J, start_vectors, steps: int, temps,
                       full_reorth: bool = False):
    levels, weights = ftl_levels(N, two_s, J, start_vectors, steps, full_reorth)
    return thermo_from_levels(levels, weights, temps)

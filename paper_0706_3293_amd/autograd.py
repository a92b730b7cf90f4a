"""Differentiable ground-state energy E0(J) of H = -sum_b J_b s(u_b).s(v_b).

Forward: Lanczos through the C ABI (hm_lanczos) and the library's host
tridiagonal solver give E0 and the lowest eigenvector c of T.
Backward: the ground-state vector psi0 = sum_k c_k v_k is recomputed on the
GPU by a second Lanczos pass that repeats the forward recurrence bit for bit
(hm_lanczos_ritz), instead of keeping the whole Krylov basis; then the bond
correlation kernel (hm_bond_corr) gives C_b = <psi0| s(u_b).s(v_b) |psi0>, and
since H is linear in J (Hellmann-Feynman) dE0/dJ_b = -C_b.
"""
import numpy as np
import torch

from .api import Basis, tridiag_lowest


def couplings_matrix(N, bonds, values):
    """Dense symmetric J with J[u, v] = J[v, u] = sum of the values of bond (u, v)."""
    J = np.zeros((N, N))
    for (u, v), val in zip(bonds, np.asarray(values, dtype=np.float64)):
        J[u, v] += val
        J[v, u] += val
    return J


class GroundStateEnergy(torch.autograd.Function):
    """E0 as a function of a vector of bond couplings (one entry per bond)."""

    @staticmethod
    def forward(ctx, Jvals, basis: Basis, bonds, v0, steps, precision="f64",
                kernel=0, tol=0.0):
        vals = Jvals.detach().to("cpu", torch.float64).numpy()
        J = couplings_matrix(basis.N, bonds, vals)
        res = basis.lanczos(J, v0, steps, precision=precision, kernel=kernel, tol=tol)
        E0, c = tridiag_lowest(res.alpha, res.beta)
        ctx.basis, ctx.bonds, ctx.v0, ctx.J = basis, list(bonds), v0, J
        ctx.opts = dict(precision=precision, kernel=kernel, tol=tol)
        ctx.steps_done, ctx.c = res.steps_done, c
        ctx.lanczos = res
        ctx.jdevice, ctx.jdtype = Jvals.device, Jvals.dtype
        return torch.tensor(E0, dtype=torch.float64, device=Jvals.device)

    @staticmethod
    def backward(ctx, grad_out):
        psi, alpha, beta = ctx.basis.ritz(ctx.J, ctx.v0, ctx.steps_done, ctx.c, **ctx.opts)
        corr = ctx.basis.bond_corr(ctx.bonds, psi)
        grad = -float(grad_out) * torch.tensor(corr, dtype=torch.float64)
        return (grad.to(ctx.jdevice, ctx.jdtype), None, None, None, None, None, None, None)


def ground_state_energy(Jvals, basis, bonds, v0, steps, precision="f64", kernel=0, tol=0.0):
    """E0(J) with autograd support (see GroundStateEnergy)."""
    return GroundStateEnergy.apply(Jvals, basis, bonds, v0, steps, precision, kernel, tol)


def ground_state(basis: Basis, J, v0, steps, precision="f64", kernel=0, tol=0.0):
    """E0, psi0 (device FP64, normalized) and the Lanczos coefficients."""
    res = basis.lanczos(J, v0, steps, precision=precision, kernel=kernel, tol=tol)
    E0, c = tridiag_lowest(res.alpha, res.beta)
    psi, _, _ = basis.ritz(J, v0, res.steps_done, c, precision=precision, kernel=kernel, tol=tol)
    return E0, psi, res

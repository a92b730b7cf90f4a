"""Batched Lanczos over many (basis, couplings, start vectors) instances in one
persistent launch (hm_lanczos_batched): argument marshalling only."""
import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from ._lib import check, lib
from .api import _stream, tridiag_ritz


@dataclass
class BatchedResult:
    alpha: np.ndarray        # [ninst][nvec][steps]
    beta: np.ndarray         # [ninst][nvec][steps]
    E0: np.ndarray           # [ninst][nvec]
    steps_done: np.ndarray   # [ninst][nvec]

    def ritz(self, k, r):
        """Ritz values and first-component weights |z_1|^2 of pair (k, r)."""
        n = int(self.steps_done[k, r])
        return tridiag_ritz(self.alpha[k, r, :n], self.beta[k, r, : max(n - 1, 0)])


class BatchedProblem:
    """Device-resident inputs of one batched run, reusable across calls.

    bases: list of Basis (one spin s); Js: list of N_k x N_k couplings;
    V0s: list of (nvec, dim_k) start vectors (numpy or torch), same nvec.
    """

    def __init__(self, bases, Js, V0s, steps: int, tol: float = 0.0, schedule=(0, 0)):
        self.schedule = tuple(int(v) for v in schedule)   # (chunk, workgroups per CU)
        self.bases = list(bases)
        self.ninst = len(self.bases)
        self.nvec = int(V0s[0].shape[0])
        self.steps = int(steps)
        self.tol = float(tol)
        self.dv = []
        for b, V in zip(self.bases, V0s):
            t = V if torch.is_tensor(V) else torch.as_tensor(np.asarray(V))
            t = t.to("cuda", torch.float64)
            if t.shape != (self.nvec, b.dim):
                raise ValueError("each V0 must be (nvec, dim)")
            self.dv.append(t.T.contiguous())          # [dim][nvec] interleaved
        self.handles = (ctypes.c_void_p * self.ninst)(*[b.handle.value for b in self.bases])
        self.Jh = [np.ascontiguousarray(np.asarray(J, dtype=np.float64)) for J in Js]
        self.Jp = (ctypes.POINTER(ctypes.c_double) * self.ninst)(
            *[j.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for j in self.Jh])
        self.vp = (ctypes.c_void_p * self.ninst)(*[t.data_ptr() for t in self.dv])
        nbytes = ctypes.c_size_t()
        check(lib().hm_lanczos_batched_workspace(self.ninst, self.handles, self.nvec,
                                                 self.steps, ctypes.byref(nbytes)))
        self.work = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        self.rows = sum(b.dim for b in self.bases)

    def run(self) -> BatchedResult:
        n, v, s = self.ninst, self.nvec, self.steps
        alpha = np.zeros((n, v, s))
        beta = np.zeros((n, v, s))
        E0 = np.zeros((n, v))
        done = np.zeros((n, v), dtype=np.int32)
        dp = ctypes.POINTER(ctypes.c_double)
        check(lib().hm_lanczos_batched(n, self.handles, self.Jp, self.vp, v, s, self.tol,
                                       self.schedule[0], self.schedule[1],
                                       ctypes.c_void_p(self.work.data_ptr()), self.work.numel(),
                                       alpha.ctypes.data_as(dp), beta.ctypes.data_as(dp),
                                       E0.ctypes.data_as(dp),
                                       done.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       _stream()))
        return BatchedResult(alpha, beta, E0, done)


def lanczos_batched(bases, Js, V0s, steps: int, tol: float = 0.0,
                    schedule=(0, 0)) -> BatchedResult:
    """One batched run (see BatchedProblem); schedule = (items per chunk,
    workgroups per compute unit), 0 for the defaults."""
    return BatchedProblem(bases, Js, V0s, steps, tol, schedule).run()

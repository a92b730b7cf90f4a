"""Batched Lanczos over many (basis, couplings, start vectors) instances in one
persistent launch (hm_lanczos_batched): argument marshalling only."""
import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from ._lib import check, lib
from .api import _stream


@dataclass
class BatchedResult:
    alpha: np.ndarray        # [ninst][nvec][steps]
    beta: np.ndarray         # [ninst][nvec][steps]
    E0: np.ndarray           # [ninst][nvec]
    steps_done: np.ndarray   # [ninst][nvec]

    def ritz(self, k, r):
        """Ritz values and first-component weights |z_1|^2 of pair (k, r)."""
        import scipy.linalg
        n = int(self.steps_done[k, r])
        a, b = self.alpha[k, r, :n], self.beta[k, r, : max(n - 1, 0)]
        if n == 1:
            return a.copy(), np.ones(1)
        w, z = scipy.linalg.eigh_tridiagonal(a, b)
        return w, z[0] ** 2


def lanczos_batched(bases, Js, V0s, steps: int, tol: float = 0.0) -> BatchedResult:
    """bases: list of Basis (one spin s), Js: list of N_k x N_k couplings,
    V0s: list of (nvec, dim_k) start vectors (numpy or torch), same nvec."""
    ninst = len(bases)
    nvec = int(V0s[0].shape[0])
    dv = []
    for b, V in zip(bases, V0s):
        t = torch.as_tensor(np.asarray(V) if not torch.is_tensor(V) else V)
        t = t.to("cuda", torch.float64)
        if t.shape != (nvec, b.dim):
            raise ValueError("each V0 must be (nvec, dim)")
        dv.append(t.T.contiguous())             # [dim][nvec] interleaved
    handles = (ctypes.c_void_p * ninst)(*[b.handle.value for b in bases])
    Jh = [np.ascontiguousarray(np.asarray(J, dtype=np.float64)) for J in Js]
    Jp = (ctypes.POINTER(ctypes.c_double) * ninst)(
        *[j.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for j in Jh])
    vp = (ctypes.c_void_p * ninst)(*[t.data_ptr() for t in dv])
    nbytes = ctypes.c_size_t()
    check(lib().hm_lanczos_batched_workspace(ninst, handles, nvec, steps, ctypes.byref(nbytes)))
    work = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
    alpha = np.zeros((ninst, nvec, steps))
    beta = np.zeros((ninst, nvec, steps))
    E0 = np.zeros((ninst, nvec))
    done = np.zeros((ninst, nvec), dtype=np.int32)
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib().hm_lanczos_batched(ninst, handles, Jp, vp, nvec, steps, float(tol),
                                   ctypes.c_void_p(work.data_ptr()), nbytes.value,
                                   alpha.ctypes.data_as(dp), beta.ctypes.data_as(dp),
                                   E0.ctypes.data_as(dp),
                                   done.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _stream()))
    return BatchedResult(alpha, beta, E0, done)

"""Python binding of libhm: argument marshalling over the C ABI of include/hm.h.

Every step of the hot path runs in the HIP kernels of libhm.so; torch is used
only to hold device memory and to name the current HIP stream.
"""
import atexit
import ctypes
import weakref
from dataclasses import dataclass
from fractions import Fraction

import numpy as np
import torch

from . import _lib
from ._lib import HM_F32, HM_F64, HM_PREC_F32_MIXED, HM_PREC_F64, check, lib

PRECISIONS = {"f64": HM_PREC_F64, "fp64": HM_PREC_F64,
              "f32_mixed": HM_PREC_F32_MIXED, "mixed": HM_PREC_F32_MIXED}


# Live basis handles.  At interpreter exit they are freed by an atexit hook,
# which runs before torch's own exit handlers and long before the HIP runtime
# and any profiler attached to it are torn down; handles still alive after
# that (objects finalized during interpreter shutdown) are left to the
# process exit instead of calling into the runtime.
_live = weakref.WeakSet()
_exiting = False


def _free_all_at_exit():
    global _exiting
    _exiting = True
    handles = list(_live)
    if not handles or _lib._lib is None:
        return
    try:
        if torch.cuda.is_available() and torch.cuda.is_initialized():
            torch.cuda.synchronize()
    except Exception:
        pass
    for b in handles:
        b._free()


atexit.register(_free_all_at_exit)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _doubled(q, what):
    f = Fraction(q).limit_denominator(2) if not isinstance(q, Fraction) else q
    if f.denominator not in (1, 2) or abs(float(f) - float(q)) > 1e-12:
        raise ValueError(f"{what} must be an integer or half-integer, got {q}")
    return int(2 * f)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _host_dbl(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def count(n: int, two_s: int, A: int) -> int:
    """D(n, A) of Eq. (E-3-c) computed by the library."""
    out = ctypes.c_int64()
    check(lib().hm_count(n, two_s, A, ctypes.byref(out)))
    return out.value


@dataclass
class LanczosResult:
    alpha: np.ndarray
    beta: np.ndarray
    E0: float
    steps_done: int


class Basis:
    """The subspace H(M) of N spins s (Sec. 3), owning a libhm basis handle.

    Pass (N, s, M) with s and M integers or half-integers (floats or
    Fractions), or the doubled values via two_s=..., two_M=...
    """

    def __init__(self, N, s=None, M=0, *, two_s=None, two_M=None):
        two_s = two_s if two_s is not None else _doubled(s, "s")
        two_M = two_M if two_M is not None else _doubled(M, "M")
        h = ctypes.c_void_p()
        check(lib().hm_basis_init(int(N), int(two_s), int(two_M), ctypes.byref(h)))
        self._h = h
        dim = ctypes.c_int64()
        check(lib().hm_basis_dim(h, ctypes.byref(dim)))
        n_, ts, A, bits = (ctypes.c_int32() for _ in range(4))
        check(lib().hm_basis_info(h, ctypes.byref(n_), ctypes.byref(ts), ctypes.byref(A),
                                  ctypes.byref(bits)))
        self.N, self.two_s, self.A, self.bits = n_.value, ts.value, A.value, bits.value
        self.two_M = int(two_M)
        self.dim = dim.value
        self._work = {}
        _live.add(self)

    def _free(self):
        h = getattr(self, "_h", None)
        self._h = None
        self._work = {}
        if h is not None and h.value and _lib._lib is not None:
            _lib._lib.hm_basis_free(h)

    def free(self):
        """Release the handle now (waits for the device first); the object
        is unusable afterwards."""
        if getattr(self, "_h", None) is not None:
            torch.cuda.synchronize()
            self._free()

    def __del__(self):
        if _exiting:
            return                    # freed by the exit hook, or left to exit
        if getattr(self, "_h", None) is not None:
            try:
                if torch.cuda.is_available() and torch.cuda.is_initialized():
                    torch.cuda.synchronize()
            except Exception:
                pass
            self._free()

    @property
    def handle(self):
        return self._h

    def set_schedule(self, low_bits: int = 0, block_threads: int = 0, rows_per_lane: int = 0,
                     staging: int = 0, items_per_wave: int = 0):
        """Schedule of the spin-1/2 block kernel (before first device use);
        staging: 0 automatic, 1 chunked items, 2 staged blocks; items_per_wave
        sizes the grid (0: the default grid)."""
        check(lib().hm_basis_set_schedule(self._h, int(low_bits), int(block_threads),
                                          int(rows_per_lane)))
        check(lib().hm_basis_set_staging(self._h, int(staging)))
        check(lib().hm_basis_set_items_per_wave(self._h, int(items_per_wave)))

    # --- codec ------------------------------------------------------------
    def unrank(self, i: int) -> np.ndarray:
        d = (ctypes.c_uint8 * self.N)()
        check(lib().hm_unrank(self._h, int(i), d))
        return np.frombuffer(d, dtype=np.uint8).astype(np.int64)

    def rank(self, digits) -> int:
        a = np.ascontiguousarray(np.asarray(digits, dtype=np.uint8))
        if a.shape != (self.N,):
            raise ValueError("need N digits")
        out = ctypes.c_int64()
        check(lib().hm_rank(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                            ctypes.byref(out)))
        return out.value

    def unrank_dev(self, idx: torch.Tensor) -> torch.Tensor:
        """Packed states (int64 view of uint64) of device int64 indices."""
        idx = idx.contiguous()
        assert idx.is_cuda and idx.dtype == torch.int64
        out = torch.empty_like(idx)
        check(lib().hm_unrank_dev(self._h, _dptr(idx), idx.numel(), _dptr(out), _stream()))
        return out

    def rank_dev(self, states: torch.Tensor) -> torch.Tensor:
        states = states.contiguous()
        assert states.is_cuda and states.dtype == torch.int64
        out = torch.empty_like(states)
        check(lib().hm_rank_dev(self._h, _dptr(states), states.numel(), _dptr(out), _stream()))
        return out

    # --- H x --------------------------------------------------------------
    def _J(self, J):
        J, p = _host_dbl(J)
        if J.shape != (self.N, self.N):
            raise ValueError("J must be N x N")
        return J, p

    def apply(self, J, x: torch.Tensor, out: torch.Tensor = None, kernel: int = 0):
        """y = H x (Eq. (E-4-b)) for a device vector x of dim float64/float32."""
        assert x.is_cuda and x.shape == (self.dim,) and x.is_contiguous()
        dtype = {torch.float64: HM_F64, torch.float32: HM_F32}[x.dtype]
        y = torch.empty_like(x) if out is None else out
        Jh, Jp = self._J(J)
        if kernel == 0:
            check(lib().hm_apply(self._h, Jp, _dptr(x), _dptr(y), dtype, _stream()))
        else:
            check(lib().hm_apply_kernel(self._h, Jp, _dptr(x), _dptr(y), dtype, kernel,
                                        _stream()))
        return y

    # --- Lanczos ----------------------------------------------------------
    def _opts(self, precision, full_reorth, use_graph, tol, kernel):
        return _lib.LanczosOpts(PRECISIONS[precision], int(bool(full_reorth)), float(tol),
                                int(bool(use_graph)), int(kernel))

    def workspace(self, steps, opts) -> torch.Tensor:
        n = ctypes.c_size_t()
        check(lib().hm_lanczos_workspace(self._h, steps, ctypes.byref(opts), ctypes.byref(n)))
        key = n.value
        w = self._work.get(key)
        if w is None:
            self._work.clear()
            w = torch.empty(key, dtype=torch.uint8, device="cuda")
            self._work[key] = w
        return w

    def lanczos(self, J, v0: torch.Tensor, steps: int, precision="f64", full_reorth=False,
                use_graph=False, tol=0.0, kernel=0) -> LanczosResult:
        """Lanczos from the device FP64 start vector v0 (Sec. 4's repeated H x).
        use_graph: replay the step loop as one hipGraph, captured on the first
        call with these couplings, step count and options and kept with the
        handle (bitwise equal to direct launches).  Replays measured 0-3 %
        faster than direct launches; the first call pays the capture, so it
        pays off for repeated runs (more start vectors, repeated solves)."""
        assert v0.is_cuda and v0.dtype == torch.float64 and v0.shape == (self.dim,)
        v0 = v0.contiguous()
        opts = self._opts(precision, full_reorth, use_graph, tol, kernel)
        work = self.workspace(steps, opts)
        alpha = np.zeros(steps)
        beta = np.zeros(steps)
        E0 = ctypes.c_double()
        done = ctypes.c_int32()
        Jh, Jp = self._J(J)
        check(lib().hm_lanczos(self._h, Jp, _dptr(v0), steps, ctypes.byref(opts), _dptr(work),
                               work.numel(), alpha.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               beta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               ctypes.byref(E0), ctypes.byref(done), _stream()))
        k = done.value
        return LanczosResult(alpha[:k].copy(), beta[:k].copy(), E0.value, k)

    def ritz(self, J, v0: torch.Tensor, steps_done: int, c, precision="f64",
             full_reorth=False, use_graph=False, tol=0.0, kernel=0):
        """psi = sum_k c_k v_k recomputed by a second identical Lanczos pass."""
        opts = self._opts(precision, full_reorth, use_graph, tol, kernel)
        work = self.workspace(steps_done, opts)
        psi = torch.empty(self.dim, dtype=torch.float64, device=v0.device)
        c, cp = _host_dbl(c)
        alpha = np.zeros(steps_done)
        beta = np.zeros(steps_done)
        Jh, Jp = self._J(J)
        check(lib().hm_lanczos_ritz(self._h, Jp, _dptr(v0.contiguous()), steps_done, cp,
                                    ctypes.byref(opts), _dptr(work), work.numel(), _dptr(psi),
                                    alpha.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    beta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    _stream()))
        return psi, alpha, beta

    def block_lanczos(self, J, X0: torch.Tensor, steps: int):
        """Block Lanczos from the p columns of X0 (device FP64, (dim, p) or
        (p, dim)); returns the diagonal blocks A (n x p x p), the sub-diagonal
        blocks B (n-1 x p x p) and n = the block steps done."""
        assert X0.is_cuda and X0.dtype == torch.float64 and X0.dim() == 2
        if X0.shape[0] != self.dim:
            X0 = X0.T
        p = int(X0.shape[1])
        X0 = X0.contiguous()                     # row-interleaved [dim][p]
        n = ctypes.c_size_t()
        check(lib().hm_block_lanczos_workspace(self._h, p, steps, ctypes.byref(n)))
        work = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        A = np.zeros((steps, p, p))
        B = np.zeros((steps, p, p))
        done = ctypes.c_int32()
        Jh, Jp = self._J(J)
        dp = ctypes.POINTER(ctypes.c_double)
        check(lib().hm_block_lanczos(self._h, Jp, _dptr(X0), p, steps, _dptr(work), work.numel(),
                                     A.ctypes.data_as(dp), B.ctypes.data_as(dp),
                                     ctypes.byref(done), _stream()))
        k = done.value
        return A[:k].copy(), B[: max(k - 1, 0)].copy(), k

    def lowest_levels(self, J, count: int, steps: int, p: int = 4, seed: int = 0,
                      X0: torch.Tensor = None) -> np.ndarray:
        """The `count` lowest eigenvalues (with multiplicity, up to p-fold) from a
        block Lanczos run: eigenvalues of the block tridiagonal matrix (host
        FP64 dense eigensolve, the block form of the final tridiagonal step)."""
        if X0 is None:
            g = torch.Generator(device="cuda")
            g.manual_seed(int(seed))
            X0 = torch.rand((self.dim, p), generator=g, dtype=torch.float64,
                            device="cuda").mul_(2.0).sub_(1.0)
        A, B, k = self.block_lanczos(J, X0, steps)
        return block_tridiag_eigenvalues(A, B)[:count]

    def bond_corr(self, bonds, psi: torch.Tensor) -> np.ndarray:
        """<psi| s(u).s(v) |psi> for each bond (u, v) (device FP64 psi)."""
        uv = np.ascontiguousarray(np.asarray(bonds, dtype=np.int32).reshape(-1, 2))
        out = np.zeros(uv.shape[0])
        n = ctypes.c_size_t()
        check(lib().hm_bond_corr_workspace(self._h, uv.shape[0], ctypes.byref(n)))
        work = torch.empty(max(n.value, 1), dtype=torch.uint8, device=psi.device)
        check(lib().hm_bond_corr(self._h, uv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                 uv.shape[0], _dptr(psi.contiguous()), _dptr(work),
                                 work.numel(),
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 _stream()))
        return out

    def cached_couplings(self) -> int:
        """Coupling lists the handle keeps on the device (at most 4)."""
        n = ctypes.c_int32()
        check(lib().hm_basis_cached_couplings(self._h, ctypes.byref(n)))
        return n.value


def tridiag_lowest(alpha, beta):
    """Lowest eigenpair of tridiag(alpha; beta[:-1]) by the library's host solver."""
    alpha, ap = _host_dbl(alpha)
    k = alpha.shape[0]
    beta, bp = _host_dbl(np.concatenate([np.asarray(beta, dtype=np.float64)[: k - 1], [0.0]]))
    ev = ctypes.c_double()
    vec = np.zeros(k)
    check(lib().hm_tridiag_lowest(k, ap, bp, ctypes.byref(ev),
                                  vec.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return ev.value, vec


def tridiag_ritz(alpha, beta):
    """All eigenvalues of tridiag(alpha; beta[:k-1]) (ascending) and the squared
    first components of their unit eigenvectors, by the library's host solver."""
    alpha, ap = _host_dbl(alpha)
    k = alpha.shape[0]
    beta, bp = _host_dbl(np.concatenate([np.asarray(beta, dtype=np.float64)[: k - 1], [0.0]]))
    vals = np.zeros(k)
    wts = np.zeros(k)
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib().hm_tridiag_ritz(k, ap, bp, vals.ctypes.data_as(dp), wts.ctypes.data_as(dp)))
    return vals, wts


def block_tridiag_eigenvalues(A, B) -> np.ndarray:
    """Eigenvalues (ascending) of the symmetric block tridiagonal matrix with
    diagonal blocks A[k] and sub-diagonal blocks B[k] (block k+1, k), by the
    library's host solver."""
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
    n, p = A.shape[0], A.shape[1]
    B = np.ascontiguousarray(np.asarray(B, dtype=np.float64)[: max(n - 1, 0)])
    if B.shape[0] == 0:
        B = np.zeros((1, p, p))
    vals = np.zeros(n * p)
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib().hm_block_tridiag_eigenvalues(n, p, A.ctypes.data_as(dp), B.ctypes.data_as(dp),
                                             vals.ctypes.data_as(dp)))
    return vals


def set_timing(enable: bool):
    lib().hm_set_timing(int(bool(enable)))


def last_timing():
    hx = ctypes.c_double()
    n = ctypes.c_int32()
    loop = ctypes.c_double()
    lib().hm_last_timing(ctypes.byref(hx), ctypes.byref(n), ctypes.byref(loop))
    return dict(hx_ms=hx.value, hx_launches=n.value, loop_ms=loop.value)

"""ctypes binding of the C oracle (oracle/oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg; never by the product package.

Functions follow Sec. 3 (count table Eq. (E-3-c), decoding Sec. 3.1, successor
Sec. 3.1, encoding Sec. 3.2) and Sec. 4 (gather form Eq. (E-4-b)) of the paper.
Indices are 0-based, digits a_u = s - m_u, the spin is given as two_s = 2s and
the subspace by A = sum_u a_u (M = N s - A).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_intp = ctypes.POINTER(ctypes.c_int)
_dblp = ctypes.POINTER(ctypes.c_double)


def bind(path: str):
    """Load an oracle library from `path` and declare its entry points."""
    lib = ctypes.CDLL(path)
    lib.or_count_table.argtypes = [ctypes.c_int, ctypes.c_int, _i64p]
    lib.or_count_table.restype = ctypes.c_int
    lib.or_unrank.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64p,
                              ctypes.c_int64, _intp]
    lib.or_unrank.restype = ctypes.c_int
    lib.or_rank.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64p,
                            _intp]
    lib.or_rank.restype = ctypes.c_int64
    lib.or_unrank_range.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64p,
                                    ctypes.c_int64, ctypes.c_int64,
                                    ctypes.POINTER(ctypes.c_uint8)]
    lib.or_unrank_range.restype = ctypes.c_int
    lib.or_successor.argtypes = [ctypes.c_int, ctypes.c_int, _intp]
    lib.or_successor.restype = ctypes.c_int
    lib.or_apply.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64p,
                             _dblp, _dblp, _dblp]
    lib.or_apply.restype = ctypes.c_int
    lib.or_apply_rows.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  _i64p, _dblp, _dblp, _i64p, ctypes.c_int64,
                                  _dblp]
    lib.or_apply_rows.restype = ctypes.c_int
    lib.or_apply_rows_hashed.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         _i64p, _dblp, _i64p, ctypes.c_int64, _dblp]
    lib.or_apply_rows_hashed.restype = ctypes.c_int
    lib.or_max_threads.argtypes = []
    lib.or_max_threads.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _build
            _build.build()
        _lib = bind(_LIB_PATH)
    return _lib


def _ptr(arr, ctype):
    return arr.ctypes.data_as(ctypes.POINTER(ctype))


def max_threads() -> int:
    """Threads the oracle's OpenMP row loop uses."""
    return int(_load().or_max_threads())


def count_table(N: int, two_s: int, lib=None) -> np.ndarray:
    """D(n, A) for n = 0..N, A = 0..N*two_s, Eq. (E-3-c); zero elsewhere."""
    D = np.zeros((N + 1, N * two_s + 1), dtype=np.int64)
    lib = lib or _load()
    if lib.or_count_table(N, two_s, _ptr(D, ctypes.c_int64)) != 0:
        raise OverflowError("D(n, A) overflows int64")
    return D


def count(n: int, two_s: int, A: int) -> int:
    """D(n, A) with zero outside 0 <= A <= 2 n s (Sec. 3)."""
    if n < 0 or A < 0 or A > n * two_s:
        return 0
    return int(count_table(n, two_s)[n, A])


class Subspace:
    """The subspace H(M = N s - A) with its count table (oracle side)."""

    def __init__(self, N: int, two_s: int, A: int, lib=None):
        if N < 1 or two_s < 1 or A < 0 or A > N * two_s:
            raise ValueError("invalid (N, two_s, A)")
        self.N, self.two_s, self.A = N, two_s, A
        self._lib = lib or _load()
        self.D = count_table(N, two_s, self._lib)
        self.dim = int(self.D[N, A])

    def unrank(self, i: int) -> np.ndarray:
        """Digits a_1..a_N of basis state i (Sec. 3.1)."""
        a = np.zeros(self.N, dtype=np.intc)
        rc = self._lib.or_unrank(self.N, self.two_s, self.A,
                               _ptr(self.D, ctypes.c_int64), int(i),
                               _ptr(a, ctypes.c_int))
        if rc != 0:
            raise IndexError(f"index {i} outside [0, {self.dim})")
        return a.astype(np.int64)

    def unrank_range(self, first: int, n: int) -> np.ndarray:
        """Digits of basis states first .. first+n-1 as an (n, N) uint8 array,
        each decoded on its own (Sec. 3.1)."""
        out = np.zeros((n, self.N), dtype=np.uint8)
        rc = self._lib.or_unrank_range(self.N, self.two_s, self.A,
                                       _ptr(self.D, ctypes.c_int64), int(first), int(n),
                                       _ptr(out, ctypes.c_uint8))
        if rc != 0:
            raise IndexError(f"range [{first}, {first + n}) outside [0, {self.dim})")
        return out

    def rank(self, digits) -> int:
        """0-based index of the basis state with the given digits (Sec. 3.2)."""
        a = np.ascontiguousarray(np.asarray(digits, dtype=np.intc))
        if a.shape != (self.N,):
            raise ValueError("need N digits")
        r = self._lib.or_rank(self.N, self.two_s, self.A,
                            _ptr(self.D, ctypes.c_int64), _ptr(a, ctypes.c_int))
        if r < 0:
            raise ValueError("digits are not a basis state of this subspace")
        return int(r)

    def successor(self, digits):
        """Next basis state by the balls-in-boxes rule (Sec. 3.1), or None."""
        a = np.ascontiguousarray(np.asarray(digits, dtype=np.intc)).copy()
        ok = self._lib.or_successor(self.N, self.two_s, _ptr(a, ctypes.c_int))
        return a.astype(np.int64) if ok else None

    def _J(self, J):
        J = np.ascontiguousarray(np.asarray(J, dtype=np.float64))
        if J.shape != (self.N, self.N):
            raise ValueError("J must be N x N")
        return J

    def apply(self, J, x) -> np.ndarray:
        """y = H x over the whole subspace, row-gather form Eq. (E-4-b)."""
        J = self._J(J)
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        if x.shape != (self.dim,):
            raise ValueError("x must have length dim")
        y = np.empty(self.dim, dtype=np.float64)
        rc = self._lib.or_apply(self.N, self.two_s, self.A,
                              _ptr(self.D, ctypes.c_int64), _ptr(J, ctypes.c_double),
                              _ptr(x, ctypes.c_double), _ptr(y, ctypes.c_double))
        if rc != 0:
            raise RuntimeError("oracle apply failed")
        return y

    def apply_rows_hashed(self, J, rows) -> np.ndarray:
        """(H x)_i for the listed rows, with x_j = hashed_input(j) (no x array:
        checks rows of problems whose vectors do not fit in host memory)."""
        J = self._J(J)
        rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        y = np.empty(rows.shape[0], dtype=np.float64)
        rc = self._lib.or_apply_rows_hashed(self.N, self.two_s, self.A,
                                            _ptr(self.D, ctypes.c_int64),
                                            _ptr(J, ctypes.c_double),
                                            _ptr(rows, ctypes.c_int64), rows.shape[0],
                                            _ptr(y, ctypes.c_double))
        if rc != 0:
            raise RuntimeError("oracle apply_rows_hashed failed (row out of range?)")
        return y

    def apply_rows(self, J, x, rows) -> np.ndarray:
        """(H x)_i for the listed rows i only."""
        J = self._J(J)
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        y = np.empty(rows.shape[0], dtype=np.float64)
        rc = self._lib.or_apply_rows(self.N, self.two_s, self.A,
                                   _ptr(self.D, ctypes.c_int64),
                                   _ptr(J, ctypes.c_double), _ptr(x, ctypes.c_double),
                                   _ptr(rows, ctypes.c_int64), rows.shape[0],
                                   _ptr(y, ctypes.c_double))
        if rc != 0:
            raise RuntimeError("oracle apply_rows failed (row out of range?)")
        return y


def hashed_input(idx) -> np.ndarray:
    """The counter-based input of apply_rows_hashed: x_j = (top 24 bits of
    j * 0x9E3779B97F4A7C15 mod 2^64) / 2^24 - 1/2 (Knuth's multiplicative
    hash), exact in FP32 and FP64."""
    j = np.asarray(idx, dtype=np.uint64)
    h = j * np.uint64(0x9E3779B97F4A7C15)
    return (h >> np.uint64(40)).astype(np.float64) / 16777216.0 - 0.5

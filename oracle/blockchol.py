"""ctypes wrapper of the oracle's C core (``block_chol.c``) -- test infrastructure only."""
import ctypes

import numpy as np

from . import library_path

_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(library_path())
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.ob_create.restype = ctypes.c_void_p
        lib.ob_create.argtypes = [ctypes.c_int, ip]
        lib.ob_free.restype = None
        lib.ob_free.argtypes = [ctypes.c_void_p]
        lib.ob_set.restype = ctypes.c_int
        lib.ob_set.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, dp]
        lib.ob_get.restype = ctypes.c_int
        lib.ob_get.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, dp]
        lib.ob_cholesky.restype = ctypes.c_int
        lib.ob_cholesky.argtypes = [ctypes.c_void_p]
        lib.ob_solve.restype = ctypes.c_int
        lib.ob_solve.argtypes = [ctypes.c_void_p, dp, ctypes.c_int]
        lib.ob_size.restype = ctypes.c_long
        lib.ob_size.argtypes = [ctypes.c_void_p]
        _lib = lib
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class BlockMatrix:
    """An M x M grid of dense FP64 blocks (lower part), factored in place."""

    def __init__(self, sizes):
        lib = _load()
        self.sizes = [int(s) for s in sizes]
        arr = (ctypes.c_int * len(self.sizes))(*self.sizes)
        self._h = lib.ob_create(len(self.sizes), arr)
        if not self._h:
            raise MemoryError("ob_create failed")
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _load is not None:   # module globals are cleared at interpreter exit
            _load().ob_free(h)
            self._h = None

    @property
    def n(self):
        return int(self.offsets[-1])

    def set(self, i, j, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        assert a.shape == (self.sizes[i], self.sizes[j]), (a.shape, i, j)
        if _load().ob_set(self._h, i, j, _dptr(a)) != 0:
            raise ValueError("ob_set(%d, %d) failed" % (i, j))

    def get(self, i, j):
        out = np.empty((self.sizes[i], self.sizes[j]), dtype=np.float64)
        rc = _load().ob_get(self._h, i, j, _dptr(out))
        if rc < 0:
            raise ValueError("ob_get(%d, %d) failed" % (i, j))
        return out if rc == 1 else None

    def cholesky(self):
        """Factor in place; 0, or (block column + 1) of the first failing pivot block."""
        return int(_load().ob_cholesky(self._h))

    def solve(self, rhs):
        """Solve L L^T x = rhs (rows in block order); returns a new array."""
        x = np.array(rhs, dtype=np.float64, order="C", copy=True)
        squeeze = x.ndim == 1
        if squeeze:
            x = x[:, None]
        assert x.shape[0] == self.n
        if _load().ob_solve(self._h, _dptr(x), x.shape[1]) != 0:
            raise ValueError("ob_solve failed")
        return x[:, 0] if squeeze else x

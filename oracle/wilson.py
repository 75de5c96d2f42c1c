"""Oracle: matrix-free Wilson-Dirac operator (test infrastructure only).

Thin ctypes wrapper over ``oracle/wilson.c`` (plain FP64 C, OpenMP over
sites).  The operator and its conventions are documented in ``lattice.py`` and
in the C source.  Pinned in tests/test_oracle_lattice.py against the dense
matrix, the free-field symbol and trace, kappa = 0, gamma5-hermiticity and
gauge covariance.
"""
import ctypes

import numpy as np

from . import _clib
from .lattice import GAMMA5, spin_op


class WilsonOp:
    """y = M x (or M^H x) on canonical complex128 vectors of shape (n,) or (N, n)."""

    def __init__(self, dims, kappa, links, t_antiperiodic=True):
        self.dims = tuple(int(d) for d in dims)
        self.kappa = float(kappa)
        self.t_antiperiodic = bool(t_antiperiodic)
        self.V = self.dims[0] * self.dims[1] * self.dims[2] * self.dims[3]
        self.n = 12 * self.V
        self.links = np.ascontiguousarray(links, dtype=np.complex128)
        assert self.links.shape == (self.V, 4, 3, 3)
        self._dims_c = (ctypes.c_int * 4)(*self.dims)
        self.matvecs = 0

    def _apply(self, x, dagger):
        x = np.asarray(x, dtype=np.complex128)
        single = x.ndim == 1
        X = np.ascontiguousarray(x.reshape(-1, self.n))
        Y = np.empty_like(X)
        _clib.lib().oracle_wilson_apply(self._dims_c, self.kappa, int(self.t_antiperiodic),
                                        self.links.ctypes.data, X.ctypes.data, Y.ctypes.data,
                                        X.shape[0], int(dagger))
        self.matvecs += X.shape[0]
        return Y.reshape(-1) if single else Y

    @staticmethod
    def set_threads(n):
        """OpenMP threads of the C operator (all calls in this process)."""
        _clib.lib().oracle_set_threads(int(n))

    @staticmethod
    def max_threads():
        return int(_clib.lib().oracle_max_threads())

    def __call__(self, x):
        return self._apply(x, False)

    def dagger(self, x):
        return self._apply(x, True)


def gamma5(x):
    """Apply gamma5 = diag(1, 1, -1, -1) in spin to canonical vectors."""
    return spin_op(np.asarray(x), GAMMA5)

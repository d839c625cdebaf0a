"""Extended-precision backend for the CPU reference (TEST INFRASTRUCTURE ONLY).

Runs the same reference code (oracle/ww_oracle.py) on numpy object arrays of
mpmath numbers at `dps` decimal digits (default 34, about quadruple precision,
the precision the paper uses for its validation runs, Sec. 3.3 and Sec. 4.4).  Its
only purpose is to measure the rounding floor of the FP64 reference on small
problems (N <= 64): the discretisation is identical, only the arithmetic differs.

Differences from the FP64 backend, all in library-primitive steps:
  * Fourier multipliers are applied as dense real circulant matrices built from
    the same symbols (exact DFT definition, no FFT);
  * the dense solve is Gaussian elimination with partial pivoting written out on
    object arrays.
"""
from __future__ import annotations

import mpmath
import numpy as np

from . import ww_oracle as O


class MPArith:
    name = "mp"

    def __init__(self, dps: int = 34):
        self.ctx = mpmath.MPContext()
        self.ctx.dps = dps
        c = self.ctx
        self._sin = np.frompyfunc(c.sin, 1, 1)
        self._cos = np.frompyfunc(c.cos, 1, 1)
        self._exp = np.frompyfunc(c.exp, 1, 1)
        self._sqrt = np.frompyfunc(c.sqrt, 1, 1)
        self._mpf = np.frompyfunc(c.mpf, 1, 1)
        self._ops = {}

    def const(self, x):
        return self.ctx.mpf(x)

    def asarray(self, x):
        if isinstance(x, np.ndarray) and x.dtype == object:
            return x.copy()
        return self._mpf(np.asarray(x, dtype=float)).astype(object)

    def zeros(self, shape):
        z = np.empty(shape, dtype=object)
        z.fill(self.ctx.mpf(0))
        return z

    def grid(self, N):
        g = np.empty(N, dtype=object)
        for j in range(N):
            g[j] = 2 * self.ctx.pi * j / N
        return g

    def sin(self, x):
        return self._sin(x)

    def cos(self, x):
        return self._cos(x)

    def exp(self, x):
        return self._exp(x)

    def sqrt(self, x):
        return self._sqrt(x)

    def cosh_sinh(self, y):
        ey = self._exp(y)
        eyi = self._exp(-y)
        return (ey + eyi) / 2, (ey - eyi) / 2

    @property
    def pi(self):
        return self.ctx.pi

    def _operator(self, kind: str, N: int):
        """Real circulant matrix of the Fourier multiplier `kind` (same symbols as the
        FP64 backend, O.multiplier), built from the DFT definition."""
        key = (kind, N)
        if key in self._ops:
            return self._ops[key]
        c = self.ctx
        ks = np.arange(N // 2 + 1, dtype=float)
        m = O.multiplier(kind, N, ks)   # symbols are exact small integers or exp(-36 ...)
        # recompute the filter symbol in extended precision
        col = []
        for d in range(N):
            th = 2 * c.pi * d / N
            s = c.mpf(0)
            for k in range(N // 2 + 1):
                if kind == "f":
                    mk = c.exp(-36 * (c.mpf(k) / (N // 2)) ** 36)
                    mk = c.mpc(mk, 0)
                else:
                    mk = c.mpc(float(m[k].real), float(m[k].imag))
                term = mk * c.expj(k * th)
                # real-FFT half spectrum: interior modes appear twice (k and -k)
                if 0 < k < N // 2:
                    s += 2 * term.real
                else:
                    s += term.real
            col.append(s / N)
        Mop = np.empty((N, N), dtype=object)
        for i in range(N):
            for j in range(N):
                Mop[i, j] = col[(i - j) % N]
        self._ops[key] = Mop
        return Mop

    def spectral(self, kind, f):
        return self._operator(kind, f.shape[0]).dot(f)

    def lu_factor(self, A):
        A = A.copy()
        n = A.shape[0]
        piv = np.arange(n)
        for k in range(n):
            p = k + int(np.argmax([abs(A[i, k]) for i in range(k, n)]))
            if p != k:
                A[[k, p], :] = A[[p, k], :]
                piv[[k, p]] = piv[[p, k]]
            A[k + 1:, k] = A[k + 1:, k] / A[k, k]
            A[k + 1:, k + 1:] = A[k + 1:, k + 1:] - np.outer(A[k + 1:, k], A[k, k + 1:])
        return A, piv

    def lu_solve(self, lu, B):
        LU, piv = lu
        n = LU.shape[0]
        X = B[piv].copy()
        for i in range(n):                       # L y = P b (unit lower)
            X[i] = X[i] - LU[i, :i].dot(X[:i]) if i else X[i]
        for i in range(n - 1, -1, -1):           # U x = y
            X[i] = (X[i] - LU[i, i + 1:].dot(X[i + 1:])) / LU[i, i]
        return X

    def matmul(self, A, B):
        return A.dot(B)

    def sum(self, x):
        s = self.ctx.mpf(0)
        for v in np.ravel(x):
            s += v
        return s

    def where(self, c, a, b):
        return np.where(np.asarray(c, dtype=bool), a, b)

    def ge0(self, x):
        return np.frompyfunc(lambda t: t >= 0, 1, 1)(x).astype(bool)


def to_float(x):
    return np.asarray(np.vectorize(float, otypes=[float])(x))

"""Independent references used to pin the oracle (test infrastructure).

* LAPACK xGGHRD (Moler-Stewart Hessenberg-triangular reduction with Givens
  rotations), called by its exported name from the LAPACK build that ships with
  scipy.  It fixes Q e1 = e1 exactly like stage two, so by the implicit-Q theorem
  both reductions agree after a diagonal unimodular normalisation.
* Exact rational evaluation of det(A - lambda B) for tiny pencils.
"""
from __future__ import annotations

import ctypes
import glob
import os
from fractions import Fraction

import numpy as np
import scipy

_blas = None


def _openblas():
    global _blas
    if _blas is None:
        d = os.path.join(os.path.dirname(scipy.__file__), "..", "scipy.libs")
        cands = sorted(glob.glob(os.path.join(d, "libscipy_openblas*.so")))
        if not cands:
            return None
        _blas = ctypes.CDLL(cands[0])
    return _blas


def gghrd(A, B):
    """Moler-Stewart reduction of (A, B), B upper triangular, with COMPQ=COMPZ='I'.

    Returns (H, T, Q, Z) or None when the routine is not available.
    """
    L = _openblas()
    if L is None:
        return None
    cplx = np.iscomplexobj(A) or np.iscomplexobj(B)
    name = "scipy_zgghrd_" if cplx else "scipy_dgghrd_"
    if not hasattr(L, name):
        return None
    f = getattr(L, name)
    dt = np.complex128 if cplx else np.float64
    n = A.shape[0]
    a = np.array(A, dtype=dt, order="F", copy=True)
    b = np.array(B, dtype=dt, order="F", copy=True)
    q = np.zeros((n, n), dtype=dt, order="F")
    z = np.zeros((n, n), dtype=dt, order="F")
    I = ctypes.c_int
    cq, cz = ctypes.c_char(b"I"), ctypes.c_char(b"I")
    nn, ilo, ihi, ld, info = I(n), I(1), I(n), I(max(1, n)), I(0)
    P = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    f(ctypes.byref(cq), ctypes.byref(cz), ctypes.byref(nn), ctypes.byref(ilo), ctypes.byref(ihi),
      P(a), ctypes.byref(ld), P(b), ctypes.byref(ld), P(q), ctypes.byref(ld), P(z), ctypes.byref(ld),
      ctypes.byref(info), ctypes.c_size_t(1), ctypes.c_size_t(1))
    if info.value != 0:
        raise RuntimeError(f"xGGHRD info={info.value}")
    return a, b, q, z


def _sgn(x):
    a = abs(x)
    return x / a if a != 0 else 1.0


def canonical(H, T, Q, Z):
    """Normalise an HT decomposition with Q e1 fixed: positive diag(T) and subdiag(H)."""
    n = H.shape[0]
    d1 = np.ones(n, dtype=np.complex128)
    d2 = np.ones(n, dtype=np.complex128)
    d1[0] = np.conj(_sgn(Q[0, 0]))
    for i in range(n):
        d2[i] = d1[i] * np.conj(_sgn(T[i, i]))
        if i + 1 < n:
            d1[i + 1] = _sgn(H[i + 1, i]) * d2[i]
    Hc = np.conj(d1)[:, None] * H * d2[None, :]
    Tc = np.conj(d1)[:, None] * T * d2[None, :]
    Qc = Q * d1[None, :]
    Zc = Z * d2[None, :]
    return Hc, Tc, Qc, Zc


def exact_det(M):
    """Determinant of a square matrix of Fractions by exact Gaussian elimination."""
    M = [row[:] for row in M]
    n = len(M)
    det = Fraction(1)
    for c in range(n):
        p = next((i for i in range(c, n) if M[i][c] != 0), None)
        if p is None:
            return Fraction(0)
        if p != c:
            M[c], M[p] = M[p], M[c]
            det = -det
        det *= M[c][c]
        for i in range(c + 1, n):
            f = M[i][c] / M[c][c]
            if f != 0:
                for j in range(c, n):
                    M[i][j] -= f * M[c][j]
    return det


def charpoly_exact(A, B):
    """Exact coefficients (lowest degree first) of p(lam) = det(A - lam B), real float64 input."""
    n = A.shape[0]
    Af = [[Fraction(float(A[i, j])) for j in range(n)] for i in range(n)]
    Bf = [[Fraction(float(B[i, j])) for j in range(n)] for i in range(n)]
    xs = list(range(n + 1))
    ys = [exact_det([[Af[i][j] - x * Bf[i][j] for j in range(n)] for i in range(n)]) for x in xs]
    # Newton divided differences -> monomial coefficients (exact)
    coef = ys[:]
    for lvl in range(1, n + 1):
        for i in range(n, lvl - 1, -1):
            coef[i] = (coef[i] - coef[i - 1]) / (xs[i] - xs[i - lvl])
    poly = [Fraction(0)] * (n + 1)
    basis = [Fraction(1)]
    for i in range(n + 1):
        for d, b in enumerate(basis):
            poly[d] += coef[i] * b
        nb = [Fraction(0)] * (len(basis) + 1)
        for d, b in enumerate(basis):
            nb[d + 1] += b
            nb[d] -= xs[i] * b
        basis = nb
    return poly

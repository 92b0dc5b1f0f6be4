"""Seeded synthetic input generators shared by the tests and the benchmark.

This module draws random numbers and masks them to the required sparsity
pattern; it holds none of the reduction's arithmetic.  The workloads stand in
for the paper's random pencils (Section 4: random pencils with B replaced by
the triangular factor of its QR factorisation, and saddle-point pencils) with
the shapes and distributions of the benchmark configurations:

* r-HT pencil: H_ic ~ N(0,1) for i <= c + r, 0 below; T_ic ~ N(0,1) for i < c,
  T_cc = 1 + |N(0,1)|, 0 below.  Draw order: H array, T array, T diagonal, each
  a full ``standard_normal`` from ``numpy.random.default_rng(seed)`` (PCG64),
  then masked.
* complex r-HT pencil: real and imaginary parts N(0,1)/sqrt(2), drawn as a
  real-part array then an imaginary-part array, for H, then T, then the
  diagonal; T_cc = 1 + |z| (real, positive).
* dense pencil: A, B i.i.d. N(0,1) (complex: CN(0,1) as above).
* saddle-point pencil: ([X Y; Y^H 0], [I 0; 0 0]) with X = G G^T / m + I
  (symmetric positive definite) and Y random, the zero block holding a given
  fraction of the dimension (the paper uses 25% infinite eigenvalues).

All arrays are returned column-major (Fortran order).
"""
from __future__ import annotations

import numpy as np


def _mask_rht(H, T, d, r):
    n = H.shape[0]
    i, c = np.indices((n, n))
    H[i > c + r] = 0
    T[i > c] = 0
    T[np.arange(n), np.arange(n)] = d
    return np.asfortranarray(H), np.asfortranarray(T)


def rht_pencil(n: int, r: int, seed: int = 0, rng=None):
    """Real r-Hessenberg-triangular pencil (H, T) of order n (float64, column-major)."""
    rng = np.random.default_rng(seed) if rng is None else rng
    H = rng.standard_normal((n, n))
    T = rng.standard_normal((n, n))
    d = 1.0 + np.abs(rng.standard_normal(n))
    return _mask_rht(H, T, d, r)


def rht_pencil_complex(n: int, r: int, seed: int = 0, rng=None):
    """Complex r-HT pencil (complex128, column-major); T has a real positive diagonal."""
    rng = np.random.default_rng(seed) if rng is None else rng
    s = 1.0 / np.sqrt(2.0)
    H = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) * s
    T = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) * s
    z = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * s
    d = (1.0 + np.abs(z)).astype(np.complex128)
    return _mask_rht(H, T, d, r)


def dense_pencil(n: int, seed: int = 0, complex_: bool = False, rng=None):
    """Dense pencil (A, B) with i.i.d. N(0,1) (or CN(0,1)) entries, column-major."""
    rng = np.random.default_rng(seed) if rng is None else rng
    if complex_:
        s = 1.0 / np.sqrt(2.0)
        A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) * s
        B = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) * s
    else:
        A = rng.standard_normal((n, n))
        B = rng.standard_normal((n, n))
    return np.asfortranarray(A), np.asfortranarray(B)


def saddle_point_pencil(n: int, frac_inf: float = 0.25, seed: int = 0, rng=None):
    """Saddle-point pencil ([X Y; Y^T 0], [I 0; 0 0]); the zero block has round(frac_inf*n) rows."""
    rng = np.random.default_rng(seed) if rng is None else rng
    m2 = int(round(frac_inf * n))
    m1 = n - m2
    G = rng.standard_normal((m1, m1))
    X = G @ G.T / m1 + np.eye(m1)
    Y = rng.standard_normal((m1, m2))
    A = np.zeros((n, n))
    A[:m1, :m1] = X
    A[:m1, m1:] = Y
    A[m1:, :m1] = Y.T
    B = np.zeros((n, n))
    B[:m1, :m1] = np.eye(m1)
    return np.asfortranarray(A), np.asfortranarray(B)


def batch_configs(count: int = 2048, seed: int = 0, nlo: int = 32, nhi: int = 512, rs=(4, 8, 16)):
    """(n, r) for the batched workload: n uniform on [nlo, nhi], r drawn from ``rs`` until r < n/4."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(nlo, nhi + 1))
        while True:
            r = int(rng.choice(rs))
            if r < n / 4:
                break
        out.append((n, r))
    return out


def batch_pencils(count: int = 2048, seed: int = 0, nlo: int = 32, nhi: int = 512, rs=(4, 8, 16)):
    """The batched workload: list of (H, T, r); pencil b drawn from SeedSequence(seed).spawn(count)[b]."""
    cfg = batch_configs(count, seed, nlo, nhi, rs)
    ss = np.random.SeedSequence(seed).spawn(count)
    out = []
    for b, (n, r) in enumerate(cfg):
        H, T = rht_pencil(n, r, rng=np.random.default_rng(ss[b]))
        out.append((H, T, r))
    return out

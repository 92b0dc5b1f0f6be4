"""Python access to the CPU oracle (``ht_oracle.c``) -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module.  It builds and loads ``libht_oracle.so`` with
gcc (FMA contraction off) and exposes numpy-level wrappers.  Arrays are
column-major (``order='F'``) float64 / complex128.

Every routine follows the paper (Steel & Vandebril, arXiv 2301.07964):
``stage2`` is the unblocked stage-two algorithm (Section 3.1, appendix
algorithm "Reduction to Hessenberg-triangular form without blocking");
``rhess`` is the stage-one reduction (Section 2.2, appendix algorithm "Blocked
reduction to r-Hessenberg-triangular form") preceded by a QR factorisation of B
(Section 4, random-pencil experiments).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ht_oracle.c")
_LIB = os.path.join(_HERE, "libht_oracle.so")
_lib = None

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c99"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction) into oracle/libht_oracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        i64, dp, vp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p
        L.oracle_stage2_d.argtypes = [i64, i64, vp, vp, vp, vp, i64, i64, dp]
        L.oracle_stage2_z.argtypes = [i64, i64, vp, vp, vp, vp, i64, i64, dp]
        L.oracle_stage2_d.restype = L.oracle_stage2_z.restype = ctypes.c_int
        L.oracle_larfg_d.argtypes = [i64, vp, vp, vp]
        L.oracle_larfg_z.argtypes = [i64, vp, vp, vp]
        L.oracle_rq_dir_d.argtypes = [i64, vp, i64, vp]
        L.oracle_rq_dir_z.argtypes = [i64, vp, i64, vp]
        L.oracle_rq_dir_d.restype = L.oracle_rq_dir_z.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        L.oracle_get_threads.restype = ctypes.c_int
        L.oracle_stage2_flops.argtypes = [i64, i64, ctypes.c_int]
        L.oracle_stage2_flops.restype = ctypes.c_double
        if hasattr(L, "oracle_rhess_d"):
            L.oracle_rhess_d.argtypes = [i64, i64, i64, vp, vp, vp, vp, i64, dp]
            L.oracle_rhess_z.argtypes = [i64, i64, i64, vp, vp, vp, vp, i64, dp]
            L.oracle_rhess_d.restype = L.oracle_rhess_z.restype = ctypes.c_int
        _lib = L
    return _lib


def set_threads(t: int) -> int:
    """Threads for the reflector applications (results are bitwise equal for
    any count: only independent rows / columns are split).  Returns the
    previous count."""
    old = lib().oracle_get_threads()
    lib().oracle_set_threads(int(t))
    return old


def host_cores() -> int:
    """CPU cores this process may run on."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _prep(a, dt):
    return np.array(a, dtype=dt, order="F", copy=True)


def larfg(alpha, x):
    """Householder generation (LAPACK xLARFG convention). Returns (beta, v, tau), v[0] = 1."""
    x = np.asarray(x)
    cplx = np.iscomplexobj(x) or np.iscomplexobj(alpha)
    dt = np.complex128 if cplx else np.float64
    a = np.array([alpha], dtype=dt)
    xx = np.array(x, dtype=dt, copy=True)
    t = np.zeros(1, dtype=dt)
    f = lib().oracle_larfg_z if cplx else lib().oracle_larfg_d
    f(len(xx) + 1, _ptr(a), _ptr(xx), _ptr(t))
    return a[0], np.concatenate([np.ones(1, dtype=dt), xx]), t[0]


def rq_direction(B):
    """Normalised direction of the first row (conjugated) of the RQ orthogonal factor of B."""
    B = np.asarray(B)
    cplx = np.iscomplexobj(B)
    dt = np.complex128 if cplx else np.float64
    Bf = _prep(B, dt)
    m = Bf.shape[0]
    y = np.zeros(m, dtype=dt)
    f = lib().oracle_rq_dir_z if cplx else lib().oracle_rq_dir_d
    if f(m, _ptr(Bf), m, _ptr(y)) != 0:
        raise MemoryError("oracle_rq_dir failed")
    return y


def stage2(H, T, r, Q=None, Z=None, accumulate=True, jmax=-1):
    """Unblocked stage two.  Returns (H, T, Q, Z, flops).

    If ``accumulate`` and Q/Z are None, identity matrices are used (the stage-two
    factors).  ``jmax`` limits the number of sweeps (for bounded samples).
    """
    H = np.asarray(H)
    cplx = np.iscomplexobj(H) or np.iscomplexobj(T)
    dt = np.complex128 if cplx else np.float64
    n = H.shape[0]
    Hf, Tf = _prep(H, dt), _prep(T, dt)
    if accumulate:
        Qf = _prep(np.eye(n) if Q is None else Q, dt)
        Zf = _prep(np.eye(n) if Z is None else Z, dt)
    else:
        Qf = Zf = None
    fl = ctypes.c_double(0.0)
    f = lib().oracle_stage2_z if cplx else lib().oracle_stage2_d
    rc = f(n, r, _ptr(Hf), _ptr(Tf), _ptr(Qf), _ptr(Zf), max(1, n), jmax, ctypes.byref(fl))
    if rc != 0:
        raise ValueError(f"oracle_stage2 returned {rc}")
    return Hf, Tf, Qf, Zf, fl.value


def stage2_flops(n, r, is_complex=False):
    """Counted flops of the whole stage two (4 * length * vectors per reflector application)."""
    return lib().oracle_stage2_flops(n, r, 1 if is_complex else 0)


def rhess(A, B, r, p=8, Q=None, Z=None):
    """Stage one: QR of B, then the blocked reduction to r-HT form (panel width r).

    Returns (A, B, Q, Z, flops) with A_in = Q A Z^H, B_in = Q B Z^H.
    """
    A = np.asarray(A)
    cplx = np.iscomplexobj(A) or np.iscomplexobj(B)
    dt = np.complex128 if cplx else np.float64
    n = A.shape[0]
    Af, Bf = _prep(A, dt), _prep(B, dt)
    Qf = _prep(np.eye(n) if Q is None else Q, dt)
    Zf = _prep(np.eye(n) if Z is None else Z, dt)
    fl = ctypes.c_double(0.0)
    f = lib().oracle_rhess_z if cplx else lib().oracle_rhess_d
    rc = f(n, r, p, _ptr(Af), _ptr(Bf), _ptr(Qf), _ptr(Zf), max(1, n), ctypes.byref(fl))
    if rc != 0:
        raise ValueError(f"oracle_rhess returned {rc}")
    return Af, Bf, Qf, Zf, fl.value

"""paper_2301_07964_amd -- Hessenberg-triangular reduction on AMD MI355X.

Thin ctypes binding of ``libht.so`` (C ABI in ``include/ht.h``).  Every step of
the reduction runs in the HIP kernels of the library; this module only checks
tensor layouts and forwards device pointers, sizes and the current torch
stream.  It raises ``ImportError`` when the library has not been built (run
``python -m paper_2301_07964_amd.build`` or ``__graft_entry__.build()``).

Matrices are torch float64 / complex128 tensors on a HIP device in
column-major layout: ``t.stride(0) == 1`` and ``t.stride(1) == ld >= n`` (for
example ``torch.empty(n, n, device='cuda').t()`` or ``x.t().contiguous().t()``).
Method: Steel & Vandebril, "Parallel two-stage reduction to
Hessenberg-triangular form" (arXiv 2301.07964).
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libht.so")

_lib = None
_i64, _vp, _int = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
_P = ctypes.POINTER(_vp)
_PI = ctypes.POINTER(_i64)


def lib(with_torch: bool = True):
    """Load libht.so (once).

    torch is imported first so that libht.so binds to the HIP runtime torch
    already loaded (same soname): device pointers and streams are then shared.
    Raises ImportError when the library has not been built.
    """
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libht.so not built at {LIB_PATH}; run paper_2301_07964_amd/build.py")
    if with_torch:
        import torch  # noqa: F401  (loads torch's HIP runtime first)
    L = ctypes.CDLL(LIB_PATH)
    for f in ("ht_stage2_q", "ht_stage2_z_q"):
        getattr(L, f).argtypes = [_vp, _vp, _vp, _vp, _i64, _i64, _i64, _i64, _vp]
    for f in ("ht_stage2_sweeps", "ht_stage2_z_sweeps"):
        getattr(L, f).argtypes = [_vp, _vp, _vp, _vp, _i64, _i64, _i64, _i64, _i64, _vp]
        getattr(L, f).restype = _int
    L.ht_stage2_noalloc.argtypes = [_vp, _vp, _vp, _vp, _i64, _i64, _i64, _vp, _vp]
    L.ht_stage2_noalloc.restype = _int
    L.ht_stream_status.argtypes = [_vp]
    L.ht_stream_status.restype = _int
    L.ht_set_knob.argtypes = [_int, _i64]
    L.ht_set_knob.restype = _int
    L.ht_get_knob.argtypes = [_int]
    L.ht_get_knob.restype = _i64
    for f in ("ht_stage2", "ht_stage2_z", "ht_rhess", "ht_rhess_z"):
        getattr(L, f).argtypes = [_vp, _vp, _vp, _vp, _i64, _i64, _i64, _vp]
    for f in ("ht_rhess_p", "ht_rhess_z_p"):
        getattr(L, f).argtypes = [_vp, _vp, _vp, _vp, _i64, _i64, _i64, _i64, _vp]
        getattr(L, f).restype = _int
    L.ht_rhess_default_p.argtypes = [_i64, _i64]
    L.ht_rhess_default_p.restype = _i64
    for f in ("ht_stage2_q", "ht_stage2_z_q", "ht_stage2", "ht_stage2_z", "ht_rhess", "ht_rhess_z",
              "ht_stage2_batched", "ht_stage2_batched_z"):
        getattr(L, f).restype = _int
    L.ht_stage2_batched.argtypes = [_i64, _P, _P, _P, _P, _PI, _PI, _PI, _PI, _vp]
    L.ht_stage2_batched_z.argtypes = [_i64, _P, _P, _P, _P, _PI, _PI, _PI, _PI, _vp]
    L.ht_workspace_bytes.argtypes = [_i64, _i64, _i64, _int]
    L.ht_workspace_bytes.restype = _i64
    L.ht_rhess_workspace_bytes.argtypes = [_i64, _i64, _i64, _int]
    L.ht_rhess_workspace_bytes.restype = _i64
    L.ht_reserve_workspace.argtypes = [_i64, _vp]
    L.ht_reserve_workspace.restype = _int
    L.ht_default_q.argtypes = [_i64, _i64]
    L.ht_default_q.restype = _i64
    L.ht_strerror.argtypes = [_int]
    L.ht_strerror.restype = ctypes.c_char_p
    L.ht_version.restype = ctypes.c_char_p
    L.ht_last_error_message.restype = ctypes.c_char_p
    L.ht_release_workspace.restype = None
    L.ht_profile_enable.argtypes = [_int]
    L.ht_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), _PI, _int]
    L.ht_batched_completion_ms.argtypes = [ctypes.POINTER(ctypes.c_double), _i64]
    L.ht_batched_completion_ms.restype = _int
    L.ht_batched_set_tuning.argtypes = [_i64, _PI, _PI, _PI]
    L.ht_batched_set_tuning.restype = _int
    _lib = L
    _apply_batched_table(L)
    return L


def _apply_batched_table(L):
    """Hand the autotuner's batched table (autotune_table.json, key "batched":
    [n_max, r, threads] entries) to the library, if there is one."""
    import json
    path = os.path.join(_HERE, "autotune_table.json")
    if not os.path.exists(path):
        return
    with open(path) as f:
        ent = json.load(f).get("batched", [])
    if ent:
        _set_tuning(L, ent)


def _set_tuning(L, entries):
    k = len(entries)
    nm, rr, th = (_i64 * max(k, 1))(), (_i64 * max(k, 1))(), (_i64 * max(k, 1))()
    for i, (a, b, c) in enumerate(entries):
        nm[i], rr[i], th[i] = int(a), int(b), int(c)
    rc = L.ht_batched_set_tuning(k, ctypes.cast(nm, _PI), ctypes.cast(rr, _PI), ctypes.cast(th, _PI))
    if rc != 0:
        raise ValueError(f"ht_batched_set_tuning: {rc}")


def set_batched_tuning(entries):
    """Set the batched path's table: entries (n_max, r, threads), threads 64
    (one wavefront per pencil) or 256 (a workgroup); r = 0 matches any r; the
    first match decides; [] restores the built-in rule."""
    _set_tuning(lib(), list(entries))


EXPORTS = (
    "ht_stage2", "ht_stage2_z", "ht_stage2_q", "ht_stage2_z_q", "ht_stage2_sweeps", "ht_stage2_z_sweeps",
    "ht_stage2_noalloc", "ht_stream_status", "ht_set_knob", "ht_get_knob", "ht_stage2_batched",
    "ht_stage2_batched_z", "ht_rhess", "ht_rhess_z", "ht_rhess_p", "ht_rhess_z_p", "ht_rhess_default_p",
    "ht_workspace_bytes", "ht_rhess_workspace_bytes", "ht_reserve_workspace",
    "ht_release_workspace", "ht_default_q", "ht_strerror", "ht_version", "ht_last_error_message",
    "ht_profile_enable", "ht_profile_read", "ht_batched_completion_ms", "ht_batched_set_tuning",
)

# knob ids of include/ht.h
KNOB_WAIT_POLLS, KNOB_UPDATE_TILE_ROWS, KNOB_LOOKAHEAD = 1, 2, 3


def set_knob(knob: int, value: int):
    """Set a process-wide knob (KNOB_*); returns the previous value."""
    old = int(lib().ht_get_knob(knob))
    _check(lib().ht_set_knob(knob, int(value)), "ht_set_knob")
    return old


def get_knob(knob: int) -> int:
    return int(lib().ht_get_knob(knob))


def stream_status(stream=None) -> int:
    """Wait for ``stream`` and return (and clear) its device-side failure
    status: 0, or HT_ERR_TIMEOUT (5) when a bounded wait of a kernel gave up."""
    return int(lib().ht_stream_status(_stream_ptr(stream)))


PROFILE_CLASSES = ("band_copy", "generate", "update_right", "update_left", "zeroing", "update_qz", "form_factors")


def profile_enable(on: bool = True):
    """Bracket every following kernel launch with HIP events (diagnostics)."""
    lib().ht_profile_enable(1 if on else 0)


def profile_read():
    """{class: (total_ms, launches)} of the launches recorded since the last read."""
    k = len(PROFILE_CLASSES)
    ms = (ctypes.c_double * k)()
    cnt = (_i64 * k)()
    _check(lib().ht_profile_read(ms, cnt, k), "ht_profile_read")
    return {c: (ms[i], int(cnt[i])) for i, c in enumerate(PROFILE_CLASSES)}


class HTError(RuntimeError):
    def __init__(self, code: int, where: str):
        detail = lib().ht_last_error_message().decode() if code > 0 else ""
        super().__init__(f"{where}: code {code}: {lib().ht_strerror(code).decode()}"
                         + (f" ({detail})" if detail else ""))
        self.code = code


def _check(code: int, where: str):
    if code != 0:
        raise HTError(code, where)


def version() -> str:
    return lib().ht_version().decode()


def workspace_bytes(n: int, r: int, q: int = 0, complex_: bool = False) -> int:
    return int(lib().ht_workspace_bytes(n, r, q, 1 if complex_ else 0))


def rhess_workspace_bytes(n: int, r: int, p: int = 0, complex_: bool = False) -> int:
    return int(lib().ht_rhess_workspace_bytes(n, r, p, 1 if complex_ else 0))


def reserve_workspace(nbytes: int, stream=None):
    """Pre-size the library workspace of ``stream`` (default: torch's current
    stream) so that later calls on it never allocate."""
    _check(lib().ht_reserve_workspace(int(nbytes), _stream_ptr(stream)), "ht_reserve_workspace")


def default_q(n: int, r: int) -> int:
    return int(lib().ht_default_q(n, r))


def release_workspace():
    lib().ht_release_workspace()


def _torch():
    import torch
    return torch


def _layout(t, n, name, cplx):
    torch = _torch()
    if t is None:
        return None, None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    want = torch.complex128 if cplx else torch.float64
    if t.dtype != want:
        raise TypeError(f"{name} must be {want}, got {t.dtype}")
    if t.dim() != 2 or t.shape[0] != n or t.shape[1] != n:
        raise ValueError(f"{name} must be {n}x{n}")
    if n > 1 and t.stride(0) != 1:
        raise ValueError(f"{name} must be column-major (stride(0) == 1)")
    ld = t.stride(1) if n > 1 else max(1, n)
    return t.data_ptr(), ld


def _stream_ptr(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def stage2(H, T, r: int, Q=None, Z=None, q: int = 0, stream=None, jmax: int = -1):
    """Reduce the r-HT pencil (H, T) in place to Hessenberg-triangular form.

    Q, Z (optional) are updated in place: Q <- Q Q2, Z <- Z Z2.  The call is
    asynchronous on ``stream`` (default: torch's current stream).  ``jmax >=
    0`` runs only the first jmax sweeps (``ht_stage2_sweeps``).
    """
    n = H.shape[0]
    cplx = H.is_complex()
    ptrs, lds = [], []
    for t, nm in ((H, "H"), (T, "T"), (Q, "Q"), (Z, "Z")):
        p, ld = _layout(t, n, nm, cplx)
        ptrs.append(p)
        if ld is not None:
            lds.append(ld)
    if len(set(lds)) != 1:
        raise ValueError("H, T, Q, Z must share the leading dimension")
    if jmax >= 0:
        f = lib().ht_stage2_z_sweeps if cplx else lib().ht_stage2_sweeps
        _check(f(*ptrs, n, r, lds[0], q, jmax, _stream_ptr(stream)), "ht_stage2_sweeps")
    else:
        f = lib().ht_stage2_z_q if cplx else lib().ht_stage2_q
        _check(f(*ptrs, n, r, lds[0], q, _stream_ptr(stream)), "ht_stage2")
    return H, T, Q, Z


NOALLOC_SCRATCH_BYTES = 64 << 20     # HT_NOALLOC_SCRATCH_BYTES of include/ht.h


def stage2_noalloc(H, T, r: int, Q=None, Z=None, status=None, stream=None):
    """``ht_stage2_noalloc``: ht_stage2 with its workspace in the library's
    fixed device scratch, for callers that cannot allocate.  ``status`` is
    None or a one-element int32 device tensor (zeroed by the caller) into
    which a device-side wait that gives up ORs 1.  Real pencils only."""
    n = H.shape[0]
    if H.is_complex():
        raise TypeError("ht_stage2_noalloc takes real (float64) pencils")
    ptrs, lds = [], []
    for t, nm in ((H, "H"), (T, "T"), (Q, "Q"), (Z, "Z")):
        p, ld = _layout(t, n, nm, False)
        ptrs.append(p)
        if ld is not None:
            lds.append(ld)
    if len(set(lds)) != 1:
        raise ValueError("H, T, Q, Z must share the leading dimension")
    sp = None
    if status is not None:
        torch = _torch()
        if not status.is_cuda or status.dtype != torch.int32 or status.numel() < 1:
            raise ValueError("status must be an int32 device tensor")
        sp = status.data_ptr()
    _check(lib().ht_stage2_noalloc(*ptrs, n, r, lds[0], sp, _stream_ptr(stream)), "ht_stage2_noalloc")
    return H, T, Q, Z


def rhess(A, B, r: int, Q=None, Z=None, p: int = 0, stream=None):
    """Stage one: reduce the dense pencil (A, B) in place to r-HT form.

    Q, Z (optional) are updated in place: Q <- Q Q1, Z <- Z Z1.  p = 0 takes
    the library's choice of panel blocks (``rhess_default_p``).
    """
    n = A.shape[0]
    cplx = A.is_complex()
    ptrs, lds = [], []
    for t, nm in ((A, "A"), (B, "B"), (Q, "Q"), (Z, "Z")):
        pt, ld = _layout(t, n, nm, cplx)
        ptrs.append(pt)
        if ld is not None:
            lds.append(ld)
    if len(set(lds)) != 1:
        raise ValueError("A, B, Q, Z must share the leading dimension")
    f = lib().ht_rhess_z_p if cplx else lib().ht_rhess_p
    _check(f(*ptrs, n, r, lds[0], p, _stream_ptr(stream)), "ht_rhess")
    return A, B, Q, Z


def rhess_default_p(n: int, r: int) -> int:
    return int(lib().ht_rhess_default_p(n, r))


def stage2_batched(pencils, q=None, stream=None):
    """Batched stage two.  ``pencils`` is a list of (H, T, Q, Z, r) (Q/Z may be None)."""
    cnt = len(pencils)
    if cnt == 0:
        return pencils
    cplx = pencils[0][0].is_complex()
    arr = [(_vp * cnt)() for _ in range(4)]
    ns, rs, lds, qs = (_i64 * cnt)(), (_i64 * cnt)(), (_i64 * cnt)(), (_i64 * cnt)()
    for b, (H, T, Q, Z, r) in enumerate(pencils):
        n = H.shape[0]
        ld = None
        for i, (t, nm) in enumerate(((H, "H"), (T, "T"), (Q, "Q"), (Z, "Z"))):
            p, l = _layout(t, n, nm, cplx)
            arr[i][b] = p
            if l is not None:
                if ld is not None and l != ld:
                    raise ValueError("matrices of one pencil must share ld")
                ld = l
        ns[b], rs[b], lds[b] = n, r, ld
        qs[b] = 0 if q is None else (q[b] if hasattr(q, "__len__") else q)
    f = lib().ht_stage2_batched_z if cplx else lib().ht_stage2_batched
    _check(f(cnt, *[ctypes.cast(a, _P) for a in arr], ctypes.cast(ns, _PI), ctypes.cast(rs, _PI),
             ctypes.cast(lds, _PI), ctypes.cast(qs, _PI), _stream_ptr(stream)), "ht_stage2_batched")
    return pencils


def batched_completion_ms(count: int):
    """Per-pencil completion times (ms from the first pencil start, device
    clock) of the last batched call made with kernel timing enabled."""
    ms = (ctypes.c_double * count)()
    _check(lib().ht_batched_completion_ms(ms, count), "ht_batched_completion_ms")
    return list(ms)


def colmajor(x, device="cuda"):
    """Copy a numpy/torch matrix into a new column-major device tensor."""
    torch = _torch()
    t = torch.as_tensor(x)
    n0, n1 = t.shape
    out = torch.empty_strided((n0, n1), (1, max(1, n0)), dtype=t.dtype, device=device)
    out.copy_(t)
    return out


def to_numpy(t):
    """Device tensor -> numpy array (Fortran order)."""
    import numpy as np
    return np.asfortranarray(t.detach().cpu().numpy())

"""The C-ABI library loads on the CPU host and exports every function that
include/ht.h declares (no compute call: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2301_07964_amd", "libht.so")
HDR = os.path.join(ROOT, "include", "ht.h")


def declared_functions():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ht_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("ht_stage2", "ht_stage2_z", "ht_rhess", "ht_rhess_z", "ht_stage2_batched",
                 "ht_stage2_batched_z", "ht_workspace_bytes", "ht_strerror"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libht.so not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libht.so not built")
def test_host_only_entry_points():
    L = ctypes.CDLL(LIB)
    L.ht_strerror.restype = ctypes.c_char_p
    L.ht_workspace_bytes.restype = ctypes.c_int64
    L.ht_workspace_bytes.argtypes = [ctypes.c_int64] * 3 + [ctypes.c_int]
    L.ht_default_q.restype = ctypes.c_int64
    L.ht_default_q.argtypes = [ctypes.c_int64] * 2
    assert L.ht_strerror(0) == b"success"
    assert L.ht_strerror(-3) == b"invalid argument"
    assert L.ht_workspace_bytes(-1, 4, 0, 0) == -1
    assert L.ht_workspace_bytes(2, 4, 0, 0) == 0
    assert L.ht_workspace_bytes(100, 8, 0, 1) > L.ht_workspace_bytes(100, 8, 0, 0) > 0
    assert L.ht_workspace_bytes(100, 8, 9, 0) == -1          # q > r
    assert 1 <= L.ht_default_q(16384, 32) <= 32
    L.ht_rhess_workspace_bytes.restype = ctypes.c_int64
    L.ht_rhess_workspace_bytes.argtypes = [ctypes.c_int64] * 3 + [ctypes.c_int]
    assert L.ht_rhess_workspace_bytes(-1, 8, 0, 0) == -1
    assert L.ht_rhess_workspace_bytes(100, 33, 0, 0) == -1      # n_b above 32
    assert L.ht_rhess_workspace_bytes(100, 16, 5, 0) == -1      # p * n_b above 64
    assert L.ht_rhess_workspace_bytes(0, 8, 0, 0) == 0
    assert L.ht_rhess_workspace_bytes(100, 8, 0, 1) > L.ht_rhess_workspace_bytes(100, 8, 0, 0) > 0
    # the reflectors of every block of a panel fit: blocks of p*nb rows, step (p-1)*nb
    n, nb, p = 1000, 8, 8
    blocks = n // ((p - 1) * nb) + 2
    assert L.ht_rhess_workspace_bytes(n, nb, p, 0) >= 2 * blocks * (p * nb * nb + nb) * 8
    L.ht_reserve_workspace.restype = ctypes.c_int
    L.ht_reserve_workspace.argtypes = [ctypes.c_int64, ctypes.c_void_p]
    assert L.ht_reserve_workspace(-1, None) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libht.so not built")
def test_argument_errors_need_no_device():
    """Argument validation happens on the host before any HIP call."""
    L = ctypes.CDLL(LIB)
    f = L.ht_stage2
    f.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int64] * 3 + [ctypes.c_void_p]
    assert f(None, None, None, None, -1, 2, 1, None) == -5
    assert f(None, None, None, None, 4, 0, 4, None) == -6
    assert f(None, None, None, None, 4, 2, 3, None) == -7
    assert f(None, None, None, None, 4, 2, 4, None) == -1
    assert f(None, None, None, None, 0, 2, 1, None) == 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="libht.so not built")
def test_batched_argument_errors_need_no_device():
    """ht_stage2_batched validates its host arrays before any HIP call."""
    L = ctypes.CDLL(LIB)
    f = L.ht_stage2_batched
    P = ctypes.POINTER(ctypes.c_void_p)
    I = ctypes.POINTER(ctypes.c_int64)
    f.argtypes = [ctypes.c_int64, P, P, P, P, I, I, I, I, ctypes.c_void_p]
    cnt = 2
    dummy = (ctypes.c_void_p * cnt)(16, 32)      # never dereferenced on the host
    nul = (ctypes.c_void_p * cnt)(None, None)
    arr = lambda *v: (ctypes.c_int64 * cnt)(*v)
    ok = dict(n=arr(8, 9), r=arr(2, 3), ld=arr(8, 9), q=arr(0, 0))
    def call(count=cnt, H=dummy, T=dummy, n=None, r=None, ld=None, q=None):
        return f(count, H, T, nul, nul, n or ok["n"], r or ok["r"], ld or ok["ld"], q or ok["q"], None)
    assert f(-1, None, None, None, None, None, None, None, None, None) == -1
    assert f(0, None, None, None, None, None, None, None, None, None) == 0
    assert f(cnt, None, dummy, nul, nul, ok["n"], ok["r"], ok["ld"], None, None) == -2
    assert f(cnt, dummy, dummy, None, nul, ok["n"], ok["r"], ok["ld"], None, None) == -4
    assert call(n=arr(8, -1)) == -6
    assert call(r=arr(0, 3)) == -7
    assert call(ld=arr(8, 4)) == -8
    assert call(q=arr(0, 5)) == -9                 # q > min(r, n-1)
    assert call(H=nul) == -2                        # NULL H[b] with n[b] > 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="libht.so not built")
def test_knobs_need_no_device():
    """The process-wide knobs are host state: defaults, ranges and the
    unknown-knob error, without a device."""
    L = ctypes.CDLL(LIB)
    L.ht_set_knob.restype = ctypes.c_int
    L.ht_set_knob.argtypes = [ctypes.c_int, ctypes.c_int64]
    L.ht_get_knob.restype = ctypes.c_int64
    L.ht_get_knob.argtypes = [ctypes.c_int]
    WAIT_POLLS, TILE_ROWS, LOOKAHEAD = 1, 2, 3
    assert L.ht_get_knob(WAIT_POLLS) == 1 << 22
    assert L.ht_get_knob(TILE_ROWS) == 0
    assert L.ht_get_knob(LOOKAHEAD) == 1
    assert L.ht_get_knob(0) == -1 and L.ht_get_knob(4) == -1
    assert L.ht_set_knob(4, 0) == -1
    for knob, bad in ((WAIT_POLLS, -1), (TILE_ROWS, 3), (LOOKAHEAD, 3), (LOOKAHEAD, -1)):
        assert L.ht_set_knob(knob, bad) == -2
        assert L.ht_get_knob(knob) in (1 << 22, 0, 1)         # unchanged
    for v in (0, 2, 1):
        assert L.ht_set_knob(LOOKAHEAD, v) == 0 and L.ht_get_knob(LOOKAHEAD) == v

"""ctypes wrapper and build step for the oracle's C sphere encoder (se.c).

TEST INFRASTRUCTURE ONLY (part of the CPU oracle; see se.c)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_build", "libvporacle.so")
_lib = None


def build(force: bool = False) -> str:
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    src = os.path.join(_HERE, "se.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _SO + ".tmp",
                               src, "-lm"])
        os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        lib.oracle_se.restype = ctypes.c_int
        lib.oracle_se.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


BOX = np.array([complex(bx, by) for bx in (-1, 0, 1) for by in (-1, 0, 1)])


def sphere_encode_batch(W, perm, s, tau, radius=None, wsel=None):
    """Exact VP for many vectors.

    W: complex [n][n] or stacked [S][n][n] (then wsel [V] selects one per vector);
    perm: [n] or [S][n] level -> user; s: complex [n][V] user order.
    Returns (l user order [V][n], cost [V], nodes [V])."""
    lib = _load()
    W = np.ascontiguousarray(W, dtype=np.complex128)
    perm = np.asarray(perm, dtype=np.int64)
    s = np.asarray(s, dtype=np.complex128)
    n, V = s.shape
    if W.ndim == 2:
        W = W[None]
        perm = perm[None]
        wsel = np.zeros(V, dtype=np.int32)
    wsel = np.ascontiguousarray(wsel, dtype=np.int32)
    s_pi = np.take_along_axis(s.T, perm[wsel], axis=1)               # [V][n] level order
    st = np.ascontiguousarray(np.einsum("vij,vj->vi", W[wsel], s_pi))
    rad = None if radius is None else np.ascontiguousarray(radius, dtype=np.float64)
    jcode = np.zeros((V, n), dtype=np.int32)
    cost = np.zeros(V)
    nodes = np.zeros(V, dtype=np.int64)
    rc = lib.oracle_se(n, V, W.ctypes.data, wsel.ctypes.data, st.ctypes.data, float(tau),
                       None if rad is None else rad.ctypes.data,
                       jcode.ctypes.data, cost.ctypes.data, nodes.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_se failed")
    l = np.zeros((V, n), dtype=np.complex128)
    ok = jcode[:, 0] >= 0
    lv = np.where(jcode >= 0, BOX[np.maximum(jcode, 0)], 0)
    np.put_along_axis(l, perm[wsel], lv, axis=1)
    l[~ok] = 0
    return l, cost, nodes

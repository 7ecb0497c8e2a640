"""Python front end of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's cpu_baseline leg may import
this module.  It loads liboracle_vp.so, built from direct.c with gcc and
OpenMP, and wraps its functions for numpy arrays.  The definitions it
computes are stated in direct.c (Section 2.1 Green's function; Section 3.2
eq. Tk_smooth_quad smooth rule; Section 4 sparse correction matrix).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct.c")
_LIB = os.path.join(_HERE, "liboracle_vp.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> str:
    """Compile direct.c into liboracle_vp.so (gcc -O2 -fopenmp)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_smooth.argtypes = [ctypes.c_int64, _dp, _dp, _dp, _dp, _dp, _i64p, ctypes.c_int64,
                                      ctypes.c_int, _dp, _dp]
        lib.oracle_csr.argtypes = [ctypes.c_int64, _i64p, _i32p, _dp, _i64p, ctypes.c_int64,
                                   ctypes.c_int, _dp, _dp]
        lib.oracle_smooth_adjoint.argtypes = [ctypes.c_int64, _dp, _dp, _dp, ctypes.c_int64, _dp, _dp,
                                              _i64p, ctypes.c_int64, ctypes.c_int, _dp, _dp]
        lib.oracle_csr_adjoint.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _dp, _i64p,
                                           ctypes.c_int64, ctypes.c_int, _dp, _dp]
        lib.oracle_smooth_grad.argtypes = [ctypes.c_int64, _dp, _dp, _dp, _dp, _dp, _i64p,
                                           ctypes.c_int64, ctypes.c_int, _dp, _dp]
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _idx(a):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(_i64p)


def _batch(f, n):
    f = np.asarray(f, dtype=np.float64)
    if f.ndim == 1:
        f = f[None, :]
    assert f.shape[1] == n
    return np.ascontiguousarray(f)


def smooth(x, y, w, f, tx=None, ty=None, tidx=None):
    """s_b(t_i) = sum_j G(r_j, t_i) w_j f_b(r_j) with G = -(1/2pi) log|r - r0|.

    Targets default to the nodes themselves (the zero-distance self pair
    then contributes nothing).  Returns [nbatch, len(tidx) or m].
    """
    lib = _load()
    x, xp = _d(x)
    y, yp = _d(y)
    w, wp = _d(w)
    n = x.shape[0]
    if tx is None:
        tx, ty = x, y
    tx, txp = _d(tx)
    ty, typ = _d(ty)
    tidx, tip = _idx(tidx)
    mt = tx.shape[0] if tidx is None else tidx.shape[0]
    f = _batch(f, n)
    out = np.empty((f.shape[0], mt))
    lib.oracle_smooth(n, xp, yp, wp, txp, typ, tip, mt, f.shape[0], f.ctypes.data_as(_dp),
                      out.ctypes.data_as(_dp))
    return out


def csr(rowptr, col, val, f, tidx=None):
    """c_b(t_i) = sum_k C[i,k] f_b(r_k) for the CSR matrix (rowptr, col, val)."""
    lib = _load()
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val, vp = _d(val)
    m = rowptr.shape[0] - 1
    tidx, tip = _idx(tidx)
    mt = m if tidx is None else tidx.shape[0]
    f = np.asarray(f, dtype=np.float64)
    if f.ndim == 1:
        f = f[None, :]
    f = np.ascontiguousarray(f)
    n = f.shape[1]
    out = np.empty((f.shape[0], mt))
    lib.oracle_csr(n, rowptr.ctypes.data_as(_i64p), col.ctypes.data_as(_i32p), vp, tip, mt,
                   f.shape[0], f.ctypes.data_as(_dp), out.ctypes.data_as(_dp))
    return out


def evaluate(x, y, w, f, rowptr=None, col=None, val=None, tx=None, ty=None, tidx=None):
    """Full forward map: smooth part plus correction part."""
    u = smooth(x, y, w, f, tx, ty, tidx)
    if rowptr is not None:
        u = u + csr(rowptr, col, val, f, tidx)
    return u


def smooth_adjoint(x, y, w, g, tx=None, ty=None, sidx=None):
    """d_b(r_j) = w_j sum_i G(r_j, t_i) g_b(t_i)."""
    lib = _load()
    x, xp = _d(x)
    y, yp = _d(y)
    w, wp = _d(w)
    n = x.shape[0]
    if tx is None:
        tx, ty = x, y
    tx, txp = _d(tx)
    ty, typ = _d(ty)
    m = tx.shape[0]
    sidx, sip = _idx(sidx)
    ns = n if sidx is None else sidx.shape[0]
    g = _batch(g, m)
    out = np.empty((g.shape[0], ns))
    lib.oracle_smooth_adjoint(n, xp, yp, wp, m, txp, typ, sip, ns, g.shape[0],
                              g.ctypes.data_as(_dp), out.ctypes.data_as(_dp))
    return out


def csr_adjoint(rowptr, col, val, g, n, sidx=None):
    """sum_i C[i,j] g_b(t_i) for columns j (all n, or the subset sidx)."""
    lib = _load()
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val, vp = _d(val)
    m = rowptr.shape[0] - 1
    g = _batch(g, m)
    sidx, sip = _idx(sidx)
    ns = n if sidx is None else sidx.shape[0]
    out = np.empty((g.shape[0], ns))
    lib.oracle_csr_adjoint(n, m, rowptr.ctypes.data_as(_i64p), col.ctypes.data_as(_i32p), vp, sip,
                           ns, g.shape[0], g.ctypes.data_as(_dp), out.ctypes.data_as(_dp))
    return out


def evaluate_adjoint(x, y, w, g, rowptr=None, col=None, val=None, tx=None, ty=None, sidx=None):
    """Transpose of evaluate: smooth adjoint plus transposed correction."""
    d = smooth_adjoint(x, y, w, g, tx, ty, sidx)
    if rowptr is not None:
        d = d + csr_adjoint(rowptr, col, val, g, x.shape[0], sidx)
    return d


def smooth_grad(x, y, w, f, tx=None, ty=None, tidx=None):
    """Target gradient of the smooth part: [nbatch, 2, len(tidx) or m]."""
    lib = _load()
    x, xp = _d(x)
    y, yp = _d(y)
    w, wp = _d(w)
    n = x.shape[0]
    if tx is None:
        tx, ty = x, y
    tx, txp = _d(tx)
    ty, typ = _d(ty)
    tidx, tip = _idx(tidx)
    mt = tx.shape[0] if tidx is None else tidx.shape[0]
    f = _batch(f, n)
    out = np.empty((f.shape[0], 2, mt))
    lib.oracle_smooth_grad(n, xp, yp, wp, txp, typ, tip, mt, f.shape[0], f.ctypes.data_as(_dp),
                           out.ctypes.data_as(_dp))
    return out

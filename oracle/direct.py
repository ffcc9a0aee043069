"""Direct summation of the PHS kernel sums in plain C (oracle; test
infrastructure only).  Loads oracle/_direct.so, built from oracle/direct.c by
oracle/build.py; when it has not been built, the same sums are taken by the
numpy routines of phs_dense (slower, same definition).

kernel_sums(k, x_nodes, c, t): out[i] = sum_j c_j phi(|t_i - x_j|) with the
basis of eq. phs_fun and phi(0) = 0 -- the kernel part of eq. phs_interp, and
with t = x[rows] the rows of the matvec M c.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path

import numpy as np

from . import phs_dense as D

_SO = Path(__file__).resolve().parent / "_direct.so"
_lib = None


def _load():
    global _lib
    if _lib is None and _SO.exists():
        L = C.CDLL(str(_SO))
        L.oracle_direct_sums.argtypes = [C.c_int, C.c_int64, C.c_void_p, C.c_void_p,
                                         C.c_int64, C.c_void_p, C.c_void_p]
        L.oracle_direct_sums.restype = None
        L.oracle_direct_threads.restype = C.c_int
        _lib = L
    return _lib


def available() -> bool:
    return _load() is not None


def threads() -> int:
    L = _load()
    return L.oracle_direct_threads() if L is not None else 1


def kernel_sums(k: int, x_nodes: np.ndarray, c: np.ndarray, t: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x_nodes, dtype=np.float64)
    cc = np.ascontiguousarray(c, dtype=np.float64)
    tt = np.ascontiguousarray(t, dtype=np.float64)
    L = _load()
    if L is None:
        return D._compensated_row_sums(
            lambda c0, c1: D.kernel_matrix(k, tt, x[c0:c1]) * cc[None, c0:c1],
            len(tt), len(x), 1 << 16)
    out = np.empty(len(tt))
    L.oracle_direct_sums(k, len(x), x.ctypes.data, cc.ctypes.data, len(tt), tt.ctypes.data,
                         out.ctypes.data)
    return out


def matvec_rows(k: int, xi: np.ndarray, v: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """(M v)[rows] by direct summation over all nodes."""
    return kernel_sums(k, xi, v, np.asarray(xi)[np.asarray(rows)])


def eval_points(k: int, xi_nodes: np.ndarray, w: np.ndarray, beta: np.ndarray, degree: int,
                xi_targets: np.ndarray) -> np.ndarray:
    """eq. phs_interp at normalised targets: P(t) beta + sum_j w_j phi(|t - x_j|)."""
    return D.poly_block(np.asarray(xi_targets), degree) @ beta + kernel_sums(
        k, xi_nodes, w, xi_targets)

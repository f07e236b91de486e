"""The N-body sum that the fast multipole method approximates (Methods,
FMM-accelerated evaluation of integral operators: the particle sum over all
quadrature points), written out plainly in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Kernels (Methods, boundary integral formulation: the free-space Green's
functions of the Laplace and linearised Poisson-Boltzmann equations):
  Laplace  g = 1/(4 pi r);  Yukawa  g = exp(-kappa r)/(4 pi r).
Outputs are the potential sum_j g(x_i, y_j) q_j and its gradient with respect
to the target x_i; pairs at zero distance are left out.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_direct.argtypes = [ctypes.c_int64, dp, ctypes.c_int64, dp, dp,
                                      ctypes.c_int, ctypes.c_double, dp, dp]
        lib.oracle_direct.restype = None
        lib.oracle_num_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def direct(targets, sources, q, kernel: str = "laplace", kappa: float = 0.0,
           gradient: bool = True):
    """FP64 direct sum (C, OpenMP).  targets (nt,3), sources (ns,3), q (ns,).
    Returns pot (nt,) and grad (nt,3) (or None)."""
    t = np.ascontiguousarray(targets, dtype=np.float64)
    s = np.ascontiguousarray(sources, dtype=np.float64)
    qq = np.ascontiguousarray(q, dtype=np.float64)
    assert t.ndim == 2 and t.shape[1] == 3 and s.shape[1] == 3 and qq.shape == (len(s),)
    pot = np.zeros(len(t))
    grad = np.zeros((len(t), 3)) if gradient else None
    _lib().oracle_direct(len(t), _ptr(t), len(s), _ptr(s), _ptr(qq),
                         1 if kernel == "yukawa" else 0, float(kappa), _ptr(pot),
                         _ptr(grad) if gradient else None)
    return pot, grad


def num_threads() -> int:
    return int(_lib().oracle_num_threads())


def direct_numpy(targets, sources, q, kernel: str = "laplace", kappa: float = 0.0):
    """Same sum with NumPy broadcasting (tiny inputs only)."""
    d = targets[:, None, :] - sources[None, :, :]
    r = np.sqrt(np.sum(d * d, axis=2))
    with np.errstate(divide="ignore", invalid="ignore"):
        if kernel == "yukawa":
            g = np.exp(-kappa * r) / (4 * math.pi * r)
            dg = -(1 + kappa * r) * np.exp(-kappa * r) / (4 * math.pi * r ** 3)
        else:
            g = 1 / (4 * math.pi * r)
            dg = -1 / (4 * math.pi * r ** 3)
    g[r == 0] = 0.0
    dg[r == 0] = 0.0
    pot = g @ q
    grad = np.einsum("ij,ijd,j->id", dg, d, q)
    return pot, grad


def green(r, kernel: str = "laplace", kappa: float = 0.0):
    """g(r) for scalar or array r > 0."""
    r = np.asarray(r, dtype=np.float64)
    if kernel == "yukawa":
        return np.exp(-kappa * r) / (4 * math.pi * r)
    return 1 / (4 * math.pi * r)


def rel_l2(a, b) -> float:
    """Relative L2 error |a - b| / |b| over all entries."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))

"""ctypes wrapper around the FP64 Ewald code in ewald.c (oracle only).

The shared object is built by oracle/build.sh (gcc -O2 -fopenmp); build() here
compiles it on demand when it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from math import ceil, erfc, log, pi, sqrt  # noqa: F401

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libewald_oracle.so")
_lib = None

# Residual size allowed for both neglected tails (real-space erfc and
# reciprocal-space Gaussian).
TAIL = 1e-16


def build(force: bool = False) -> str:
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(os.path.join(_HERE, "ewald.c")):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _SO,
                               os.path.join(_HERE, "ewald.c"), "-lm"])
    return _SO


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_int64)
        lib.ew_field.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int, ctypes.c_int64, lp, dp, dp, ctypes.c_int]
        lib.ew_field.restype = ctypes.c_int
        lib.ew_pair.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int64,
                                dp, dp, dp, ctypes.c_int]
        lib.ew_pair.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a, t=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(t))


def cutoffs(alpha: float, L: float, tail: float = TAIL):
    """Real-space cutoff rc with erfc(alpha rc) <= tail, and the largest |m| of
    reciprocal vectors k = 2 pi m / L with exp(-k^2 / 4 alpha^2) <= tail."""
    lo, hi = 0.0, 20.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if erfc(mid) > tail:
            lo = mid
        else:
            hi = mid
    rc = hi / alpha
    kmax = 2.0 * alpha * sqrt(log(1.0 / tail))
    mmax = int(ceil(kmax * L / (2 * pi)))
    return rc, mmax


def default_alpha(n: int, L: float) -> float:
    """Splitting parameter balancing real and reciprocal work for n atoms in a cube of edge L."""
    V = L ** 3
    return max(2.0 / L, 2.9 * (n / V ** 2) ** (1.0 / 6.0))


def field(x, q, L: float, targets=None, alpha: float | None = None, nthreads: int = 0):
    """Potential phi_t = sum_j q_j phi_EW(x_t - x_j) (self term = self images) and
    field E_t = sum_j q_j G(x_t - x_j) at the target atoms."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    n = x.shape[0]
    tg = np.arange(n, dtype=np.int64) if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    a = default_alpha(n, L) if alpha is None else alpha
    rc, mmax = cutoffs(a, L)
    phi = np.zeros(tg.shape[0])
    E = np.zeros((tg.shape[0], 3))
    rcode = lib.ew_field(n, _ptr(x), _ptr(q), L, a, rc, mmax, tg.shape[0], _ptr(tg, ctypes.c_int64),
                         _ptr(phi), _ptr(E), nthreads)
    if rcode != 0:
        raise RuntimeError("ew_field failed")
    return phi, E


def pair(r, L: float, alpha: float | None = None, nthreads: int = 0):
    """Pair kernel phi_EW(r) and G(r) = -grad phi_EW(r) for displacements r [n,3].
    A zero displacement gives the self-image value and G = 0."""
    lib = _load()
    r = np.ascontiguousarray(np.atleast_2d(r), dtype=np.float64)
    a = 2.0 / L if alpha is None else alpha
    rc, mmax = cutoffs(a, L)
    phi = np.zeros(r.shape[0])
    G = np.zeros((r.shape[0], 3))
    rcode = lib.ew_pair(L, a, rc, mmax, r.shape[0], _ptr(r), _ptr(phi), _ptr(G), nthreads)
    if rcode != 0:
        raise RuntimeError("ew_pair failed")
    return phi, G

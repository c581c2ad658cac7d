"""Extended-precision local solve (x87 long double) -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` and ``bench.py``'s accuracy report may import this module.
It evaluates the plain definitions of the optimal-test elimination (§2.3)

    K_e = B^H G^{-1} B,   l_e = B^H G^{-1} l,   eta = sqrt(r^H G^{-1} r)

for given FP64 inputs with a 64-bit significand (unit roundoff 2^-64), so its
result is the exact solve of those FP64 inputs to far below FP64 working
accuracy.  Comparing an FP64 solve of the same inputs against it measures
that solve's own forward error; comparing the extended solves of two
independently formed FP64 systems measures how far their formation roundoff
alone moves the exact answer.

The arithmetic is in ``xsolve.c`` (compiled with gcc, no fast-math); the
library is built next to it on first use, or by ``build()``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "xsolve.c")
LIB = os.path.join(HERE, "libxsolve.so")

_lib = None


def build() -> str:
    """Compiles xsolve.c into libxsolve.so (always)."""
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC], check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.xsolve.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp]
        lib.xsolve.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def local_solve_ext(G, B, l, r=None, with_ynorm=False):
    """(K_e, l_e, eta) of the FP64 inputs G (n x n Hermitian positive
    definite; its lower triangle is read), B (n x k), l (n) and residual r
    (n, or None: eta = None), evaluated in extended precision and rounded to
    FP64 once at the end.  with_ynorm: also ||y|| = sqrt(l^H G^{-1} l), the
    scale of l_e (|l_e,a| <= sqrt(K_aa) ||y||)."""
    lib = _load()
    G = np.ascontiguousarray(G, dtype=np.complex128)
    B = np.ascontiguousarray(B, dtype=np.complex128)
    l = np.ascontiguousarray(l, dtype=np.complex128)
    n, k = B.shape
    assert G.shape == (n, n) and l.shape == (n,)
    rr = None if r is None else np.ascontiguousarray(r, dtype=np.complex128)
    K = np.empty((k, k), np.complex128)
    le = np.empty(k, np.complex128)
    e2 = np.zeros(2, np.float64)
    rc = lib.xsolve(n, k, _ptr(G), _ptr(B), _ptr(l), _ptr(rr) if rr is not None else None, _ptr(K), _ptr(le),
                    _ptr(e2))
    if rc != 0:
        raise ValueError(f"xsolve: G not positive definite (pivot {rc})")
    eta = None if r is None else float(np.sqrt(max(e2[0], 0.0)))
    if with_ynorm:
        return K, le, eta, float(np.sqrt(max(e2[1], 0.0)))
    return K, le, eta

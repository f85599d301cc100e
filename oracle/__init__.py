"""Reference oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct CPU implementations of what the tuned path
computes.  Only ``tests/``, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It never imports the product package and
the product never imports it; the two share no code.

* :func:`ref_gemm` / :func:`ref_gemm_at` -- FP64 definition of
  ``C = alpha*A*B + beta*C0`` (C source in ``ref_gemm.c``), plus
  ``T = |A||B|`` for the elementwise error bound.
* :func:`gemm_tolerance` -- the acceptance bound for an FP32 result.
* :mod:`oracle.ptune_ref` -- post-processing, the library cost function,
  brute-force portability tuning and the dispatch rule (Sec. IV, Sec. V).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ref_gemm.c")
_LIB = os.path.join(_HERE, "libref_gemm.so")

# Unit roundoff of IEEE binary32 (round to nearest).
U32 = 2.0 ** -24


def build(force: bool = True) -> str:
    """Compile ``ref_gemm.c`` into ``libref_gemm.so`` with gcc + OpenMP.

    No ``-ffast-math``: the oracle relies on IEEE FP64 semantics.  No
    ``-march=native``: the library may be built on one host and run on another.
    """
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
             "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"],
            check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64, f64 = ctypes.c_int64, ctypes.c_double
        vp = ctypes.c_void_p
        lib.ref_gemm.argtypes = [i64, i64, i64, f64, vp, i64, vp, i64, f64, vp, i64,
                                 vp, vp, vp]
        lib.ref_gemm.restype = ctypes.c_int
        lib.ref_gemm_at.argtypes = [i64, i64, i64, f64, vp, i64, vp, i64, f64, vp, i64,
                                    i64, vp, vp, vp, vp, vp]
        lib.ref_gemm_at.restype = ctypes.c_int
        lib.ref_threads.argtypes = []
        lib.ref_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def threads() -> int:
    """Number of OpenMP threads the oracle uses (OMP_NUM_THREADS or all cores)."""
    return int(_load().ref_threads())


def _mat(x, rows, cols, name):
    """Return (pointer, row stride in elements) of a row-major FP32 matrix view."""
    if x is None:
        return None, max(1, cols)
    x = np.asarray(x)
    if x.dtype != np.float32 or x.ndim != 2 or x.shape != (rows, cols):
        raise ValueError(f"{name}: expected float32 array of shape {(rows, cols)}, "
                         f"got {x.dtype} {x.shape}")
    if x.size == 0:
        return x.ctypes.data, max(1, cols)
    if (cols > 1 and x.strides[1] != 4) or x.strides[0] % 4 != 0:
        raise ValueError(f"{name}: rows must be contiguous FP32")
    ld = max(x.strides[0] // 4, max(1, cols)) if rows > 1 else max(1, cols)
    return x.ctypes.data, ld


def ref_gemm(A, B, alpha=1.0, beta=0.0, C0=None, M=None, N=None, K=None):
    """FP64 reference of ``alpha*A@B + beta*C0``.

    ``A`` is M x K, ``B`` is K x N, ``C0`` is M x N (FP32, row-major; views
    with a row stride larger than the width are allowed).  Returns
    ``(Cref, S, T)`` as dense FP64 arrays: the reference result, the plain
    product ``A@B`` and ``|A|@|B|``.
    """
    if A is not None:
        M, K = A.shape if M is None else (M, K)
    if B is not None:
        K2, N2 = B.shape
        K = K2 if K is None else K
        N = N2 if N is None else N
    if C0 is not None:
        M = C0.shape[0] if M is None else M
        N = C0.shape[1] if N is None else N
    pa, lda = _mat(A, M, K, "A")
    pb, ldb = _mat(B, K, N, "B")
    pc, ldc = _mat(C0, M, N, "C0")
    Cref = np.empty((M, N), np.float64)
    S = np.empty((M, N), np.float64)
    T = np.empty((M, N), np.float64)
    rc = _load().ref_gemm(M, N, K, float(alpha), pa, lda, pb, ldb, float(beta), pc, ldc,
                          Cref.ctypes.data, S.ctypes.data, T.ctypes.data)
    if rc != 0:
        raise ValueError(f"ref_gemm rejected its arguments (rc={rc})")
    return Cref, S, T


def ref_gemm_at(A, B, rows, cols, alpha=1.0, beta=0.0, C0=None):
    """Reference values at the given (row, col) positions only."""
    M, K = A.shape
    N = B.shape[1]
    pa, lda = _mat(A, M, K, "A")
    pb, ldb = _mat(B, K, N, "B")
    pc, ldc = _mat(C0, M, N, "C0")
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    n = rows.size
    Cref = np.empty(n, np.float64)
    S = np.empty(n, np.float64)
    T = np.empty(n, np.float64)
    rc = _load().ref_gemm_at(M, N, K, float(alpha), pa, lda, pb, ldb, float(beta), pc, ldc,
                             n, rows.ctypes.data, cols.ctypes.data,
                             Cref.ctypes.data, S.ctypes.data, T.ctypes.data)
    if rc != 0:
        raise ValueError(f"ref_gemm_at rejected its arguments (rc={rc})")
    return Cref, S, T


def gemm_tolerance(K, alpha, beta, S, T, C0=None):
    """Elementwise acceptance bound for an FP32 GEMM result.

    ``4*K*u*|alpha|*T`` bounds FP32 accumulation of K products (the textbook
    dot-product bound gamma_K ~= K*u with a factor 4 of headroom).  When the
    epilogue rounds (alpha != 1, or beta != 0), ``2*u*(|alpha*S| + |beta*C0|)``
    is added for the scaling and the addition of ``beta*C0``.  With alpha == 1
    and beta == 0 the bound is exactly ``4*K*2^-24*T``.
    """
    tol = 4.0 * K * U32 * abs(alpha) * np.asarray(T, np.float64)
    if alpha != 1.0 or beta != 0.0:
        extra = abs(alpha) * np.abs(S)
        if beta != 0.0:
            extra = extra + abs(beta) * np.abs(np.asarray(C0, np.float64))
        tol = tol + 2.0 * U32 * extra
    return tol

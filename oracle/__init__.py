"""CPU oracle for Low(A*phi(A)) mod p — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It never imports the GPU library and the GPU library
never imports it.

* ``oracle.c``      the definition written out (exact integer triple loops),
                    plus the field helpers of Section 4 (Legendre, Tonelli-Shanks,
                    Algorithm 2) and a Freivalds check.
* ``alg1_model.py`` a plain model of Algorithm 1 (Section 3) with every
                    intermediate kept, used to pin the algebra on small cases.
* ``brute.py``      arbitrary-precision brute force for tiny inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, EPRIME, ERANGE = 0, -1, -2, -3


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (plain -O2, OpenMP, no host-specific ISA).
    ORACLE_LIBRARY names a library built elsewhere (the tests' sanitizer build),
    which is then used as it is."""
    if os.environ.get("ORACLE_LIBRARY"):
        return os.environ["ORACLE_LIBRARY"]
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        i64, P = ctypes.c_int64, ctypes.c_void_p
        L.oracle_is_prime.argtypes = [i64]
        L.oracle_is_prime.restype = ctypes.c_int
        L.oracle_powmod.argtypes = [i64, i64, i64]
        L.oracle_powmod.restype = i64
        L.oracle_legendre.argtypes = [i64, i64]
        L.oracle_legendre.restype = ctypes.c_int
        L.oracle_inverse.argtypes = [i64, i64]
        L.oracle_inverse.restype = i64
        L.oracle_sqrt_mod.argtypes = [i64, i64]
        L.oracle_sqrt_mod.restype = i64
        L.oracle_sos.argtypes = [i64, i64, P, P, P]
        L.oracle_sos.restype = ctypes.c_int
        L.oracle_syrk_modp.argtypes = [i64, i64, i64, P, i64, P, i64, ctypes.c_int]
        L.oracle_syrk_modp.restype = ctypes.c_int
        L.oracle_syrk_entries.argtypes = [i64, i64, i64, P, i64, i64, P, P, P]
        L.oracle_syrk_entries.restype = ctypes.c_int
        L.oracle_herk_modp2.argtypes = [i64, i64, i64, P, P, i64, P, P, i64, ctypes.c_int]
        L.oracle_herk_modp2.restype = ctypes.c_int
        L.oracle_herk_entries.argtypes = [i64, i64, i64, P, P, i64, i64, P, P, P, P]
        L.oracle_herk_entries.restype = ctypes.c_int
        L.oracle_freivalds_syrk.argtypes = [i64, i64, i64, P, i64, P, i64, P, P, P]
        L.oracle_freivalds_syrk.restype = ctypes.c_int
        L.oracle_freivalds_herk.argtypes = [i64, i64, i64, P, P, i64, P, P, i64, P, P, P, P, P, P]
        L.oracle_freivalds_herk.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _chk(st):
    if st != OK:
        raise OracleError(f"oracle status {st}")


def _i64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def is_prime(p):
    return bool(lib().oracle_is_prime(p))


def legendre(a, p):
    return lib().oracle_legendre(a, p)


def sqrt_mod(a, p):
    return lib().oracle_sqrt_mod(a, p)


def inverse(a, p):
    return lib().oracle_inverse(a, p)


def sos(p, k=-1):
    """Algorithm 2: returns (a, b, s) with a^2+b^2 = k mod p; s = non-residue used (0 if none)."""
    a, b, s = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _chk(lib().oracle_sos(p, k, ctypes.byref(a), ctypes.byref(b), ctypes.byref(s)))
    return a.value, b.value, s.value


def syrk_modp(A, p, full=False):
    """Lower triangle (or full matrix) of A*A^T mod p; strict upper is 0 unless full."""
    A = _i64(A)
    n, k = A.shape
    C = np.zeros((n, n), dtype=np.int64)
    _chk(lib().oracle_syrk_modp(n, k, p, _ptr(A), max(k, 1), _ptr(C), max(n, 1), int(full)))
    return C


def syrk_update(A, C, p, alpha=1, beta=0, trans=False):
    """The SYRK update form of Section 7: alpha Low(op(A) op(A)^T) + beta Low(C) mod p,
    op(A) = A or A^T; the strict upper triangle of the result is C's."""
    Aop = np.asarray(A, dtype=np.int64)
    if trans:
        Aop = Aop.T
    X = syrk_modp(Aop, p)
    C = _i64(C)
    low = np.tril(np.ones(C.shape, dtype=bool))
    out = C.copy()
    out[low] = (alpha * X[low] + beta * C[low]) % p
    return out


def syrk_entries(A, p, rows, cols):
    A = _i64(A)
    n, k = A.shape
    rows, cols = _i64(rows), _i64(cols)
    out = np.zeros(len(rows), dtype=np.int64)
    _chk(lib().oracle_syrk_entries(n, k, p, _ptr(A), max(k, 1), len(rows), _ptr(rows),
                                   _ptr(cols), _ptr(out)))
    return out


def herk_modp2(Ar, Ai, p, full=False):
    """(Re, Im) of the lower triangle (or full) of A*A^H over F_p[i]/(i^2+1)."""
    Ar, Ai = _i64(Ar), _i64(Ai)
    n, k = Ar.shape
    Cr = np.zeros((n, n), dtype=np.int64)
    Ci = np.zeros((n, n), dtype=np.int64)
    _chk(lib().oracle_herk_modp2(n, k, p, _ptr(Ar), _ptr(Ai), max(k, 1), _ptr(Cr), _ptr(Ci),
                                 max(n, 1), int(full)))
    return Cr, Ci


def herk_entries(Ar, Ai, p, rows, cols):
    Ar, Ai = _i64(Ar), _i64(Ai)
    n, k = Ar.shape
    rows, cols = _i64(rows), _i64(cols)
    re = np.zeros(len(rows), dtype=np.int64)
    im = np.zeros(len(rows), dtype=np.int64)
    _chk(lib().oracle_herk_entries(n, k, p, _ptr(Ar), _ptr(Ai), max(k, 1), len(rows),
                                   _ptr(rows), _ptr(cols), _ptr(re), _ptr(im)))
    return re, im


def freivalds_syrk(A, C, p, x):
    """(y_c, y_a) = (Sym(C) x, A (A^T x)) mod p; equal for a correct lower triangle C."""
    A, C, x = _i64(A), _i64(C), _i64(x)
    n, k = A.shape
    yc = np.zeros(n, dtype=np.int64)
    ya = np.zeros(n, dtype=np.int64)
    _chk(lib().oracle_freivalds_syrk(n, k, p, _ptr(A), max(k, 1), _ptr(C), max(n, 1), _ptr(x),
                                     _ptr(yc), _ptr(ya)))
    return yc, ya


def freivalds_herk(Ar, Ai, Cr, Ci, p, xr, xi):
    """((Re, Im) of Herm(C) x, (Re, Im) of A (A^H x)) mod p; equal for a correct C."""
    Ar, Ai, Cr, Ci = _i64(Ar), _i64(Ai), _i64(Cr), _i64(Ci)
    xr, xi = _i64(xr), _i64(xi)
    n, k = Ar.shape
    out = [np.zeros(n, dtype=np.int64) for _ in range(4)]
    _chk(lib().oracle_freivalds_herk(n, k, p, _ptr(Ar), _ptr(Ai), max(k, 1), _ptr(Cr), _ptr(Ci),
                                     max(n, 1), _ptr(xr), _ptr(xi), *[_ptr(v) for v in out]))
    return (out[0], out[1]), (out[2], out[3])


def num_threads():
    return lib().oracle_num_threads()

"""Python access to the CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this package.  The product
path (the HIP library and its binding) never loads it.

The oracle is plain C++ (``oracle.cpp``) compiled with gcc and OpenMP; it is built on first use if the shared object
is missing or older than its source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_LL = ctypes.POINTER(ctypes.c_longlong)


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            L.oracle_boys.argtypes = [ctypes.c_int, ctypes.c_double, _D]
            L.oracle_basis_create.restype = ctypes.c_void_p
            L.oracle_basis_create.argtypes = [ctypes.c_int, _I, _I, _D, _D, _D]
            L.oracle_basis_destroy.argtypes = [ctypes.c_void_p]
            L.oracle_nbf.argtypes = [ctypes.c_void_p]
            L.oracle_nbf.restype = ctypes.c_int
            L.oracle_eri_quartet.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, _D]
            L.oracle_eri_tensor.argtypes = [ctypes.c_void_p, _D]
            L.oracle_schwarz.argtypes = [ctypes.c_void_p, _D]
            L.oracle_jk_direct.argtypes = [ctypes.c_void_p, ctypes.c_int, _D, ctypes.c_double, _D, _D]
            L.oracle_jk_symmetric.argtypes = [ctypes.c_void_p, ctypes.c_int, _D, ctypes.c_double, _D, _D, _LL,
                                              ctypes.c_int, _I]
            L.oracle_j_block.argtypes = [ctypes.c_void_p, _D, ctypes.c_double, ctypes.c_int, ctypes.c_int, _D]
            L.oracle_k_block.argtypes = [ctypes.c_void_p, _D, ctypes.c_double, ctypes.c_int, ctypes.c_int, _D]
            L.oracle_num_threads.restype = ctypes.c_int
            L.oracle_set_num_threads.argtypes = [ctypes.c_int]
            _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _ip(a: np.ndarray):
    return a.ctypes.data_as(_I)


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def boys(mmax: int, T: float) -> np.ndarray:
    out = np.zeros(mmax + 1)
    lib().oracle_boys(int(mmax), float(T), _dp(out))
    return out


def set_threads(n: int) -> None:
    lib().oracle_set_num_threads(int(n))


def num_threads() -> int:
    return int(lib().oracle_num_threads())


class Basis:
    """Normalised contracted Cartesian basis held by the oracle."""

    def __init__(self, shells):
        self._keep = [np.ascontiguousarray(shells.l, dtype=np.int32),
                      np.ascontiguousarray(shells.nprim, dtype=np.int32),
                      np.ascontiguousarray(shells.center, dtype=np.float64).reshape(-1),
                      np.ascontiguousarray(shells.alpha, dtype=np.float64),
                      np.ascontiguousarray(shells.coef, dtype=np.float64)]
        l, k, c, a, co = self._keep
        self.l = l.copy()
        self.nshell = int(l.shape[0])
        h = lib().oracle_basis_create(self.nshell, _ip(l), _ip(k), _dp(c), _dp(a), _dp(co))
        if not h:
            raise ValueError("oracle: invalid basis (l must be 0..2, K >= 1)")
        self.h = ctypes.c_void_p(h)
        self.nbf = int(lib().oracle_nbf(self.h))
        n = [ncart(int(x)) for x in l]
        self.offsets = np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int64)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().oracle_basis_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def eri(self, a: int, b: int, c: int, d: int) -> np.ndarray:
        la, lb, lc, ld = (int(self.l[x]) for x in (a, b, c, d))
        out = np.zeros((ncart(la), ncart(lb), ncart(lc), ncart(ld)))
        lib().oracle_eri_quartet(self.h, a, b, c, d, _dp(out))
        return out

    def eri_tensor(self) -> np.ndarray:
        N = self.nbf
        out = np.zeros((N, N, N, N))
        lib().oracle_eri_tensor(self.h, _dp(out))
        return out

    def schwarz(self) -> np.ndarray:
        Q = np.zeros((self.nshell, self.nshell))
        lib().oracle_schwarz(self.h, _dp(Q))
        return Q

    def _stack(self, Ds):
        Ds = [np.ascontiguousarray(D, dtype=np.float64) for D in Ds]
        return np.ascontiguousarray(np.stack(Ds)), len(Ds)

    def jk_direct(self, Ds, tau: float = 0.0):
        D, m = self._stack(Ds)
        J = np.zeros_like(D)
        K = np.zeros_like(D)
        lib().oracle_jk_direct(self.h, m, _dp(D), float(tau), _dp(J), _dp(K))
        return J, K

    def jk_symmetric(self, Ds, tau: float = 0.0, bra_sample=None):
        D, m = self._stack(Ds)
        J = np.zeros_like(D)
        K = np.zeros_like(D)
        counts = np.zeros(2, dtype=np.int64)
        if bra_sample is None:
            lib().oracle_jk_symmetric(self.h, m, _dp(D), float(tau), _dp(J), _dp(K),
                                      counts.ctypes.data_as(_LL), 0, None)
        else:
            s = np.ascontiguousarray(bra_sample, dtype=np.int32)
            lib().oracle_jk_symmetric(self.h, m, _dp(D), float(tau), _dp(J), _dp(K),
                                      counts.ctypes.data_as(_LL), int(s.shape[0]), _ip(s))
        return J, K, counts

    def j_block(self, D, a: int, b: int, tau: float = 0.0) -> np.ndarray:
        D = np.ascontiguousarray(D, dtype=np.float64)
        out = np.zeros((ncart(int(self.l[a])), ncart(int(self.l[b]))))
        lib().oracle_j_block(self.h, _dp(D), float(tau), a, b, _dp(out))
        return out

    def k_block(self, D, a: int, d: int, tau: float = 0.0) -> np.ndarray:
        D = np.ascontiguousarray(D, dtype=np.float64)
        out = np.zeros((ncart(int(self.l[a])), ncart(int(self.l[d]))))
        lib().oracle_k_block(self.h, _dp(D), float(tau), a, d, _dp(out))
        return out


def fock_parts(J: np.ndarray, K: np.ndarray, D: np.ndarray):
    """G = J - K/2 and E2 = 1/2 sum_ij D_ij G_ij."""
    G = J - 0.5 * K
    return G, 0.5 * float(np.sum(D * G))

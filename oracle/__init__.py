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
            L.oracle_one_electron.argtypes = [ctypes.c_void_p, ctypes.c_int, _D, _D, _D, _D, _D]
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


def nuclear_repulsion(Z, R) -> float:
    """E_nuc = sum_{A<B} Z_A Z_B / |R_A - R_B| (bohr, hartree)."""
    Z = np.asarray(Z, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64).reshape(-1, 3)
    e = 0.0
    for a in range(len(Z)):
        for b in range(a):
            e += Z[a] * Z[b] / float(np.linalg.norm(R[a] - R[b]))
    return e


def one_electron(basis: "Basis", Z, R):
    """Overlap S, kinetic T and nuclear attraction V matrices (Eq. (2)-(4)) for point nuclei Z at R."""
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1)
    N = basis.nbf
    S, T, V = (np.zeros((N, N)) for _ in range(3))
    lib().oracle_one_electron(basis.h, int(Z.shape[0]), _dp(Z), _dp(R), _dp(S), _dp(T), _dp(V))
    return S, T, V


def rhf(shells, Z, R, nocc: int, tau: float = 0.0, max_iter: int = 200, e_conv: float = 1e-12,
        d_conv: float = 1e-10):
    """Restricted closed-shell Hartree-Fock by plain Roothaan iteration (Szabo-Ostlund Sec. 3.4.6): symmetric
    orthogonalisation X = S^{-1/2}, core-Hamiltonian guess, P = 2 C_occ C_occ^T, F = H + J(P) - K(P)/2,
    E = 1/2 tr P (H + F) + E_nuc.  No acceleration, no damping."""
    O = Basis(shells)
    S, T, V = one_electron(O, Z, R)
    H = T + V
    s, U = np.linalg.eigh(S)
    X = U @ np.diag(s ** -0.5) @ U.T
    N = O.nbf
    P = np.zeros((N, N))
    e_old = 0.0
    for it in range(1, max_iter + 1):
        J, K, _ = O.jk_symmetric([P], tau=tau)
        F = H + J[0] - 0.5 * K[0]
        e_el = 0.5 * float(np.sum(P * (H + F)))
        eps, Cp = np.linalg.eigh(X.T @ F @ X)
        C = X @ Cp
        Pn = 2.0 * C[:, :nocc] @ C[:, :nocc].T
        dP = float(np.max(np.abs(Pn - P)))
        P = Pn
        if it > 1 and abs(e_el - e_old) < e_conv and dP < d_conv:
            break
        e_old = e_el
    else:
        raise RuntimeError("oracle rhf: no convergence in %d iterations" % max_iter)
    e_nuc = nuclear_repulsion(Z, R)
    return {"E_elec": e_el, "E_nuc": e_nuc, "E_total": e_el + e_nuc, "P": P, "C": C, "eps": eps,
            "iterations": it, "S": S, "T": T, "V": V}


def mix_homo_lumo(C: np.ndarray, n: int, theta: float) -> np.ndarray:
    """Rotates the highest occupied (index n-1) and lowest virtual (index n) columns of C by the angle theta:
    c_h' = cos(theta) c_h + sin(theta) c_l, c_l' = -sin(theta) c_h + cos(theta) c_l (a guess that breaks the
    spatial and spin symmetry of a closed-shell start; no change if theta = 0 or n is 0 or nbf)."""
    C = C.copy()
    if theta != 0.0 and 0 < n < C.shape[1]:
        h, l = C[:, n - 1].copy(), C[:, n].copy()
        C[:, n - 1] = np.cos(theta) * h + np.sin(theta) * l
        C[:, n] = -np.sin(theta) * h + np.cos(theta) * l
    return C


def uhf(shells, Z, R, nalpha: int, nbeta: int, tau: float = 0.0, guess_mix: float = 0.0, max_iter: int = 500,
        e_conv: float = 1e-12, d_conv: float = 1e-10):
    """Unrestricted Hartree-Fock (the paper's URHF; Pople-Nesbet equations, Szabo-Ostlund Sec. 3.8) by plain
    iteration: X = S^{-1/2}, core-Hamiltonian guess for both spins (the alpha guess optionally rotated by
    mix_homo_lumo), P^s = C^s_occ C^s_occ^T, F^s = H + J(P^a + P^b) - K(P^s),
    E = 1/2 tr[(P^a + P^b) H + P^a F^a + P^b F^b] + E_nuc.  No acceleration, no damping."""
    O = Basis(shells)
    S, T, V = one_electron(O, Z, R)
    H = T + V
    s, U = np.linalg.eigh(S)
    X = U @ np.diag(s ** -0.5) @ U.T
    _, Cp = np.linalg.eigh(X.T @ H @ X)
    C0 = X @ Cp
    Ca = mix_homo_lumo(C0, nalpha, guess_mix)
    Cb = C0
    Pa = Ca[:, :nalpha] @ Ca[:, :nalpha].T
    Pb = Cb[:, :nbeta] @ Cb[:, :nbeta].T
    e_old = 0.0
    for it in range(1, max_iter + 1):
        J, K, _ = O.jk_symmetric([Pa, Pb], tau=tau)
        Jt = J[0] + J[1]
        Fa, Fb = H + Jt - K[0], H + Jt - K[1]
        e_el = 0.5 * float(np.sum((Pa + Pb) * H + Pa * Fa + Pb * Fb))
        ea, Ca = np.linalg.eigh(X.T @ Fa @ X)
        eb, Cb = np.linalg.eigh(X.T @ Fb @ X)
        Ca, Cb = X @ Ca, X @ Cb
        Pan = Ca[:, :nalpha] @ Ca[:, :nalpha].T
        Pbn = Cb[:, :nbeta] @ Cb[:, :nbeta].T
        dP = float(max(np.max(np.abs(Pan - Pa)), np.max(np.abs(Pbn - Pb))))
        Pa, Pb = Pan, Pbn
        if it > 1 and abs(e_el - e_old) < e_conv and dP < d_conv:
            break
        e_old = e_el
    else:
        raise RuntimeError("oracle uhf: no convergence in %d iterations" % max_iter)
    e_nuc = nuclear_repulsion(Z, R)
    s2 = spin_contamination(S, Pa, Pb, nalpha, nbeta)
    return {"E_elec": e_el, "E_nuc": e_nuc, "E_total": e_el + e_nuc, "Pa": Pa, "Pb": Pb, "Ca": Ca, "Cb": Cb,
            "eps_a": ea, "eps_b": eb, "iterations": it, "S": S, "H": H, "S2": s2}


def spin_contamination(S, Pa, Pb, nalpha: int, nbeta: int) -> float:
    """<S^2> of a single determinant of nalpha alpha and nbeta beta spin orbitals (Szabo-Ostlund Sec. 3.8):
    S_z (S_z + 1) + nbeta - sum_ij |<i alpha|j beta>|^2, the overlap sum being tr(P^a S P^b S)."""
    sz = 0.5 * (nalpha - nbeta)
    return sz * (sz + 1.0) + nbeta - float(np.sum((Pa @ S) * (Pb @ S).T))


def mo_integrals_ovov(eri: np.ndarray, C: np.ndarray, nocc: int, nfrozen: int = 0) -> np.ndarray:
    """(ia|jb) = sum_{mu nu lam sig} C_mu,i C_nu,a (mu nu|lam sig) C_lam,j C_sig,b for active occupied i, j
    (nfrozen <= i < nocc) and virtual a, b (>= nocc): the four-index transformation written out, one index at a
    time, from the AO tensor eri[mu, nu, lam, sig]."""
    Co = C[:, nfrozen:nocc]
    Cv = C[:, nocc:]
    t = np.einsum("mi,mnls->inls", Co, eri, optimize=False)
    t = np.einsum("na,inls->ials", Cv, t, optimize=False)
    t = np.einsum("lj,ials->iajs", Co, t, optimize=False)
    return np.einsum("sb,iajs->iajb", Cv, t, optimize=False)


def mp2_closed_shell(ovov: np.ndarray, eps: np.ndarray, nocc: int, nfrozen: int = 0):
    """Closed-shell second-order Moller-Plesset energy from canonical orbitals (Szabo-Ostlund Sec. 6.5, the
    spin-adapted form the paper's MP2 follows): E2 = sum_{ijab} (ia|jb) [2 (ia|jb) - (ib|ja)] / D_ijab with
    D_ijab = e_i + e_j - e_a - e_b.  Returns (E2, E_os, E_ss): E_os = sum (ia|jb)^2 / D (opposite spins),
    E_ss = sum (ia|jb) [(ia|jb) - (ib|ja)] / D (same spins), E2 = E_os + E_ss."""
    eo = eps[nfrozen:nocc]
    ev = eps[nocc:]
    D = eo[:, None, None, None] - ev[None, :, None, None] + eo[None, None, :, None] - ev[None, None, None, :]
    V = ovov
    Vx = V.transpose(0, 3, 2, 1)  # (ib|ja) at [i, a, j, b]
    e_os = float(np.sum(V * V / D))
    e_ss = float(np.sum(V * (V - Vx) / D))
    return e_os + e_ss, e_os, e_ss


def fock_parts(J: np.ndarray, K: np.ndarray, D: np.ndarray):
    """G = J - K/2 and E2 = 1/2 sum_ij D_ij G_ij."""
    G = J - 0.5 * K
    return G, 0.5 * float(np.sum(D * G))

"""Python binding of libuqc (ctypes over include/uqc.h): argument marshalling only.

Every step of the integral and Fock-build path runs in the HIP library.  PyTorch supplies device memory and the
stream: device tensors are passed to the library as raw pointers and the context launches on the current torch
stream.  If the shared library cannot be loaded, every call raises; there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import threading
import weakref
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libuqc.so")

UQC_OK, UQC_PENDING = 0, 1
UQC_E_ARG, UQC_E_UNSUPPORTED, UQC_E_NOMEM, UQC_E_DEVICE = -1, -2, -3, -4
UQC_E_NOT_SYMMETRIC, UQC_E_NOT_FOUND, UQC_E_BUSY = -5, -6, -7
FP64, MIXED = 0, 1
RYS = 2  # uqc_eri_block(s) only: the same integrals by Rys quadrature
MAX_CLASS_STATS = 96
MAX_ITER = 64

EXPORTED = ["uqc_fock_opts_default", "uqc_init", "uqc_finalize", "uqc_last_error", "uqc_basis_create",
            "uqc_basis_destroy", "uqc_basis_info", "uqc_schwarz", "uqc_eri_block", "uqc_eri_blocks",
            "uqc_fock_build", "uqc_boys", "uqc_server_create", "uqc_submit", "uqc_poll", "uqc_server_drain",
            "uqc_server_destroy", "uqc_one_electron", "uqc_scf_opts_default", "uqc_scf_rhf", "uqc_fock_build_uhf",
            "uqc_scf_uhf", "uqc_mp2", "uqc_fock_build_noalloc"]


class UqcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("uqc status %d: %s" % (status, msg))
        self.status = status


PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong, ctypes.c_longlong)


class FockOpts(ctypes.Structure):
    _fields_ = [("schwarz_tau", ctypes.c_double), ("precision", ctypes.c_int), ("fp64_bound", ctypes.c_double),
                ("timing", ctypes.c_int), ("progress", PROGRESS_FN), ("progress_user", ctypes.c_void_p),
                ("max_items_per_launch", ctypes.c_longlong), ("exchange_scale", ctypes.c_double),
                ("streams", ctypes.c_int), ("fp64_boys_T", ctypes.c_double)]


class ScfOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("e_conv", ctypes.c_double), ("d_conv", ctypes.c_double),
                ("diis_size", ctypes.c_int), ("fock", FockOpts), ("guess_mix", ctypes.c_double)]


class ScfResult(ctypes.Structure):
    _fields_ = [("E_total", ctypes.c_double), ("E_elec", ctypes.c_double), ("E_nuc", ctypes.c_double),
                ("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("error", ctypes.c_double),
                ("ms", ctypes.c_double), ("fock_ms", ctypes.c_double), ("quartets", ctypes.c_longlong),
                ("s2", ctypes.c_double)]


class Mp2Result(ctypes.Structure):
    _fields_ = [("e2", ctypes.c_double), ("e_os", ctypes.c_double), ("e_ss", ctypes.c_double),
                ("quartets", ctypes.c_longlong), ("ao_ms", ctypes.c_double), ("transform_ms", ctypes.c_double),
                ("energy_ms", ctypes.c_double), ("ms", ctypes.c_double), ("transform_flops", ctypes.c_double),
                ("batches", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("E2", ctypes.c_double), ("quartets", ctypes.c_longlong), ("quartets_screened", ctypes.c_longlong),
                ("prim_quartets", ctypes.c_longlong), ("fp64_quartets", ctypes.c_longlong),
                ("flops", ctypes.c_double), ("ms", ctypes.c_double), ("eri_ms", ctypes.c_double),
                ("nclass", ctypes.c_int), ("class_id", ctypes.c_int * MAX_CLASS_STATS),
                ("class_ms", ctypes.c_double * MAX_CLASS_STATS), ("class_flops", ctypes.c_double * MAX_CLASS_STATS),
                ("class_quartets", ctypes.c_longlong * MAX_CLASS_STATS)]

    def as_dict(self):
        d = {k: getattr(self, k) for k in ("E2", "quartets", "quartets_screened", "prim_quartets", "fp64_quartets",
                                           "flops", "ms", "eri_ms")}
        d["classes"] = [{"id": int(self.class_id[i]), "ms": float(self.class_ms[i]),
                         "flops": float(self.class_flops[i]), "quartets": int(self.class_quartets[i])}
                        for i in range(self.nclass)]
        return d


_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


class Request(ctypes.Structure):
    _fields_ = [("nshell", ctypes.c_int), ("l", _I), ("nprim", _I), ("center", _D), ("alpha", _D), ("coef", _D),
                ("D0", _D), ("n_iter", ctypes.c_int), ("ncol", ctypes.c_int), ("eps", ctypes.c_double),
                ("seed", ctypes.c_ulonglong), ("opts", FockOpts), ("arrival_ms", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("n_iter", ctypes.c_int), ("nbf", ctypes.c_int), ("E2", ctypes.c_double * MAX_ITER),
                ("submit_ms", ctypes.c_double), ("admit_ms", ctypes.c_double), ("finish_ms", ctypes.c_double),
                ("quartets", ctypes.c_longlong), ("J", _D), ("K", _D), ("G", _D), ("D", _D),
                ("device_bytes", ctypes.c_longlong), ("steps", ctypes.c_int)]


_lock = threading.Lock()
_lib = None

# Live handles, closed children-first when their context closes and at interpreter exit (before the HIP runtime's
# own teardown), so no library call ever runs on a freed context.
_live = {"server": weakref.WeakSet(), "basis": weakref.WeakSet(), "ctx": weakref.WeakSet()}


@atexit.register
def _close_all():
    for kind in ("server", "basis", "ctx"):
        for obj in list(_live[kind]):
            try:
                obj.close()
            except Exception:
                pass


def _close_children(ctx):
    for kind in ("server", "basis"):
        for obj in list(_live[kind]):
            if getattr(obj, "ctx", None) is ctx:
                obj.close()


def load(build_if_missing: bool = True):
    """Loads libuqc.so (building it first if it does not exist)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            if not build_if_missing:
                raise OSError("libuqc.so is not built (python -m paper_1303_4916_amd.build)")
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.uqc_fock_opts_default.argtypes = [ctypes.POINTER(FockOpts)]
        L.uqc_fock_opts_default.restype = None
        L.uqc_init.argtypes = [ctypes.c_int, vp, ctypes.POINTER(vp)]
        L.uqc_finalize.argtypes = [vp]
        L.uqc_last_error.restype = ctypes.c_char_p
        L.uqc_basis_create.argtypes = [vp, ctypes.c_int, _I, _I, _D, _D, _D, ctypes.POINTER(vp)]
        L.uqc_basis_destroy.argtypes = [vp]
        L.uqc_basis_info.argtypes = [vp, _I, _I]
        L.uqc_schwarz.argtypes = [vp, _D]
        L.uqc_eri_block.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _D]
        L.uqc_eri_blocks.argtypes = [vp, ctypes.c_int, _I, ctypes.c_int, _D]
        L.uqc_fock_build.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(FockOpts), ctypes.POINTER(Stats)]
        L.uqc_fock_build_noalloc.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(FockOpts), ctypes.POINTER(Stats)]
        L.uqc_boys.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _D, _D]
        L.uqc_server_create.argtypes = [vp, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(vp)]
        L.uqc_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_longlong)]
        L.uqc_poll.argtypes = [vp, ctypes.c_longlong, ctypes.POINTER(Result)]
        L.uqc_server_drain.argtypes = [vp]
        L.uqc_server_destroy.argtypes = [vp]
        L.uqc_one_electron.argtypes = [vp, ctypes.c_int, _D, _D, vp, vp, vp]
        L.uqc_scf_opts_default.argtypes = [ctypes.POINTER(ScfOpts)]
        L.uqc_scf_opts_default.restype = None
        L.uqc_scf_rhf.argtypes = [vp, ctypes.c_int, _D, _D, ctypes.c_int, ctypes.POINTER(ScfOpts), _D, _D,
                                  ctypes.POINTER(ScfResult)]
        L.uqc_fock_build_uhf.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(FockOpts),
                                         ctypes.POINTER(Stats)]
        L.uqc_scf_uhf.argtypes = [vp, ctypes.c_int, _D, _D, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ScfOpts), _D,
                                  _D, _D, _D, ctypes.POINTER(ScfResult)]
        L.uqc_mp2.argtypes = [vp, _D, _D, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_size_t,
                              ctypes.POINTER(Mp2Result)]
        for name in EXPORTED:
            if name not in ("uqc_fock_opts_default", "uqc_last_error", "uqc_scf_opts_default"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
        return L


def _check(st: int):
    if st != UQC_OK:
        msg = load().uqc_last_error()
        raise UqcError(st, msg.decode() if msg else "")


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _ip(a: np.ndarray):
    return a.ctypes.data_as(_I)


def scf_opts(max_iter: int = 100, e_conv: float = 1e-10, d_conv: float = 1e-8, diis_size: int = 8,
             fock: FockOpts = None, guess_mix: float = 0.0) -> ScfOpts:
    """Options of uqc_scf_rhf / uqc_scf_uhf (library defaults unless given)."""
    o = ScfOpts()
    load().uqc_scf_opts_default(ctypes.byref(o))
    o.max_iter = int(max_iter)
    o.e_conv = float(e_conv)
    o.d_conv = float(d_conv)
    o.diis_size = int(diis_size)
    o.guess_mix = float(guess_mix)
    if fock is not None:
        o.fock = fock
    return o


def default_opts(tau: float = 1e-12, precision: int = FP64, fp64_bound: float = 1e-8, timing: bool = False,
                 progress=None, max_items_per_launch: int = 0, exchange_scale: float = 1.0,
                 streams: int | None = None, fp64_boys_T: float | None = None):
    """Fock-build options.  progress: None or a callable(class_id, items_done, items_total) called after every
    class sub-launch has completed on the device (on one stream the build then waits for each one).
    max_items_per_launch: cap on the work items of one class-kernel launch (0: the library default).
    exchange_scale: weight x of exchange (G = J - (x/2) K; spin densities G^s = J - x K^s).  streams: HIP streams
    the class launches are spread over (None: the library default).  fp64_boys_T: mixed precision, Boys arguments
    above it evaluated in FP64 (None: the library default, 30)."""
    o = FockOpts()
    load().uqc_fock_opts_default(ctypes.byref(o))
    o.schwarz_tau = float(tau)
    o.precision = int(precision)
    o.fp64_bound = float(fp64_bound)
    o.timing = 1 if timing else 0
    o.max_items_per_launch = int(max_items_per_launch)
    o.exchange_scale = float(exchange_scale)
    if streams is not None:
        o.streams = int(streams)
    if fp64_boys_T is not None:
        o.fp64_boys_T = float(fp64_boys_T)
    if progress is not None:
        fn = PROGRESS_FN(lambda user, cid, done, total: progress(int(cid), int(done), int(total)))
        o.progress = fn
        o._progress_ref = fn  # keeps the C callback alive as long as the options object
    return o


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


class Context:
    """A device context; ``stream`` is a raw hipStream_t (int) or None for the library's own stream."""

    def __init__(self, device: int = 0, stream: Optional[int] = None):
        L = load()
        h = ctypes.c_void_p()
        _check(L.uqc_init(int(device), ctypes.c_void_p(stream) if stream else None, ctypes.byref(h)))
        self.h = h
        self.device = device
        _live["ctx"].add(self)

    @classmethod
    def for_torch(cls, device: int = 0):
        """Context launching on torch's current stream of ``device``."""
        import torch
        s = torch.cuda.current_stream(device)
        return cls(device, int(s.cuda_stream) if s.cuda_stream else None)

    def close(self):
        if getattr(self, "h", None):
            _close_children(self)
            load().uqc_finalize(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def boys(self, T, mmax: int, precision: int = FP64) -> np.ndarray:
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(-1)
        out = np.zeros((T.shape[0], mmax + 1))
        _check(load().uqc_boys(self.h, int(precision), int(mmax), int(T.shape[0]), _dp(T), _dp(out)))
        return out


class Basis:
    """A basis of contracted Cartesian shells (``workloads.Shells``-like object) on a context."""

    def __init__(self, ctx: Context, shells):
        L = load()
        self.ctx = ctx
        self._arrs = [np.ascontiguousarray(shells.l, dtype=np.int32),
                      np.ascontiguousarray(shells.nprim, dtype=np.int32),
                      np.ascontiguousarray(shells.center, dtype=np.float64).reshape(-1),
                      np.ascontiguousarray(shells.alpha, dtype=np.float64),
                      np.ascontiguousarray(shells.coef, dtype=np.float64)]
        l, k, c, a, co = self._arrs
        self.l = l.copy()
        self.nshell = int(l.shape[0])
        h = ctypes.c_void_p()
        _check(L.uqc_basis_create(ctx.h, self.nshell, _ip(l), _ip(k), _dp(c), _dp(a), _dp(co), ctypes.byref(h)))
        self.h = h
        nbf = ctypes.c_int()
        offs = np.zeros(self.nshell, dtype=np.int32)
        _check(L.uqc_basis_info(self.h, ctypes.byref(nbf), _ip(offs)))
        self.nbf = int(nbf.value)
        self.offsets = offs.astype(np.int64)
        _live["basis"].add(self)

    def close(self):
        if getattr(self, "h", None):
            load().uqc_basis_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def schwarz(self) -> np.ndarray:
        Q = np.zeros((self.nshell, self.nshell))
        _check(load().uqc_schwarz(self.h, _dp(Q)))
        return Q

    def eri_block(self, a: int, b: int, c: int, d: int, precision: int = FP64) -> np.ndarray:
        if not all(0 <= x < self.nshell for x in (a, b, c, d)):
            out = np.zeros(1)  # the library rejects the indices before writing anything
            _check(load().uqc_eri_block(self.h, a, b, c, d, int(precision), _dp(out)))
        shp = tuple(ncart(int(self.l[x])) for x in (a, b, c, d))
        out = np.zeros(shp)
        _check(load().uqc_eri_block(self.h, a, b, c, d, int(precision), _dp(out)))
        return out

    def eri_blocks(self, quartets, precision: int = FP64):
        q = np.ascontiguousarray(quartets, dtype=np.int32).reshape(-1, 4)
        sizes = [int(np.prod([ncart(int(self.l[x])) for x in row])) for row in q]
        out = np.zeros(int(sum(sizes)))
        _check(load().uqc_eri_blocks(self.h, int(q.shape[0]), _ip(q), int(precision), _dp(out)))
        res, pos = [], 0
        for row, n in zip(q, sizes):
            res.append(out[pos:pos + n].reshape([ncart(int(self.l[x])) for x in row]))
            pos += n
        return res

    def eri_tensor(self, precision: int = FP64) -> np.ndarray:
        ns = self.nshell
        quartets = np.array([(a, b, c, d) for a in range(ns) for b in range(ns) for c in range(ns)
                             for d in range(ns)], dtype=np.int32)
        blocks = self.eri_blocks(quartets, precision)
        N = self.nbf
        T = np.zeros((N, N, N, N))
        o = self.offsets
        for (a, b, c, d), blk in zip(quartets, blocks):
            na, nb, nc, nd = blk.shape
            T[o[a]:o[a] + na, o[b]:o[b] + nb, o[c]:o[c] + nc, o[d]:o[d] + nd] = blk
        return T

    def fock_build_ptr(self, D_ptr: int, J_ptr: int, K_ptr: int, G_ptr: int, opts: FockOpts = None) -> Stats:
        """Raw-pointer build (device or host pointers, all of the same kind)."""
        st = Stats()
        o = opts if opts is not None else default_opts()
        _check(load().uqc_fock_build(self.h, ctypes.c_void_p(D_ptr), ctypes.c_void_p(J_ptr) if J_ptr else None,
                                     ctypes.c_void_p(K_ptr) if K_ptr else None,
                                     ctypes.c_void_p(G_ptr) if G_ptr else None, ctypes.byref(o), ctypes.byref(st)))
        return st

    def fock_build_noalloc_ptr(self, D_ptr: int, J_ptr: int, K_ptr: int, G_ptr: int,
                               opts: FockOpts = None) -> Stats:
        """uqc_fock_build_noalloc on raw device pointers (the library allocates nothing; see include/uqc.h)."""
        st = Stats()
        o = opts if opts is not None else default_opts()
        _check(load().uqc_fock_build_noalloc(self.h, ctypes.c_void_p(D_ptr),
                                             ctypes.c_void_p(J_ptr) if J_ptr else None,
                                             ctypes.c_void_p(K_ptr) if K_ptr else None,
                                             ctypes.c_void_p(G_ptr) if G_ptr else None, ctypes.byref(o),
                                             ctypes.byref(st)))
        return st

    def fock_build(self, D, opts: FockOpts = None, want=("J", "K", "G")):
        """D: numpy array (host path) or torch tensor on the device (device path).  Returns (J, K, G, stats) with
        outputs of the same kind as D (None for those not requested)."""
        N = self.nbf
        try:
            import torch
            is_t = isinstance(D, torch.Tensor)
        except Exception:
            is_t = False
        if is_t:
            if D.dtype != torch.float64 or not D.is_contiguous() or tuple(D.shape) != (N, N):
                raise ValueError("D must be a contiguous float64 %dx%d tensor" % (N, N))
            outs = {k: (torch.empty((N, N), dtype=torch.float64, device=D.device) if k in want else None)
                    for k in ("J", "K", "G")}
            ptr = lambda t: int(t.data_ptr()) if t is not None else 0
            st = self.fock_build_ptr(int(D.data_ptr()), ptr(outs["J"]), ptr(outs["K"]), ptr(outs["G"]), opts)
            return outs["J"], outs["K"], outs["G"], st
        D = np.ascontiguousarray(D, dtype=np.float64)
        if D.shape != (N, N):
            raise ValueError("D must be %dx%d" % (N, N))
        outs = {k: (np.zeros((N, N)) if k in want else None) for k in ("J", "K", "G")}
        ptr = lambda a: a.ctypes.data if a is not None else 0
        st = self.fock_build_ptr(D.ctypes.data, ptr(outs["J"]), ptr(outs["K"]), ptr(outs["G"]), opts)
        return outs["J"], outs["K"], outs["G"], st

    def fock_build_uhf(self, Da, Db, opts: FockOpts = None, want=("J", "Ka", "Kb", "Ga", "Gb")):
        """Spin-density build: Da, Db numpy arrays (host path) or torch tensors on the device (device path).  Returns
        a dict with J, Ka, Kb, Ga, Gb (outputs of the same kind as the inputs; None for those not requested) and
        "stats"."""
        N = self.nbf
        names = ("J", "Ka", "Kb", "Ga", "Gb")
        try:
            import torch
            is_t = isinstance(Da, torch.Tensor)
        except Exception:
            is_t = False
        if is_t:
            for D in (Da, Db):
                if D.dtype != torch.float64 or not D.is_contiguous() or tuple(D.shape) != (N, N):
                    raise ValueError("densities must be contiguous float64 %dx%d tensors" % (N, N))
            outs = {k: (torch.empty((N, N), dtype=torch.float64, device=Da.device) if k in want else None)
                    for k in names}
            ptr = lambda t: ctypes.c_void_p(int(t.data_ptr())) if t is not None else None
        else:
            Da = np.ascontiguousarray(Da, dtype=np.float64)
            Db = np.ascontiguousarray(Db, dtype=np.float64)
            if Da.shape != (N, N) or Db.shape != (N, N):
                raise ValueError("densities must be %dx%d" % (N, N))
            outs = {k: (np.zeros((N, N)) if k in want else None) for k in names}
            ptr = lambda a: ctypes.c_void_p(a.ctypes.data) if a is not None else None
        st = Stats()
        o = opts if opts is not None else default_opts()
        _check(load().uqc_fock_build_uhf(self.h, ptr(Da), ptr(Db), *[ptr(outs[k]) for k in names], ctypes.byref(o),
                                         ctypes.byref(st)))
        outs["stats"] = st
        return outs


    def one_electron(self, Z, R, want=("S", "T", "V")):
        """Overlap, kinetic and nuclear-attraction matrices for nuclei Z[natom] at R[natom][3] (host numpy arrays
        out; None for those not requested)."""
        Z = np.ascontiguousarray(Z, dtype=np.float64).reshape(-1)
        R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1)
        if R.shape[0] != 3 * Z.shape[0]:
            raise ValueError("R must hold 3 coordinates per nucleus")
        N = self.nbf
        outs = {k: (np.zeros((N, N)) if k in want else None) for k in ("S", "T", "V")}
        ptr = lambda a: ctypes.c_void_p(a.ctypes.data) if a is not None else None
        _check(load().uqc_one_electron(self.h, int(Z.shape[0]), _dp(Z), _dp(R), ptr(outs["S"]), ptr(outs["T"]),
                                       ptr(outs["V"])))
        return outs["S"], outs["T"], outs["V"]

    def scf_rhf(self, Z, R, nocc: int, opts: ScfOpts = None):
        """Restricted closed-shell Hartree-Fock; returns a dict with the energies, iteration count, convergence
        flag, final error, timings, the density P and the orbital energies."""
        Z = np.ascontiguousarray(Z, dtype=np.float64).reshape(-1)
        R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1)
        if R.shape[0] != 3 * Z.shape[0]:
            raise ValueError("R must hold 3 coordinates per nucleus")
        N = self.nbf
        P = np.zeros((N, N))
        eps = np.zeros(N)
        res = ScfResult()
        o = opts if opts is not None else scf_opts()
        _check(load().uqc_scf_rhf(self.h, int(Z.shape[0]), _dp(Z), _dp(R), int(nocc), ctypes.byref(o), _dp(P),
                                  _dp(eps), ctypes.byref(res)))
        return {"E_total": res.E_total, "E_elec": res.E_elec, "E_nuc": res.E_nuc, "iterations": res.iterations,
                "converged": bool(res.converged), "error": res.error, "ms": res.ms, "fock_ms": res.fock_ms,
                "quartets": res.quartets, "P": P, "eps": eps}

    def mp2(self, C, eps, nocc: int, nfrozen: int = 0, tau: float = 0.0, batch_bytes: int = 0):
        """Closed-shell MP2 correlation energy for canonical orbitals C[mu, p] and energies eps (host arrays);
        returns a dict with e2, e_os, e_ss, the AO quartet count, stage timings, the transformation FLOPs and the
        number of AO batches.  batch_bytes > 0 caps the device memory of one AO batch (0: free memory decides)."""
        N = self.nbf
        C = np.ascontiguousarray(C, dtype=np.float64)
        eps = np.ascontiguousarray(eps, dtype=np.float64).reshape(-1)
        if C.shape != (N, N) or eps.shape[0] != N:
            raise ValueError("C must be %dx%d and eps of length %d" % (N, N, N))
        r = Mp2Result()
        _check(load().uqc_mp2(self.h, _dp(C), _dp(eps), int(nocc), int(nfrozen), float(tau),
                              ctypes.c_size_t(int(batch_bytes)), ctypes.byref(r)))
        return {k: getattr(r, k) for k, _ in Mp2Result._fields_}

    def scf_uhf(self, Z, R, nalpha: int, nbeta: int, opts: ScfOpts = None):
        """Unrestricted Hartree-Fock; returns a dict with the energies, iteration count, convergence flag, final
        error, <S^2>, timings, the spin densities Pa, Pb and the orbital energies eps_a, eps_b."""
        Z = np.ascontiguousarray(Z, dtype=np.float64).reshape(-1)
        R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1)
        if R.shape[0] != 3 * Z.shape[0]:
            raise ValueError("R must hold 3 coordinates per nucleus")
        N = self.nbf
        Pa, Pb = np.zeros((N, N)), np.zeros((N, N))
        ea, eb = np.zeros(N), np.zeros(N)
        res = ScfResult()
        o = opts if opts is not None else scf_opts()
        _check(load().uqc_scf_uhf(self.h, int(Z.shape[0]), _dp(Z), _dp(R), int(nalpha), int(nbeta), ctypes.byref(o),
                                  _dp(Pa), _dp(Pb), _dp(ea), _dp(eb), ctypes.byref(res)))
        return {"E_total": res.E_total, "E_elec": res.E_elec, "E_nuc": res.E_nuc, "iterations": res.iterations,
                "converged": bool(res.converged), "error": res.error, "s2": res.s2, "ms": res.ms,
                "fock_ms": res.fock_ms, "quartets": res.quartets, "Pa": Pa, "Pb": Pb, "eps_a": ea, "eps_b": eb}


class Server:
    """Continuous-batching Fock-build server (see include/uqc.h)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_slots: int):
        h = ctypes.c_void_p()
        _check(load().uqc_server_create(ctx.h, ctypes.c_size_t(int(hbm_budget_bytes)), int(max_slots),
                                        ctypes.byref(h)))
        self.h = h
        self.ctx = ctx
        self._keep = {}
        _live["server"].add(self)

    def submit(self, shells, D0, n_iter: int = 8, ncol: int = 1, eps: float = 0.05, seed: int = 0,
               opts: FockOpts = None, arrival_ms: float = 0.0) -> int:
        arrs = [np.ascontiguousarray(shells.l, dtype=np.int32), np.ascontiguousarray(shells.nprim, dtype=np.int32),
                np.ascontiguousarray(shells.center, dtype=np.float64).reshape(-1),
                np.ascontiguousarray(shells.alpha, dtype=np.float64),
                np.ascontiguousarray(shells.coef, dtype=np.float64), np.ascontiguousarray(D0, dtype=np.float64)]
        r = Request()
        r.nshell = int(arrs[0].shape[0])
        r.l, r.nprim = _ip(arrs[0]), _ip(arrs[1])
        r.center, r.alpha, r.coef, r.D0 = _dp(arrs[2]), _dp(arrs[3]), _dp(arrs[4]), _dp(arrs[5])
        r.n_iter, r.ncol, r.eps, r.seed = int(n_iter), int(ncol), float(eps), int(seed)
        r.opts = opts if opts is not None else default_opts()
        r.arrival_ms = float(arrival_ms)
        t = ctypes.c_longlong()
        _check(load().uqc_submit(self.h, ctypes.byref(r), ctypes.byref(t)))
        self._keep[int(t.value)] = int(arrs[5].shape[0])
        return int(t.value)

    def poll(self, ticket: int, want_matrices: bool = True):
        """None while pending; a dict once finished (raises on a failed request)."""
        res = Result()
        n = self._keep.get(ticket, 0)
        mats = {}
        if want_matrices and n:
            for k in ("J", "K", "G", "D"):
                mats[k] = np.zeros((n, n))
                setattr(res, k, _dp(mats[k]))
        st = load().uqc_poll(self.h, ctypes.c_longlong(ticket), ctypes.byref(res))
        if st == UQC_PENDING:
            return None
        _check(st)
        self._keep.pop(ticket, None)
        out = {"n_iter": res.n_iter, "nbf": res.nbf, "E2": [res.E2[i] for i in range(res.n_iter)],
               "submit_ms": res.submit_ms, "admit_ms": res.admit_ms, "finish_ms": res.finish_ms,
               "quartets": res.quartets, "device_bytes": res.device_bytes, "steps": res.steps}
        out.update(mats)
        return out

    def drain(self):
        _check(load().uqc_server_drain(self.h))

    def close(self):
        if getattr(self, "h", None):
            load().uqc_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

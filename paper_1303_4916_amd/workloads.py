"""Seeded synthetic inputs for the ERI / Fock-build path.

This module only *draws* inputs: atom positions, shell angular momenta, contraction depths, exponents,
contraction coefficients (for normalised primitives) and symmetric positive semi-definite densities.  It holds none
of the integral arithmetic (no normalisation, no overlaps, no Boys function), so both the CPU oracle and the HIP
library can consume it without sharing any of the method's code.

Basis functions are contracted Cartesian Gaussians (paper, Sec. "Implementation details", Eq. 1).  Units are bohr.

Workloads (sizes follow the five synthetic configurations of the benchmark definition):

* ``cube``     -- 8 atoms uniform in a 6 bohr cube (min separation 1.5), s(K=3)+p(K=3) per atom, N = 32.
* ``lattice``  -- n atoms on a jittered cubic lattice (spacing 2.5, jitter U(-0.3, 0.3)), 2s1p1d per atom
                  (Cartesian d, N = 11 per atom), exponents log-uniform in [0.05, 200].
* ``stream``   -- Poisson arrivals of lattice molecules of log-uniform size (serving workload).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np


@dataclasses.dataclass
class Shells:
    """A list of contracted Cartesian shells in input order.

    l[s]       angular momentum of shell s (0, 1, 2)
    nprim[s]   contraction depth K of shell s
    center     (nshell, 3) float64, bohr
    alpha      concatenated primitive exponents, sum(nprim) entries
    coef       concatenated contraction coefficients for *normalised* primitives
    atom[s]    index of the atom the shell sits on (informational)
    """

    l: np.ndarray
    nprim: np.ndarray
    center: np.ndarray
    alpha: np.ndarray
    coef: np.ndarray
    atom: np.ndarray

    @property
    def nshell(self) -> int:
        return int(self.l.shape[0])

    @property
    def nbf(self) -> int:
        return int(sum((int(x) + 1) * (int(x) + 2) // 2 for x in self.l))

    def offsets(self) -> np.ndarray:
        n = [(int(x) + 1) * (int(x) + 2) // 2 for x in self.l]
        return np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int64)

    def translated(self, shift: Sequence[float]) -> "Shells":
        return dataclasses.replace(self, center=self.center + np.asarray(shift, dtype=np.float64)[None, :])

    def subset(self, idx: Sequence[int]) -> "Shells":
        idx = list(idx)
        starts = np.concatenate([[0], np.cumsum(self.nprim)[:-1]])
        a = np.concatenate([self.alpha[starts[i]:starts[i] + self.nprim[i]] for i in idx])
        c = np.concatenate([self.coef[starts[i]:starts[i] + self.nprim[i]] for i in idx])
        return Shells(self.l[idx].copy(), self.nprim[idx].copy(), self.center[idx].copy(), a, c,
                      self.atom[idx].copy())


def _exponents(rng: np.random.Generator, k: int, lo: float, hi: float) -> np.ndarray:
    """k exponents log-uniform in [lo, hi], sorted descending, redrawn while two are within 1 %."""
    while True:
        a = np.exp(rng.uniform(math.log(lo), math.log(hi), size=k))
        a = np.sort(a)[::-1]
        if k == 1 or np.all(a[:-1] / a[1:] > 1.01):
            return a


def _make_shells(rng: np.random.Generator, centers: np.ndarray, per_atom: Sequence[tuple],
                 lo: float, hi: float) -> Shells:
    ls, ks, cs, als, cos, at = [], [], [], [], [], []
    for ia, R in enumerate(centers):
        for (l, k) in per_atom:
            ls.append(l)
            ks.append(k)
            cs.append(R)
            als.append(_exponents(rng, k, lo, hi))
            cos.append(rng.uniform(0.1, 1.0, size=k))
            at.append(ia)
    return Shells(np.asarray(ls, dtype=np.int32), np.asarray(ks, dtype=np.int32),
                  np.asarray(cs, dtype=np.float64).reshape(-1, 3),
                  np.concatenate(als).astype(np.float64), np.concatenate(cos).astype(np.float64),
                  np.asarray(at, dtype=np.int32))


def cube_positions(rng: np.random.Generator, n: int = 8, side: float = 6.0, min_sep: float = 1.5) -> np.ndarray:
    while True:
        x = rng.uniform(0.0, side, size=(n, 3))
        d = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
        d[np.arange(n), np.arange(n)] = np.inf
        if d.min() >= min_sep:
            return x


def lattice_positions(rng: np.random.Generator, n: int, spacing: float = 2.5, jitter: float = 0.3) -> np.ndarray:
    side = int(math.ceil(round(n ** (1.0 / 3.0), 9)))
    while side ** 3 < n:
        side += 1
    g = np.stack(np.meshgrid(np.arange(side), np.arange(side), np.arange(side), indexing="ij"), -1).reshape(-1, 3)
    pick = rng.permutation(g.shape[0])[:n]
    pos = g[pick].astype(np.float64) * spacing
    pos += rng.uniform(-jitter, jitter, size=pos.shape)
    return pos


def random_density(rng: np.random.Generator, nbf: int, ncol: int, trace: float) -> np.ndarray:
    """Symmetric PSD D = C C^T with C ~ N(0,1)^{nbf x ncol}, scaled to tr(D) = trace."""
    C = rng.standard_normal((nbf, ncol))
    D = C @ C.T
    D *= trace / np.trace(D)
    return 0.5 * (D + D.T)


@dataclasses.dataclass
class Workload:
    name: str
    shells: Shells
    densities: List[np.ndarray]
    tau: float
    natoms: int


def cube(seed: int = 1) -> Workload:
    """8 atoms, s(K=3)+p(K=3) each, exponents log-uniform [0.1, 50]; one density with trace 8; unscreened."""
    rng = np.random.default_rng(seed)
    pos = cube_positions(rng)
    sh = _make_shells(rng, pos, [(0, 3), (1, 3)], 0.1, 50.0)
    D = random_density(rng, sh.nbf, 4, 8.0)
    return Workload("cube8_sp_K3", sh, [D], 0.0, 8)


def lattice_shells(natoms: int, seed: int, k_s: int = 3, k_s_core: int = None, k_p: int = 3, k_d: int = 1,
                   lo: float = 0.05, hi: float = 200.0) -> Shells:
    """2s1p1d per atom on a jittered cubic lattice.  ``k_s_core`` overrides the first (tighter) s shell's depth."""
    rng = np.random.default_rng(seed)
    pos = lattice_positions(rng, natoms)
    per_atom = [(0, k_s_core if k_s_core else k_s), (0, k_s), (1, k_p), (2, k_d)]
    return _make_shells(rng, pos, per_atom, lo, hi)


def lattice(natoms: int = 60, seed: int = 2, ndens: int = 10, dens_seeds: Sequence[int] = None,
            tau: float = 1e-12, k_s_core: int = None, k_d: int = 1, ncol: int = 30) -> Workload:
    sh = lattice_shells(natoms, seed, k_s_core=k_s_core, k_d=k_d)
    if dens_seeds is None:
        dens_seeds = [10 * seed + i for i in range(ndens)]
    Ds = [random_density(np.random.default_rng(s), sh.nbf, min(ncol, sh.nbf), float(natoms)) for s in dens_seeds]
    return Workload(f"lattice{natoms}_2s1p1d", sh, Ds, tau, natoms)


def medium(ndens: int = 10) -> Workload:
    """60 atoms, N = 660, K = 3/3/3/1 (s, s, p, d), tau = 1e-12, densities seeded 20..29."""
    return lattice(60, seed=2, ndens=ndens, dens_seeds=list(range(20, 20 + ndens)), tau=1e-12)


def mixed150(ndens: int = 1) -> Workload:
    """150 atoms, N = 1650, first s shell K = 6, tau = 1e-12."""
    return lattice(150, seed=3, ndens=ndens, dens_seeds=list(range(30, 30 + ndens)), tau=1e-12, k_s_core=6)


def large400(ndens: int = 1, k_d: int = 3) -> Workload:
    """400 atoms, N = 4400, K = 3 on every shell (d included), tau = 1e-11."""
    return lattice(400, seed=5, ndens=ndens, dens_seeds=list(range(50, 50 + ndens)), tau=1e-11, k_d=k_d)


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    natoms: int
    shells: Shells
    D0: np.ndarray


def stream(nreq: int = 512, rate_hz: float = 200.0, seed: int = 4, min_atoms: int = 4, max_atoms: int = 120,
           ncol_per_atom: float = 0.5) -> List[Request]:
    """Poisson arrivals; molecule sizes log-uniform in [min_atoms, max_atoms]; geometry seed 1000 + id."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=nreq)
    t = np.cumsum(gaps) - gaps[0]
    sizes = np.rint(np.exp(rng.uniform(math.log(min_atoms), math.log(max_atoms), size=nreq))).astype(int)
    out = []
    for i in range(nreq):
        sh = lattice_shells(int(sizes[i]), 1000 + i)
        D0 = random_density(np.random.default_rng(100000 + i), sh.nbf, max(1, int(sizes[i] * ncol_per_atom)),
                            float(sizes[i]))
        out.append(Request(i, float(t[i]), int(sizes[i]), sh, D0))
    return out


def random_quartet_shells(seed: int, ls: Sequence[int], k: int = 2, spread: float = 1.5,
                          lo: float = 0.2, hi: float = 5.0) -> Shells:
    """Four (or any number of) shells with the given angular momenta at random nearby centres (small tests)."""
    rng = np.random.default_rng(seed)
    cs, als, cos = [], [], []
    for _ in ls:
        cs.append(rng.uniform(-spread, spread, size=3))
        als.append(_exponents(rng, k, lo, hi))
        cos.append(rng.uniform(0.1, 1.0, size=k))
    n = len(ls)
    return Shells(np.asarray(ls, dtype=np.int32), np.full(n, k, dtype=np.int32), np.asarray(cs),
                  np.concatenate(als), np.concatenate(cos), np.arange(n, dtype=np.int32))


def h2_sto3g(R: float = 1.4, zeta: float = 1.24) -> Shells:
    """Minimal-basis H2: two 1s STO-3G functions (zeta-scaled exponents) on the z axis, R bohr apart."""
    a = np.array([2.22766, 0.405771, 0.109818]) * zeta ** 2
    c = np.array([0.154329, 0.535328, 0.444635])
    return Shells(np.array([0, 0], dtype=np.int32), np.array([3, 3], dtype=np.int32),
                  np.array([[0.0, 0.0, 0.0], [0.0, 0.0, R]]), np.concatenate([a, a]), np.concatenate([c, c]),
                  np.array([0, 1], dtype=np.int32))

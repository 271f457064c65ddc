"""Brute-force numerical quadrature of contracted one-electron integrals (test-only checker).

Independent of the oracle and of the HIP path: no Hermite expansion, no recursion, no Boys function.

  overlap      S_ab = prod_x int a_x(x) b_x(x) dx
  kinetic      T_ab = 1/2 <grad a | grad b> = 1/2 sum_x int a_x' b_x' dx * (overlaps of the other two directions)
               (the symmetric first-derivative form, not the second-derivative form)
  attraction   V_ab = -Z (2/sqrt(pi)) int_0^inf prod_x int a_x b_x exp(-u^2 (x - C_x)^2) dx du
               (1/|r - C| = (2/sqrt(pi)) int_0^inf exp(-u^2 |r - C|^2) du)

with a_x(x) = (x - A_x)^i exp(-alpha (x - A_x)^2).  Each one-dimensional integrand is a polynomial times one
Gaussian, done exactly by Gauss-Hermite after completing the square; the u-integral is mapped to t in (0, 1) and
summed with Gauss-Legendre nodes, doubling the count until successive results agree.  Normalisation is numerical
(the same 1D rule), as in quad_eri.
"""
from __future__ import annotations

import math

import numpy as np

from quad_eri import _comp_coefs, cart_list

_GH_X, _GH_W = np.polynomial.hermite.hermgauss(10)  # exact to degree 19


def _moment(g: float, m: float, A: float, B: float, i: int, j: int, deriv: bool, a: float, b: float) -> float:
    """int f_i(x - A) f_j(x - B) exp(-g (x - m)^2) dx, f_k(y) = y^k, or with both factors differentiated."""
    s = 1.0 / math.sqrt(g)
    x = m + _GH_X * s
    if deriv:
        fa = (i * (x - A) ** (i - 1) if i > 0 else 0.0) - 2.0 * a * (x - A) ** (i + 1)
        fb = (j * (x - B) ** (j - 1) if j > 0 else 0.0) - 2.0 * b * (x - B) ** (j + 1)
    else:
        fa = (x - A) ** i
        fb = (x - B) ** j
    return float(np.sum(_GH_W * fa * fb) * s)


def _prim(la, lb, a, b, A, B, nuclei, nodes):
    """Primitive S, T, V blocks (unnormalised Cartesian primitives)."""
    ca, cb = cart_list(la), cart_list(lb)
    g = a + b
    m = (a * A + b * B) / g
    pre = np.exp(-a * b / g * (A - B) ** 2)  # per direction
    S = np.zeros((len(ca), len(cb)))
    T = np.zeros_like(S)
    V = np.zeros_like(S)
    for i, pa in enumerate(ca):
        for j, pb in enumerate(cb):
            s1 = [pre[k] * _moment(g, m[k], A[k], B[k], pa[k], pb[k], False, a, b) for k in range(3)]
            d1 = [pre[k] * _moment(g, m[k], A[k], B[k], pa[k], pb[k], True, a, b) for k in range(3)]
            S[i, j] = s1[0] * s1[1] * s1[2]
            T[i, j] = 0.5 * (d1[0] * s1[1] * s1[2] + s1[0] * d1[1] * s1[2] + s1[0] * s1[1] * d1[2])
    t, w = np.polynomial.legendre.leggauss(nodes)
    t = 0.5 * (t + 1.0)
    w = 0.5 * w
    u = math.sqrt(g) * t / np.sqrt(1.0 - t * t)
    dudt = math.sqrt(g) * (1.0 - t * t) ** (-1.5)
    u2 = u * u
    gg = a + b + u2                                  # [nodes]
    ys = _GH_X[None, :] / np.sqrt(gg)[:, None]       # [nodes, gh]
    for Z, C in nuclei:
        # per direction k and power pair (i, j): int (x-A)^i (x-B)^j exp(-a(x-A)^2 - b(x-B)^2 - u^2 (x-C)^2) dx
        tab = []
        for k in range(3):
            mm = (a * A[k] + b * B[k] + u2 * C[k]) / gg
            e0 = a * A[k] ** 2 + b * B[k] ** 2 + u2 * C[k] ** 2 - gg * mm * mm
            x = mm[:, None] + ys
            scale = np.exp(-e0) / np.sqrt(gg)
            tk = {}
            for i in range(la + 1):
                for j in range(lb + 1):
                    tk[(i, j)] = scale * np.sum(_GH_W[None, :] * (x - A[k]) ** i * (x - B[k]) ** j, axis=1)
            tab.append(tk)
        for i, pa in enumerate(ca):
            for j, pb in enumerate(cb):
                f = tab[0][(pa[0], pb[0])] * tab[1][(pa[1], pb[1])] * tab[2][(pa[2], pb[2])]
                V[i, j] -= Z * (2.0 / math.sqrt(math.pi)) * float(np.sum(w * dudt * f))
    return S, T, V


def one_electron_block(shells, a: int, b: int, nuclei, rtol: float = 1e-12, max_nodes: int = 2048):
    """Contracted S, T, V blocks for shells a, b of a ``workloads.Shells`` list; nuclei = [(Z, centre), ...]."""
    starts = np.concatenate([[0], np.cumsum(shells.nprim)[:-1]])
    ls = [int(shells.l[s]) for s in (a, b)]
    al = [shells.alpha[starts[s]:starts[s] + shells.nprim[s]] for s in (a, b)]
    co = [shells.coef[starts[s]:starts[s] + shells.nprim[s]] for s in (a, b)]
    cen = [np.asarray(shells.center[s], dtype=np.float64) for s in (a, b)]
    cc = [_comp_coefs(ls[x], al[x], co[x]) for x in range(2)]
    nuc = [(float(Z), np.asarray(C, dtype=np.float64)) for Z, C in nuclei]

    def total(nodes):
        acc = [0.0, 0.0, 0.0]
        for p1, e1 in enumerate(al[0]):
            for p2, e2 in enumerate(al[1]):
                blk = _prim(ls[0], ls[1], e1, e2, cen[0], cen[1], nuc, nodes)
                w = np.outer(np.array([x[p1] for x in cc[0]]), np.array([x[p2] for x in cc[1]]))
                acc = [acc[k] + w * blk[k] for k in range(3)]
        return acc

    nodes = 32
    prev = total(nodes)
    while nodes < max_nodes:
        nodes *= 2
        cur = total(nodes)
        if np.max(np.abs(cur[2] - prev[2])) <= rtol * max(np.max(np.abs(cur[2])), 1e-300):
            return cur
        prev = cur
    raise RuntimeError("quadrature did not converge")

"""Brute-force numerical quadrature of contracted electron-repulsion integrals (test-only checker).

Independent of both the oracle and the HIP path: no Boys function, no recursion, no closed-form normalisation.

  1/r12 = (2/sqrt(pi)) int_0^inf exp(-u^2 r12^2) du, so
  (ab|cd) = (2/sqrt(pi)) int_0^inf I_x(u) I_y(u) I_z(u) du,
  I_x(u) = int int (x1-Ax)^ax (x1-Bx)^bx (x2-Cx)^cx (x2-Dx)^dx
                 exp(-a(x1-Ax)^2 - b(x1-Bx)^2 - c(x2-Cx)^2 - d(x2-Dx)^2 - u^2 (x1-x2)^2) dx1 dx2.

Each I_x is a polynomial times a 2D positive-definite Gaussian: completing the square and a Cholesky change of
variables turns it into a Gauss-Hermite product rule that is exact for the polynomial degrees involved.  The
u-integral is mapped to t in (0,1) by u = sqrt(rho) t / sqrt(1-t^2), which makes the integrand smooth, and is
summed with Gauss-Legendre nodes, doubling the count until successive results agree.

Normalisation (every Cartesian component normalised on its own, coefficients referring to normalised primitives)
is also done numerically with 1D Gauss-Hermite overlaps.
"""
from __future__ import annotations

import math

import numpy as np

_GH_X, _GH_W = np.polynomial.hermite.hermgauss(8)  # weight exp(-y^2), exact to degree 15


def cart_list(l: int):
    out = []
    for x in range(l, -1, -1):
        for y in range(l - x, -1, -1):
            out.append((x, y, l - x - y))
    return out


def _gauss_moment_1d(power: int, g: float) -> float:
    """int x^power exp(-g x^2) dx by Gauss-Hermite (exact for power <= 15)."""
    s = 1.0 / math.sqrt(g)
    return float(np.sum(_GH_W * (_GH_X * s) ** power) * s)


def _comp_coefs(l: int, alpha: np.ndarray, coef: np.ndarray):
    """Per-component coefficients c_p * n_p / sqrt(S) with numerical primitive and contracted normalisation."""
    out = []
    for (lx, ly, lz) in cart_list(l):
        n = np.array([1.0 / math.sqrt(_gauss_moment_1d(2 * lx, 2 * a) * _gauss_moment_1d(2 * ly, 2 * a) *
                                      _gauss_moment_1d(2 * lz, 2 * a)) for a in alpha])
        cc = coef * n
        S = 0.0
        for i, ai in enumerate(alpha):
            for j, aj in enumerate(alpha):
                g = ai + aj
                S += cc[i] * cc[j] * (_gauss_moment_1d(2 * lx, g) * _gauss_moment_1d(2 * ly, g) *
                                      _gauss_moment_1d(2 * lz, g))
        out.append(cc / math.sqrt(S))
    return out


def _I2d(u2: np.ndarray, a, b, c, d, A, B, C, D, lmax_ab: int, lmax_cd: int) -> np.ndarray:
    """I[u, ia, ib, ic, id] for one Cartesian direction, powers 0..2 each (only those needed are used)."""
    nu = u2.shape[0]
    M11 = a + b + u2
    M22 = c + d + u2
    M12 = -u2
    b1 = a * A + b * B
    b2 = c * C + d * D
    det = M11 * M22 - M12 * M12
    m1 = (M22 * b1 - M12 * b2) / det
    m2 = (-M12 * b1 + M11 * b2) / det
    c0 = a * A * A + b * B * B + c * C * C + d * D * D
    pref = np.exp(b1 * m1 + b2 * m2 - c0)
    # Cholesky M = L L^T, L = [[l11, 0], [l21, l22]];  x = m + L^{-T} y
    l11 = np.sqrt(M11)
    l21 = M12 / l11
    l22 = np.sqrt(M22 - l21 * l21)
    # L^{-T} = [[1/l11, -l21/(l11 l22)], [0, 1/l22]]
    y1 = _GH_X[:, None]
    y2 = _GH_X[None, :]
    W = (_GH_W[:, None] * _GH_W[None, :])
    x1 = m1[:, None, None] + y1[None] / l11[:, None, None] - (l21 / (l11 * l22))[:, None, None] * y2[None]
    x2 = m2[:, None, None] + y2[None] / l22[:, None, None]
    jac = 1.0 / (l11 * l22)
    fa = [(x1 - A) ** k for k in range(3)]
    fb = [(x1 - B) ** k for k in range(3)]
    fc = [(x2 - C) ** k for k in range(3)]
    fd = [(x2 - D) ** k for k in range(3)]
    out = np.zeros((nu, 3, 3, 3, 3))
    for ia in range(3):
        for ib in range(3):
            if ia + ib > lmax_ab + 2:
                continue
            fab = fa[ia] * fb[ib]
            for ic in range(3):
                for id_ in range(3):
                    v = np.sum(W[None] * fab * fc[ic] * fd[id_], axis=(1, 2))
                    out[:, ia, ib, ic, id_] = v * jac * pref
    return out


def _prim_quartet(ls, exps, centers, nodes: int) -> np.ndarray:
    la, lb, lc, ld = ls
    a, b, c, d = exps
    A, B, C, D = centers
    p, q = a + b, c + d
    rho = p * q / (p + q)
    t, w = np.polynomial.legendre.leggauss(nodes)
    t = 0.5 * (t + 1.0)
    w = 0.5 * w
    u = math.sqrt(rho) * t / np.sqrt(1.0 - t * t)
    dudt = math.sqrt(rho) * (1.0 - t * t) ** (-1.5)
    u2 = u * u
    Ix = [_I2d(u2, a, b, c, d, A[k], B[k], C[k], D[k], la + lb, lc + ld) for k in range(3)]
    ca, cb, cc, cd = cart_list(la), cart_list(lb), cart_list(lc), cart_list(ld)
    out = np.zeros((len(ca), len(cb), len(cc), len(cd)))
    for i, pa in enumerate(ca):
        for j, pb in enumerate(cb):
            for k, pc in enumerate(cc):
                for l, pd in enumerate(cd):
                    f = (Ix[0][:, pa[0], pb[0], pc[0], pd[0]] * Ix[1][:, pa[1], pb[1], pc[1], pd[1]] *
                         Ix[2][:, pa[2], pb[2], pc[2], pd[2]])
                    out[i, j, k, l] = (2.0 / math.sqrt(math.pi)) * np.sum(w * dudt * f)
    return out


def eri_block(shells, a: int, b: int, c: int, d: int, rtol: float = 1e-13, max_nodes: int = 1024) -> np.ndarray:
    """Contracted block (ab|cd) of a ``workloads.Shells`` list, by quadrature."""
    starts = np.concatenate([[0], np.cumsum(shells.nprim)[:-1]])
    idx = (a, b, c, d)
    ls = [int(shells.l[s]) for s in idx]
    al = [shells.alpha[starts[s]:starts[s] + shells.nprim[s]] for s in idx]
    co = [shells.coef[starts[s]:starts[s] + shells.nprim[s]] for s in idx]
    cen = [shells.center[s] for s in idx]
    cc = [_comp_coefs(ls[x], al[x], co[x]) for x in range(4)]

    def total(nodes):
        acc = 0.0
        for p1, e1 in enumerate(al[0]):
            for p2, e2 in enumerate(al[1]):
                for p3, e3 in enumerate(al[2]):
                    for p4, e4 in enumerate(al[3]):
                        blk = _prim_quartet(ls, (e1, e2, e3, e4), cen, nodes)
                        w = np.einsum("i,j,k,l->ijkl", np.array([x[p1] for x in cc[0]]),
                                      np.array([x[p2] for x in cc[1]]), np.array([x[p3] for x in cc[2]]),
                                      np.array([x[p4] for x in cc[3]]))
                        acc = acc + w * blk
        return acc

    nodes = 32
    prev = total(nodes)
    while nodes < max_nodes:
        nodes *= 2
        cur = total(nodes)
        if np.max(np.abs(cur - prev)) <= rtol * max(np.max(np.abs(cur)), 1e-300):
            return cur
        prev = cur
    raise RuntimeError("quadrature did not converge")

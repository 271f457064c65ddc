#!/usr/bin/env python3
"""Generator of the Rys quadrature table (build step): roots and weights of the n-point Rys rule, n = 1..5.

The n-point rule has nodes x_r = t_r^2 in (0, 1) and weights W_r > 0 with
    F_k(T) = int_0^1 t^{2k} exp(-T t^2) dt = sum_r W_r x_r^k    for k = 0 .. 2n-1,
i.e. the Gauss rule of the weight x^{-1/2} exp(-T x) / 2 on [0, 1] (Rys, Dupuis and King).  For T < kTmax the
roots and weights of every n are fitted on unit intervals [i, i+1) by Chebyshev polynomials of degree kDeg,
interpolating values computed in extended precision: a discretised Stieltjes procedure on a 400-point
Gauss-Legendre rule in t (extended-precision nodes from Newton's method), the Jacobi matrix's eigenvalues by
bisection on its Sturm sequence, the weights as Christoffel numbers.  For T >= kTmax the rule is the generalised
Gauss-Laguerre rule (alpha = -1/2) scaled, x_r = y_r / T and W_r = w_r / (2 sqrt(T)) (the interval [1, inf) then
carries a relative share below 1e-17 of every moment up to x^9); its nodes and weights are written too.  The generator checks its fits
against direct evaluations at points between the interpolation nodes and stops if any is off by more than 2e-15
(relative, weights; absolute, nodes).

Usage: gen_rys.py OUTDIR   (writes rys_consts.h and rys_table.h)
"""
from __future__ import annotations

import os
import sys

import numpy as np

LD = np.longdouble
NMAX = 5
TMAX = 64
DEG = 15
NGL = 400


def gauss_legendre_01(m: int):
    """Gauss-Legendre nodes and weights on [0, 1] in extended precision (Newton on P_m from Chebyshev guesses)."""
    xs, ws = [], []
    for i in range(1, m + 1):
        x = LD(np.cos(np.pi * (i - 0.25) / (m + 0.5)))
        for _ in range(100):
            p0, p1 = LD(1), x
            for k in range(2, m + 1):
                p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
            dp = m * (x * p1 - p0) / (x * x - 1)
            dx = p1 / dp
            x -= dx
            if abs(dx) < LD(1e-21):
                break
        p0, p1 = LD(1), x
        for k in range(2, m + 1):
            p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
        dp = m * (x * p1 - p0) / (x * x - 1)
        xs.append((1 - x) / 2)
        ws.append(LD(1) / ((1 - x * x) * dp * dp))  # 2/((1-x^2)P'^2) on [-1,1], halved for [0,1]
    return np.array(xs, dtype=LD), np.array(ws, dtype=LD)


GL_T, GL_W = gauss_legendre_01(NGL)


def rys_rule(n: int, T) -> tuple:
    """Nodes x_r (ascending) and weights W_r of the n-point Rys rule at T, extended precision."""
    T = LD(T)
    x = GL_T * GL_T
    om = GL_W * np.exp(-T * x)
    alpha, beta = [], []
    pm, p = np.zeros_like(x), np.ones_like(x)
    norm_prev = None
    for k in range(n):
        nk = np.sum(om * p * p)
        a = np.sum(om * x * p * p) / nk
        b = np.sum(om) if k == 0 else nk / norm_prev
        alpha.append(a)
        beta.append(b)
        pm, p = p, (x - a) * p - (b * pm if k > 0 else 0)
        norm_prev = nk

    def sturm_count(lam):  # eigenvalues of the Jacobi matrix below lam
        c, d = 0, LD(1)
        for k in range(n):
            d = (alpha[k] - lam) - (beta[k] / d if k > 0 else 0)
            if d == 0:
                d = LD(1e-40)
            if d < 0:
                c += 1
        return c

    roots = []
    for r in range(n):
        lo, hi = LD(0), LD(1)
        for _ in range(200):
            mid = (lo + hi) / 2
            if sturm_count(mid) > r:
                hi = mid
            else:
                lo = mid
            if hi - lo < LD(1e-21):
                break
        roots.append((lo + hi) / 2)
    weights = []
    for xr in roots:  # Christoffel numbers: 1 / sum_k p_k(x_r)^2 / ||p_k||^2
        s, q0, q1 = LD(0), LD(0), LD(1)
        nrm = beta[0]
        for k in range(n):
            s += q1 * q1 / nrm
            q0, q1 = q1, (xr - alpha[k]) * q1 - (beta[k] * q0 if k > 0 else 0)
            if k + 1 < n:
                nrm = nrm * beta[k + 1]
        weights.append(1 / s)
    return np.array(roots, dtype=LD), np.array(weights, dtype=LD)


def cheb_fit(vals):
    """Chebyshev coefficients c_j of the interpolant through values at the DEG+1 Chebyshev points of [-1, 1]."""
    m = DEG + 1
    c = []
    for j in range(m):
        s = LD(0)
        for k in range(m):
            s += vals[k] * np.cos(LD(np.pi) * j * (k + LD(0.5)) / m)
        c.append(s * (1 if j == 0 else 2) / m)
    return c


def cheb_eval(c, u):
    b1 = b2 = 0.0
    for cj in reversed(c[1:]):
        b1, b2 = 2 * u * b1 - b2 + cj, b1
    return u * b1 - b2 + c[0]


def table():
    """rows[n][i] = (coefficients of x_1..x_n, coefficients of W_1..W_n) on [i, i+1)."""
    m = DEG + 1
    pts = [np.cos(np.pi * (k + 0.5) / m) for k in range(m)]
    out = {}
    for n in range(1, NMAX + 1):
        rows = []
        for i in range(TMAX):
            xs, ws = [], []
            for u in pts:
                x, w = rys_rule(n, LD(i) + (LD(u) + 1) / 2)
                xs.append(x)
                ws.append(w)
            xs, ws = np.array(xs), np.array(ws)
            rows.append(([cheb_fit(xs[:, r]) for r in range(n)], [cheb_fit(ws[:, r]) for r in range(n)]))
        out[n] = rows
    return out


def check(tab, rng):
    worst = 0.0
    for n in range(1, NMAX + 1):
        for T in np.concatenate([rng.uniform(0, TMAX, 200), [0.0, 1e-9, TMAX - 1e-9]]):
            i = min(int(T), TMAX - 1)
            u = 2 * (T - i) - 1
            x, w = rys_rule(n, T)
            cx, cw = tab[n][i]
            for r in range(n):
                ex = abs(cheb_eval([float(c) for c in cx[r]], u) - float(x[r]))
                ew = abs(cheb_eval([float(c) for c in cw[r]], u) - float(w[r])) / float(w[r])
                worst = max(worst, ex, ew)
    if worst > 2e-15:
        raise SystemExit("gen_rys: fit error %.3g above 2e-15" % worst)
    return worst


def main(outdir):
    from scipy.special import roots_genlaguerre
    os.makedirs(outdir, exist_ok=True)
    tab = table()
    worst = check(tab, np.random.default_rng(5))
    offs = [sum(2 * k * TMAX * (DEG + 1) for k in range(1, n)) for n in range(1, NMAX + 2)]
    c = ["// Generated by gen_rys.py: constants of the Rys quadrature table (n = 1..%d roots).  Do not edit." % NMAX,
         "// Fit error %.2g (worst over the check points)." % worst, "#pragma once", "",
         "constexpr int kRysNmax = %d;      // roots" % NMAX,
         "constexpr int kRysTmax = %d;     // fitted on [0, kRysTmax), unit intervals" % TMAX,
         "constexpr int kRysDeg = %d;      // Chebyshev degree" % DEG,
         "// table layout: for n = 1..kRysNmax, interval i = 0..kRysTmax-1: n node fits then n weight fits of",
         "// kRysDeg+1 coefficients each, the block of n starting at kRysOff[n-1]; from kRysOff[kRysNmax] the",
         "// generalised Gauss-Laguerre (alpha = -1/2) nodes y_r of n = 1..kRysNmax (n-major, kRysNlag values), then",
         "// their weights w_r",
         "constexpr int kRysOff[%d] = {%s};" % (NMAX + 1, ", ".join(str(v) for v in offs)),
         "constexpr int kRysNlag = %d;" % (NMAX * (NMAX + 1) // 2),
         "constexpr int kRysTabSize = %d;" % (offs[-1] + NMAX * (NMAX + 1)), ""]
    vals = []
    for n in range(1, NMAX + 1):
        for i in range(TMAX):
            cx, cw = tab[n][i]
            for r in range(n):
                vals += [float(v) for v in cx[r]]
            for r in range(n):
                vals += [float(v) for v in cw[r]]
    ys, wl = [], []
    for n in range(1, NMAX + 1):
        y, w = roots_genlaguerre(n, -0.5)
        ys += [float(v) for v in y]
        wl += [float(v) for v in w]
    vals += ys + wl
    assert len(vals) == offs[-1] + NMAX * (NMAX + 1)
    h = ["// Generated by gen_rys.py: the Rys quadrature table (layout in rys_consts.h).  Do not edit.",
         "#pragma once", '#include "rys_consts.h"', "", "static const double kRysTab[kRysTabSize] = {"]
    for k in range(0, len(vals), 4):
        h.append("    " + ", ".join("%.17g" % v for v in vals[k:k + 4]) + ",")
    h.append("};")
    for name, lines in (("rys_consts.h", c), ("rys_table.h", h)):
        text = "\n".join(lines) + "\n"
        path = os.path.join(outdir, name)
        if os.path.exists(path) and open(path).read() == text:
            continue
        with open(path, "w") as f:
            f.write(text)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                                "generated"))

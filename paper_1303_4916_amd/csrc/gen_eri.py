#!/usr/bin/env python3
"""Generator of the per-class electron-repulsion-integral device code (build step).

For every canonical class (la lb | lc ld) with l <= 2, la >= lb, lc >= ld and (la, lb) >= (lc, ld) in pair-class
order, it writes straight-line device code for

  * the Obara-Saika vertical recursion (Head-Gordon-Pople form) that builds, per primitive quartet, the integrals
    [e0|f0]^(0) for e in la..la+lb and f in lc..lc+ld from the Boys values [00|00]^(m), and adds them to the
    contracted accumulators (FP64 accumulation whatever the recursion's precision);
  * the horizontal recursion, applied once per contracted quartet, that moves angular momentum from a to b and from
    c to d:  (a, b+1_i| = (a+1_i, b| + AB_i (a, b|  and  |c, d+1_i) = |c+1_i, d) + CD_i |c, d);
  * a frozen table of algorithmic operation counts per class (FMA = 2 FLOPs), used for roofline accounting.

The quantity computed is the integral of Eq. (5) over the contracted Cartesian Gaussians of Eq. (1); this is one
exact route to it (the paper itself uses Rys quadrature).

Vertical recursion (W - P = WP, W - Q = WQ, rho = zeta eta / (zeta + eta)):
  [a+1_i 0|00]^(m) = PA_i [a0|00]^(m) + WP_i [a0|00]^(m+1)
                     + a_i/(2 zeta) ([a-1_i 0|00]^(m) - rho/zeta [a-1_i 0|00]^(m+1))
  [e0|c+1_i 0]^(m) = QC_i [e0|c0]^(m) + WQ_i [e0|c0]^(m+1)
                     + c_i/(2 eta) ([e0|c-1_i 0]^(m) - rho/eta [e0|c-1_i 0]^(m+1))
                     + e_i/(2(zeta+eta)) [e-1_i 0|c0]^(m+1)

Usage: gen_eri.py OUTDIR   (writes eri_classes.h and eri_flops.json)
"""
from __future__ import annotations

import json
import os
import sys

PAIR_CLASSES = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)]  # pair-class order: ss, ps, pp, ds, dp, dd
LET = "spdfg"


def comps(l):
    return [(x, y, l - x - y) for x in range(l, -1, -1) for y in range(l - x, -1, -1)]


def ncart(l):
    return (l + 1) * (l + 2) // 2


def classes():
    out = []
    for bi, (la, lb) in enumerate(PAIR_CLASSES):
        for ki, (lc, ld) in enumerate(PAIR_CLASSES):
            if ki <= bi:
                out.append((la, lb, lc, ld))
    return out


def cname(c):
    return "".join(LET[x] for x in c)


def sub(t, i, k=1):
    t = list(t)
    t[i] -= k
    return tuple(t)


def add(t, i, k=1):
    t = list(t)
    t[i] += k
    return tuple(t)


class Vrr:
    """Emits the vertical recursion for one class as SSA statements over type T."""

    def __init__(self, la, lb, lc, ld):
        self.la, self.lb, self.lc, self.ld = la, lb, lc, ld
        self.L = la + lb + lc + ld
        self.lines = []
        self.memo = {}
        self.fma = 0
        self.mul = 0
        self.add = 0
        self.used_consts = set()

    def name(self, e, f, m):
        return "v%d%d%d_%d%d%d_%d" % (e + f + (m,))

    def get(self, e, f, m):
        if min(e) < 0 or min(f) < 0:
            return None
        key = (e, f, m)
        if key in self.memo:
            return self.memo[key]
        if sum(f) == 0:
            if sum(e) == 0:
                nm = "F%d" % m
                self.memo[key] = nm
                return nm
            # bra step: pick the direction with the smallest positive power (drops the a_i - 1 term if it is 1)
            i = min((x for x in range(3) if e[x] > 0), key=lambda x: (e[x], x))
            e1 = sub(e, i)
            a = self.get(e1, f, m)
            b = self.get(e1, f, m + 1)
            expr = "fma(PA%s, %s, WP%s * %s)" % ("xyz"[i], a, "xyz"[i], b)
            self.fma += 1
            self.mul += 1
            if e1[i] > 0:
                e2 = sub(e1, i)
                c = self.get(e2, f, m)
                d = self.get(e2, f, m + 1)
                k = e1[i]
                self.used_consts.add(("oz", k))
                expr = "fma(oz%d, %s, fma(-ozr%d, %s, %s))" % (k, c, k, d, expr)
                self.fma += 2
        else:
            # ket step: prefer a direction whose power is 1 (no c_i - 1 term) and whose bra power is 0
            i = min((x for x in range(3) if f[x] > 0), key=lambda x: (f[x] > 1, e[x] > 0, f[x], x))
            f1 = sub(f, i)
            a = self.get(e, f1, m)
            b = self.get(e, f1, m + 1)
            expr = "fma(QC%s, %s, WQ%s * %s)" % ("xyz"[i], a, "xyz"[i], b)
            self.fma += 1
            self.mul += 1
            if f1[i] > 0:
                f2 = sub(f1, i)
                c = self.get(e, f2, m)
                d = self.get(e, f2, m + 1)
                k = f1[i]
                self.used_consts.add(("oe", k))
                expr = "fma(oe%d, %s, fma(-oer%d, %s, %s))" % (k, c, k, d, expr)
                self.fma += 2
            if e[i] > 0:
                g = self.get(sub(e, i), f1, m + 1)
                k = e[i]
                self.used_consts.add(("oze", k))
                expr = "fma(oze%d, %s, %s)" % (k, g, expr)
                self.fma += 1
        nm = self.name(e, f, m)
        self.lines.append("const T %s = %s;" % (nm, expr))
        self.memo[key] = nm
        return nm

    def targets(self):
        es = [c for l in range(self.la, self.la + self.lb + 1) for c in comps(l)]
        fs = [c for l in range(self.lc, self.lc + self.ld + 1) for c in comps(l)]
        return es, fs


def gen_vrr(c):
    la, lb, lc, ld = c
    v = Vrr(la, lb, lc, ld)
    es, fs = v.targets()
    acc_lines = []
    for ie, e in enumerate(es):
        for jf, f in enumerate(fs):
            nm = v.get(e, f, 0)
            acc_lines.append("acc[%d] += (double)%s;" % (ie * len(fs) + jf, nm))
    return v, es, fs, acc_lines


def interleave(v, acc_lines):
    """VRR statements with every accumulation placed right after the statement that defines its target, so a
    target's register can be released as soon as its last use as an intermediate is past."""
    where = {}
    for line in acc_lines:
        nm = line.split("(double)")[1].rstrip(";")
        where.setdefault(nm, []).append(line)
    out = []
    for line in v.lines:
        out.append(line)
        nm = line.split()[2]
        out.extend(where.pop(nm, []))
    for rest in where.values():  # targets that are Boys values themselves (class (ss|ss))
        out.extend(rest)
    return out


class Hrr:
    """Horizontal recursion programme on one side (bra or ket), as a list of (target, src1, src2, dir)."""

    def __init__(self, la, lb):
        self.la, self.lb = la, lb
        self.steps = []
        self.memo = {}

    def get(self, a, b):
        key = (a, b)
        if key in self.memo:
            return self.memo[key]
        if sum(b) == 0:
            self.memo[key] = ("src", a)
            return self.memo[key]
        i = min((x for x in range(3) if b[x] > 0), key=lambda x: (b[x], x))
        b1 = sub(b, i)
        s1 = self.get(add(a, i), b1)
        s2 = self.get(a, b1)
        node = ("tmp", len(self.steps))
        self.steps.append((node, s1, s2, i))
        self.memo[key] = node
        return node

    def build(self):
        outs = []
        for a in comps(self.la):
            for b in comps(self.lb):
                outs.append(self.get(a, b))
        return outs


def gen_hrr(c, es, fs):
    """Contracted [e0|f0] (acc) -> (ab|cd) (out), choosing the cheaper of bra-first / ket-first."""
    la, lb, lc, ld = c
    hb = Hrr(la, lb)
    bra_outs = hb.build()
    hk = Hrr(lc, ld)
    ket_outs = hk.build()
    na, nb, nc, nd = ncart(la), ncart(lb), ncart(lc), ncart(ld)
    eidx = {e: i for i, e in enumerate(es)}
    fidx = {f: i for i, f in enumerate(fs)}
    NF = len(fs)
    cost_ket_first = len(hk.steps) * len(es) + len(hb.steps) * nc * nd
    cost_bra_first = len(hb.steps) * len(fs) + len(hk.steps) * na * nb
    lines = []
    if len(hb.steps) == 0 and len(hk.steps) == 0:
        for i in range(na * nb):
            for k in range(nc * nd):
                lines.append("out[%d] = acc[%d];" % (i * nc * nd + k, i * NF + k))
        return lines, 0
    ket_first = cost_ket_first <= cost_bra_first
    # stage 1 over the first side, for every component of the other side's source range
    if ket_first:
        # for each e: ket programme from acc[e][f] to K1[e][cd]
        for ie, e in enumerate(es):
            def ref(node, ie=ie):
                if node[0] == "src":
                    return "acc[%d]" % (ie * NF + fidx[node[1]])
                return "hk%d_%d" % (ie, node[1])
            for (node, s1, s2, i) in hk.steps:
                lines.append("const double hk%d_%d = fma(CD%s, %s, %s);" % (ie, node[1], "xyz"[i], ref(s2), ref(s1)))
            for kcd, node in enumerate(ket_outs):
                lines.append("const double k1_%d_%d = %s;" % (ie, kcd, ref(node)))
        for kcd in range(nc * nd):
            def ref2(node, kcd=kcd):
                if node[0] == "src":
                    return "k1_%d_%d" % (eidx[node[1]], kcd)
                return "hb%d_%d" % (kcd, node[1])
            for (node, s1, s2, i) in hb.steps:
                lines.append("const double hb%d_%d = fma(AB%s, %s, %s);" % (kcd, node[1], "xyz"[i], ref2(s2), ref2(s1)))
            for iab, node in enumerate(bra_outs):
                lines.append("out[%d] = %s;" % (iab * nc * nd + kcd, ref2(node)))
        flops = 2 * (len(hk.steps) * len(es) + len(hb.steps) * nc * nd)
    else:
        for jf, f in enumerate(fs):
            def ref(node, jf=jf):
                if node[0] == "src":
                    return "acc[%d]" % (eidx[node[1]] * NF + jf)
                return "hb%d_%d" % (jf, node[1])
            for (node, s1, s2, i) in hb.steps:
                lines.append("const double hb%d_%d = fma(AB%s, %s, %s);" % (jf, node[1], "xyz"[i], ref(s2), ref(s1)))
            for iab, node in enumerate(bra_outs):
                lines.append("const double b1_%d_%d = %s;" % (iab, jf, ref(node)))
        for iab in range(na * nb):
            def ref2(node, iab=iab):
                if node[0] == "src":
                    return "b1_%d_%d" % (iab, fidx[node[1]])
                return "hk%d_%d" % (iab, node[1])
            for (node, s1, s2, i) in hk.steps:
                lines.append("const double hk%d_%d = fma(CD%s, %s, %s);" % (iab, node[1], "xyz"[i], ref2(s2), ref2(s1)))
            for kcd, node in enumerate(ket_outs):
                lines.append("out[%d] = %s;" % (iab * nc * nd + kcd, ref2(node)))
        flops = 2 * (len(hb.steps) * len(fs) + len(hk.steps) * na * nb)
    return lines, flops


def setup_flops(L):
    """Per-primitive-quartet set-up outside the recursion: zeta+eta, 1/(zeta+eta) (counted as 1), rho, PQ, T,
    WP, WQ, recursion constants, prefactor with sqrt (counted as 1), Boys (Taylor of order 7 at F_L: 7 mul +
    7 fma; downward recursion 2 per order; exp counted as 1) and scaling of the L+1 Boys values."""
    f = 1 + 1 + 3 + 3 + 5 + 6 + 6 + 4 + 4
    f += 14 + 1 + (3 * L if L > 0 else 0)
    f += L + 1
    return f


def _write(path, text):
    """Writes only when the content changes, so incremental builds see unchanged headers as up to date."""
    if os.path.exists(path):
        with open(path) as f:
            if f.read() == text:
                return
    with open(path, "w") as f:
        f.write(text)


def main(outdir):
    os.makedirs(outdir, exist_ok=True)
    hdr = []
    hdr.append("// Generated by gen_eri.py: per-class vertical and horizontal recursions.  Do not edit.")
    hdr.append("#pragma once")
    hdr.append("")
    table = {}
    for c in classes():
        la, lb, lc, ld = c
        v, es, fs, acc_lines = gen_vrr(c)
        hrr_lines, hrr_flops = gen_hrr(c, es, fs)
        L = la + lb + lc + ld
        nacc = len(es) * len(fs)
        consts = sorted(v.used_consts)
        nm = cname(c)
        hdr.append("// class (%s%s|%s%s): %d accumulators, L = %d" % (LET[la], LET[lb], LET[lc], LET[ld], nacc, L))
        hdr.append("template <> struct EriClass<%d, %d, %d, %d> {" % c)
        hdr.append("  static constexpr int L = %d;" % L)
        hdr.append("  static constexpr int NACC = %d;" % nacc)
        hdr.append("  static constexpr int NA = %d, NB = %d, NC = %d, ND = %d;" % (ncart(la), ncart(lb), ncart(lc),
                                                                                    ncart(ld)))
        hdr.append("  template <typename T>")
        hdr.append("  __device__ static __forceinline__ void vrr(const T* __restrict__ F, const PrimGeom<T>& g, "
                   "double* __restrict__ acc) {")
        hdr.append("    const T PAx = g.PA[0], PAy = g.PA[1], PAz = g.PA[2];")
        hdr.append("    const T WPx = g.WP[0], WPy = g.WP[1], WPz = g.WP[2];")
        hdr.append("    const T QCx = g.QC[0], QCy = g.QC[1], QCz = g.QC[2];")
        hdr.append("    const T WQx = g.WQ[0], WQy = g.WQ[1], WQz = g.WQ[2];")
        for m in range(L + 1):
            hdr.append("    const T F%d = F[%d];" % (m, m))
        for (kind, k) in consts:
            if kind == "oz":
                hdr.append("    const T oz%d = T(%d) * g.o2z, ozr%d = oz%d * g.roz;" % (k, k, k, k))
            elif kind == "oe":
                hdr.append("    const T oe%d = T(%d) * g.o2e, oer%d = oe%d * g.roe;" % (k, k, k, k))
            else:
                hdr.append("    const T oze%d = T(%d) * g.o2ze;" % (k, k))
        for line in interleave(v, acc_lines):
            hdr.append("    " + line)
        hdr.append("    (void)PAx; (void)PAy; (void)PAz; (void)WPx; (void)WPy; (void)WPz;")
        hdr.append("    (void)QCx; (void)QCy; (void)QCz; (void)WQx; (void)WQy; (void)WQz;")
        hdr.append("  }")
        hdr.append("  __device__ static __forceinline__ void hrr(const double* __restrict__ acc, const double ABx, "
                   "const double ABy, const double ABz, const double CDx, const double CDy, const double CDz, "
                   "double* __restrict__ out) {")
        for line in hrr_lines:
            hdr.append("    " + line)
        hdr.append("    (void)ABx; (void)ABy; (void)ABz; (void)CDx; (void)CDy; (void)CDz;")
        hdr.append("  }")
        hdr.append("};")
        hdr.append("")
        nout = ncart(la) * ncart(lb) * ncart(lc) * ncart(ld)
        vrr_flops = 2 * v.fma + v.mul + v.add
        table[nm] = {
            "class": list(c),
            "L": L,
            "nacc": nacc,
            "nout": nout,
            "vrr_flops": vrr_flops,
            "setup_flops": setup_flops(L),
            "acc_flops": nacc,
            "f_prim": vrr_flops + setup_flops(L) + nacc,
            "hrr_flops": hrr_flops,
            "digest_flops": 12 * nout,
            "f_contr": hrr_flops + 12 * nout,
            "vrr_terms": len(v.lines),
        }
    _write(os.path.join(outdir, "eri_classes.h"), "\n".join(hdr) + "\n")
    # frozen FLOP model, also as a C table (class order = generation order)
    lines = ["// Generated by gen_eri.py: algorithmic FLOPs per primitive quartet and per contracted quartet.",
             "#pragma once", "static const double kClassFlopsPrim[%d] = {" % len(table)]
    lines.append(", ".join("%d" % table[cname(c)]["f_prim"] for c in classes()) + "};")
    lines.append("static const double kClassFlopsContr[%d] = {" % len(table))
    lines.append(", ".join("%d" % table[cname(c)]["f_contr"] for c in classes()) + "};")
    _write(os.path.join(outdir, "eri_flops.h"), "\n".join(lines) + "\n")
    _write(os.path.join(outdir, "eri_flops.json"), json.dumps(table, indent=1, sort_keys=True) + "\n")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                                "generated"))

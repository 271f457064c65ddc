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

import itertools
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



# ------------------------------------------------------------------------------------------------------------------
# Team evaluation of the largest classes.  The six permutations of the Cartesian axes map the set of [e0|f0]
# targets (and of (ab|cd) outputs) onto itself.  A team of six lanes evaluates one contracted quartet: lane p runs
# the recursion for one representative of every orbit with its geometry vectors relabelled by p, which yields the
# true integrals of the permuted components.  Every lane runs identical straight-line code, each holds about a
# sixth of the accumulators, and the horizontal recursion reads the values it needs from the other lanes.
#   relabel:  P(t, p)_i = t[p[i]]           (geometry seen by lane p: V_lane = P(V, p))
#   inverse:  Q(t, p)[p[i]] = t[i]          (lane p's representative r stands for the true component Q(r, p))
#   Q(Q(t, pi), p) = Q(t, p o pi) with (p o pi)[i] = p[pi[i]]
# ------------------------------------------------------------------------------------------------------------------
PERMS = list(itertools.permutations(range(3)))
TEAM_CLASSES = [(2, 1, 2, 1), (2, 2, 1, 1), (2, 2, 2, 0), (2, 2, 2, 1), (2, 2, 2, 2)]
TEAM_SIZE = 6
# classes whose lanes digest every output as soon as it is formed (all six partial blocks live at once) instead
# of holding the outputs for three two-block passes: (dd|dd) has 224 outputs per lane, too many to hold
TEAM_STREAM_DIGEST = {(2, 2, 2, 2)}


def perm_q(t, p):
    u = [0, 0, 0]
    for i in range(3):
        u[p[i]] = t[i]
    return tuple(u)


def perm_compose(p, q):
    return tuple(p[q[i]] for i in range(3))


def binom(n, k):
    return [[1], [1, 1], [1, 2, 1]][n][k]


def orbit_rep(x, act):
    """x: tuple of component triples; returns (representative, perm index pi with act(rep, pi) == x)."""
    orb = [(tuple(act(t, p) for t in x), ip) for ip, p in enumerate(PERMS)]
    rep = min(o for o, _ in orb)
    # find pi with Q(rep, pi) == x
    for ip, p in enumerate(PERMS):
        if tuple(act(t, p) for t in rep) == x:
            return rep, ip
    raise AssertionError


def gen_team(c):
    la, lb, lc, ld = c
    v = Vrr(la, lb, lc, ld)
    es, fs = v.targets()
    targets = [(e, f) for e in es for f in fs]
    reps = sorted({orbit_rep(t, perm_q)[0] for t in targets})
    rep_idx = {r: i for i, r in enumerate(reps)}
    acc_lines = []
    for i, (e, f) in enumerate(reps):
        nm = v.get(e, f, 0)
        acc_lines.append("acc[%d] += (double)%s;" % (i, nm))
    vrr_lines = interleave(v, acc_lines)
    # outputs and their orbits
    ca, cb, cc, cd = comps(la), comps(lb), comps(lc), comps(ld)
    outs = [(a, b, cx, d) for a in ca for b in cb for cx in cc for d in cd]
    out_reps = sorted({orbit_rep(o, perm_q)[0] for o in outs})
    hl = []       # horizontal recursion + digest lines
    leaf = {}     # (rep index, perm index) -> name

    def get_leaf(e, f):
        r, ip = orbit_rep((e, f), perm_q)
        if r == (e, f):
            ip = 0  # identity: the lane's own accumulator
        key = (rep_idx[r], ip)
        if key not in leaf:
            nm = "lf%d_%d" % key
            if ip == 0:
                hl.append("const double %s = acc[%d];" % (nm, key[0]))
            else:
                hl.append("const double %s = fetch(acc[%d], src[%d]);" % (nm, key[0], ip))
            leaf[key] = nm
        return leaf[key]

    mono = {}

    def get_mono(kind, m):
        if sum(m) == 0:
            return None
        key = (kind, m)
        if key not in mono:
            nm = "%s%d%d%d" % ((kind,) + m)
            fac = []
            for i, ax in enumerate("xyz"):
                fac += ["%s%s" % (kind, ax)] * m[i]
            hl.append("const double %s = %s;" % (nm, " * ".join(fac)))
            mono[key] = nm
        return mono[key]

    half = {}
    flops = [0]

    def get_half(e, cx, d):
        key = (e, cx, d)
        if key in half:
            return half[key]
        terms = []
        for kx in range(d[0] + 1):
            for ky in range(d[1] + 1):
                for kz in range(d[2] + 1):
                    k = (kx, ky, kz)
                    f = tuple(cx[i] + k[i] for i in range(3))
                    coef = binom(d[0], kx) * binom(d[1], ky) * binom(d[2], kz)
                    mnm = get_mono("CD", tuple(d[i] - k[i] for i in range(3)))
                    terms.append((coef, mnm, get_leaf(e, f)))
        nm = "h%d" % len(half)
        expr = None
        for coef, mnm, lf in terms:
            t = lf if mnm is None else "%s * %s" % (mnm, lf)
            if coef != 1:
                t = "%d.0 * %s" % (coef, t) if mnm is None else "(%d.0 * %s) * %s" % (coef, mnm, lf)
            expr = t if expr is None else "%s + %s" % (expr, t)
            flops[0] += 2
        hl.append("const double %s = %s;" % (nm, expr))
        half[key] = nm
        return nm

    na, nb, nc, nd = ncart(la), ncart(lb), ncart(lc), ncart(ld)
    ia, ib, ic, idd = ({t: i for i, t in enumerate(x)} for x in (ca, cb, cc, cd))
    masks = []
    stream = []   # the same outputs, each digested at once into all six partial blocks (streaming form)
    stream_lds = []  # streaming form against the team's LDS copies of the density slices and partial blocks
    emits = []  # each output handed to a caller's functor as soon as it is formed: e(output index, weighted value)
    for o in out_reps:
        a, b, cx, d = o
        terms = []
        for kx in range(b[0] + 1):
            for ky in range(b[1] + 1):
                for kz in range(b[2] + 1):
                    k = (kx, ky, kz)
                    e = tuple(a[i] + k[i] for i in range(3))
                    coef = binom(b[0], kx) * binom(b[1], ky) * binom(b[2], kz)
                    mnm = get_mono("AB", tuple(b[i] - k[i] for i in range(3)))
                    terms.append((coef, mnm, get_half(e, cx, d)))
        expr = None
        for coef, mnm, hn in terms:
            t = hn if mnm is None else "%s * %s" % (mnm, hn)
            if coef != 1:
                t = "%d.0 * %s" % (coef, t)
            expr = t if expr is None else "%s + %s" % (expr, t)
            flops[0] += 2
        # owners: one lane per coset of the stabiliser
        stab = [ip for ip, p in enumerate(PERMS) if tuple(perm_q(t, p) for t in o) == o]
        mask = 0
        for ip, p in enumerate(PERMS):
            coset = [PERMS.index(perm_compose(p, PERMS[s])) for s in stab]
            if ip == min(coset):
                mask |= 1 << ip
        masks.append(mask)
        wexpr = "w" if mask == (1 << TEAM_SIZE) - 1 else "(((%d >> pidx) & 1) ? w : 0.0)" % mask
        hl.append("out[%d] = (%s) * %s;" % (len(masks) - 1, expr, wexpr))
        emits.append("e(%d, (%s) * %s);" % (len(masks) - 1, expr, wexpr))
        i, j, k, l = ia[a], ib[b], ic[cx], idd[d]
        stream.append("{ const double x = (%s) * %s;" % (expr, wexpr))
        stream.append("  jab[%d] = fma(x, dcd[%d], jab[%d]); jcd[%d] = fma(x, dab[%d], jcd[%d]);"
                      % (i * nb + j, k * nd + l, i * nb + j, k * nd + l, i * nb + j, k * nd + l))
        stream.append("  kac[%d] = fma(x, dbd[%d], kac[%d]); kad[%d] = fma(x, dbc[%d], kad[%d]);"
                      % (i * nc + k, j * nd + l, i * nc + k, i * nd + l, j * nc + k, i * nd + l))
        stream.append("  kbc[%d] = fma(x, dad[%d], kbc[%d]); kbd[%d] = fma(x, dac[%d], kbd[%d]); }"
                      % (j * nc + k, i * nd + l, j * nc + k, j * nd + l, i * nc + k, j * nd + l))
        # true-index offsets from the lane's component maps pA..pD (frame component -> true component)
        stream_lds.append("{ const double x = (%s) * %s;" % (expr, wexpr))
        stream_lds.append("  const int ij = pA[%d] * %d + pB[%d], kl = pC[%d] * %d + pD[%d], "
                          "ik = pA[%d] * %d + pC[%d], il = pA[%d] * %d + pD[%d], "
                          "jk = pB[%d] * %d + pC[%d], jl = pB[%d] * %d + pD[%d];"
                          % (i, nb, j, k, nd, l, i, nc, k, i, nd, l, j, nc, k, j, nd, l))
        stream_lds.append("  if constexpr (WITH_J) { atomic_add_lds(t_jab + ij, x * s_cd[kl]); "
                          "atomic_add_lds(t_jcd + kl, x * s_ab[ij]); }")
        stream_lds.append("  atomic_add_lds(t_kac + ik, x * s_bd[jl]); atomic_add_lds(t_kad + il, x * s_bc[jk]); "
                          "atomic_add_lds(t_kbc + jk, x * s_ad[il]); atomic_add_lds(t_kbd + jl, x * s_ac[ik]); }")
    # Digest passes over the lane's weighted outputs, two partial blocks each (the same pairing as the 64-ket
    # kernels): P = 0: x = out.D_cd -> J_ab, y = out.D_ab -> J_cd; P = 1: x = out.D_bd -> K_ac, y = out.D_ac -> K_bd;
    # P = 2: x = out.D_bc -> K_ad, y = out.D_ad -> K_bc.  D slices and partials are in the lane's own frame; every
    # partial is assigned at its first term (no zero fill) and untouched ones are set to zero.
    digest = []
    sizes = [(na * nb, nc * nd), (na * nc, nb * nd), (na * nd, nb * nc)]
    for P in range(3):
        lines = []
        seen_x, seen_y = set(), set()
        for n, o in enumerate(out_reps):
            a, b, cx, d = o
            i, j, k, l = ia[a], ib[b], ic[cx], idd[d]
            xe, d1e, ye, d2e = [(i * nb + j, k * nd + l, k * nd + l, i * nb + j),
                                (i * nc + k, j * nd + l, j * nd + l, i * nc + k),
                                (i * nd + l, j * nc + k, j * nc + k, i * nd + l)][P]
            for arr, e, darr, de, seen in (("x", xe, "d1", d1e, seen_x), ("y", ye, "d2", d2e, seen_y)):
                if e in seen:
                    lines.append("%s[%d] = fma(out[%d], %s[%d], %s[%d]);" % (arr, e, n, darr, de, arr, e))
                else:
                    lines.append("%s[%d] = out[%d] * %s[%d];" % (arr, e, n, darr, de))
                    seen.add(e)
        for e in range(sizes[P][0]):
            if e not in seen_x:
                lines.append("x[%d] = 0.0;" % e)
        for e in range(sizes[P][1]):
            if e not in seen_y:
                lines.append("y[%d] = 0.0;" % e)
        digest.append(lines)
    # the streaming form shares the memoised intermediate lines of the horizontal recursion
    hrr_stream = [x for x in hl if not x.startswith("out[")]
    pos = 0
    merged, merged_lds, merged_emit = [], [], []
    for x in hl:
        if x.startswith("out["):
            merged += stream[4 * pos:4 * pos + 4]
            merged_lds += stream_lds[4 * pos:4 * pos + 4]
            merged_emit.append(emits[pos])
            pos += 1
        else:
            merged.append(x)
            merged_lds.append(x)
            merged_emit.append(x)
    return {"vrr": vrr_lines, "nrep": len(reps), "reps": reps, "out_reps": out_reps, "hrr": hl,
            "digest": digest, "hrr_digest": merged, "hrr_digest_lds": merged_lds, "hrr_emit": merged_emit,
            "masks": masks, "v": v, "hrr_flops": flops[0]}


def perm_comp_table():
    """kPermComp[l][p][k]: index in the shell of true component Q(comps(l)[k], p)."""
    rows = []
    for l in range(3):
        cl = comps(l)
        idx = {t: i for i, t in enumerate(cl)}
        rows.append([[idx[perm_q(t, p)] for t in cl] + [0] * (6 - len(cl)) for p in PERMS])
    return rows

# Transcendental operations per primitive quartet, counted apart from the FLOPs: the reciprocal square root of
# zeta + eta (1/(zeta+eta) is its square, and the prefactor takes its other factor) and exp(-T) of the Boys
# function's downward recursion.
TRANS_PER_PRIM = 2


def setup_flops(L):
    """Per-primitive-quartet FLOPs outside the recursion: zeta+eta (1), 1/(zeta+eta) as the square of
    1/sqrt(zeta+eta) (1), rho, PQ, T, WP, WQ, recursion constants, prefactor (the square root itself is one of the
    TRANS_PER_PRIM transcendental operations, not a FLOP), Boys (Taylor of order 7 at F_L: 7 mul + 7 fma; downward
    recursion 2 per order; exp(-T) is the other transcendental operation) and scaling of the L+1 Boys values."""
    f = 1 + 1 + 3 + 3 + 5 + 6 + 6 + 4 + 3
    f += 14 + (3 * L if L > 0 else 0)
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
            "trans_per_prim": TRANS_PER_PRIM,
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
             "#pragma once", "static constexpr double kClassFlopsPrim[%d] = {" % len(table)]
    lines.append(", ".join("%d" % table[cname(c)]["f_prim"] for c in classes()) + "};")
    lines.append("static constexpr double kClassFlopsContr[%d] = {" % len(table))
    lines.append(", ".join("%d" % table[cname(c)]["f_contr"] for c in classes()) + "};")
    lines.append("// 1 where the Fock-build kernel of the class is the six-lane team kernel (10 ket pairs per wavefront)")
    lines.append("static constexpr int kClassTeam[%d] = {%s};" % (len(table), ", ".join(
        "1" if c in TEAM_CLASSES else "0" for c in classes())))
    _write(os.path.join(outdir, "eri_flops.h"), "\n".join(lines) + "\n")
    _write(os.path.join(outdir, "eri_flops.json"), json.dumps(table, indent=1, sort_keys=True) + "\n")
    # team classes
    th = ["// Generated by gen_eri.py: six-lane team evaluation of the largest classes.  Do not edit.", "#pragma once",
          ""]
    pc = perm_comp_table()
    th.append("static constexpr int kPermAxes[6][3] = {%s};" % ", ".join(
        "{%d, %d, %d}" % p for p in PERMS))
    th.append("static constexpr int kPermCompose[6][6] = {%s};" % ", ".join(
        "{%s}" % ", ".join(str(PERMS.index(perm_compose(p, q))) for q in PERMS) for p in PERMS))
    th.append("static constexpr int kPermComp[3][6][6] = {%s};" % ", ".join(
        "{%s}" % ", ".join("{%s}" % ", ".join(str(x) for x in row) for row in pc[l]) for l in range(3)))
    th.append("")
    for c in TEAM_CLASSES:
        t = gen_team(c)
        v = t["v"]
        L = sum(c)
        th.append("// class (%s%s|%s%s): %d orbit representatives of %d targets, %d representative outputs"
                  % (LET[c[0]], LET[c[1]], LET[c[2]], LET[c[3]], t["nrep"], len(v.targets()[0]) * len(v.targets()[1]),
                     len(t["out_reps"])))
        th.append("template <> struct TeamClass<%d, %d, %d, %d> {" % c)
        th.append("  static constexpr int L = %d;" % L)
        th.append("  static constexpr int NREP = %d;" % t["nrep"])
        th.append("  static constexpr int NA = %d, NB = %d, NC = %d, ND = %d;" % tuple(ncart(x) for x in c))
        th.append("  template <typename T>")
        th.append("  __device__ static __forceinline__ void vrr(const T* __restrict__ F, const PrimGeom<T>& g, "
                  "double* __restrict__ acc) {")
        th.append("    const T PAx = g.PA[0], PAy = g.PA[1], PAz = g.PA[2];")
        th.append("    const T WPx = g.WP[0], WPy = g.WP[1], WPz = g.WP[2];")
        th.append("    const T QCx = g.QC[0], QCy = g.QC[1], QCz = g.QC[2];")
        th.append("    const T WQx = g.WQ[0], WQy = g.WQ[1], WQz = g.WQ[2];")
        for m in range(L + 1):
            th.append("    const T F%d = F[%d];" % (m, m))
        for (kind, k) in sorted(v.used_consts):
            if kind == "oz":
                th.append("    const T oz%d = T(%d) * g.o2z, ozr%d = oz%d * g.roz;" % (k, k, k, k))
            elif kind == "oe":
                th.append("    const T oe%d = T(%d) * g.o2e, oer%d = oe%d * g.roe;" % (k, k, k, k))
            else:
                th.append("    const T oze%d = T(%d) * g.o2ze;" % (k, k))
        for line in t["vrr"]:
            th.append("    " + line)
        th.append("    (void)PAx; (void)PAy; (void)PAz; (void)WPx; (void)WPy; (void)WPz;")
        th.append("    (void)QCx; (void)QCy; (void)QCz; (void)WQx; (void)WQy; (void)WQz;")
        th.append("  }")
        th.append("  static constexpr int NOUT = %d;  // representative outputs held by a lane" % len(t["out_reps"]))
        th.append("  static constexpr bool STREAM = %s;" % ("true" if c in TEAM_STREAM_DIGEST else "false"))
        cab = [comps(x) for x in c]
        th.append("  // frame component indices (a, b, c, d) of each representative output (the order of hrr's out)")
        th.append("  static constexpr unsigned char OUT_IDX[%d][4] = {%s};" % (len(t["out_reps"]), ", ".join(
            "{%s}" % ", ".join(str(cab[x].index(o[x])) for x in range(4)) for o in t["out_reps"])))
        if c in TEAM_STREAM_DIGEST:
            th.append("  __device__ static __forceinline__ void hrr_digest(const double* __restrict__ acc, "
                      "const int* __restrict__ src, int pidx, double w, double ABx, double ABy, double ABz, "
                      "double CDx, double CDy, double CDz, const double* __restrict__ dab, "
                      "const double* __restrict__ dcd, const double* __restrict__ dbd, "
                      "const double* __restrict__ dbc, const double* __restrict__ dad, "
                      "const double* __restrict__ dac, double* __restrict__ jab, double* __restrict__ jcd, "
                      "double* __restrict__ kac, double* __restrict__ kad, double* __restrict__ kbc, "
                      "double* __restrict__ kbd) {")
            for line in t["hrr_digest"]:
                th.append("    " + line)
            th.append("    (void)ABx; (void)ABy; (void)ABz; (void)CDx; (void)CDy; (void)CDz; (void)src; (void)pidx;")
            th.append("  }")
            # the same, with the density slices read from and the partial blocks added into the team's LDS copies
            # (true component order; pA..pD: the lane's maps from frame to true components)
            th.append("  template <bool WITH_J>")
            th.append("  __device__ static __forceinline__ void hrr_digest_lds(const double* __restrict__ acc, "
                      "const int* __restrict__ src, int pidx, double w, double ABx, double ABy, double ABz, "
                      "double CDx, double CDy, double CDz, const double* s_ab, const double* s_cd, "
                      "const double* s_ac, const double* s_ad, const double* s_bc, const double* s_bd, "
                      "double* t_jab, double* t_jcd, double* t_kac, double* t_kad, double* t_kbc, double* t_kbd, "
                      "const int* pA, const int* pB, const int* pC, const int* pD) {")
            for line in t["hrr_digest_lds"]:
                th.append("    " + line)
            th.append("    (void)ABx; (void)ABy; (void)ABz; (void)CDx; (void)CDy; (void)CDz; (void)src; (void)pidx;")
            th.append("  }")
        # the same outputs handed one by one to e(n, value) as they are formed (nothing held for all of them)
        th.append("  template <class E>")
        th.append("  __device__ static __forceinline__ void hrr_emit(const double* __restrict__ acc, "
                  "const int* __restrict__ src, int pidx, double w, double ABx, double ABy, double ABz, "
                  "double CDx, double CDy, double CDz, E& e) {")
        for line in t["hrr_emit"]:
            th.append("    " + line)
        th.append("    (void)ABx; (void)ABy; (void)ABz; (void)CDx; (void)CDy; (void)CDz; (void)src; (void)pidx;")
        th.append("  }")
        th.append("  __device__ static __forceinline__ void hrr(const double* __restrict__ acc, "
                  "const int* __restrict__ src, int pidx, double w, double ABx, double ABy, double ABz, "
                  "double CDx, double CDy, double CDz, double* __restrict__ out) {")
        for line in t["hrr"]:
            th.append("    " + line)
        th.append("    (void)ABx; (void)ABy; (void)ABz; (void)CDx; (void)CDy; (void)CDz; (void)src; (void)pidx;")
        th.append("  }")
        for P in range(3):
            th.append("  __device__ static __forceinline__ void digest%d(const double* __restrict__ out, "
                      "const double* __restrict__ d1, const double* __restrict__ d2, double* __restrict__ x, "
                      "double* __restrict__ y) {" % P)
            for line in t["digest"][P]:
                th.append("    " + line)
            th.append("  }")
        th.append("};")
        th.append("")
    _write(os.path.join(outdir, "eri_team.h"), "\n".join(th) + "\n")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                                "generated"))

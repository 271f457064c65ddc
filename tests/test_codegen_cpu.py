"""CPU check of the generated recursions (no GPU): the straight-line vertical and horizontal recursion statements
that gen_eri.py emits for the device are executed here in Python, for single-primitive shells, and compared with
the oracle (McMurchie-Davidson) after removing its primitive normalisation.  This catches generator mistakes (a
dropped term, a wrong index or coefficient) independently of the HIP compiler and the device."""
import importlib.util
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_1303_4916_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_spec = importlib.util.spec_from_file_location("gen_eri", os.path.join(ROOT, "paper_1303_4916_amd", "csrc",
                                                                       "gen_eri.py"))
gen = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(gen)


def _fma(a, b, c):
    return a * b + c


def _run_class(c, A, B, C, D, al, be, ga, de):
    la, lb, lc, ld = c
    v, es, fs, acc_lines = gen.gen_vrr(c)
    hrr_lines, _ = gen.gen_hrr(c, es, fs)
    z, e = al + be, ga + de
    P = (al * A + be * B) / z
    Q = (ga * C + de * D) / e
    ze = z + e
    rho = z * e / ze
    PQ = P - Q
    T = rho * float(PQ @ PQ)
    L = la + lb + lc + ld
    pref = (2 * math.pi ** 2.5 / (z * e * math.sqrt(ze)) * math.exp(-al * be / z * float((A - B) @ (A - B))) *
            math.exp(-ga * de / e * float((C - D) @ (C - D))))
    F = oracle.boys(L, T) * pref
    env = {"fma": _fma}
    for m in range(L + 1):
        env["F%d" % m] = F[m]
    for i, ax in enumerate("xyz"):
        env["PA" + ax] = P[i] - A[i]
        env["WP" + ax] = -(e / ze) * PQ[i]
        env["QC" + ax] = Q[i] - C[i]
        env["WQ" + ax] = (z / ze) * PQ[i]
        env["AB" + ax] = A[i] - B[i]
        env["CD" + ax] = C[i] - D[i]
    o2z, o2e, o2ze, roz, roe = 0.5 / z, 0.5 / e, 0.5 / ze, e / ze, z / ze
    for k in range(1, 9):
        env["oz%d" % k] = k * o2z
        env["ozr%d" % k] = k * o2z * roz
        env["oe%d" % k] = k * o2e
        env["oer%d" % k] = k * o2e * roe
        env["oze%d" % k] = k * o2ze
    nacc = len(es) * len(fs)
    env["acc"] = np.zeros(nacc)
    nout = gen.ncart(la) * gen.ncart(lb) * gen.ncart(lc) * gen.ncart(ld)
    env["out"] = np.zeros(nout)
    code = []
    for line in v.lines + acc_lines + hrr_lines:
        line = re.sub(r"^const (T|double) ", "", line).rstrip(";")
        line = line.replace("(double)", "")
        code.append(line)
    exec("\n".join(code), env)
    return env["out"].reshape(gen.ncart(la), gen.ncart(lb), gen.ncart(lc), gen.ncart(ld))


def _norm(a, comp):
    lx, ly, lz = comp
    l = lx + ly + lz
    df = lambda n: float(np.prod(np.arange(n, 0, -2))) if n > 0 else 1.0
    return (2 * a / math.pi) ** 0.75 * (4 * a) ** (l / 2) / math.sqrt(df(2 * lx - 1) * df(2 * ly - 1) * df(2 * lz - 1))


@pytest.mark.parametrize("c", gen.classes(), ids=gen.cname)
def test_generated_recursions_match_oracle(c):
    rng = np.random.default_rng(sum(x * 3 ** i for i, x in enumerate(c)) + 17)
    cen = rng.uniform(-1.5, 1.5, size=(4, 3))
    ex = np.exp(rng.uniform(math.log(0.2), math.log(6.0), size=4))
    sh = wl.Shells(np.array(c, np.int32), np.ones(4, np.int32), cen, ex, np.ones(4), np.arange(4, dtype=np.int32))
    ref = oracle.Basis(sh).eri(0, 1, 2, 3)
    raw = _run_class(c, *cen, *ex)
    comps = [gen.comps(l) for l in c]
    scale = np.einsum("i,j,k,l->ijkl", *[np.array([_norm(ex[s], cp) for cp in comps[s]]) for s in range(4)])
    got = raw * scale
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_flop_table_is_complete():
    import json
    t = json.load(open(os.path.join(ROOT, "paper_1303_4916_amd", "csrc", "generated", "eri_flops.json")))
    assert len(t) == 21
    for k, v in t.items():
        assert v["f_prim"] > 0 and v["f_contr"] >= 12 * v["nout"]

"""CPU emulation of the six-lane team evaluation generated for the largest classes (no GPU).

Each emulated lane p runs the generated representative recursion with its geometry vectors relabelled by the axis
permutation p, reads the values it needs from the other lanes as the device code does (source lane p o pi), and
digests its representative outputs in its own frame with densities gathered at permuted component indices.  The
test checks that (1) the owned outputs of the six lanes cover the true block exactly once and equal the oracle
(after removing the oracle's primitive normalisation), and (2) the per-lane digests, added at their true indices,
equal the digest of the oracle block."""
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


def _norm(a, comp):
    lx, ly, lz = comp
    l = lx + ly + lz
    df = lambda n: float(np.prod(np.arange(n, 0, -2))) if n > 0 else 1.0
    return (2 * a / math.pi) ** 0.75 * (4 * a) ** (l / 2) / math.sqrt(df(2 * lx - 1) * df(2 * ly - 1) * df(2 * lz - 1))


def _geometry(A, B, C, D, al, be, ga, de):
    z, e = al + be, ga + de
    P = (al * A + be * B) / z
    Q = (ga * C + de * D) / e
    ze = z + e
    PQ = P - Q
    T = z * e / ze * float(PQ @ PQ)
    pref = (2 * math.pi ** 2.5 / (z * e * math.sqrt(ze)) * math.exp(-al * be / z * float((A - B) @ (A - B))) *
            math.exp(-ga * de / e * float((C - D) @ (C - D))))
    return dict(PA=P - A, WP=-(e / ze) * PQ, QC=Q - C, WQ=(z / ze) * PQ, AB=A - B, CD=C - D, T=T, pref=pref,
                o2z=0.5 / z, o2e=0.5 / e, o2ze=0.5 / ze, roz=e / ze, roe=z / ze)


def _lane_env(geo, p, L):
    env = {"fma": _fma}
    F = oracle.boys(L, geo["T"]) * geo["pref"]
    for m in range(L + 1):
        env["F%d" % m] = F[m]
    for name in ("PA", "WP", "QC", "WQ", "AB", "CD"):
        V = geo[name]
        for i, ax in enumerate("xyz"):
            env[name + ax] = V[p[i]]  # geometry relabelled for lane p
    for k in range(1, 9):
        env["oz%d" % k] = k * geo["o2z"]
        env["ozr%d" % k] = k * geo["o2z"] * geo["roz"]
        env["oe%d" % k] = k * geo["o2e"]
        env["oer%d" % k] = k * geo["o2e"] * geo["roe"]
        env["oze%d" % k] = k * geo["o2ze"]
    return env


@pytest.mark.parametrize("c", gen.TEAM_CLASSES, ids=gen.cname)
def test_team_emulation_matches_oracle(c):
    la, lb, lc, ld = c
    t = gen.gen_team(c)
    rng = np.random.default_rng(sum(x * 3 ** i for i, x in enumerate(c)) + 99)
    cen = rng.uniform(-1.5, 1.5, size=(4, 3))
    ex = np.exp(rng.uniform(math.log(0.3), math.log(5.0), size=4))
    sh = wl.Shells(np.array(c, np.int32), np.ones(4, np.int32), cen, ex, np.ones(4), np.arange(4, dtype=np.int32))
    ref = oracle.Basis(sh).eri(0, 1, 2, 3)
    comps = [gen.comps(l) for l in c]
    scale = np.einsum("i,j,k,l->ijkl", *[np.array([_norm(ex[s], cp) for cp in comps[s]]) for s in range(4)])
    raw_ref = ref / scale
    geo = _geometry(*cen, *ex)
    L = la + lb + lc + ld
    # phase 1: every lane's representative accumulators
    vrr_code = "\n".join(re.sub(r"^const (T|double) ", "", x).rstrip(";").replace("(double)", "") for x in t["vrr"])
    accs = []
    for p in gen.PERMS:
        env = _lane_env(geo, p, L)
        env["acc"] = np.zeros(t["nrep"])
        exec(vrr_code, env)
        accs.append(env["acc"])
    # phase 2: per lane, the horizontal recursion on its representative outputs, with cross-lane reads
    comp_tab = [[gen.PERMS.index(gen.perm_compose(p, q)) for q in gen.PERMS] for p in gen.PERMS]
    na, nb, nc, nd = (len(x) for x in comps)
    covered = np.zeros((na, nb, nc, nd), dtype=int)
    got = np.zeros((na, nb, nc, nd))
    rngD = np.random.default_rng(5)
    N = na + nb + nc + nd
    Dm = rngD.standard_normal((N, N))
    Dm = Dm + Dm.T
    off = [0, na, na + nb, na + nb + nc]
    true_dig = {k: np.zeros(n) for k, n in [("jab", na * nb), ("jcd", nc * nd), ("kac", na * nc), ("kad", na * nd),
                                             ("kbc", nb * nc), ("kbd", nb * nd)]}
    pc_tab = gen.perm_comp_table()
    for ip, p in enumerate(gen.PERMS):
        env = _lane_env(geo, p, L)
        env["acc"] = accs[ip]
        env["src"] = comp_tab[ip]
        env["pidx"] = ip
        env["w"] = 1.0
        env["_acc"] = accs
        env["out"] = np.zeros(len(t["out_reps"]))
        code = []
        for line in t["hrr"]:
            line = re.sub(r"^const double ", "", line).rstrip(";")
            line = re.sub(r"fetch\(acc\[(\d+)\], src\[(\d+)\]\)", r"_acc[src[\2]][\1]", line)
            line = re.sub(r"\(\(\((\d+) >> pidx\) & 1\) \? w : 0\.0\)", r"(w if ((\1 >> pidx) & 1) else 0.0)", line)
            code.append(line)
        exec("\n".join(code), env)
        rec = env["out"]
        # map representative outputs to true components; owned ones only (a zero weight marks the others)
        pcs = [pc_tab[l][ip] for l in c]
        for n, (o, mask) in enumerate(zip(t["out_reps"], t["masks"])):
            if not (mask >> ip) & 1:
                assert rec[n] == 0.0
                continue
            idx = tuple(gen.comps(c[s]).index(gen.perm_q(o[s], p)) for s in range(4))
            covered[idx] += 1
            got[idx] = rec[n]
        # the generated digest passes, in the lane's frame, with densities gathered at permuted indices; their
        # partial blocks are added at the true indices (as the device does into LDS)
        D1 = lambda r, cc: Dm[r, cc]
        Pa, Pb, Pc, Pd = (lambda x: off[0] + pcs[0][x]), (lambda x: off[1] + pcs[1][x]), \
            (lambda x: off[2] + pcs[2][x]), (lambda x: off[3] + pcs[3][x])
        slices = [
            (np.array([D1(Pc(k), Pd(l)) for k in range(nc) for l in range(nd)]),
             np.array([D1(Pa(i), Pb(j)) for i in range(na) for j in range(nb)]),
             ("jab", na, nb, 0, 1), ("jcd", nc, nd, 2, 3)),
            (np.array([D1(Pb(j), Pd(l)) for j in range(nb) for l in range(nd)]),
             np.array([D1(Pa(i), Pc(k)) for i in range(na) for k in range(nc)]),
             ("kac", na, nc, 0, 2), ("kbd", nb, nd, 1, 3)),
            (np.array([D1(Pb(j), Pc(k)) for j in range(nb) for k in range(nc)]),
             np.array([D1(Pa(i), Pd(l)) for i in range(na) for l in range(nd)]),
             ("kad", na, nd, 0, 3), ("kbc", nb, nc, 1, 2)),
        ]
        for P, (d1, d2, xs, ys) in enumerate(slices):
            penv = {"fma": _fma, "out": rec, "d1": d1, "d2": d2, "x": np.full(xs[1] * xs[2], np.nan),
                    "y": np.full(ys[1] * ys[2], np.nan)}
            exec("\n".join(x.rstrip(";") for x in t["digest"][P]), penv)
            assert not np.any(np.isnan(penv["x"])) and not np.any(np.isnan(penv["y"]))
            for arr, (name, n1, n2, s1, s2) in ((penv["x"], xs), (penv["y"], ys)):
                for u in range(n1):
                    for v_ in range(n2):
                        tu, tv = pcs[s1][u], pcs[s2][v_]
                        true_dig[name][tu * n2 + tv] += arr[u * n2 + v_]
    assert np.all(covered == 1)
    assert np.max(np.abs(got - raw_ref)) <= 1e-12 * np.max(np.abs(raw_ref))
    # reference digest of the full true block
    v = raw_ref
    Dab, Dcd = Dm[off[0]:off[0] + na, off[1]:off[1] + nb], Dm[off[2]:off[2] + nc, off[3]:off[3] + nd]
    Dbd, Dbc = Dm[off[1]:off[1] + nb, off[3]:off[3] + nd], Dm[off[1]:off[1] + nb, off[2]:off[2] + nc]
    Dad, Dac = Dm[off[0]:off[0] + na, off[3]:off[3] + nd], Dm[off[0]:off[0] + na, off[2]:off[2] + nc]
    refd = {"jab": np.einsum("ijkl,kl->ij", v, Dcd).ravel(), "jcd": np.einsum("ijkl,ij->kl", v, Dab).ravel(),
            "kac": np.einsum("ijkl,jl->ik", v, Dbd).ravel(), "kad": np.einsum("ijkl,jk->il", v, Dbc).ravel(),
            "kbc": np.einsum("ijkl,il->jk", v, Dad).ravel(), "kbd": np.einsum("ijkl,ik->jl", v, Dac).ravel()}
    for k in refd:
        assert np.max(np.abs(true_dig[k] - refd[k])) <= 1e-12 * max(np.max(np.abs(refd[k])), 1e-300), k


def _stream_lds_python(lines):
    """The generated LDS streaming digest as Python: atomic_add_lds(t_X + i, v) adds v into block X at i."""
    out = []
    for line in lines:
        s = line.strip()
        if s.startswith("{ const double x = "):
            out.append("x = " + s[len("{ const double x = "):].rstrip(";"))
        elif s.startswith("const int ij = "):
            out += [a.strip() for a in s[len("const int "):].rstrip(";").split(", ")]
        elif "atomic_add_lds" in s:
            cond = s.startswith("if constexpr (WITH_J)")
            calls = re.findall(r"atomic_add_lds\(t_(\w+) \+ (\w+), ([^;]*)\);", s)
            assert calls, s
            for blk, idx, val in calls:
                out.append(("if WITH_J: " if cond else "") + "_add('%s', %s, %s)" % (blk, idx, val))
        else:
            s = re.sub(r"^const double ", "", s).rstrip(";")
            out.append(s)
    code = "\n".join(out)
    code = re.sub(r"fetch\(acc\[(\d+)\], src\[(\d+)\]\)", r"_acc[src[\2]][\1]", code)
    code = re.sub(r"\(\(\((\d+) >> pidx\) & 1\) \? w : 0\.0\)", r"(w if ((\1 >> pidx) & 1) else 0.0)", code)
    return code


@pytest.mark.parametrize("c", sorted(gen.TEAM_STREAM_DIGEST), ids=gen.cname)
@pytest.mark.parametrize("with_j", [True, False])
def test_team_stream_lds_digest_matches_oracle(c, with_j):
    """The streaming digest that reads the team's density slices from, and adds its contributions into, shared
    true-index blocks (LDS on the device): the six lanes' contributions equal the digest of the oracle block."""
    la, lb, lc, ld = c
    t = gen.gen_team(c)
    rng = np.random.default_rng(sum(x * 3 ** i for i, x in enumerate(c)) + 7)
    cen = rng.uniform(-1.5, 1.5, size=(4, 3))
    ex = np.exp(rng.uniform(math.log(0.3), math.log(5.0), size=4))
    sh = wl.Shells(np.array(c, np.int32), np.ones(4, np.int32), cen, ex, np.ones(4), np.arange(4, dtype=np.int32))
    ref = oracle.Basis(sh).eri(0, 1, 2, 3)
    comps = [gen.comps(l) for l in c]
    scale = np.einsum("i,j,k,l->ijkl", *[np.array([_norm(ex[s], cp) for cp in comps[s]]) for s in range(4)])
    v = ref / scale
    geo = _geometry(*cen, *ex)
    L = la + lb + lc + ld
    vrr_code = "\n".join(re.sub(r"^const (T|double) ", "", x).rstrip(";").replace("(double)", "") for x in t["vrr"])
    accs = []
    for p in gen.PERMS:
        env = _lane_env(geo, p, L)
        env["acc"] = np.zeros(t["nrep"])
        exec(vrr_code, env)
        accs.append(env["acc"])
    na, nb, nc, nd = (len(x) for x in comps)
    Dm = np.random.default_rng(11).standard_normal((na + nb + nc + nd,) * 2)
    Dm = Dm + Dm.T
    o = [0, na, na + nb, na + nb + nc]
    blk = lambda s1, n1, s2, n2: Dm[o[s1]:o[s1] + n1, o[s2]:o[s2] + n2]
    S = {"s_ab": blk(0, na, 1, nb).ravel(), "s_cd": blk(2, nc, 3, nd).ravel(), "s_ac": blk(0, na, 2, nc).ravel(),
         "s_ad": blk(0, na, 3, nd).ravel(), "s_bc": blk(1, nb, 2, nc).ravel(), "s_bd": blk(1, nb, 3, nd).ravel()}
    tot = {k: np.zeros(n) for k, n in [("jab", na * nb), ("jcd", nc * nd), ("kac", na * nc), ("kad", na * nd),
                                        ("kbc", nb * nc), ("kbd", nb * nd)]}

    def _add(name, i, val):
        tot[name][i] += val

    comp_tab = [[gen.PERMS.index(gen.perm_compose(p, q)) for q in gen.PERMS] for p in gen.PERMS]
    pc_tab = gen.perm_comp_table()
    code = _stream_lds_python(t["hrr_digest_lds"])
    for ip, p in enumerate(gen.PERMS):
        env = _lane_env(geo, p, L)
        env.update(S)
        env.update(acc=accs[ip], src=comp_tab[ip], pidx=ip, w=1.0, _acc=accs, _add=_add, WITH_J=with_j,
                   pA=pc_tab[la][ip], pB=pc_tab[lb][ip], pC=pc_tab[lc][ip], pD=pc_tab[ld][ip])
        exec(code, env)
    refd = {"jab": np.einsum("ijkl,kl->ij", v, S["s_cd"].reshape(nc, nd)).ravel(),
            "jcd": np.einsum("ijkl,ij->kl", v, S["s_ab"].reshape(na, nb)).ravel(),
            "kac": np.einsum("ijkl,jl->ik", v, S["s_bd"].reshape(nb, nd)).ravel(),
            "kad": np.einsum("ijkl,jk->il", v, S["s_bc"].reshape(nb, nc)).ravel(),
            "kbc": np.einsum("ijkl,il->jk", v, S["s_ad"].reshape(na, nd)).ravel(),
            "kbd": np.einsum("ijkl,ik->jl", v, S["s_ac"].reshape(na, nc)).ravel()}
    for k in refd:
        if not with_j and k in ("jab", "jcd"):
            assert not np.any(tot[k]), k
            continue
        assert np.max(np.abs(tot[k] - refd[k])) <= 1e-12 * max(np.max(np.abs(refd[k])), 1e-300), k


@pytest.mark.parametrize("c", gen.TEAM_CLASSES, ids=gen.cname)
def test_team_emit_stores_match_oracle(c):
    """The per-output form used for the MP2 batch stores (hrr_emit): each lane hands every representative output to
    e(n, value) as it is formed; the device stores the nonzero ones at the true components of the frame indices
    OUT_IDX[n] (the order of out_reps).  Emulated for the six lanes: the stored elements cover the true block once,
    with the oracle's values, and the copies of the non-owning lanes are zero."""
    la, lb, lc, ld = c
    t = gen.gen_team(c)
    rng = np.random.default_rng(sum(x * 5 ** i for i, x in enumerate(c)) + 7)
    cen = rng.uniform(-1.5, 1.5, size=(4, 3))
    ex = np.exp(rng.uniform(math.log(0.3), math.log(5.0), size=4))
    sh = wl.Shells(np.array(c, np.int32), np.ones(4, np.int32), cen, ex, np.ones(4), np.arange(4, dtype=np.int32))
    ref = oracle.Basis(sh).eri(0, 1, 2, 3)
    comps = [gen.comps(l) for l in c]
    scale = np.einsum("i,j,k,l->ijkl", *[np.array([_norm(ex[s], cp) for cp in comps[s]]) for s in range(4)])
    raw_ref = ref / scale
    geo = _geometry(*cen, *ex)
    L = la + lb + lc + ld
    vrr_code = "\n".join(re.sub(r"^const (T|double) ", "", x).rstrip(";").replace("(double)", "") for x in t["vrr"])
    accs = []
    for p in gen.PERMS:
        env = _lane_env(geo, p, L)
        env["acc"] = np.zeros(t["nrep"])
        exec(vrr_code, env)
        accs.append(env["acc"])
    comp_tab = [[gen.PERMS.index(gen.perm_compose(p, q)) for q in gen.PERMS] for p in gen.PERMS]
    pc_tab = gen.perm_comp_table()
    # the frame component indices the generator writes as OUT_IDX
    out_idx = [tuple(comps[s].index(o[s]) for s in range(4)) for o in t["out_reps"]]
    code = []
    for line in t["hrr_emit"]:
        line = re.sub(r"^const double ", "", line).rstrip(";")
        line = re.sub(r"fetch\(acc\[(\d+)\], src\[(\d+)\]\)", r"_acc[src[\2]][\1]", line)
        line = re.sub(r"\(\(\((\d+) >> pidx\) & 1\) \? w : 0\.0\)", r"(w if ((\1 >> pidx) & 1) else 0.0)", line)
        code.append(line)
    assert sum(1 for x in code if x.startswith("e(")) == len(t["out_reps"])
    written = np.zeros(raw_ref.shape, dtype=int)
    got = np.zeros(raw_ref.shape)
    for ip, p in enumerate(gen.PERMS):
        env = _lane_env(geo, p, L)
        env.update({"acc": accs[ip], "src": comp_tab[ip], "pidx": ip, "w": 1.0, "_acc": accs})
        pcs = [pc_tab[l][ip] for l in c]
        seen = []

        def e(n, v, ip=ip, pcs=pcs, seen=seen):
            seen.append(n)
            owner = (t["masks"][n] >> ip) & 1
            if not owner:
                assert v == 0.0
            if v == 0.0:  # not stored (the buffer is zero beforehand)
                return
            idx = tuple(pcs[s][out_idx[n][s]] for s in range(4))
            written[idx] += 1
            got[idx] = v

        env["e"] = e
        exec("\n".join(code), env)
        assert seen == list(range(len(t["out_reps"])))
    tol = 1e-12 * np.max(np.abs(raw_ref))
    assert np.all(written <= 1)
    assert np.all((written == 1) | (np.abs(raw_ref) <= tol))  # an element never stored is a vanishing integral
    assert np.max(np.abs(got - raw_ref)) <= tol


def test_generated_headers_are_current(tmp_path):
    """The committed generated headers (recursions, team forms with their OUT_IDX tables, FLOP tables) are what
    the generator writes now, byte for byte."""
    gen.main(str(tmp_path))
    made = sorted(os.listdir(tmp_path))
    assert made
    for name in made:
        with open(os.path.join(tmp_path, name), "rb") as f:
            new = f.read()
        with open(os.path.join(ROOT, "paper_1303_4916_amd", "csrc", "generated", name), "rb") as f:
            assert f.read() == new, name

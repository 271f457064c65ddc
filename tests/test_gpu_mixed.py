"""GPU parity of the mixed-precision path (FP32 primitive recursions, FP64 contraction and J/K accumulation) against
the CPU oracle and against the FP64 GPU path, through the C ABI.

Bounds (the oracle evaluates every integral in FP64 with a long-double Boys function):
* ERI blocks with every primitive recursion in FP32 (uqc_eri_blocks with UQC_MIXED; no FP64 routing): largest
  absolute error 2e-6 (integrals of the tightest core shells reach about 10, FP32 carries 6e-8 relative), and per
  element |ERI_mixed - ERI_oracle| <= 5e-3 Q_ab Q_cd + 1e-12, with Q_ab Q_cd the Schwarz bound of the quartet
  (|(ij|kl)| <= Q_ab Q_cd).  The bound relative to Q_ab Q_cd is loose because the horizontal recursion, run in FP64
  on the contracted FP32 results, amplifies their rounding by about |AB|^l_b |CD|^l_d: for distant d-shell pairs
  it reaches 1e-3 (measured on this sample: 1.5e-3 at Q_ab Q_cd = 8e-9).  This is why the Fock build routes every
  quartet with Q_ab Q_cd above a bound (1e-8 by default) to FP64; the FP32 ones then move J and K by at most
  5e-3 x 1e-8 each.  The 1e-12 floor covers integrals far below the screening threshold, whose FP32 intermediates
  fall out of FP32's range.
* Fock builds with the default routing (and 1e-6): |E2_mixed - E2_fp64| <= 1e-6 Eh (the benchmark's energy
  criterion) and the same against the oracle; ||G_mixed - G_fp64||_F / ||G_fp64||_F <= 1e-7; max |G_mixed -
  G_fp64| <= 1e-5; J, K, G within 1e-6 of each matrix's largest element against the oracle's definition of Eq. (12).
* Every quartet in FP32 (routing bound 1): the energy criterion does not hold (measured |dE2| 2.1e-6 Eh at 12
  atoms), which is the reason for the routing; the test bounds it at 1e-5 Eh and 1e-4 relative in J, K, G.
"""
import numpy as np
import pytest

import oracle
from paper_1303_4916_amd import uqc
from paper_1303_4916_amd import workloads as wl

pytestmark = pytest.mark.gpu

CLASSES = [(la, lb, lc, ld) for la in range(3) for lb in range(la + 1) for lc in range(3) for ld in range(lc + 1)
           if (la, lb) >= (lc, ld)]
ERI_REL_SCHWARZ = 5e-3
ERI_ABS = 2e-6
ERI_FLOOR = 1e-12
E2_BOUND = 1e-6
G_FROB = 1e-7
G_MAX = 1e-5


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = uqc.Context(0)
    yield c
    c.close()


def class_sample(l, rng, per_class, pair_index):
    """Uniform sample of canonical quartets (a >= b, c >= d, (ab) >= (cd) in pair order) of every class: shells of
    the class's angular momenta drawn at random, then each pair and the two pairs put in canonical order."""
    by_l = [np.flatnonzero(l == x) for x in range(3)]
    out = []
    for (la, lb, lc, ld) in CLASSES:
        for _ in range(per_class):
            a, b, c, d = (int(rng.choice(by_l[x])) for x in (la, lb, lc, ld))
            if la == lb and b > a:
                a, b = b, a
            if lc == ld and d > c:
                c, d = d, c
            if (la, lb) == (lc, ld) and pair_index(c, d) > pair_index(a, b):
                a, b, c, d = c, d, a, b
            out.append((a, b, c, d))
    return np.array(out, dtype=np.int32)


def compact_sample(sh, rng, per_class):
    """Quartets of every class whose four shells sit on one atom or on two neighbouring atoms (the largest
    integrals, where an FP32 error is largest in absolute terms)."""
    atoms = sh.atom
    pos = np.array([sh.center[np.flatnonzero(atoms == i)[0]] for i in range(int(atoms.max()) + 1)])
    out = []
    for (la, lb, lc, ld) in CLASSES:
        for _ in range(per_class):
            i = int(rng.integers(0, len(pos)))
            dist = np.linalg.norm(pos - pos[i], axis=1)
            near = np.flatnonzero(dist < 3.2)
            q = []
            for x in (la, lb, lc, ld):
                at = int(rng.choice(near))
                q.append(int(rng.choice(np.flatnonzero((atoms == at) & (sh.l == x)))))
            out.append(tuple(q))
    return np.array(out, dtype=np.int32)


def test_mixed_eri_blocks_sampled_vs_oracle(ctx):
    """150-atom lattice (first s shell K = 6): 100 uniformly drawn canonical quartets of each of the 21 classes plus
    20 compact ones per class, every recursion in FP32, element by element against the oracle; the FP64 path on the
    same quartets at the FP64 bound."""
    w = wl.mixed150(ndens=1)
    sh = w.shells
    B = uqc.Basis(ctx, sh)
    O = oracle.Basis(sh)
    Q = B.schwarz()
    rng = np.random.default_rng(31)
    q = np.concatenate([class_sample(sh.l, rng, 100, lambda x, y: x * (x + 1) // 2 + y),
                        compact_sample(sh, rng, 20)])
    assert len(q) >= 2100 and len({tuple(sorted(sh.l[list(x)])) for x in q}) >= 15
    mixed = B.eri_blocks(q, uqc.MIXED)
    fp64 = B.eri_blocks(q, uqc.FP64)
    rel, absd, f64 = [], [], []
    for (a, b, c, d), m, f in zip(q, mixed, fp64):
        ref = O.eri(int(a), int(b), int(c), int(d))
        err = float(np.max(np.abs(m - ref)))
        absd.append(err)
        rel.append(max(err - ERI_FLOOR, 0.0) / max(Q[a, b] * Q[c, d], 1e-300))
        f64.append(float(np.max(np.abs(f - ref))) / max(float(np.max(np.abs(ref))), 1e-4))
    rel, absd = np.array(rel), np.array(absd)
    worst = np.argsort(rel)[::-1][:5]
    print("mixed ERI sample: %d quartets, max |dERI| %.3e, |dERI|/(Q_ab Q_cd): max %.3e, 99%% %.3e, median %.3e; "
          "FP64 max rel %.3e; worst %s" % (
              len(q), absd.max(), rel.max(), np.percentile(rel, 99), np.median(rel), max(f64),
              [(tuple(int(x) for x in q[i]), tuple(int(sh.l[x]) for x in q[i]), float(absd[i]),
                float(Q[q[i][0], q[i][1]] * Q[q[i][2], q[i][3]])) for i in worst]))
    assert max(f64) <= 1e-10
    assert absd.max() <= ERI_ABS
    assert rel.max() <= ERI_REL_SCHWARZ, (q[int(np.argmax(rel))], rel.max())


@pytest.fixture(scope="module")
def small_lattice(ctx):
    """12 atoms with a K = 6 core s shell, tau = 1e-12: the oracle's J, K, G and E2 and the FP64 GPU build."""
    w = wl.lattice(12, seed=41, ndens=1, tau=1e-12, k_s_core=6)
    B = uqc.Basis(ctx, w.shells)
    D = w.densities[0]
    Jr, Kr, _ = oracle.Basis(w.shells).jk_symmetric([D], tau=w.tau)
    Gr, E2r = oracle.fock_parts(Jr[0], Kr[0], D)
    return w, B, (Jr[0], Kr[0], Gr, E2r), B.fock_build(D, uqc.default_opts(tau=w.tau))


@pytest.mark.parametrize("bound", [1e-8, 1e-6, 1.0])
def test_mixed_fock_small_lattice_vs_oracle(small_lattice, bound):
    """The closed-shell mixed build (whole quartets in FP64 above the bound; 1.0 leaves almost every quartet in
    FP32) against the oracle's J, K, G and E2 and against the FP64 build."""
    w, B, (Jr, Kr, Gr, E2r), (J6, K6, G6, st6) = small_lattice
    D = w.densities[0]
    J, K, G, st = B.fock_build(D, uqc.default_opts(tau=w.tau, precision=uqc.MIXED, fp64_bound=bound))
    rel = {n: float(np.max(np.abs(x - r)) / np.max(np.abs(r))) for n, x, r in (("J", J, Jr), ("K", K, Kr),
                                                                                ("G", G, Gr))}
    print("bound %g: FP64 quartets %d of %d, |dE2| vs oracle %.3e, vs FP64 %.3e, max rel dJ/dK/dG %s" % (
        bound, st.fp64_quartets, st.quartets, abs(st.E2 - E2r), abs(st.E2 - st6.E2), rel))
    assert st.fp64_quartets < st.quartets and st.quartets == st6.quartets
    if bound >= 1.0:
        assert st.fp64_quartets <= 0.01 * st.quartets
    if bound >= 1.0:  # every quartet in FP32: outside the energy criterion, bounded loosely
        assert max(rel.values()) <= 1e-4
        assert abs(st.E2 - E2r) <= 1e-5 and abs(st.E2 - st6.E2) <= 1e-5
        return
    assert max(rel.values()) <= 1e-6
    assert abs(st.E2 - E2r) <= E2_BOUND, (st.E2, E2r)
    assert abs(st.E2 - st6.E2) <= E2_BOUND
    assert np.linalg.norm(G - G6) <= G_FROB * np.linalg.norm(G6)
    assert np.max(np.abs(G - G6)) <= G_MAX


@pytest.mark.parametrize("boys_t", [0.0, 10.0, 30.0])
def test_mixed_fock_boys_cutoff_option(small_lattice, boys_t):
    """fp64_boys_T moves the FP32/FP64 split of the Boys evaluation (0: every Boys argument in FP64, 30: the FP32
    table's whole range); at every setting the mixed build meets the same bounds against the oracle and the FP64
    build, and a setting below 30 changes the result (it takes effect)."""
    w, B, (Jr, Kr, Gr, E2r), (J6, K6, G6, st6) = small_lattice
    D = w.densities[0]
    J, K, G, st = B.fock_build(D, uqc.default_opts(tau=w.tau, precision=uqc.MIXED, fp64_boys_T=boys_t))
    assert abs(st.E2 - E2r) <= E2_BOUND and abs(st.E2 - st6.E2) <= E2_BOUND
    assert np.linalg.norm(G - G6) <= G_FROB * np.linalg.norm(G6)
    assert np.max(np.abs(G - Gr)) <= 1e-6 * np.max(np.abs(Gr))
    if boys_t < 30.0:
        _, _, G30, _ = B.fock_build(D, uqc.default_opts(tau=w.tau, precision=uqc.MIXED))
        assert np.any(G != G30)


@pytest.mark.parametrize("boys_t", [-1.0, 30.5, float("nan")])
def test_mixed_fock_boys_cutoff_out_of_range(small_lattice, boys_t):
    w, B, _, _ = small_lattice
    with pytest.raises(uqc.UqcError) as e:
        B.fock_build(w.densities[0], uqc.default_opts(tau=w.tau, precision=uqc.MIXED, fp64_boys_T=boys_t))
    assert e.value.status == uqc.UQC_E_ARG and "fp64_boys_T" in str(e.value)


@pytest.fixture(scope="module")
def mixed150(ctx):
    """150 atoms, N = 1650, first s shell K = 6, tau = 1e-12: one FP64 and one mixed build of the same density."""
    import torch
    w = wl.mixed150(ndens=1)
    B = uqc.Basis(ctx, w.shells)
    D = torch.from_numpy(w.densities[0]).cuda()
    out = {}
    for name, prec in (("fp64", uqc.FP64), ("mixed", uqc.MIXED)):
        J, K, G, st = B.fock_build(D, uqc.default_opts(tau=w.tau, precision=prec))
        out[name] = (J.cpu().numpy(), K.cpu().numpy(), G.cpu().numpy(), st)
    return w, B, out


def test_mixed_fock_150_atoms_vs_fp64(mixed150):
    w, B, out = mixed150
    J6, K6, G6, s6 = out["fp64"]
    Jm, Km, Gm, sm = out["mixed"]
    assert sm.quartets == s6.quartets and sm.fp64_quartets < sm.quartets
    assert abs(sm.E2 - s6.E2) <= E2_BOUND, (sm.E2, s6.E2)
    assert np.linalg.norm(Gm - G6) <= G_FROB * np.linalg.norm(G6)
    assert np.max(np.abs(Gm - G6)) <= G_MAX
    print("150 atoms: E2 %.10f, |dE2| %.3e Eh, |dG|_F/|G|_F %.3e, max|dG| %.3e, FP64 quartets %d of %d" % (
        s6.E2, abs(sm.E2 - s6.E2), np.linalg.norm(Gm - G6) / np.linalg.norm(G6), np.max(np.abs(Gm - G6)),
        sm.fp64_quartets, sm.quartets))


def test_fock_150_atoms_sampled_blocks_vs_oracle(mixed150):
    """At the full 150-atom size, J and K shell blocks of both builds, one or two per pair class, recomputed one by
    one by the oracle's definition of Eq. (12) with the same screening: FP64 within 1e-10 and mixed within 1e-6 of
    the matrix's largest element."""
    w, B, out = mixed150
    O = oracle.Basis(w.shells)
    D = w.densities[0]
    off = B.offsets
    rng = np.random.default_rng(151)
    l = w.shells.l
    picks = []
    for (la, lb) in [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)]:
        picks.append((int(rng.choice(np.flatnonzero(l == la))), int(rng.choice(np.flatnonzero(l == lb)))))
    for (a, b) in picks:
        na, nb = oracle.ncart(int(l[a])), oracle.ncart(int(l[b]))
        jb = O.j_block(D, a, b, tau=w.tau)
        kb = O.k_block(D, a, b, tau=w.tau)
        for name, tol in (("fp64", 1e-10), ("mixed", 1e-6)):
            J, K, _, _ = out[name]
            assert np.max(np.abs(J[off[a]:off[a] + na, off[b]:off[b] + nb] - jb)) <= tol * np.max(np.abs(J)), (
                name, "J", a, b)
            assert np.max(np.abs(K[off[a]:off[a] + na, off[b]:off[b] + nb] - kb)) <= tol * np.max(np.abs(K)), (
                name, "K", a, b)

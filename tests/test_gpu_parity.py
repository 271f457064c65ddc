"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Tolerance (FP64 mode): norm-wise relative error max|GPU - oracle| / max|oracle| <= 1e-10 per ERI block and per J,
K, G matrix, with an absolute floor of 1e-14 for blocks whose largest element is below 1e-4 (elementwise relative
error is ill-posed for elements near zero).  The oracle shares no code with the HIP path; both read the same seeded
inputs from paper_1303_4916_amd.workloads.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1303_4916_amd import uqc
from paper_1303_4916_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-10


def close(got, ref, tol=TOL, floor=1e-14):
    m = float(np.max(np.abs(ref))) if np.size(ref) else 0.0
    err = float(np.max(np.abs(np.asarray(got) - np.asarray(ref)))) if np.size(ref) else 0.0
    bound = tol * m if m >= 1e-4 else max(tol * m, floor)
    return err <= bound, err, m


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = uqc.Context(0)
    yield c
    c.close()


# ----------------------------------------------------------------------------------------------- Boys function
def test_boys_fp64_matches_oracle(ctx):
    T = np.concatenate([[0.0, 1e-12, 1e-6, 0.05, 0.0499999, 0.1, 39.9, 39.95, 39.9999, 40.0, 40.0001, 41.0, 55.0,
                         120.0, 700.0, 1e4], np.linspace(0, 45, 2001)])
    got = ctx.boys(T, 8, uqc.FP64)
    ref = np.array([oracle.boys(8, t) for t in T])
    rel = np.max(np.abs(got - ref) / ref)
    assert rel <= 5e-14, rel


@pytest.mark.parametrize("mmax", range(9))
def test_boys_fp64_every_order_around_its_asymptotic_cut(ctx, mmax):
    # the order-L evaluation switches to the asymptotic form at T_L = 37, 41, ..., 60 (L = 0..8)
    cut = [37, 41, 44, 47, 50, 53, 55, 58, 60][mmax]
    T = np.concatenate([np.linspace(0, 70, 1401), cut + np.array([-1e-9, -1e-6, -0.01, 0.0, 1e-9, 1e-6, 0.01, 0.5])])
    got = ctx.boys(T, mmax, uqc.FP64)
    ref = np.array([oracle.boys(mmax, t) for t in T])
    rel = np.max(np.abs(got - ref) / ref)
    assert rel <= 5e-14, rel


def test_boys_fp64_asymptotic_is_exact_to_rounding(ctx):
    # beyond T_0 = 37, F_0(T) = sqrt(pi / T) / 2 to well below double rounding (erfc(sqrt(37)) ~ 1e-17): this pins
    # the device reciprocal square root (hardware estimate + one third-order step) to a few rounding errors
    T = np.geomspace(37.0, 1e8, 4001)
    got = ctx.boys(T, 0, uqc.FP64)[:, 0]
    ref = np.sqrt(np.pi / T) / 2
    rel = np.max(np.abs(got - ref) / ref)
    assert rel <= 1e-15, rel


def test_boys_fp32_matches_oracle(ctx):
    T = np.linspace(0, 30, 3001)
    got = ctx.boys(T, 8, uqc.MIXED)
    ref = np.array([oracle.boys(8, t) for t in T])
    rel = np.max(np.abs(got - ref) / ref)
    assert rel <= 2e-6, rel


# ----------------------------------------------------------------------------------------------- ERI blocks
CLASSES = [(la, lb, lc, ld) for la in range(3) for lb in range(la + 1) for lc in range(3) for ld in range(lc + 1)
           if (la, lb) >= (lc, ld)]


@pytest.mark.parametrize("ls", CLASSES, ids=lambda x: "".join("spd"[i] for i in x))
def test_eri_block_every_class(ctx, ls):
    sh = wl.random_quartet_shells(200 + sum(v * 3 ** i for i, v in enumerate(ls)), ls, k=3)
    B = uqc.Basis(ctx, sh)
    O = oracle.Basis(sh)
    for q in [(0, 1, 2, 3), (1, 0, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0), (0, 1, 0, 1), (2, 2, 3, 3), (0, 0, 0, 0)]:
        ok, err, m = close(B.eri_block(*q), O.eri(*q))
        assert ok, (q, err, m)


def test_full_tensor_cube(ctx):
    w = wl.cube()
    B = uqc.Basis(ctx, w.shells)
    O = oracle.Basis(w.shells)
    T = B.eri_tensor()
    R = O.eri_tensor()
    ok, err, m = close(T, R)
    assert ok, (err, m)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1)]:
        assert np.max(np.abs(T - T.transpose(perm))) <= 1e-13 * m


# ------------------------------------------------------------------------------------ Rys quadrature (UQC_RYS)
@pytest.mark.parametrize("ls", CLASSES, ids=lambda x: "".join("spd"[i] for i in x))
def test_eri_block_every_class_rys(ctx, ls):
    """The same blocks by Rys quadrature (the paper's method) against the oracle's McMurchie-Davidson integrals."""
    sh = wl.random_quartet_shells(200 + sum(v * 3 ** i for i, v in enumerate(ls)), ls, k=3)
    B = uqc.Basis(ctx, sh)
    O = oracle.Basis(sh)
    for q in [(0, 1, 2, 3), (1, 0, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0), (0, 1, 0, 1), (2, 2, 3, 3), (0, 0, 0, 0)]:
        ok, err, m = close(B.eri_block(*q, precision=uqc.RYS), O.eri(*q))
        assert ok, (q, err, m)


def test_full_tensor_cube_rys(ctx):
    w = wl.cube()
    B = uqc.Basis(ctx, w.shells)
    T = B.eri_tensor(precision=uqc.RYS)
    ok, err, m = close(T, oracle.Basis(w.shells).eri_tensor())
    assert ok, (err, m)
    # both GPU methods on a lattice with distant pairs (large T: the asymptotic rule)
    sh = wl.lattice(6, seed=12, ndens=1).shells
    B2 = uqc.Basis(ctx, sh)
    rng = np.random.default_rng(3)
    q = rng.integers(0, B2.nshell, size=(400, 4)).astype(np.int32)
    for x, y in zip(B2.eri_blocks(q, uqc.FP64), B2.eri_blocks(q, uqc.RYS)):
        ok, err, m = close(y, x)
        assert ok, (err, m)


def test_schwarz_bounds(ctx):
    w = wl.lattice(6, seed=12, ndens=1)
    B = uqc.Basis(ctx, w.shells)
    O = oracle.Basis(w.shells)
    q1, q2 = B.schwarz(), O.schwarz()
    assert np.max(np.abs(q1 - q2)) <= 1e-12 * np.max(q2)


# ----------------------------------------------------------------------------------------------- Fock builds
def _check_fock(B, O, D, tau, J, K, G, st):
    Jr, Kr = O.jk_direct([D], tau=tau) if B.nshell <= 24 else O.jk_symmetric([D], tau=tau)[:2]
    Jr, Kr = Jr[0], Kr[0]
    Gr, E2r = oracle.fock_parts(Jr, Kr, D)
    for got, ref, name in [(J, Jr, "J"), (K, Kr, "K"), (G, Gr, "G")]:
        ok, err, m = close(got, ref)
        assert ok, (name, err, m)
    assert abs(st.E2 - E2r) <= 1e-10 * abs(E2r)


def test_fock_cube_unscreened(ctx):
    w = wl.cube()
    B = uqc.Basis(ctx, w.shells)
    O = oracle.Basis(w.shells)
    D = w.densities[0]
    J, K, G, st = B.fock_build(D, uqc.default_opts(tau=0.0))
    assert st.quartets == 9316 and st.quartets_screened == 0
    _check_fock(B, O, D, 0.0, J, K, G, st)


@pytest.mark.parametrize("natoms,seed,tau", [(5, 21, 1e-12), (9, 22, 1e-10), (12, 23, 1e-12)])
def test_fock_lattice_screened(ctx, natoms, seed, tau):
    w = wl.lattice(natoms, seed=seed, ndens=2, tau=tau)
    B = uqc.Basis(ctx, w.shells)
    O = oracle.Basis(w.shells)
    for D in w.densities:
        J, K, G, st = B.fock_build(D, uqc.default_opts(tau=tau))
        _check_fock(B, O, D, tau, J, K, G, st)


def test_fock_device_pointers_match_host(ctx):
    import torch
    w = wl.lattice(6, seed=31, ndens=1)
    B = uqc.Basis(ctx, w.shells)
    D = w.densities[0]
    J, K, G, st = B.fock_build(D)
    Dt = torch.from_numpy(D).cuda()
    Jt, Kt, Gt, st2 = B.fock_build(Dt)
    torch.cuda.synchronize()
    for a, b in [(J, Jt), (K, Kt), (G, Gt)]:
        ok, err, m = close(b.cpu().numpy(), a, tol=1e-13)
        assert ok, (err, m)
    assert abs(st.E2 - st2.E2) <= 1e-13 * abs(st.E2)


@pytest.mark.parametrize("streams", [1, 3])
def test_fock_split_launches_and_progress(ctx, streams):
    """Class launches split into many small ones (7 work items each, ragged ends) give the same J, K, G as single
    launches; the progress report reaches every class's item total, in increasing steps, with the class launches on
    one stream (a wait after each) and on three (reports after all are queued)."""
    w = wl.lattice(9, seed=35, ndens=1, tau=1e-12)
    B = uqc.Basis(ctx, w.shells)
    O = oracle.Basis(w.shells)
    D = w.densities[0]
    J1, K1, G1, st1 = B.fock_build(D, uqc.default_opts(tau=1e-12))
    seen = {}

    def report(cid, done, total):
        prev = seen.get(cid, (0, total))
        assert prev[1] == total and done > prev[0] and done <= total
        seen[cid] = (done, total)

    J2, K2, G2, st2 = B.fock_build(D, uqc.default_opts(tau=1e-12, progress=report, max_items_per_launch=7,
                                                        streams=streams))
    assert seen and all(done == total for done, total in seen.values())
    assert any(total > 7 for _, total in seen.values())
    for a, b in [(J1, J2), (K1, K2), (G1, G2)]:
        ok, err, m = close(b, a, tol=1e-13)
        assert ok, (err, m)
    assert st1.quartets == st2.quartets
    _check_fock(B, O, D, 1e-12, J2, K2, G2, st2)


@pytest.mark.parametrize("streams", [2, 3, 4])
def test_fock_several_streams(ctx, streams):
    """Class launches spread over several HIP streams (joined back before the final pass) give the one-stream J, K,
    G up to atomic-order rounding and match the oracle; timing still reports every class; the spin-density build
    takes the same path; out-of-range stream counts are rejected."""
    w = wl.lattice(9, seed=36, ndens=1, tau=1e-12)
    B = uqc.Basis(ctx, w.shells)
    O = oracle.Basis(w.shells)
    D = w.densities[0]
    J1, K1, G1, st1 = B.fock_build(D, uqc.default_opts(tau=1e-12, streams=1))
    for rep in range(2):  # the second build orders classes by the first one's FLOPs
        J2, K2, G2, st2 = B.fock_build(D, uqc.default_opts(tau=1e-12, streams=streams, timing=True))
        for a, b in [(J1, J2), (K1, K2), (G1, G2)]:
            ok, err, m = close(b, a, tol=1e-13)
            assert ok, (rep, err, m)
        assert st1.quartets == st2.quartets and st2.nclass > 1 and all(
            st2.class_ms[c] > 0 for c in range(st2.nclass))
    _check_fock(B, O, D, 1e-12, J2, K2, G2, st2)
    Db = 0.5 * D
    one = B.fock_build_uhf(D, Db, uqc.default_opts(tau=1e-12, streams=1), want=("Ga", "Gb"))
    many = B.fock_build_uhf(D, Db, uqc.default_opts(tau=1e-12, streams=streams), want=("Ga", "Gb"))
    for k in ("Ga", "Gb"):
        ok, err, m = close(many[k], one[k], tol=1e-13)
        assert ok, (k, err, m)
    for bad in (-1, 5):
        with pytest.raises(uqc.UqcError) as e:
            B.fock_build(D, uqc.default_opts(tau=1e-12, streams=bad))
        assert e.value.status == uqc.UQC_E_ARG


def test_fock_zero_and_linear(ctx):
    w = wl.lattice(4, seed=33, ndens=2)
    B = uqc.Basis(ctx, w.shells)
    N = B.nbf
    J0, K0, G0, st0 = B.fock_build(np.zeros((N, N)))
    assert np.all(J0 == 0) and np.all(K0 == 0) and st0.E2 == 0
    D1, D2 = w.densities
    J1, K1, _, _ = B.fock_build(D1)
    J2, K2, _, _ = B.fock_build(D2)
    J3, K3, _, _ = B.fock_build(0.3 * D1 - 1.7 * D2)
    assert np.max(np.abs(J3 - (0.3 * J1 - 1.7 * J2))) <= 1e-13 * np.max(np.abs(J1)) * 10
    assert np.max(np.abs(K3 - (0.3 * K1 - 1.7 * K2))) <= 1e-13 * np.max(np.abs(K1)) * 10


# ----------------------------------------------------------------------------------------------- errors
def test_errors(ctx):
    w = wl.lattice(3, seed=34, ndens=1)
    B = uqc.Basis(ctx, w.shells)
    D = w.densities[0].copy()
    D[0, 1] += 1e-3
    with pytest.raises(uqc.UqcError) as e:
        B.fock_build(D)
    assert e.value.status == uqc.UQC_E_NOT_SYMMETRIC
    D = w.densities[0].copy()
    D[2, 2] = np.nan
    with pytest.raises(uqc.UqcError) as e:
        B.fock_build(D)
    assert e.value.status == uqc.UQC_E_NOT_SYMMETRIC
    with pytest.raises(uqc.UqcError) as e:
        B.eri_block(0, 1, 2, B.nshell)
    assert e.value.status == uqc.UQC_E_ARG
    sh = wl.random_quartet_shells(1, (3, 0), k=1)
    with pytest.raises(uqc.UqcError) as e:
        uqc.Basis(ctx, sh)
    assert e.value.status == uqc.UQC_E_UNSUPPORTED
    sh = wl.random_quartet_shells(1, (1, 0), k=1)
    sh.alpha[0] = -1.0
    with pytest.raises(uqc.UqcError) as e:
        uqc.Basis(ctx, sh)
    assert e.value.status == uqc.UQC_E_ARG
    # the basis is still usable after rejected calls
    J, K, G, st = B.fock_build(w.densities[0])
    assert np.isfinite(st.E2)


# ----------------------------------------------------------------------------------------------- full size
@pytest.fixture(scope="module")
def medium(ctx):
    w = wl.medium(ndens=3)
    B = uqc.Basis(ctx, w.shells)
    return w, B


def test_medium_sampled_blocks_match_oracle(medium):
    """60 atoms, N = 660, tau = 1e-12, the benchmark's launch configuration: J and K blocks, two per pair class
    (ss, ps, pp, ds, dp, dd) and both shell orders, on three of the densities, computed one by one by the oracle's
    definition of Eq. (12) (same screening rule), within 1e-10 of the matrix's largest element."""
    w, B = medium
    O = oracle.Basis(w.shells)
    rng = np.random.default_rng(7)
    off = B.offsets
    l = np.asarray(B.l)
    for D in w.densities[:3]:
        J, K, G, st = B.fock_build(D, uqc.default_opts(tau=w.tau))
        picks = []
        for (la, lb) in [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)]:
            for rep in range(2):
                a = int(rng.choice(np.flatnonzero(l == la)))
                b = int(rng.choice(np.flatnonzero(l == lb)))
                picks.append((a, b) if rep == 0 else (b, a))
        for (a, b) in picks:
            na, nb = oracle.ncart(int(l[a])), oracle.ncart(int(l[b]))
            jb = O.j_block(D, a, b, tau=w.tau)
            kb = O.k_block(D, a, b, tau=w.tau)
            assert np.max(np.abs(J[off[a]:off[a] + na, off[b]:off[b] + nb] - jb)) <= TOL * np.max(np.abs(J)), (
                "J", a, b)
            assert np.max(np.abs(K[off[a]:off[a] + na, off[b]:off[b] + nb] - kb)) <= TOL * np.max(np.abs(K)), (
                "K", a, b)


def test_medium_properties(medium):
    w, B = medium
    D1, D2 = w.densities[:2]
    J1, K1, G1, s1 = B.fock_build(D1, uqc.default_opts(tau=w.tau))
    J2, K2, G2, s2 = B.fock_build(D2, uqc.default_opts(tau=w.tau))
    assert s1.quartets == s2.quartets and s1.quartets > 1e7
    for J, K in [(J1, K1), (J2, K2)]:
        assert np.max(np.abs(J - J.T)) <= 1e-14 * np.max(np.abs(J)) * 10
        assert np.max(np.abs(K - K.T)) <= 1e-14 * np.max(np.abs(K)) * 10
    for D, J, K, st in [(D1, J1, K1, s1), (D2, J2, K2, s2)]:
        trJ, trK = float(np.sum(D * J)), float(np.sum(D * K))
        assert 0 < trK <= trJ
        assert abs(st.E2 - 0.5 * (trJ - 0.5 * trK)) <= 1e-12 * st.E2
    # a second build of the same density reproduces the first up to atomic-order rounding
    J1b, K1b, G1b, s1b = B.fock_build(D1, uqc.default_opts(tau=w.tau))
    assert np.max(np.abs(G1b - G1)) <= 1e-13 * np.max(np.abs(G1))

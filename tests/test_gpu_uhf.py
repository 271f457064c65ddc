"""GPU tests of the spin-density Fock build (uqc_fock_build_uhf), the exchange weight of the Fock build
(exchange_scale) and the unrestricted Hartree-Fock driver (uqc_scf_uhf), against the CPU oracle.

  * J(Da + Db), K(Da), K(Db), G^s = J - x K^s and E2 = 1/2 sum (Da Ga + Db Gb) match the oracle's definitions to
    1e-10 of each matrix's largest element, unscreened and screened, host and device pointers, several tiles and a
    ragged tail; equal spin densities reproduce the closed-shell build;
  * the closed-shell build with exchange weight x gives G = J - (x/2) K and the matching E2;
  * UHF: hydrogen atom and H2 triplet (textbook values), closed-shell H2 equal to the restricted driver, stretched
    H2 broken-symmetry solution and open-shell hydrogen-like lattices equal to the oracle's plain iteration (energy
    1e-9 Eh, densities, <S^2>, occupied orbital energies); argument errors.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1303_4916_amd import uqc
from paper_1303_4916_amd import workloads as wl

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def ctx():
    c = uqc.Context(0)
    yield c
    c.close()


def _nuclei(sh, charge=1.0):
    nat = int(np.max(sh.atom)) + 1
    R = np.array([sh.center[np.where(sh.atom == a)[0][0]] for a in range(nat)])
    return np.full(nat, float(charge)), R


def _golden():
    vals = {}
    with open(os.path.join(HERE, "golden", "h2_sto3g.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            vals[k] = float(v)
    return vals


def _spin_densities(nbf, seed, na, nb):
    rng = np.random.default_rng(seed)
    ca = rng.standard_normal((nbf, na))
    cb = rng.standard_normal((nbf, nb))
    return ca @ ca.T / nbf, cb @ cb.T / nbf


def _close(a, b, tol):
    scale = max(1.0, float(np.max(np.abs(b))))
    assert float(np.max(np.abs(a - b))) <= tol * scale, float(np.max(np.abs(a - b)))


@pytest.mark.parametrize("natoms,seed,tau", [(5, 61, 0.0), (9, 62, 1e-12), (12, 63, 1e-10)])
@pytest.mark.parametrize("device", [False, True])
def test_fock_uhf_matches_oracle(ctx, natoms, seed, tau, device):
    print("fock_uhf", natoms, seed, tau, device, flush=True)
    sh = wl.lattice(natoms, seed=seed, ndens=1).shells
    B = uqc.Basis(ctx, sh)
    Da, Db = _spin_densities(sh.nbf, seed, 5, 3)
    opts = uqc.default_opts(tau=tau, exchange_scale=0.75)
    if device:
        import torch
        r = B.fock_build_uhf(torch.from_numpy(Da).cuda(), torch.from_numpy(Db).cuda(), opts)
        r = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in r.items()}
    else:
        r = B.fock_build_uhf(Da, Db, opts)
    O = oracle.Basis(sh)
    J, K, _ = O.jk_symmetric([Da, Db], tau=tau)
    Jt = J[0] + J[1]
    Ga, Gb = Jt - 0.75 * K[0], Jt - 0.75 * K[1]
    _close(r["J"], Jt, 1e-10)
    _close(r["Ka"], K[0], 1e-10)
    _close(r["Kb"], K[1], 1e-10)
    _close(r["Ga"], Ga, 1e-10)
    _close(r["Gb"], Gb, 1e-10)
    e2 = 0.5 * float(np.sum(Da * Ga + Db * Gb))
    assert abs(r["stats"].E2 - e2) <= 1e-10 * max(1.0, abs(e2))
    B.close()


def test_fock_uhf_equal_spins_is_closed_shell(ctx):
    sh = wl.lattice(9, seed=64, ndens=1).shells
    B = uqc.Basis(ctx, sh)
    D = wl.random_density(np.random.default_rng(5), sh.nbf, 6, 9.0)
    J, K, G, st = B.fock_build(D)
    r = B.fock_build_uhf(0.5 * D, 0.5 * D, want=("J", "Ga", "Gb"))
    _close(r["J"], J, 1e-12)
    _close(r["Ga"], G, 1e-12)
    _close(r["Gb"], G, 1e-12)
    assert abs(r["stats"].E2 - st.E2) <= 1e-12 * abs(st.E2)
    assert r["Ka"] is None and r["Kb"] is None
    B.close()


@pytest.mark.parametrize("x", [0.0, 0.2, 1.0])
def test_exchange_scale_closed_shell(ctx, x):
    sh = wl.lattice(5, seed=65, ndens=1).shells
    B = uqc.Basis(ctx, sh)
    D = wl.random_density(np.random.default_rng(6), sh.nbf, 4, 5.0)
    J, K, G, st = B.fock_build(D, uqc.default_opts(tau=0.0, exchange_scale=x))
    Jo, Ko, _ = oracle.Basis(sh).jk_symmetric([D])
    _close(G, Jo[0] - 0.5 * x * Ko[0], 1e-10)
    assert abs(st.E2 - 0.5 * float(np.sum(D * (Jo[0] - 0.5 * x * Ko[0])))) <= 1e-10 * max(1.0, abs(st.E2))
    _close(G, J - 0.5 * x * K, 1e-13)
    B.close()


def test_fock_uhf_rejects_bad_input(ctx):
    sh = wl.lattice(3, seed=66, ndens=1).shells
    B = uqc.Basis(ctx, sh)
    Da, Db = _spin_densities(sh.nbf, 3, 2, 1)
    Db[0, 1] += 1.0
    with pytest.raises(uqc.UqcError) as e:
        B.fock_build_uhf(Da, Db)
    assert e.value.status == uqc.UQC_E_NOT_SYMMETRIC
    with pytest.raises(uqc.UqcError) as e:
        B.fock_build_uhf(Da, Da, uqc.default_opts(exchange_scale=float("nan")))
    assert e.value.status == uqc.UQC_E_ARG
    B.close()


def _h_atom():
    h2 = wl.h2_sto3g()
    return wl.Shells(h2.l[:1].copy(), h2.nprim[:1].copy(), h2.center[:1].copy(), h2.alpha[:3].copy(),
                     h2.coef[:3].copy(), np.zeros(1, dtype=np.int32))


def test_uhf_hydrogen_atom_and_h2_triplet(ctx):
    g = _golden()
    sh = _h_atom()
    B = uqc.Basis(ctx, sh)
    r = B.scf_uhf([1.0], sh.center, 1, 0)
    assert r["converged"]
    assert abs(r["E_total"] - (g["T11"] + g["V1_11"])) <= 1e-4
    assert abs(r["E_total"] - oracle.uhf(sh, [1.0], sh.center, 1, 0)["E_total"]) <= 1e-10
    assert abs(r["s2"] - 0.75) <= 1e-12
    B.close()
    sh = wl.h2_sto3g()
    B = uqc.Basis(ctx, sh)
    r = B.scf_uhf([1.0, 1.0], sh.center, 2, 0)
    ref = oracle.uhf(sh, [1.0, 1.0], sh.center, 2, 0)
    assert r["converged"]
    assert abs(r["E_total"] - (g["h_gg"] + g["h_uu"] + g["J_gu"] - g["K_gu"] + 1.0 / 1.4)) <= 3e-4
    assert abs(r["E_total"] - ref["E_total"]) <= 1e-10
    assert abs(r["s2"] - 2.0) <= 1e-10
    assert np.max(np.abs(r["Pb"])) == 0.0
    B.close()


def test_uhf_closed_shell_equals_rhf(ctx):
    sh = wl.lattice(4, seed=43, ndens=1).shells
    Z, R = _nuclei(sh)
    B = uqc.Basis(ctx, sh)
    o = uqc.scf_opts(e_conv=1e-11, d_conv=1e-9, fock=uqc.default_opts(tau=0.0))
    ru = B.scf_uhf(Z, R, 2, 2, o)
    rr = B.scf_rhf(Z, R, 2, o)
    assert ru["converged"] and rr["converged"]
    assert abs(ru["E_total"] - rr["E_total"]) <= 1e-10
    assert np.max(np.abs(ru["Pa"] - ru["Pb"])) <= 1e-8
    assert np.max(np.abs(ru["Pa"] + ru["Pb"] - rr["P"])) <= 1e-7
    assert abs(ru["s2"]) <= 1e-8
    B.close()


def test_uhf_stretched_h2_broken_symmetry(ctx):
    sh = wl.h2_sto3g(R=4.0)
    Z, R = [1.0, 1.0], sh.center
    B = uqc.Basis(ctx, sh)
    r = B.scf_uhf(Z, R, 1, 1, uqc.scf_opts(guess_mix=np.pi / 4, e_conv=1e-11, d_conv=1e-9))
    ref = oracle.uhf(sh, Z, R, 1, 1, guess_mix=np.pi / 4)
    rr = oracle.rhf(sh, Z, R, nocc=1)
    assert r["converged"]
    assert abs(r["E_total"] - ref["E_total"]) <= 1e-9
    assert abs(r["s2"] - ref["S2"]) <= 1e-6
    assert r["E_total"] < rr["E_total"] - 1e-3  # below the restricted solution
    assert np.max(np.abs(r["Pa"] + r["Pb"] - ref["Pa"] - ref["Pb"])) <= 1e-6
    B.close()


@pytest.mark.parametrize("natoms,seed,na,nb,diis", [(3, 7, 2, 1, 8), (4, 43, 3, 1, 8), (6, 5, 4, 2, 8),
                                                      (4, 43, 3, 1, 0)])
def test_uhf_open_shell_lattice_matches_oracle(ctx, natoms, seed, na, nb, diis):
    print("uhf", natoms, seed, na, nb, diis, flush=True)
    sh = wl.lattice(natoms, seed=seed, ndens=1).shells
    Z, R = _nuclei(sh)
    B = uqc.Basis(ctx, sh)
    r = B.scf_uhf(Z, R, na, nb, uqc.scf_opts(diis_size=diis, max_iter=500, e_conv=1e-11, d_conv=1e-9,
                                             fock=uqc.default_opts(tau=0.0)))
    ref = oracle.uhf(sh, Z, R, na, nb)
    assert r["converged"], r["iterations"]
    assert abs(r["E_total"] - ref["E_total"]) <= 1e-9
    assert np.max(np.abs(r["Pa"] - ref["Pa"])) <= 1e-6
    assert np.max(np.abs(r["Pb"] - ref["Pb"])) <= 1e-6
    assert abs(r["s2"] - ref["S2"]) <= 1e-7
    assert np.max(np.abs(r["eps_a"][:na] - ref["eps_a"][:na])) <= 1e-7
    assert np.max(np.abs(r["eps_b"][:nb] - ref["eps_b"][:nb])) <= 1e-7
    if diis:
        assert r["iterations"] <= ref["iterations"] + 1
    B.close()


def test_uhf_rejects_bad_arguments(ctx):
    sh = wl.lattice(3, seed=7, ndens=1).shells
    Z, R = _nuclei(sh)
    B = uqc.Basis(ctx, sh)
    for na, nb in ((-1, 1), (0, 0), (B.nbf + 1, 0), (1, B.nbf + 1)):
        with pytest.raises(uqc.UqcError) as e:
            B.scf_uhf(Z, R, na, nb)
        assert e.value.status == uqc.UQC_E_ARG
    with pytest.raises(uqc.UqcError) as e:
        B.scf_uhf(Z, R, 2, 1, uqc.scf_opts(guess_mix=float("inf")))
    assert e.value.status == uqc.UQC_E_ARG
    r = B.scf_uhf(Z, R, 2, 1, uqc.scf_opts(max_iter=3))
    assert r["iterations"] == 3 and not r["converged"]
    B.close()


@pytest.mark.parametrize("x", [0.0, 0.2, 0.5])
def test_scf_with_scaled_exchange_textbook(ctx, x):
    # minimal-basis H2: the occupied orbital is fixed by symmetry, so with G = J - (x/2) K the closed-shell energy is
    # 2 h_gg + (2 - x) J_gg + 1/R (textbook molecular-orbital integrals); the H atom (one function, one electron)
    # in the unrestricted driver has E = H_11 + (1 - x) (11|11) / 2
    g = _golden()
    sh = wl.h2_sto3g()
    B = uqc.Basis(ctx, sh)
    r = B.scf_rhf([1.0, 1.0], sh.center, 1, uqc.scf_opts(fock=uqc.default_opts(exchange_scale=x)))
    assert r["converged"]
    assert abs(r["E_total"] - (2 * g["h_gg"] + (2 - x) * g["J_gg"] + 1 / 1.4)) <= 3e-4
    B.close()
    sh = _h_atom()
    B = uqc.Basis(ctx, sh)
    r = B.scf_uhf([1.0], sh.center, 1, 0, uqc.scf_opts(fock=uqc.default_opts(exchange_scale=x)))
    assert r["converged"]
    assert abs(r["E_total"] - (g["T11"] + g["V1_11"] + 0.5 * (1 - x) * g["(11|11)"])) <= 2e-4
    B.close()


def test_spin_build_full_size(ctx):
    """60 atoms, N = 660, tau = 1e-12 (the benchmark's launch configuration): sampled J, Ka, Kb blocks of the
    spin-density build against the oracle's definitions computed one by one, and over every element
    K(Da) + K(Db) = K(Da + Db) and J(Da + Db) from the closed-shell build of Da + Db (linearity)."""
    w = wl.medium(ndens=2)
    B = uqc.Basis(ctx, w.shells)
    Da, Db = 0.55 * w.densities[0], 0.45 * w.densities[1]
    o = uqc.default_opts(tau=w.tau)
    r = B.fock_build_uhf(Da, Db, o)
    J, K, G, st = B.fock_build(Da + Db, o)
    assert np.max(np.abs(r["J"] - J)) <= 1e-12 * np.max(np.abs(J))
    assert np.max(np.abs(r["Ka"] + r["Kb"] - K)) <= 1e-12 * np.max(np.abs(K))
    assert r["stats"].quartets == st.quartets
    O = oracle.Basis(w.shells)
    off = B.offsets
    rng = np.random.default_rng(17)
    picks = [(0, 0), (5, 2)] + [tuple(int(x) for x in rng.integers(0, B.nshell, size=2)) for _ in range(2)]
    for a, b in picks:
        na, nb = oracle.ncart(int(B.l[a])), oracle.ncart(int(B.l[b]))
        blocks = [("J", r["J"], O.j_block(Da + Db, a, b, tau=w.tau)), ("Ka", r["Ka"], O.k_block(Da, a, b, tau=w.tau)),
                  ("Kb", r["Kb"], O.k_block(Db, a, b, tau=w.tau))]
        for name, M, ref in blocks:
            got = M[off[a]:off[a] + na, off[b]:off[b] + nb]
            assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(M)), (name, a, b)
    B.close()


def test_spin_build_mixed_precision(ctx):
    """Mixed precision (FP32 recursions, FP64 accumulation) in the one-pass spin build: E2 within 1e-6 Eh of the
    FP64 spin build on a 12-atom lattice, the matrices within 1e-6 of their largest element, and some quartets
    routed to FP32."""
    sh = wl.lattice(12, seed=63, ndens=1).shells
    B = uqc.Basis(ctx, sh)
    Da, Db = _spin_densities(sh.nbf, 63, 6, 5)
    r64 = B.fock_build_uhf(Da, Db, uqc.default_opts(tau=1e-12))
    rmx = B.fock_build_uhf(Da, Db, uqc.default_opts(tau=1e-12, precision=uqc.MIXED))
    assert abs(rmx["stats"].E2 - r64["stats"].E2) <= 1e-6
    for k in ("J", "Ka", "Kb", "Ga", "Gb"):
        assert np.max(np.abs(rmx[k] - r64[k])) <= 1e-6 * np.max(np.abs(r64[k])), k
    assert rmx["stats"].fp64_quartets < rmx["stats"].quartets
    B.close()

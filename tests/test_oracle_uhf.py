"""Pins of the oracle's unrestricted Hartree-Fock iteration (the paper's URHF; Pople-Nesbet equations), against facts
that do not come from the oracle:

  * the hydrogen atom in the textbook minimal basis: one electron in one function, E = T_11 + V_11 (values of
    tests/golden/h2_sto3g.txt);
  * the H2 triplet in that basis: both alpha spin orbitals filled, E = h_gg + h_uu + J_gu - K_gu + 1/R from the
    textbook molecular-orbital integrals (tests/golden/h2_sto3g.txt), and <S^2> = 2;
  * a closed-shell start with equal spins stays restricted: the energy equals the textbook closed-shell value and
    the pinned restricted oracle, P^a = P^b, <S^2> = 0;
  * dissociation: at R = 20 bohr the broken-symmetry solution has the energy of two separate atoms and <S^2> = 1;
  * invariants of a converged open-shell lattice: P^s S P^s = P^s, tr(P^s S) = n_s, F^s P^s S = S P^s F^s,
    <S^2> >= S_z (S_z + 1), and exchanging the spin labels leaves the energy unchanged.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1303_4916_amd import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    vals = {}
    with open(os.path.join(HERE, "golden", "h2_sto3g.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            vals[k] = float(v)
    return vals


def _h_atom():
    h2 = wl.h2_sto3g()
    return wl.Shells(h2.l[:1].copy(), h2.nprim[:1].copy(), h2.center[:1].copy(), h2.alpha[:3].copy(),
                     h2.coef[:3].copy(), np.zeros(1, dtype=np.int32))


def _h2(R):
    sh = wl.h2_sto3g(R=R)
    return sh, [1.0, 1.0], sh.center


def test_hydrogen_atom():
    g = _golden()
    sh = _h_atom()
    r = oracle.uhf(sh, [1.0], sh.center, nalpha=1, nbeta=0)
    assert abs(r["E_total"] - (g["T11"] + g["V1_11"])) <= 1e-4
    assert abs(r["S2"] - 0.75) <= 1e-12


def test_h2_triplet_textbook():
    g = _golden()
    sh, Z, R = _h2(1.4)
    r = oracle.uhf(sh, Z, R, nalpha=2, nbeta=0)
    e = g["h_gg"] + g["h_uu"] + g["J_gu"] - g["K_gu"] + 1.0 / 1.4
    assert abs(r["E_total"] - e) <= 3e-4
    assert abs(r["S2"] - 2.0) <= 1e-12
    # the closed-shell values from the same integrals (consistency of the stored table)
    assert abs(2 * g["h_gg"] + g["J_gg"] - g["E_elec"]) <= 2e-4


def test_h2_closed_shell_stays_restricted():
    g = _golden()
    sh, Z, R = _h2(1.4)
    r = oracle.uhf(sh, Z, R, nalpha=1, nbeta=1)
    ref = oracle.rhf(sh, Z, R, nocc=1)
    assert abs(r["E_total"] - g["E_total"]) <= 1e-4
    assert abs(r["E_total"] - ref["E_total"]) <= 1e-10
    assert np.max(np.abs(r["Pa"] - r["Pb"])) <= 1e-10
    assert np.max(np.abs(r["Pa"] + r["Pb"] - ref["P"])) <= 1e-8
    assert abs(r["S2"]) <= 1e-10


def test_h2_dissociation_broken_symmetry():
    g = _golden()
    sh, Z, R = _h2(20.0)
    r = oracle.uhf(sh, Z, R, nalpha=1, nbeta=1, guess_mix=np.pi / 4)
    atom = oracle.uhf(_h_atom(), [1.0], _h_atom().center, nalpha=1, nbeta=0)
    rr = oracle.rhf(sh, Z, R, nocc=1)
    assert abs(r["E_total"] - 2 * (g["T11"] + g["V1_11"])) <= 2e-4
    assert abs(r["E_total"] - 2 * atom["E_total"]) <= 1e-8      # size consistency of the separated atoms
    assert abs(r["S2"] - 1.0) <= 1e-6
    assert r["E_total"] < rr["E_total"] - 0.1                   # the restricted solution dissociates wrongly
    # one electron of each spin, on different atoms
    Sd = r["S"]
    qa = np.diag(r["Pa"] @ Sd)
    qb = np.diag(r["Pb"] @ Sd)
    assert abs(qa[0] - qb[1]) <= 1e-6 and min(abs(qa[0] - 1.0), abs(qa[0])) <= 1e-6 and abs(qa[0] - qb[0]) > 0.99


@pytest.mark.parametrize("natoms,seed,na,nb,flip", [(3, 7, 2, 1, True), (4, 43, 3, 1, True), (6, 5, 4, 2, False)])
def test_open_shell_lattice_invariants(natoms, seed, na, nb, flip):
    sh = wl.lattice(natoms, seed=seed, ndens=1).shells
    R = np.unique(sh.center, axis=0)
    Z = np.ones(R.shape[0])
    r = oracle.uhf(sh, Z, R, nalpha=na, nbeta=nb)
    S, H = r["S"], r["H"]
    O = oracle.Basis(sh)
    J, K, _ = O.jk_symmetric([r["Pa"], r["Pb"]])
    for P, Kx, n in ((r["Pa"], K[0], na), (r["Pb"], K[1], nb)):
        F = H + J[0] + J[1] - Kx
        assert np.max(np.abs(P @ S @ P - P)) <= 1e-10
        assert abs(np.trace(P @ S) - n) <= 1e-10
        assert np.max(np.abs(F @ P @ S - S @ P @ F)) <= 1e-7
    sz = 0.5 * (na - nb)
    assert r["S2"] >= sz * (sz + 1) - 1e-10
    if flip:
        f = oracle.uhf(sh, Z, R, nalpha=nb, nbeta=na)
        assert abs(f["E_total"] - r["E_total"]) <= 1e-9
        assert np.max(np.abs(f["Pa"] - r["Pb"])) <= 1e-6

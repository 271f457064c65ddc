"""Pins of the oracle's second-order Moller-Plesset energy (the paper's MP2; closed-shell spin-adapted formula) and
of its four-index transformation, against facts that do not come from those functions:

  * the textbook minimal-basis H2: only the g -> u double excitation exists, so E2 = K_gu^2 / (2 (e_g - e_u))
    with K_gu, e_g, e_u from tests/golden/h2_sto3g.txt (-0.0132 Eh);
  * the spin-orbital definition E2 = 1/4 sum_{ijab} |<ij||ab>|^2 / (e_i + e_j - e_a - e_b) over spin orbitals,
    from a full one-shot MO transformation written here, on small lattices, with and without frozen core, and its
    opposite-spin part (i, j of different spin);
  * size consistency: two H2 molecules 60 bohr apart have twice the energy of one;
  * signs: E_os < 0 and E_ss <= 0 for closed-shell ground states.
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


def _mp2(sh, Z, R, nocc, nfrozen=0):
    r = oracle.rhf(sh, Z, R, nocc=nocc)
    eri = oracle.Basis(sh).eri_tensor()
    V = oracle.mo_integrals_ovov(eri, r["C"], nocc, nfrozen)
    return oracle.mp2_closed_shell(V, r["eps"], nocc, nfrozen), r, eri


def _spin_orbital_mp2(eri, C, eps, nocc, nfrozen):
    """1/4 sum |<ij||ab>|^2 / D over spin orbitals; spin orbital 2p is alpha, 2p+1 beta of spatial orbital p."""
    mo = np.einsum("mp,nq,mnls,lr,st->pqrt", C, C, eri, C, C, optimize=True)  # (pq|rt), chemists' notation
    n = C.shape[1]
    occ = [s for p in range(nfrozen, nocc) for s in (2 * p, 2 * p + 1)]
    vir = [s for p in range(nocc, n) for s in (2 * p, 2 * p + 1)]

    def g(p, q, r, s):  # <pq|rs> = (pr|qs) with spin integration
        if p % 2 != r % 2 or q % 2 != s % 2:
            return 0.0
        return mo[p // 2, r // 2, q // 2, s // 2]

    e = e_os = 0.0
    for i in occ:
        for j in occ:
            for a in vir:
                for b in vir:
                    x = g(i, j, a, b) - g(i, j, b, a)
                    d = eps[i // 2] + eps[j // 2] - eps[a // 2] - eps[b // 2]
                    e += 0.25 * x * x / d
                    if i % 2 != j % 2:
                        e_os += 0.25 * x * x / d  # the loop visits (i alpha, j beta) and (i beta, j alpha)
    return e, e_os


def _nuclei(sh):
    nat = int(np.max(sh.atom)) + 1
    R = np.array([sh.center[np.where(sh.atom == a)[0][0]] for a in range(nat)])
    return np.ones(nat), R


def test_h2_textbook():
    g = _golden()
    sh = wl.h2_sto3g()
    (e2, e_os, e_ss), r, _ = _mp2(sh, [1.0, 1.0], sh.center, 1)
    assert abs(e2 - g["K_gu"] ** 2 / (2 * (g["eps1"] - g["eps2"]))) <= 2e-5
    assert abs(e2 - (-0.0132)) <= 1e-4
    assert e_ss == pytest.approx(0.0, abs=1e-15)  # one occupied spatial orbital: no same-spin pairs
    assert e2 == e_os


@pytest.mark.parametrize("natoms,seed,nfrozen", [(2, 3, 0), (4, 43, 0), (4, 43, 1)])
def test_spin_orbital_definition(natoms, seed, nfrozen):
    sh = wl.lattice(natoms, seed=seed, ndens=1).shells
    Z, R = _nuclei(sh)
    nocc = natoms // 2
    (e2, e_os, e_ss), r, eri = _mp2(sh, Z, R, nocc, nfrozen)
    ref, ref_os = _spin_orbital_mp2(eri, r["C"], r["eps"], nocc, nfrozen)
    assert abs(e2 - ref) <= 1e-12 * max(1.0, abs(ref))
    assert abs(e_os - ref_os) <= 1e-12 * max(1.0, abs(ref_os))
    assert e_os < 0 and e_ss <= 1e-15


def test_size_consistency():
    one = wl.h2_sto3g(R=1.4)
    (e1, _, _), _, _ = _mp2(one, [1.0, 1.0], one.center, 1)
    shift = np.array([0.0, 60.0, 0.0])
    two = wl.Shells(np.concatenate([one.l, one.l]), np.concatenate([one.nprim, one.nprim]),
                    np.concatenate([one.center, one.center + shift]), np.concatenate([one.alpha, one.alpha]),
                    np.concatenate([one.coef, one.coef]), np.array([0, 1, 2, 3], dtype=np.int32))
    (e2, _, _), _, _ = _mp2(two, [1.0] * 4, two.center, 2)
    assert abs(e2 - 2 * e1) <= 1e-10

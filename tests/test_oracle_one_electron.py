"""Pins of the oracle's one-electron integrals (Eq. (2)-(4)) and of its restricted Hartree-Fock iteration, against
facts that do not come from the oracle:

  * brute-force quadrature (tests/quad_one.py: no Hermite expansion, no Boys function, kinetic energy in the
    symmetric first-derivative form) for every shell-pair class up to (d|d), with two nuclei;
  * closed forms for s primitives: S = (pi/p)^{3/2} e^{-mu R^2}, T = mu (3 - 2 mu R^2) S,
    V = -Z (2 pi/p) e^{-mu R^2} F_0(p |P-C|^2) with F_0(x) = sqrt(pi/x) erf(sqrt(x)) / 2 (math.erf);
  * the textbook minimal-basis H2 example (tests/golden/h2_sto3g.txt, 4 decimals);
  * invariants: S symmetric with unit diagonal and positive definite, T positive definite, translation invariance,
    rotation invariance of the generalized spectra of (T, S) and (V, S); for the converged SCF the commutator
    F P S - S P F vanishes, P S P = 2 P, tr(P S) = 2 nocc, and the energy lies below the core-guess energy.
"""
import math
import os

import numpy as np
import pytest

import oracle
import quad_one
from paper_1303_4916_amd import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
NUC = [(1.0, np.array([0.3, -0.2, 0.5])), (3.0, np.array([-1.0, 0.7, 0.1]))]


def _golden():
    vals = {}
    with open(os.path.join(HERE, "golden", "h2_sto3g.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            vals[k] = float(v)
    return vals


def _blocks(sh, Z, R):
    O = oracle.Basis(sh)
    S, T, V = oracle.one_electron(O, Z, R)
    return O, S, T, V


@pytest.mark.parametrize("ls", [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (0, 2), (1, 2)])
def test_one_electron_matches_quadrature(ls):
    sh = wl.random_quartet_shells(40 + 3 * ls[0] + ls[1], ls, k=2)
    ref = quad_one.one_electron_block(sh, 0, 1, NUC)
    O, S, T, V = _blocks(sh, [z for z, _ in NUC], np.array([c for _, c in NUC]))
    na, nb = ref[0].shape
    o = O.offsets
    for name, M, R in (("S", S, ref[0]), ("T", T, ref[1]), ("V", V, ref[2])):
        got = M[o[0]:o[0] + na, o[1]:o[1] + nb]
        assert np.max(np.abs(got - R)) <= 1e-12 * max(np.max(np.abs(R)), 1e-3), (name, ls)


def test_s_primitive_closed_forms():
    rng = np.random.default_rng(11)
    for _ in range(20):
        a, b = np.exp(rng.uniform(math.log(0.1), math.log(20.0), size=2))
        A, B, C = rng.uniform(-2.0, 2.0, size=(3, 3))
        Z = float(rng.uniform(0.5, 8.0))
        sh = wl.Shells(np.zeros(2, np.int32), np.ones(2, np.int32), np.stack([A, B]), np.array([a, b]),
                       np.ones(2), np.arange(2, dtype=np.int32))
        _, S, T, V = _blocks(sh, [Z], C[None, :])
        p = a + b
        mu = a * b / p
        R2 = float(np.sum((A - B) ** 2))
        P = (a * A + b * B) / p
        x = p * float(np.sum((P - C) ** 2))
        na, nb = (2 * a / math.pi) ** 0.75, (2 * b / math.pi) ** 0.75
        s = na * nb * (math.pi / p) ** 1.5 * math.exp(-mu * R2)
        t = mu * (3.0 - 2.0 * mu * R2) * s
        f0 = 1.0 if x < 1e-12 else 0.5 * math.sqrt(math.pi / x) * math.erf(math.sqrt(x))
        v = -Z * na * nb * (2.0 * math.pi / p) * math.exp(-mu * R2) * f0
        assert abs(S[0, 1] - s) <= 1e-14 * (1.0 + mu * R2)
        assert abs(T[0, 1] - t) <= 1e-13 * (1.0 + mu * R2) * max(abs(t), mu * abs(s))
        assert abs(V[0, 1] - v) <= 1e-13 * (1.0 + mu * R2 + x) * abs(v)


def test_h2_sto3g_one_electron_and_scf_textbook():
    g = _golden()
    sh = wl.h2_sto3g()
    O, S, T, V = _blocks(sh, [1.0, 1.0], sh.center)
    V1 = oracle.one_electron(O, [1.0, 0.0], sh.center)[2]
    H = T + V
    got = {"S12": S[0, 1], "T11": T[0, 0], "T12": T[0, 1], "V1_11": V1[0, 0], "V1_12": V1[0, 1], "V1_22": V1[1, 1],
           "H11": H[0, 0], "H12": H[0, 1]}
    r = oracle.rhf(sh, [1.0, 1.0], sh.center, nocc=1)
    got.update({"eps1": r["eps"][0], "eps2": r["eps"][1], "E_elec": r["E_elec"], "E_total": r["E_total"]})
    for k, v in got.items():
        assert abs(v - g[k]) <= 1.1e-4, (k, v, g[k])
    assert abs(r["E_nuc"] - 1.0 / 1.4) <= 1e-15


def test_one_electron_invariants():
    w = wl.lattice(4, seed=41, ndens=1)
    sh = w.shells
    nat = int(np.max(sh.atom)) + 1
    R = np.array([sh.center[np.where(sh.atom == a)[0][0]] for a in range(nat)])
    Z = np.arange(1, nat + 1, dtype=np.float64)
    O, S, T, V = _blocks(sh, Z, R)
    for M in (S, T, V):
        assert np.max(np.abs(M - M.T)) <= 1e-14 * np.max(np.abs(M))
    assert np.max(np.abs(np.diag(S) - 1.0)) <= 1e-13
    assert np.min(np.linalg.eigvalsh(S)) > 0 and np.min(np.linalg.eigvalsh(T)) > 0
    # translation
    shift = np.array([0.37, -1.1, 2.3])
    sh2 = wl.Shells(sh.l, sh.nprim, sh.center + shift, sh.alpha, sh.coef, sh.atom)
    _, S2, T2, V2 = _blocks(sh2, Z, R + shift)
    for a, b in ((S, S2), (T, T2), (V, V2)):
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))
    # rotation: the span of every full Cartesian shell is closed under rotation, so the generalized eigenvalues of
    # (T, S) and (V, S) do not change
    rng = np.random.default_rng(5)
    Qm, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    sh3 = wl.Shells(sh.l, sh.nprim, sh.center @ Qm.T, sh.alpha, sh.coef, sh.atom)
    _, S3, T3, V3 = _blocks(sh3, Z, R @ Qm.T)

    def gen_eig(M, Sm):
        s, U = np.linalg.eigh(Sm)
        X = U @ np.diag(s ** -0.5) @ U.T
        return np.sort(np.linalg.eigvalsh(X.T @ M @ X))

    for M, M3 in ((T, T3), (V, V3)):
        e1, e3 = gen_eig(M, S), gen_eig(M3, S3)
        assert np.max(np.abs(e1 - e3)) <= 1e-9 * np.max(np.abs(e1))


def test_rhf_converged_properties():
    """A small lattice of hydrogen-like centres (Z = 1 per atom, even electron count): the converged density commutes
    with F in the S metric, is idempotent in that metric, holds the right electron count, and the SCF energy is
    below the energy of the core-Hamiltonian guess."""
    w = wl.lattice(4, seed=43, ndens=1)
    sh = w.shells
    nat = int(np.max(sh.atom)) + 1
    R = np.array([sh.center[np.where(sh.atom == a)[0][0]] for a in range(nat)])
    Z = np.ones(nat)
    nocc = nat // 2
    r = oracle.rhf(sh, Z, R, nocc=nocc)
    S, P = r["S"], r["P"]
    H = r["T"] + r["V"]
    O = oracle.Basis(sh)
    J, K, _ = O.jk_symmetric([P])
    F = H + J[0] - 0.5 * K[0]
    comm = F @ P @ S - S @ P @ F
    assert np.max(np.abs(comm)) <= 1e-7 * np.max(np.abs(F))
    assert np.max(np.abs(P @ S @ P - 2.0 * P)) <= 1e-9 * np.max(np.abs(P))
    assert abs(float(np.sum(P * S)) - 2 * nocc) <= 1e-9
    # energy of the core guess (first iteration density)
    s, U = np.linalg.eigh(S)
    X = U @ np.diag(s ** -0.5) @ U.T
    _, Cp = np.linalg.eigh(X.T @ H @ X)
    C = X @ Cp
    P0 = 2.0 * C[:, :nocc] @ C[:, :nocc].T
    J0, K0, _ = O.jk_symmetric([P0])
    F0 = H + J0[0] - 0.5 * K0[0]
    e0 = 0.5 * float(np.sum(P0 * (H + F0)))
    assert r["E_elec"] < e0

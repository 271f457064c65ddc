"""GPU tests of the closed-shell MP2 energy (uqc_mp2: AO tensor from the quartet kernels, four GEMM quarter
transformations, energy reduction) against the CPU oracle and against properties that hold at any size.

  * textbook minimal-basis H2 (-0.0132 Eh) and small lattices with the oracle's orbitals: E2, E_os, E_ss within
    1e-10 of the oracle's definition, with and without frozen core;
  * the whole GPU pipeline (restricted SCF, then MP2) against the oracle's;
  * screened (tau = 1e-12) against unscreened AO tensors;
  * at nbf = 220 and 440, beyond the oracle's reach (440: beyond one nbf^4 AO tensor): two copies of a lattice 300
    bohr apart, each with the monomer's orbitals, have twice the MP2 energy of one (size consistency);
  * the AO integrals in many small batches against the oracle and the single-batch result;
  * argument errors, and no virtual orbitals giving E2 = 0.
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


def _nuclei(sh):
    nat = int(np.max(sh.atom)) + 1
    R = np.array([sh.center[np.where(sh.atom == a)[0][0]] for a in range(nat)])
    return np.ones(nat), R


def _oracle_mp2(sh, C, eps, nocc, nfrozen=0):
    eri = oracle.Basis(sh).eri_tensor()
    V = oracle.mo_integrals_ovov(eri, C, nocc, nfrozen)
    return oracle.mp2_closed_shell(V, eps, nocc, nfrozen)


def test_mp2_h2_textbook(ctx):
    sh = wl.h2_sto3g()
    r = oracle.rhf(sh, [1.0, 1.0], sh.center, nocc=1)
    B = uqc.Basis(ctx, sh)
    m = B.mp2(r["C"], r["eps"], 1)
    e, _, _ = _oracle_mp2(sh, r["C"], r["eps"], 1)
    assert abs(m["e2"] - e) <= 1e-13
    assert abs(m["e2"] - (-0.0132)) <= 1e-4
    assert m["e_ss"] == pytest.approx(0.0, abs=1e-16)
    B.close()


@pytest.mark.parametrize("natoms,seed,nfrozen", [(4, 43, 0), (6, 55, 0), (6, 55, 1), (8, 71, 2)])
def test_mp2_matches_oracle(ctx, natoms, seed, nfrozen):
    print("mp2", natoms, seed, nfrozen, flush=True)
    sh = wl.lattice(natoms, seed=seed, ndens=1).shells
    Z, R = _nuclei(sh)
    nocc = natoms // 2
    r = oracle.rhf(sh, Z, R, nocc=nocc)
    B = uqc.Basis(ctx, sh)
    m = B.mp2(r["C"], r["eps"], nocc, nfrozen)
    e, eos, ess = _oracle_mp2(sh, r["C"], r["eps"], nocc, nfrozen)
    assert abs(m["e2"] - e) <= 1e-10 * abs(e)
    assert abs(m["e_os"] - eos) <= 1e-10 * abs(eos)
    assert abs(m["e_ss"] - ess) <= 1e-10 * max(abs(ess), 1e-12)
    assert m["quartets"] > 0 and m["transform_flops"] > 0
    B.close()


def test_mp2_gpu_pipeline_and_screening(ctx):
    sh = wl.lattice(6, seed=55, ndens=1).shells
    Z, R = _nuclei(sh)
    B = uqc.Basis(ctx, sh)
    s = B.scf_rhf(Z, R, 3, uqc.scf_opts(e_conv=1e-12, d_conv=1e-10, fock=uqc.default_opts(tau=0.0)))
    assert s["converged"]
    # canonical orbitals of the converged Fock matrix, on the host from the GPU's density-derived Fock matrix
    S, T, V = B.one_electron(Z, R)
    _, _, G, _ = B.fock_build(s["P"], uqc.default_opts(tau=0.0))
    F = T + V + G
    w, U = np.linalg.eigh(S)
    X = U @ np.diag(w ** -0.5) @ U.T
    eps, Cp = np.linalg.eigh(X.T @ F @ X)
    C = X @ Cp
    m = B.mp2(C, eps, 3)
    ref = oracle.rhf(sh, Z, R, nocc=3)
    e, _, _ = _oracle_mp2(sh, ref["C"], ref["eps"], 3)
    assert abs(m["e2"] - e) <= 1e-8
    ms = B.mp2(C, eps, 3, tau=1e-12)
    assert abs(ms["e2"] - m["e2"]) <= 1e-10
    assert ms["quartets"] <= m["quartets"]
    B.close()


def test_mp2_batched_matches_oracle_and_unbatched(ctx):
    """The AO integrals in many small ket-pair batches (each transformed over its first index at once) give the
    oracle's energies and the single-batch result."""
    sh = wl.lattice(8, seed=71, ndens=1).shells
    Z, R = _nuclei(sh)
    r = oracle.rhf(sh, Z, R, nocc=4)
    B = uqc.Basis(ctx, sh)
    one = B.mp2(r["C"], r["eps"], 4, 1)
    many = B.mp2(r["C"], r["eps"], 4, 1, batch_bytes=8 << 20)
    e, eos, ess = _oracle_mp2(sh, r["C"], r["eps"], 4, 1)
    assert one["batches"] == 1 and many["batches"] > 10
    assert many["quartets"] == one["quartets"]
    for m in (one, many):
        assert abs(m["e2"] - e) <= 1e-10 * abs(e)
        assert abs(m["e_os"] - eos) <= 1e-10 * abs(eos)
        assert abs(m["e_ss"] - ess) <= 1e-10 * max(abs(ess), 1e-12)
    assert abs(many["e2"] - one["e2"]) <= 1e-12 * abs(one["e2"])
    with pytest.raises(uqc.UqcError) as ex:  # a batch must hold the widest shell pair's columns
        B.mp2(r["C"], r["eps"], 4, 1, batch_bytes=1 << 20)
    assert ex.value.status == uqc.UQC_E_NOMEM
    B.close()


@pytest.mark.parametrize("natoms", [10, 20])
def test_mp2_size_consistency(ctx, natoms):
    # the dimer takes the monomer's orbitals on both sites (block-diagonal C, energies repeated): its MP2 energy is
    # twice the monomer's up to the dispersion-like cross terms, O(R^-6) (the dimer's own SCF would differ at order
    # mu / R^2 through the electrostatics of the two polar monomers); nbf = 220 and 440, the latter beyond what one
    # nbf^4 AO tensor (300 GB) would allow.  For the 20-atom monomers the cross term is 8.6e-9 Eh at 100 bohr and
    # 1.2e-11 Eh at 300 bohr (the factor 3^6), so the copies sit 300 bohr apart
    mono = wl.lattice(natoms, seed=81, ndens=1).shells
    Z, R = _nuclei(mono)
    shift = np.array([300.0, 0.0, 0.0])
    dim = wl.Shells(np.concatenate([mono.l, mono.l]), np.concatenate([mono.nprim, mono.nprim]),
                    np.concatenate([mono.center, mono.center + shift]), np.concatenate([mono.alpha, mono.alpha]),
                    np.concatenate([mono.coef, mono.coef]), np.concatenate([mono.atom, mono.atom + natoms]))
    no = natoms // 2
    B = uqc.Basis(ctx, mono)
    s = B.scf_rhf(Z, R, no, uqc.scf_opts(e_conv=1e-12, d_conv=1e-10))
    assert s["converged"]
    S, T, V = B.one_electron(Z, R)
    _, _, G, _ = B.fock_build(s["P"])
    w, U = np.linalg.eigh(S)
    X = U @ np.diag(w ** -0.5) @ U.T
    eps, Cp = np.linalg.eigh(X.T @ (T + V + G) @ X)
    C = X @ Cp
    e_mono = B.mp2(C, eps, no)
    n = B.nbf
    B.close()
    order = list(range(no)) + list(range(n, n + no)) + list(range(no, n)) + list(range(n + no, 2 * n))
    Cd = np.zeros((2 * n, 2 * n))
    Cd[:n, :n] = C
    Cd[n:, n:] = C
    Cd = Cd[:, order]
    ed = np.concatenate([eps, eps])[order]
    Bd = uqc.Basis(ctx, dim)
    print("mp2 size consistency nbf", Bd.nbf, flush=True)
    e_dim = Bd.mp2(Cd, ed, 2 * no)
    if natoms == 20:  # the batching is exact: twice as many batches, the same energy
        e_more = Bd.mp2(Cd, ed, 2 * no, batch_bytes=8 << 30)
        assert e_more["batches"] > e_dim["batches"]
        assert abs(e_more["e2"] - e_dim["e2"]) <= 1e-12 * abs(e_dim["e2"])
    Bd.close()
    print("mp2 dimer nbf %d: %d batches, %.0f ms (AO %.0f, transformations %.0f)" % (
        2 * n, e_dim["batches"], e_dim["ms"], e_dim["ao_ms"], e_dim["transform_ms"]), flush=True)
    assert e_dim["e2"] < 0
    assert abs(e_dim["e2"] - 2 * e_mono["e2"]) <= 1e-9 * abs(e_dim["e2"])
    assert abs(e_dim["e_os"] - 2 * e_mono["e_os"]) <= 1e-9 * abs(e_dim["e_os"])


def test_mp2_errors_and_no_virtuals(ctx):
    sh = wl.h2_sto3g()
    B = uqc.Basis(ctx, sh)
    C = np.eye(2)
    for nocc, nf in ((0, 0), (3, 0), (1, 1), (1, -1)):
        with pytest.raises(uqc.UqcError) as e:
            B.mp2(C, np.array([-1.0, 1.0]), nocc, nf)
        assert e.value.status == uqc.UQC_E_ARG
    with pytest.raises(uqc.UqcError) as e:
        B.mp2(C, np.array([1.0, -1.0]), 1)  # virtual below occupied
    assert e.value.status == uqc.UQC_E_ARG
    assert B.mp2(C, np.array([-1.0, -0.5]), 2)["e2"] == 0.0
    B.close()

"""GPU tests of the one-electron integrals (uqc_one_electron, Eq. (2)-(4)) and of the restricted Hartree-Fock
driver (uqc_scf_rhf) against the CPU oracle.

  * S, T, V for every shell-pair class (lattices with s, p, d shells and several nuclei) match the oracle to 1e-12 of
    each matrix's largest element; the device-pointer path matches the host path;
  * the textbook minimal-basis H2 SCF (E = -1.1167 Eh, orbital energies) and small hydrogen-like lattices: energies
    equal the oracle's plain Roothaan iteration to 1e-9 Eh and densities agree, with and without DIIS;
  * stopping at max_iter is reported as not converged; bad arguments are rejected.
"""
import numpy as np
import pytest

import oracle
from paper_1303_4916_amd import uqc
from paper_1303_4916_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = uqc.Context(0)
    yield c
    c.close()


def _nuclei(sh, charge=None):
    nat = int(np.max(sh.atom)) + 1
    R = np.array([sh.center[np.where(sh.atom == a)[0][0]] for a in range(nat)])
    Z = np.arange(1, nat + 1, dtype=np.float64) if charge is None else np.full(nat, float(charge))
    return Z, R


@pytest.mark.parametrize("natoms,seed", [(3, 51), (6, 52)])
def test_one_electron_matches_oracle(ctx, natoms, seed):
    sh = wl.lattice(natoms, seed=seed, ndens=1).shells
    Z, R = _nuclei(sh)
    B = uqc.Basis(ctx, sh)
    S, T, V = B.one_electron(Z, R)
    So, To, Vo = oracle.one_electron(oracle.Basis(sh), Z, R)
    for name, a, b in (("S", S, So), ("T", T, To), ("V", V, Vo)):
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b)), name
    B.close()


def test_one_electron_device_pointers(ctx):
    import torch
    sh = wl.lattice(4, seed=53, ndens=1).shells
    Z, R = _nuclei(sh)
    B = uqc.Basis(ctx, sh)
    S, T, V = B.one_electron(Z, R)
    N = B.nbf
    St, Tt, Vt = (torch.empty((N, N), dtype=torch.float64, device="cuda") for _ in range(3))
    uqc._check(uqc.load().uqc_one_electron(B.h, len(Z), uqc._dp(np.ascontiguousarray(Z)),
                                           uqc._dp(np.ascontiguousarray(R.reshape(-1))), St.data_ptr(),
                                           Tt.data_ptr(), Vt.data_ptr()))
    torch.cuda.synchronize()
    for a, b in ((S, St), (T, Tt), (V, Vt)):
        assert np.max(np.abs(a - b.cpu().numpy())) == 0.0
    # no nuclei: V = 0
    _, _, V0 = B.one_electron(np.zeros(0), np.zeros((0, 3)))
    assert np.all(V0 == 0.0)
    B.close()


def test_scf_h2_textbook(ctx):
    sh = wl.h2_sto3g()
    B = uqc.Basis(ctx, sh)
    r = B.scf_rhf([1.0, 1.0], sh.center, nocc=1)
    ref = oracle.rhf(sh, [1.0, 1.0], sh.center, nocc=1)
    assert r["converged"]
    assert abs(r["E_total"] - ref["E_total"]) <= 1e-10
    assert abs(r["E_total"] - (-1.1167)) <= 1e-4
    assert np.max(np.abs(r["eps"] - ref["eps"])) <= 1e-8
    assert np.max(np.abs(r["P"] - ref["P"])) <= 1e-8
    B.close()


@pytest.mark.parametrize("natoms,seed,diis", [(4, 43, 8), (4, 43, 0), (6, 55, 8)])
def test_scf_lattice_matches_oracle(ctx, natoms, seed, diis):
    sh = wl.lattice(natoms, seed=seed, ndens=1).shells
    Z, R = _nuclei(sh, charge=1.0)
    nocc = natoms // 2
    B = uqc.Basis(ctx, sh)
    r = B.scf_rhf(Z, R, nocc, uqc.scf_opts(diis_size=diis, max_iter=200, e_conv=1e-11, d_conv=1e-9,
                                           fock=uqc.default_opts(tau=0.0)))
    ref = oracle.rhf(sh, Z, R, nocc=nocc, tau=0.0)
    assert r["converged"], r["iterations"]
    assert abs(r["E_total"] - ref["E_total"]) <= 1e-9
    assert abs(r["E_nuc"] - ref["E_nuc"]) <= 1e-12
    assert np.max(np.abs(r["P"] - ref["P"])) <= 1e-6
    assert np.max(np.abs(r["eps"][:nocc + 1] - ref["eps"][:nocc + 1])) <= 1e-7
    if diis:
        assert r["iterations"] <= ref["iterations"] + 1
    B.close()


def test_scf_stops_at_max_iter_and_rejects_bad_arguments(ctx):
    sh = wl.lattice(4, seed=43, ndens=1).shells
    Z, R = _nuclei(sh, charge=1.0)
    B = uqc.Basis(ctx, sh)
    r = B.scf_rhf(Z, R, 2, uqc.scf_opts(max_iter=2))
    assert r["iterations"] == 2 and not r["converged"]
    for nocc in (0, B.nbf + 1):
        with pytest.raises(uqc.UqcError) as e:
            B.scf_rhf(Z, R, nocc)
        assert e.value.status == uqc.UQC_E_ARG
    with pytest.raises(uqc.UqcError) as e:
        B.scf_rhf(Z, R, 2, uqc.scf_opts(diis_size=17))
    assert e.value.status == uqc.UQC_E_ARG
    B.close()

"""uqc_fock_build_noalloc (the Fock build that allocates nothing, its workspace in a fixed device array) against
uqc_fock_build, through the C ABI.

The two entry points run the same kernels on the same plan; only the order of the atomic additions differs, so
J, K, G agree to 1e-13 of each matrix's largest element and E2 to 1e-13 relative, and the quartet counts are equal.
Two calls in a row share the fixed array: the second, on a smaller basis, must not see the first one's contents.
"""
import numpy as np
import pytest

import oracle
from paper_1303_4916_amd import uqc
from paper_1303_4916_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-13


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = uqc.Context(0)
    yield c
    c.close()


def _dev(B):
    import torch
    N = B.nbf
    return [torch.empty((N, N), dtype=torch.float64, device="cuda") for _ in range(3)]


def _ptrs(D, outs):
    return int(D.data_ptr()), int(outs[0].data_ptr()), int(outs[1].data_ptr()), int(outs[2].data_ptr())


def _close(a, b, tol=TOL):
    return float(np.max(np.abs(a - b))) <= tol * float(np.max(np.abs(b)))


@pytest.mark.parametrize("precision", [uqc.FP64, uqc.MIXED])
def test_noalloc_matches_fock_build_two_calls(ctx, precision):
    import torch
    big = wl.lattice(12, seed=71, ndens=1, tau=1e-12)
    small = wl.lattice(5, seed=72, ndens=1, tau=1e-12)
    cases = []
    for w in (big, small):
        B = uqc.Basis(ctx, w.shells)
        D = torch.from_numpy(w.densities[0]).cuda()
        ref = _dev(B)
        opts = uqc.default_opts(tau=w.tau, precision=precision)
        st_ref = B.fock_build_ptr(*_ptrs(D, ref), opts)  # also makes the plan for these options
        cases.append((w, B, D, ref, st_ref, opts))
    torch.cuda.synchronize()
    got = []
    for (w, B, D, ref, st_ref, opts) in cases:  # two calls in a row: the second on the smaller basis
        outs = _dev(B)
        st = B.fock_build_noalloc_ptr(*_ptrs(D, outs), opts)
        got.append((outs, st))
    torch.cuda.synchronize()
    for (w, B, D, ref, st_ref, opts), (outs, st) in zip(cases, got):
        for a, b in zip(outs, ref):
            assert _close(a.cpu().numpy(), b.cpu().numpy())
        assert abs(st.E2 - st_ref.E2) <= TOL * abs(st_ref.E2)
        assert st.quartets == st_ref.quartets and st.prim_quartets == st_ref.prim_quartets
        assert st.fp64_quartets == st_ref.fp64_quartets
    # and the FP64 result is the oracle's (Eq. (12), same screening rule)
    if precision == uqc.FP64:
        w, B, D = cases[1][0], cases[1][1], cases[1][2]
        Jr, Kr, _ = oracle.Basis(w.shells).jk_symmetric([w.densities[0]], tau=w.tau)
        Gr, E2r = oracle.fock_parts(Jr[0], Kr[0], w.densities[0])
        outs, st = got[1]
        for a, r in zip(outs, (Jr[0], Kr[0], Gr)):
            assert _close(a.cpu().numpy(), r, 1e-10)
        assert abs(st.E2 - E2r) <= 1e-10 * abs(E2r)


def test_noalloc_repeated_and_null_outputs(ctx):
    """Repeated calls give the same result (each clears what it accumulates into); J or K may be left out."""
    import torch
    w = wl.lattice(9, seed=73, ndens=2, tau=1e-12)
    B = uqc.Basis(ctx, w.shells)
    opts = uqc.default_opts(tau=w.tau)
    Ds = [torch.from_numpy(D).cuda() for D in w.densities]
    refs = []
    for D in Ds:
        r = _dev(B)
        refs.append((r, B.fock_build_ptr(*_ptrs(D, r), opts)))
    for rep in range(2):
        for D, (r, st_ref) in zip(Ds, refs):
            outs = _dev(B)
            st = B.fock_build_noalloc_ptr(int(D.data_ptr()), 0, 0, int(outs[2].data_ptr()), opts)
            torch.cuda.synchronize()
            assert _close(outs[2].cpu().numpy(), r[2].cpu().numpy())
            assert abs(st.E2 - st_ref.E2) <= TOL * abs(st_ref.E2)


def test_noalloc_errors(ctx):
    import torch
    w = wl.lattice(4, seed=74, ndens=1, tau=1e-12)
    B = uqc.Basis(ctx, w.shells)
    N = B.nbf
    D = torch.from_numpy(w.densities[0]).cuda()
    outs = _dev(B)
    # no plan for these options yet
    with pytest.raises(uqc.UqcError) as e:
        B.fock_build_noalloc_ptr(*_ptrs(D, outs), uqc.default_opts(tau=1e-11))
    assert e.value.status == uqc.UQC_E_ARG
    B.fock_build_ptr(*_ptrs(D, outs), uqc.default_opts(tau=1e-11))
    B.fock_build_noalloc_ptr(*_ptrs(D, outs), uqc.default_opts(tau=1e-11))
    # host pointers, timing, spin builds are not for this entry point
    Dh = np.ascontiguousarray(w.densities[0])
    Jh = np.zeros((N, N))
    with pytest.raises(uqc.UqcError) as e:
        B.fock_build_noalloc_ptr(Dh.ctypes.data, Jh.ctypes.data, 0, 0, uqc.default_opts(tau=1e-11))
    assert e.value.status == uqc.UQC_E_ARG
    with pytest.raises(uqc.UqcError) as e:
        B.fock_build_noalloc_ptr(*_ptrs(D, outs), uqc.default_opts(tau=1e-11, timing=True))
    assert e.value.status == uqc.UQC_E_ARG
    # a non-symmetric density is still rejected
    Dn = D.clone()
    Dn[0, 1] += 1e-3
    with pytest.raises(uqc.UqcError) as e:
        B.fock_build_noalloc_ptr(*_ptrs(Dn, outs), uqc.default_opts(tau=1e-11))
    assert e.value.status == uqc.UQC_E_NOT_SYMMETRIC
    # more basis functions than the fixed array holds
    big = wl.lattice_shells(94, 75)
    assert big.nbf > 1024
    Bb = uqc.Basis(ctx, big)
    Db = torch.zeros((big.nbf, big.nbf), dtype=torch.float64, device="cuda")
    ob = _dev(Bb)
    with pytest.raises(uqc.UqcError) as e:
        Bb.fock_build_noalloc_ptr(*_ptrs(Db, ob), uqc.default_opts())
    assert e.value.status == uqc.UQC_E_ARG
    Bb.close()

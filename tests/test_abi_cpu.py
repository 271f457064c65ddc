"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every declared entry point, and its
host-only logic (defaults, argument checks that precede any device call) behaves as documented."""
import ctypes
import os
import re

import pytest

from paper_1303_4916_amd import uqc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "uqc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"\b(uqc_[a-z_0-9]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = uqc.load()
    declared = _declared()
    assert len(declared) >= 17
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(uqc.EXPORTED) == declared


def test_library_has_gfx950_code_object():
    data = open(uqc.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_default_options():
    o = uqc.default_opts()
    assert o.schwarz_tau == 1e-12 and o.precision == uqc.FP64 and o.fp64_bound == 1e-8 and o.timing == 0
    assert o.streams == 3 and o.fp64_boys_T == 30.0  # the last field: the Python mirror matches the C layout
    assert not o.progress and o.max_items_per_launch == 0 and o.exchange_scale == 1.0
    assert uqc.default_opts(fp64_boys_T=12.5).fp64_boys_T == 12.5


def test_null_arguments_rejected_before_device_use():
    L = uqc.load()
    assert L.uqc_init(0, None, None) == uqc.UQC_E_ARG
    assert b"NULL" in L.uqc_last_error()
    assert L.uqc_basis_create(None, 1, None, None, None, None, None, None) == uqc.UQC_E_ARG
    assert L.uqc_fock_build(None, None, None, None, None, None, None) == uqc.UQC_E_ARG
    assert L.uqc_eri_block(None, 0, 0, 0, 0, 0, None) == uqc.UQC_E_ARG
    assert L.uqc_poll(None, 1, None) == uqc.UQC_E_ARG
    assert L.uqc_server_destroy(None) == uqc.UQC_E_ARG
    assert L.uqc_one_electron(None, 0, None, None, None, None, None) == uqc.UQC_E_ARG
    assert L.uqc_scf_rhf(None, 0, None, None, 1, None, None, None, None) == uqc.UQC_E_ARG
    assert L.uqc_fock_build_uhf(None, None, None, None, None, None, None, None, None, None) == uqc.UQC_E_ARG
    assert L.uqc_scf_uhf(None, 0, None, None, 1, 0, None, None, None, None, None, None) == uqc.UQC_E_ARG
    assert L.uqc_mp2(None, None, None, 1, 0, 0.0, 0, None) == uqc.UQC_E_ARG
    assert L.uqc_fock_build_noalloc(None, None, None, None, None, None, None) == uqc.UQC_E_ARG
    o = uqc.scf_opts()
    assert o.max_iter == 100 and o.e_conv == 1e-10 and o.d_conv == 1e-8 and o.diis_size == 8
    assert o.guess_mix == 0.0
    assert o.fock.schwarz_tau == 1e-12 and o.fock.precision == uqc.FP64


def test_init_without_device_reports_device_error():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is visible")
    except Exception:
        pass
    L = uqc.load()
    h = ctypes.c_void_p()
    assert L.uqc_init(0, None, ctypes.byref(h)) == uqc.UQC_E_DEVICE
    assert L.uqc_last_error() != b""


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the public structs have the C compiler's sizes and field offsets."""
    import subprocess
    fields = {"uqc_fock_opts": (uqc.FockOpts, ["schwarz_tau", "precision", "fp64_bound", "timing", "progress",
                                                 "progress_user", "max_items_per_launch", "exchange_scale",
                                                 "streams"]),
              "uqc_stats": (uqc.Stats, [f for f, _ in uqc.Stats._fields_]),
              "uqc_scf_opts": (uqc.ScfOpts, [f for f, _ in uqc.ScfOpts._fields_]),
              "uqc_scf_result": (uqc.ScfResult, [f for f, _ in uqc.ScfResult._fields_]),
              "uqc_mp2_result": (uqc.Mp2Result, [f for f, _ in uqc.Mp2Result._fields_]),
              "uqc_request": (uqc.Request, [f for f, _ in uqc.Request._fields_]),
              "uqc_result": (uqc.Result, [f for f, _ in uqc.Result._fields_])}
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "uqc.h"', "int main(void) {"]
    for st, (_, fl) in fields.items():
        src.append('printf("%%s %%zu\\n", "%s", sizeof(%s));' % (st, st))
        for f in fl:
            src.append('printf("%%s.%%s %%zu\\n", "%s", "%s", offsetof(%s, %s));' % (st, f, st, f))
    src.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)])
    out = dict(line.rsplit(" ", 1) for line in subprocess.check_output([str(exe)]).decode().split("\n") if line)
    for st, (cls, fl) in fields.items():
        assert int(out[st]) == ctypes.sizeof(cls), st
        for f in fl:
            assert int(out[st + "." + f]) == getattr(cls, f).offset, (st, f)

"""Build step of libuqc: generate the per-class recursions, compile every HIP source for gfx950, link libuqc.so.

Usage:  python -m paper_1303_4916_amd.build [--incremental] [--jobs N]

The library lands in this package directory (in-tree), objects in <repo>/_build.  Every translation unit of the
quartet kernels holds one angular-momentum class, so the classes compile in parallel.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
GEN = os.path.join(CSRC, "generated")
OBJ = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libuqc.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled (they have produced silently wrong results on these devices); the host
# compilation pass warns that it does not know the feature, which is harmless.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]

PAIR = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)]

# classes whose quartet kernel is asked to fit a given number of wavefronts per SIMD, one more than the compiler's
# own register choice gives (none to a few dozen bytes of spill, measured faster per class); the others keep the
# compiler's choice (for them one more wavefront costs 130-340 bytes of spill per lane and was slower)
WAVES_PER_EU = {(2, 0, 1, 1): 2, (2, 1, 2, 1): 2, (2, 2, 1, 1): 2, (1, 1, 0, 0): 4, (1, 0, 1, 0): 4, (2, 0, 1, 0): 3}
# classes that do not keep their K_ac sums in LDS (the slots cost a wavefront per SIMD); none since the ket pairs
# of a bin are ordered by their kept primitive count: (dp|ps) had been the one, and with its kets' first-shell runs
# shorter its K_ac atomics doubled without the slots (275.6 ms per 150-atom build; 181.6 ms with them)
KAC_NOT_IN_LDS = set()
# classes whose FP64 Fock-build kernel reads the Boys rows from an LDS copy of its slice (measured per class: every
# plain class gains or breaks even except (ds|ps), (ds|pp) and (ds|ds), which run more wavefronts per SIMD without
# the rows' LDS and lose with it; (ds|ds): one workgroup per CU with the rows, two without, 132 vs 98.5 ms at 150
# atoms)
BOYS_LDS = {(0, 0, 0, 0), (1, 0, 0, 0), (1, 0, 1, 0), (1, 1, 0, 0), (2, 0, 0, 0), (1, 1, 1, 0), (2, 1, 0, 0),
            (2, 2, 0, 0), (1, 1, 1, 1), (2, 1, 1, 0), (2, 1, 1, 1), (2, 1, 2, 0), (2, 2, 1, 0)}


def classes():
    out = []
    for bi, (la, lb) in enumerate(PAIR):
        for ki in range(bi + 1):
            lc, ld = PAIR[ki]
            out.append((la, lb, lc, ld))
    return out


def _team_classes():
    import importlib.util
    spec = importlib.util.spec_from_file_location("gen_eri", os.path.join(CSRC, "gen_eri.py"))
    g = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(g)
    return set(g.TEAM_CLASSES)


def _units():
    headers = [os.path.join(CSRC, h) for h in ("uqc_internal.h", "uqc_device_common.h", "uqc_eri_impl.h",
                                               "uqc_api_internal.h")]
    headers += [os.path.join(GEN, "eri_classes.h"), os.path.join(GEN, "eri_flops.h"),
                os.path.join(ROOT, "include", "uqc.h"), os.path.join(CSRC, "uqc_one.h"),
                os.path.join(GEN, "one_electron.h")]
    units = []
    team = _team_classes()
    headers = headers + [os.path.join(CSRC, "uqc_eri_team.h"), os.path.join(GEN, "eri_team.h"),
                         os.path.join(CSRC, "uqc_rys.h"), os.path.join(GEN, "rys_consts.h"),
                         os.path.join(GEN, "rys_table.h")]
    for i, (la, lb, lc, ld) in enumerate(classes()):
        units.append((os.path.join(CSRC, "uqc_eri_class.hip"), os.path.join(OBJ, "eri_class_%02d.o" % i),
                      ["-DUQC_CLASS_ID=%d" % i, "-DUQC_LA=%d" % la, "-DUQC_LB=%d" % lb, "-DUQC_LC=%d" % lc,
                       "-DUQC_LD=%d" % ld, "-DUQC_TEAM=%d" % (1 if (la, lb, lc, ld) in team else 0)] +
                      (["-DUQC_WAVES_ATTR=__attribute__((amdgpu_waves_per_eu(%d)))" % WAVES_PER_EU[(la, lb, lc, ld)]]
                       if (la, lb, lc, ld) in WAVES_PER_EU else []) +
                      (["-DUQC_KAC_LDS=0"] if (la, lb, lc, ld) in KAC_NOT_IN_LDS else []) +
                      (["-DUQC_BOYS_LDS=1"] if (la, lb, lc, ld) in BOYS_LDS else []), headers))
    for src in ("uqc_kernels.hip", "uqc_one.hip", "uqc_mp2.hip", "uqc_noalloc.hip", "uqc_api.cpp", "uqc_serve.cpp",
                "uqc_scf.cpp"):
        units.append((os.path.join(CSRC, src), os.path.join(OBJ, os.path.splitext(src)[0] + ".o"), [], headers))
    # heaviest classes first so they start early
    units.sort(key=lambda u: -int(u[2][0].split("=")[1]) if u[2] else 0)
    return units


def _command(unit):
    src, obj, defs, _ = unit
    return [HIPCC] + FLAGS + defs + ["-c", src, "-o", obj]


def _stale(unit):
    """An object is rebuilt when it is missing, older than a source it depends on, or was compiled with another
    command line (recorded next to it)."""
    src, obj, _, deps = unit
    if not os.path.exists(obj) or not os.path.exists(obj + ".cmd"):
        return True
    if open(obj + ".cmd").read() != " ".join(_command(unit)):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in [src] + deps if os.path.exists(d))


def _compile(unit):
    obj = unit[1]
    cmd = _command(unit)
    t = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    with open(obj + ".cmd", "w") as f:
        f.write(" ".join(cmd))
    return os.path.basename(obj), time.time() - t


def build(incremental: bool = False, jobs: int = None, verbose: bool = True) -> str:
    os.makedirs(OBJ, exist_ok=True)
    for gen in ("gen_eri.py", "gen_one.py"):
        subprocess.check_call([sys.executable, os.path.join(CSRC, gen), GEN])
    # the Rys table takes ~15 s to compute: regenerated only when missing or older than its generator
    rys_out = [os.path.join(GEN, f) for f in ("rys_consts.h", "rys_table.h")]
    if any(not os.path.exists(f) or os.path.getmtime(f) < os.path.getmtime(os.path.join(CSRC, "gen_rys.py"))
           for f in rys_out):
        subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_rys.py"), GEN])
    units = _units()
    todo = [u for u in units if not incremental or _stale(u)]
    jobs = jobs or min(16, os.cpu_count() or 4)
    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for name, dt in ex.map(_compile, todo):
            if verbose:
                print("  compiled %-22s %6.1f s" % (name, dt), flush=True)
    objs = [u[1] for u in units]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built %s in %.1f s" % (LIB, time.time() - t0), flush=True)
    return LIB


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--incremental", action="store_true")
    ap.add_argument("--jobs", type=int, default=None)
    a = ap.parse_args()
    build(a.incremental, a.jobs)


if __name__ == "__main__":
    main()

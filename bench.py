#!/usr/bin/env python3
"""Benchmark: FP64 Fock builds G(D) = J(D) - K(D)/2 on one MI355X.

Workload (one step = one Fock build of the whole path: density preparation, every screened shell-quartet class
kernel with its J/K digest, finalisation to J, K, G and E2) on the medium synthetic system: 60 atoms on a jittered
2.5 bohr lattice, 2s1p1d Cartesian shells per atom (K = 3/3/3/1), N = 660 basis functions, Schwarz threshold 1e-12,
ten fresh PSD densities (trace 60) cycled over the steps.  The basis plan (normalisation, pair data, Schwarz bounds,
work lists) is built once before the timed region and reported separately (plan_ms).  Densities and outputs stay
in device memory (torch tensors); the call is synchronous.

Printed: one JSON line with the metric, the per-build latency percentiles, the roofline line of the dominant
class kernel (algorithmic FLOPs from the frozen per-class operation counts / its average launch time measured with
HIP events on the library's stream) and the oracle timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "shell quartets/s and Fock builds/s at ≤1e-6 Eh vs FP64; p50/p99 build latency"
FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CUs x 2.4 GHz x 128 FP64 FLOP/clk/CU
CLASS_NAME = "spd"


def class_name(cid: int) -> str:
    mixed = cid >= 10000
    c = cid % 10000
    digits = [c // 1000, (c // 100) % 10, (c // 10) % 10, c % 10]
    return "(" + "".join(CLASS_NAME[d] for d in digits[:2]) + "|" + "".join(CLASS_NAME[d] for d in digits[2:]) + \
           ")" + ("-mixed" if mixed else "")


def cpu_baseline(w, target_s: float = 15.0):
    """The oracle, unchanged, on a bounded uniform sample of bra shell pairs of the same workload: all their
    canonical ket partners, the same screening rule, one density.  Scaled to shell quartets/s."""
    import oracle
    nthreads = min(os.cpu_count() or 1, 16)
    oracle.set_threads(nthreads)
    O = oracle.Basis(w.shells)
    O.schwarz()  # screening bounds (part of the oracle's set-up, not timed)
    ns = O.nshell
    npair = ns * (ns + 1) // 2
    rng = np.random.default_rng(1234)
    order = rng.permutation(npair).astype(np.int32)
    D = w.densities[0]
    n = 16
    t_used = 0.0
    kept = 0
    t0 = time.perf_counter()
    pos = 0
    while pos < npair:
        take = order[pos:pos + n]
        t = time.perf_counter()
        _, _, cnt = O.jk_symmetric([D], tau=w.tau, bra_sample=take)
        dt = time.perf_counter() - t
        t_used += dt
        kept += int(cnt[0])
        pos += len(take)
        if time.perf_counter() - t0 >= target_s:
            break
        n = max(16, int(len(take) * min(4.0, max(1.2, (target_s - t_used) / max(dt, 1e-3) * 0.5))))
    return {"value": kept / t_used, "unit": "shell quartets/s", "cores": nthreads, "kind": "oracle",
            "sample": "%d of %d bra shell pairs (uniform, seed 1234) x all canonical kets, tau=%g, 1 density: "
                      "%d quartets in %.1f s" % (pos, npair, w.tau, kept, t_used)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-mixed", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (the Fock build would shard by "
              "bra-pair work lists with one all-reduce of J and K; not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1303_4916_amd import uqc
    from paper_1303_4916_amd import workloads as wl

    w = wl.medium(ndens=10)
    ctx = uqc.Context(0)
    t = time.perf_counter()
    B = uqc.Basis(ctx, w.shells)
    plan_ms = (time.perf_counter() - t) * 1e3
    N = B.nbf
    Ds = [torch.from_numpy(D).cuda() for D in w.densities]
    J = torch.empty((N, N), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    G = torch.empty_like(J)
    torch.cuda.synchronize()
    opts = uqc.default_opts(tau=w.tau, timing=True)
    t = time.perf_counter()
    st0 = B.fock_build_ptr(Ds[0].data_ptr(), J.data_ptr(), K.data_ptr(), G.data_ptr(), opts)  # plan for this tau
    first_ms = (time.perf_counter() - t) * 1e3
    for i in range(a.warmup):
        B.fock_build_ptr(Ds[i % len(Ds)].data_ptr(), J.data_ptr(), K.data_ptr(), G.data_ptr(), opts)
    torch.cuda.synchronize()
    lat = []
    cls_ms = {}
    cls_flops = {}
    cls_q = {}
    E2s = []
    t0 = time.perf_counter()
    for i in range(a.steps):
        ts = time.perf_counter()
        st = B.fock_build_ptr(Ds[i % len(Ds)].data_ptr(), J.data_ptr(), K.data_ptr(), G.data_ptr(), opts)
        lat.append((time.perf_counter() - ts) * 1e3)
        E2s.append(st.E2)
        for c in range(st.nclass):
            cid = int(st.class_id[c])
            cls_ms[cid] = cls_ms.get(cid, 0.0) + float(st.class_ms[c])
            cls_flops[cid] = float(st.class_flops[c])
            cls_q[cid] = int(st.class_quartets[c])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    q = int(st0.quartets)
    ms_per_step = elapsed * 1e3 / a.steps
    dom = max(cls_ms, key=lambda k: cls_ms[k])
    dom_avg_ms = cls_ms[dom] / a.steps
    achieved = cls_flops[dom] / (dom_avg_ms * 1e-3) / 1e12
    eri_ms = sum(cls_ms.values()) / a.steps
    total_flops = float(st0.flops)
    out = {
        "metric": METRIC,
        "value": q * a.steps / elapsed,
        "unit": "shell quartets/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "lattice60_2s1p1d: 60 atoms, N=660, K=3/3/3/1, tau=1e-12, FP64, 10 densities",
                   "natoms": 60, "nbf": N, "tau": w.tau, "precision": "fp64"},
        "fock_builds_per_s": a.steps / elapsed,
        "p50_build_ms": float(np.percentile(lat, 50)),
        "p99_build_ms": float(np.percentile(lat, 99)),
        "plan_ms": plan_ms,
        "first_build_ms": first_ms,
        "quartets_per_build": q,
        "quartets_screened_per_build": int(st0.quartets_screened),
        "prim_quartets_per_build": int(st0.prim_quartets),
        "algorithmic_flops_per_build": total_flops,
        "algorithmic_tflops": total_flops * a.steps / elapsed / 1e12,
        "eri_kernel_ms_per_build": eri_ms,
        "E2_first": E2s[0],
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "kernel": "k_digest " + class_name(dom), "kernel_avg_ms": dom_avg_ms,
                     "kernel_flops_per_launch": cls_flops[dom]},
        "classes": {class_name(k): {"ms": cls_ms[k] / a.steps, "quartets": cls_q[k],
                                    "tflops": cls_flops[k] / (cls_ms[k] / a.steps * 1e-3) / 1e12}
                    for k in sorted(cls_ms, key=lambda k: -cls_ms[k])},
    }
    if not a.no_mixed:
        mo = uqc.default_opts(tau=w.tau, precision=uqc.MIXED)
        B.fock_build_ptr(Ds[0].data_ptr(), J.data_ptr(), K.data_ptr(), G.data_ptr(), mo)
        nm = max(2, a.steps // 2)
        t = time.perf_counter()
        errs = []
        for i in range(nm):
            stm = B.fock_build_ptr(Ds[i % len(Ds)].data_ptr(), J.data_ptr(), K.data_ptr(), G.data_ptr(), mo)
            errs.append(abs(stm.E2 - E2s[i % len(E2s)]) if i < len(E2s) else float("nan"))
        tm = (time.perf_counter() - t) / nm
        out["mixed"] = {"fock_builds_per_s": 1.0 / tm, "speedup_vs_fp64": ms_per_step / (tm * 1e3),
                        "max_abs_E2_error_vs_fp64_Eh": float(np.nanmax(errs)),
                        "fp64_quartets_per_build": int(stm.fp64_quartets)}
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_seconds)
    print(json.dumps(out), flush=True)
    B.close()
    ctx.close()


if __name__ == "__main__":
    main()

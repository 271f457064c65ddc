#!/usr/bin/env python3
"""Benchmark: FP64 Fock builds G(D) = J(D) - K(D)/2 on one MI355X.

Workload (one step = one Fock build of the whole path: density preparation, every screened shell-quartet class
kernel with its J/K digest, finalisation to J, K, G and E2) on the 150-atom synthetic system: 150 atoms on a jittered
2.5 bohr lattice, 2s1p1d Cartesian shells per atom, the first (tighter) s shell contracted from 6 primitives and the
others K = 3/3/1 (s, p, d), N = 1650 basis functions, Schwarz threshold 1e-12, one PSD density of trace 150.  The
basis plan (normalisation, pair data, Schwarz bounds, work lists) is built once before the timed region and reported
separately (plan_ms).  Densities and outputs stay in device memory (torch tensors); the call is synchronous.

The timed builds use the library's default launch configuration (class kernels spread over three HIP streams).
Printed: one JSON line with the metric, the per-build latency percentiles, the roofline line of the dominant
class kernel (algorithmic FLOPs from the frozen per-class operation counts / its average launch time measured with
HIP events on the stream it runs on, in a second pass of builds with every class launch on one stream), the
mixed-precision leg against FP64 (energy, Fock-matrix and sampled ERI errors, speed), the 60-atom workload of the
medium configuration (N = 660, ten densities) as extra keys, and the oracle timed on a bounded sample on the host
cores.
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
TRAFFIC_FILES = {"lattice150": os.path.join(ROOT, "profiles", "traffic_lattice150_fp64.json"),
                 "medium": os.path.join(ROOT, "profiles", "traffic_medium60_fp64.json")}
TRAFFIC_FILE = TRAFFIC_FILES["lattice150"]


# Sources of the Fock-build kernels (the class-kernel unit and the headers it includes, the prepare/finalize unit,
# the generators and what they wrote, and the build step that sets per-class compile options); host-only files (the
# C ABI, SCF driver, server) do not change the kernels.
KERNEL_SOURCES = ("uqc_eri_class.hip", "uqc_eri_impl.h", "uqc_eri_team.h", "uqc_rys.h", "uqc_device_common.h",
                  "uqc_internal.h", "uqc_kernels.hip")


def kernel_sources_sha256() -> str:
    """Hash of every source the Fock-build kernels are built from (traffic counters are only valid for these); the
    Rys table headers are generated at build time from gen_rys.py, which is hashed, so they are left out."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1303_4916_amd", "csrc")
    names = [os.path.join(csrc, f) for f in KERNEL_SOURCES]
    names += sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith(".py"))
    names.append(os.path.join(ROOT, "paper_1303_4916_amd", "build.py"))
    gen = os.path.join(csrc, "generated")
    names += sorted(os.path.join(gen, f) for f in os.listdir(gen)
                    if f.endswith((".h", ".json")) and f not in ("rys_consts.h", "rys_table.h"))
    for n in names:
        h.update(os.path.basename(n).encode())
        h.update(open(n, "rb").read())
    return h.hexdigest()


def summarize_pmc(fetch_csv: str, write_csv: str, copy_fetch_csv: str, copy_write_csv: str, out: str, cmd: str,
                  builds: int = 0):
    """Per-kernel HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (KiB per dispatch), each scaled
    by the counter's reading for a plain 1 GiB device-to-device copy (bytes known).  builds > 0: the Fock builds of
    the counted run, so that bytes per build (a class may run as several dispatches per build) can be derived."""
    import csv

    def per_kernel(path, counter):
        acc = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            k = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("uqc::", "")
            v = acc.setdefault(k, [0.0, set()])
            v[0] += float(r["Counter_Value"])
            v[1].add(r["Dispatch_Id"])
        return {k: (v[0], len(v[1])) for k, v in acc.items()}

    cf, cw = per_kernel(copy_fetch_csv, "FETCH_SIZE"), per_kernel(copy_write_csv, "WRITE_SIZE")
    ck = max(cf, key=lambda k: cf[k][0])
    gib_kib = float(1 << 20)
    f_scale = gib_kib / (cf[ck][0] / cf[ck][1])
    w_scale = gib_kib / (cw[ck][0] / cw[ck][1]) if ck in cw else 1.0
    kf, kw = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    kernels = {}
    for k in kf:
        fb = kf[k][0] / kf[k][1] * f_scale * 1024
        wb = (kw[k][0] / kw[k][1] * w_scale * 1024) if k in kw else 0.0
        kernels[k] = {"fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb, "launches": kf[k][1]}
    doc = {"command": cmd, "copy_kernel": ck, "fetch_scale": f_scale, "write_scale": w_scale,
           "kernel_sources_sha256": kernel_sources_sha256(), "kernels": kernels}
    if builds:
        doc["builds"] = builds
    with open(out, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
    return doc


def summarize_stats(stats_path: str, out: str, cmd: str, title: str, builds: int = 0):
    """Markdown table of a rocprofv3 kernel summary: the --stats CSV (Name, Calls, AverageNs, TotalDurationNs,
    Percentage) or, for the database format, the per-kernel aggregate of its dispatches.  builds > 0 adds the time
    per Fock build (a class whose work list exceeds the per-launch cap runs as several dispatches per build)."""
    import csv
    rows = []
    if stats_path.endswith(".db"):
        import sqlite3
        con = sqlite3.connect(stats_path)
        agg = {}
        for name, dur in con.execute("select name, duration from kernels"):
            v = agg.setdefault(name, [0, 0.0])
            v[0] += 1
            v[1] += float(dur)
        tot = sum(v[1] for v in agg.values()) or 1.0
        src = [(n, v[0], v[1] / v[0], v[1], 100.0 * v[1] / tot) for n, v in agg.items()]
    else:
        src = [(r["Name"], int(r["Calls"]), float(r["AverageNs"]), float(r["TotalDurationNs"]), float(r["Percentage"]))
               for r in csv.DictReader(open(stats_path))]
    for name, calls, avg_ns, tot_ns, pct in src:
        k = name.split("(")[0].replace("void ", "").replace("uqc::", "")
        rows.append((k, calls, avg_ns * 1e-6, tot_ns * 1e-6, pct) + ((tot_ns * 1e-6 / builds,) if builds else ()))
    rows.sort(key=lambda r: -r[3])
    head = "| kernel | calls | avg ms | total ms | % |" + (" ms per build |" if builds else "")
    lines = ["# %s -- rocprofv3 kernel stats" % title, "", "Command (from the repository root):", "", "```", cmd,
             "```", "", "kernel_sources_sha256: %s" % kernel_sources_sha256(), ""]
    if builds:
        lines += ["Fock builds in the run: %d." % builds, ""]
    lines += [head, "|---|---|---|---|---|" + ("---|" if builds else "")]
    fmt = "| %s | %d | %.3f | %.2f | %.1f |" + (" %.2f |" if builds else "")
    lines += [fmt % r for r in rows]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def traffic_for(kernel_key: str, path: str = None):
    """HBM bytes per launch of a kernel from the committed counter summary, or None if the kernels changed since."""
    try:
        doc = json.load(open(path or TRAFFIC_FILE))
    except Exception:
        return None
    if doc.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    # the largest classes run as the team kernel (k_digest_team), the others as k_digest
    k = doc["kernels"].get(kernel_key) or doc["kernels"].get(kernel_key.replace("k_digest<", "k_digest_team<"))
    if not k:
        return None
    per_launch = k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]
    # per Fock build (the unit the achieved rate is measured in) when the counted run's build count is recorded
    return per_launch * k["launches"] / doc["builds"] if doc.get("builds") else per_launch
FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CUs x 2.4 GHz x 128 FP64 FLOP/clk/CU
CLASS_NAME = "spd"


def class_name(cid: int) -> str:
    mixed = cid >= 10000
    c = cid % 10000
    digits = [c // 1000, (c // 100) % 10, (c // 10) % 10, c % 10]
    return "(" + "".join(CLASS_NAME[d] for d in digits[:2]) + "|" + "".join(CLASS_NAME[d] for d in digits[2:]) + \
           ")" + ("-mixed" if mixed else "")


def cartesian_per_quartet(cid: int) -> int:
    """Cartesian integrals n_a n_b n_c n_d of one shell quartet of class id la*1000 + lb*100 + lc*10 + ld."""
    c = cid % 10000
    return int(np.prod([(l + 1) * (l + 2) // 2 for l in (c // 1000, (c // 100) % 10, (c // 10) % 10, c % 10)]))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def dom_kernel_key(cid: int) -> str:
    """rocprofv3 short name of the FP64/mixed closed-shell (one density) class kernel with this class id."""
    c = cid % 10000
    ls = [c // 1000, (c // 100) % 10, (c // 10) % 10, c % 10]
    return "k_digest<%d, %d, %d, %d, %s, 1>" % (ls[0], ls[1], ls[2], ls[3], "true" if cid >= 10000 else "false")


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
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
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
    ap.add_argument("--workload", default="lattice150",
                    choices=["lattice150", "medium", "mixed150", "large400", "large400kd1", "serve", "scf", "uhf",
                             "mp2", "rys", "oracle-c1", "copy"],
                    help="lattice150 (default, the benchmark line: 150 atoms, N=1650); medium: the same line on the "
                         "60-atom workload; mixed150 / large400: one-build mixed vs FP64 accuracy and speed; serve: "
                         "Poisson request stream through the continuous-batching server")
    ap.add_argument("--no-medium", action="store_true", help="leave out the 60-atom extra keys")
    ap.add_argument("--traffic-out", default=None, help="--summarize-pmc: output file (default: lattice150's)")
    ap.add_argument("--nreq", type=int, default=32, help="serve: requests taken from the 512-request stream")
    ap.add_argument("--rate", type=float, default=200.0,
                    help="serve: mean arrival rate in requests/s (the stream's 200, or a sustainable rate)")
    ap.add_argument("--oracle-quartets", type=int, default=2000,
                    help="ERI sample size of the accuracy legs (oracle against both precisions)")
    ap.add_argument("--fp64-bound", type=float, default=None,
                    help="mixed150/large400: the mixed leg's FP64 routing bound (default: the library's 1e-8)")
    ap.add_argument("--streams", type=int, default=None,
                    help="HIP streams the class launches of one Fock build are spread over (default: the library's)")
    ap.add_argument("--fp64-only", action="store_true",
                    help="mixed150/large400/serve: time the FP64 leg only (no mixed build, no mixed-vs-FP64 errors)")
    ap.add_argument("--summarize-pmc", nargs=5, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV",
                                                         "COPY_WRITE_CSV", "CMD"),
                    help="write the per-kernel traffic summary from rocprofv3 counter CSVs and exit")
    ap.add_argument("--summarize-stats", nargs=4, metavar=("STATS_CSV_OR_DB", "OUT_MD", "CMD", "TITLE"),
                    help="write a markdown summary of a rocprofv3 kernel stats CSV (or results database) and exit")
    ap.add_argument("--builds", type=int, default=0,
                    help="--summarize-stats / --summarize-pmc: Fock builds in the profiled run")
    a = ap.parse_args()
    if a.summarize_stats:
        summarize_stats(*a.summarize_stats, builds=a.builds)
        return
    if a.summarize_pmc:
        summarize_pmc(*a.summarize_pmc[:4], a.traffic_out or TRAFFIC_FILE, a.summarize_pmc[4], builds=a.builds)
        return
    if a.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (the Fock build would shard by "
              "bra-pair work lists with one all-reduce of J and K; not built).", file=sys.stderr)
        sys.exit(2)

    if a.workload == "serve":
        return bench_serve(a)
    if a.workload == "copy":
        return bench_copy(a)
    if a.workload == "scf":
        return bench_scf(a)
    if a.workload == "uhf":
        return bench_uhf(a)
    if a.workload == "mp2":
        return bench_mp2(a)
    if a.workload == "rys":
        return bench_rys(a)
    if a.workload == "oracle-c1":
        return bench_oracle_c1(a)
    if a.workload in ("mixed150", "large400", "large400kd1"):
        return bench_mixed(a)

    out = bench_fock(a)
    print(json.dumps(out), flush=True)


WORKLOAD_NAMES = {
    "lattice150": "lattice150_2s1p1d: 150 atoms, N=1650, first s K=6, K=3/3/1 otherwise, tau=1e-12, FP64, 1 density",
    "medium": "lattice60_2s1p1d: 60 atoms, N=660, K=3/3/3/1, tau=1e-12, FP64, 10 densities",
}


def fock_leg(B, Ds, tau, steps, warmup, streams, one_stream_builds, traffic_path):
    """Timed FP64 builds (the library's default launch configuration), then a pass of `one_stream_builds` builds
    with every class launch on one stream and HIP-event timing per class (roofline of the dominant class kernel)."""
    import torch
    from paper_1303_4916_amd import uqc
    N = B.nbf
    J = torch.empty((N, N), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    G = torch.empty_like(J)
    torch.cuda.synchronize()
    opts = uqc.default_opts(tau=tau, streams=streams)
    sopts = uqc.default_opts(tau=tau, timing=True, streams=1)
    build = lambda i, o: B.fock_build_ptr(Ds[i % len(Ds)].data_ptr(), J.data_ptr(), K.data_ptr(), G.data_ptr(), o)
    t = time.perf_counter()
    st0 = build(0, opts)  # makes the plan for this tau
    first_ms = (time.perf_counter() - t) * 1e3
    for i in range(warmup):
        build(i, opts)
    torch.cuda.synchronize()
    lat, E2s = [], []
    t0 = time.perf_counter()
    for i in range(steps):
        ts = time.perf_counter()
        st = build(i, opts)
        lat.append((time.perf_counter() - ts) * 1e3)
        E2s.append(st.E2)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    G0 = None
    if len(Ds) == 1:
        G0 = G.cpu().numpy().copy()
    cls_ms, cls_flops, cls_q = {}, {}, {}
    n1 = max(1, min(steps, one_stream_builds))
    t1 = time.perf_counter()
    for i in range(n1):
        st = build(i, sopts)
        for c in range(st.nclass):
            cid = int(st.class_id[c])
            cls_ms[cid] = cls_ms.get(cid, 0.0) + float(st.class_ms[c])
            cls_flops[cid] = float(st.class_flops[c])
            cls_q[cid] = int(st.class_quartets[c])
    torch.cuda.synchronize()
    serial_ms = (time.perf_counter() - t1) * 1e3 / n1
    q = int(st0.quartets)
    dom = max(cls_ms, key=lambda k: cls_ms[k])
    dom_avg_ms = cls_ms[dom] / n1
    achieved = cls_flops[dom] / (dom_avg_ms * 1e-3) / 1e12
    total_flops = float(st0.flops)
    res = {
        "value": q * steps / elapsed,
        "ms_per_step": elapsed * 1e3 / steps,
        "fock_builds_per_s": steps / elapsed,
        "p50_build_ms": float(np.percentile(lat, 50)),
        "p99_build_ms": float(np.percentile(lat, 99)),
        "first_build_ms": first_ms,
        "quartets_per_build": q,
        "quartets_screened_per_build": int(st0.quartets_screened),
        "prim_quartets_per_build": int(st0.prim_quartets),
        "prim_quartets_per_s": int(st0.prim_quartets) * steps / elapsed,
        "cartesian_integrals_per_s": sum(cls_q[k] * cartesian_per_quartet(k) for k in cls_q) * steps / elapsed,
        "algorithmic_flops_per_build": total_flops,
        "algorithmic_tflops": total_flops * steps / elapsed / 1e12,
        "one_stream_ms_per_build": serial_ms,
        "one_stream_builds": n1,
        "eri_kernel_ms_per_build_one_stream": sum(cls_ms.values()) / n1,
        "E2_first": E2s[0],
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": traffic_for(dom_kernel_key(dom), traffic_path),
                     "kernel": "k_digest " + class_name(dom), "kernel_avg_ms": dom_avg_ms,
                     "kernel_flops_per_launch": cls_flops[dom],
                     "per": "the class's work in one Fock build (time, FLOPs and traffic summed over its dispatches)",
                     "timed_in": "the one-stream pass of the same builds (each kernel alone on the chip)"},
        "classes": {class_name(k): {"ms": cls_ms[k] / n1, "quartets": cls_q[k],
                                    "tflops": cls_flops[k] / (cls_ms[k] / n1 * 1e-3) / 1e12}
                    for k in sorted(cls_ms, key=lambda k: -cls_ms[k])},
    }
    return res, E2s, G0, (J, K, G)


def mixed_leg(B, Ds, tau, builds, streams, E2_fp64, G_fp64, bufs):
    """Mixed-precision builds of the same densities: speed and error against the FP64 builds."""
    import torch
    from paper_1303_4916_amd import uqc
    J, K, G = bufs
    mo = uqc.default_opts(tau=tau, precision=uqc.MIXED, streams=streams)
    B.fock_build_ptr(Ds[0].data_ptr(), J.data_ptr(), K.data_ptr(), G.data_ptr(), mo)  # plan for this routing
    torch.cuda.synchronize()
    nm = max(1, builds)
    errs = []
    t = time.perf_counter()
    for i in range(nm):
        stm = B.fock_build_ptr(Ds[i % len(Ds)].data_ptr(), J.data_ptr(), K.data_ptr(), G.data_ptr(), mo)
        errs.append(abs(stm.E2 - E2_fp64[i % len(E2_fp64)]) if i < len(E2_fp64) else float("nan"))
    torch.cuda.synchronize()
    tm = (time.perf_counter() - t) / nm
    out = {"fock_builds_per_s": 1.0 / tm, "ms_per_build": tm * 1e3, "fp64_bound": float(mo.fp64_bound),
           "max_abs_E2_error_vs_fp64_Eh": float(np.nanmax(errs)),
           "meets_1e-6_Eh": bool(np.nanmax(errs) <= 1e-6),
           "fp64_quartets_per_build": int(stm.fp64_quartets), "quartets_per_build": int(stm.quartets),
           "fp32_share_of_quartets": 1.0 - stm.fp64_quartets / max(1, stm.quartets)}
    if G_fp64 is not None:
        Gm = G.cpu().numpy()
        out["G_frobenius_rel_error_vs_fp64"] = float(np.linalg.norm(Gm - G_fp64) / np.linalg.norm(G_fp64))
        out["G_max_abs_error_vs_fp64"] = float(np.max(np.abs(Gm - G_fp64)))
    return out, tm


def eri_sample_errors(B, shells, n, seed):
    """Largest ERI error of both precisions against the oracle on a uniform sample of canonical shell quartets."""
    import oracle
    from paper_1303_4916_amd import uqc
    q = _sample_quartets(B.nshell, n, seed)
    O = oracle.Basis(shells)
    e64 = em = ref_max = 0.0
    for (qa, qb, qc, qd), x64, xm in zip(q, B.eri_blocks(q, uqc.FP64), B.eri_blocks(q, uqc.MIXED)):
        r = O.eri(int(qa), int(qb), int(qc), int(qd))
        e64 = max(e64, float(np.max(np.abs(x64 - r))))
        em = max(em, float(np.max(np.abs(xm - r))))
        ref_max = max(ref_max, float(np.max(np.abs(r))))
    return {"quartets": int(len(q)), "max_abs_eri_error_fp64": e64, "max_abs_eri_error_mixed": em,
            "max_abs_eri": ref_max, "sample": "uniform over canonical shell quartets, seed %d" % seed}


def bench_fock(a):
    """The benchmark line: FP64 Fock builds of the chosen workload (default: 150 atoms), the mixed leg, the 60-atom
    workload as extra keys, the oracle on a bounded sample of the same workload."""
    import torch
    from paper_1303_4916_amd import uqc
    from paper_1303_4916_amd import workloads as wl

    w = wl.mixed150(ndens=1) if a.workload == "lattice150" else wl.medium(ndens=10)
    ctx = uqc.Context(0)
    t = time.perf_counter()
    B = uqc.Basis(ctx, w.shells)
    plan_ms = (time.perf_counter() - t) * 1e3
    Ds = [torch.from_numpy(D).cuda() for D in w.densities]
    big = a.workload == "lattice150"
    print("%s: N=%d, plan %.0f ms" % (w.name, B.nbf, plan_ms), file=sys.stderr, flush=True)
    res, E2s, G0, bufs = fock_leg(B, Ds, w.tau, a.steps, a.warmup, a.streams, 3 if big else a.steps,
                                  TRAFFIC_FILES[a.workload])
    print("  FP64: %.1f ms per build, %.3e quartets/s" % (res["ms_per_step"], res["value"]), file=sys.stderr,
          flush=True)
    opts = uqc.default_opts(tau=w.tau, streams=a.streams)
    out = {
        "metric": METRIC,
        "value": res.pop("value"),
        "unit": "shell quartets/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": res.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_NAMES[a.workload], "natoms": w.natoms, "nbf": B.nbf, "tau": w.tau,
                   "precision": "fp64", "streams": int(opts.streams)},
        "plan_ms": plan_ms,
    }
    out.update(res)
    if not a.no_mixed:
        m, tm = mixed_leg(B, Ds, w.tau, 3 if big else max(2, a.steps // 2), a.streams, E2s, G0, bufs)
        m["speedup_vs_fp64"] = out["ms_per_step"] / (tm * 1e3)
        out["mixed"] = m
        print("  mixed: %.1f ms per build, |dE2| %.2e Eh" % (tm * 1e3, m["max_abs_E2_error_vs_fp64_Eh"]),
              file=sys.stderr, flush=True)
        out["mixed"]["oracle_sample"] = eri_sample_errors(B, w.shells, a.oracle_quartets, 31)
    if big and not a.no_medium:
        wm = wl.medium(ndens=10)
        Bm = uqc.Basis(ctx, wm.shells)
        Dm = [torch.from_numpy(D).cuda() for D in wm.densities]
        rm, _, _, _ = fock_leg(Bm, Dm, wm.tau, 10, 2, a.streams, 10, TRAFFIC_FILES["medium"])
        out["medium60"] = {"workload": WORKLOAD_NAMES["medium"], "quartets_per_s": rm["value"],
                           "fock_builds_per_s": rm["fock_builds_per_s"], "ms_per_build": rm["ms_per_step"],
                           "p50_build_ms": rm["p50_build_ms"], "p99_build_ms": rm["p99_build_ms"],
                           "algorithmic_tflops": rm["algorithmic_tflops"], "roofline": rm["roofline"]}
        Bm.close()
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_seconds)
    B.close()
    ctx.close()
    return out


def _sample_quartets(nshell: int, n: int, seed: int) -> np.ndarray:
    """Uniform sample of canonical shell quartets (a>=b, c>=d, ab>=cd)."""
    rng = np.random.default_rng(seed)
    npair = nshell * (nshell + 1) // 2
    out = []
    while len(out) < n:
        p = rng.integers(0, npair, size=(4 * n, 2))
        p.sort(axis=1)
        for cd, ab in p:
            a = int((np.sqrt(8 * ab + 1) - 1) // 2)
            b = int(ab - a * (a + 1) // 2)
            c = int((np.sqrt(8 * cd + 1) - 1) // 2)
            d = int(cd - c * (c + 1) // 2)
            out.append((a, b, c, d))
            if len(out) == n:
                break
    return np.array(out, dtype=np.int32)


def bench_mixed(a):
    """Mixed precision (FP32 recursions, FP64 accumulation) vs the FP64 path on one system: full-build G and E2
    errors, ERI-block errors of both precisions vs the oracle on a uniform sample of canonical quartets."""
    import torch
    from paper_1303_4916_amd import uqc
    from paper_1303_4916_amd import workloads as wl
    import oracle

    if a.workload == "mixed150":
        w = wl.mixed150(ndens=1)
    else:
        w = wl.large400(ndens=1, k_d=1 if a.workload == "large400kd1" else 3)
    ctx = uqc.Context(0)
    t = time.perf_counter()
    B = uqc.Basis(ctx, w.shells)
    plan_ms = (time.perf_counter() - t) * 1e3
    N = B.nbf
    D = torch.from_numpy(w.densities[0]).cuda()
    J = torch.empty((N, N), dtype=torch.float64, device="cuda")
    K = torch.empty_like(J)
    G = torch.empty_like(J)
    res = {}
    print("%s: N=%d, plan %.0f ms" % (w.name, N, plan_ms), file=sys.stderr, flush=True)
    def report(cid, done, total):
        print("    class %s: %d of %d work items" % (class_name(cid), done, total), file=sys.stderr, flush=True)

    legs = [("fp64", uqc.default_opts(tau=w.tau, timing=True, progress=report)),
            ("mixed", uqc.default_opts(tau=w.tau, precision=uqc.MIXED, timing=True, progress=report,
                                       fp64_bound=a.fp64_bound if a.fp64_bound is not None else 1e-8))]
    for name, opts in legs[:1] if a.fp64_only else legs:
        times = []
        for rep in range(max(1, a.steps)):
            torch.cuda.synchronize()
            t = time.perf_counter()
            st = B.fock_build_ptr(D.data_ptr(), J.data_ptr(), K.data_ptr(), G.data_ptr(), opts)
            times.append(time.perf_counter() - t)
            print("  %s build %d: %.1f ms" % (name, rep, times[-1] * 1e3), file=sys.stderr, flush=True)
        res[name] = {"ms": 1e3 * min(times), "E2": st.E2, "G": G.cpu().numpy().copy(), "quartets": st.quartets,
                     "fp64_quartets": st.fp64_quartets, "flops": st.flops}
    mixed = "mixed" in res
    q = _sample_quartets(B.nshell, a.oracle_quartets, 31)
    O = oracle.Basis(w.shells)
    oracle.set_threads(min(os.cpu_count() or 1, 16))
    e64 = em = ref_max = 0.0
    b64 = B.eri_blocks(q, uqc.FP64)
    bm = B.eri_blocks(q, uqc.MIXED) if mixed else b64
    for (qa, qb, qc, qd), x64, xm in zip(q, b64, bm):
        r = O.eri(int(qa), int(qb), int(qc), int(qd))
        e64 = max(e64, float(np.max(np.abs(x64 - r))))
        em = max(em, float(np.max(np.abs(xm - r))))
        ref_max = max(ref_max, float(np.max(np.abs(r))))
    head = res["mixed"] if mixed else res["fp64"]
    out = {
        "metric": METRIC,
        "value": head["quartets"] / (head["ms"] * 1e-3),
        "unit": "shell quartets/s",
        "n_gpus": 1, "steps": a.steps, "warmup": 0,
        "ms_per_step": head["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 recursions + f64 accumulation" if mixed else "f64", "data": "synthetic",
        "config": {"workload": w.name + {"mixed150": ": 150 atoms, N=1650, first s K=6, tau=1e-12",
                                         "large400": ": 400 atoms, N=4400, K=3 on every shell, tau=1e-11",
                                         "large400kd1": ": 400 atoms, N=4400, K=3 on s and p, K=1 on d, "
                                                        "tau=1e-11"}[a.workload],
                   "nbf": N, "tau": w.tau,
                   "fp64_bound": (a.fp64_bound if a.fp64_bound is not None else uqc.default_opts().fp64_bound)
                   if mixed else None},
        "plan_ms": plan_ms,
        "fp64_build_ms": res["fp64"]["ms"],
        "quartets_per_build": res["fp64"]["quartets"],
        "E2_fp64": res["fp64"]["E2"],
        "oracle_sample": {"quartets": int(len(q)), "max_abs_eri_error_fp64": e64,
                          "max_abs_eri": ref_max, "sample": "uniform over canonical shell quartets, seed 31"},
        "fp64_tflops_algorithmic": res["fp64"]["flops"] / (res["fp64"]["ms"] * 1e-3) / 1e12,
    }
    if mixed:
        G64, Gm = res["fp64"]["G"], res["mixed"]["G"]
        out.update({
            "mixed_build_ms": res["mixed"]["ms"],
            "mixed_speedup_vs_fp64": res["fp64"]["ms"] / res["mixed"]["ms"],
            "mixed_fp64_routed_quartets": res["mixed"]["fp64_quartets"],
            "abs_E2_error_mixed_vs_fp64_Eh": abs(res["mixed"]["E2"] - res["fp64"]["E2"]),
            "G_frobenius_rel_error_mixed_vs_fp64": float(np.linalg.norm(Gm - G64) / np.linalg.norm(G64)),
            "G_max_abs_error_mixed_vs_fp64": float(np.max(np.abs(Gm - G64))),
        })
        out["oracle_sample"]["max_abs_eri_error_mixed"] = em
    print(json.dumps(out), flush=True)
    B.close()
    ctx.close()


def bench_scf(a):
    """Restricted Hartree-Fock on the medium lattice (60 centres, unit nuclear charges, 30 doubly occupied orbitals,
    2s1p1d basis, N = 660): the whole SCF on the GPU (one-electron integrals, orthogonalisation, DIIS, Fock builds,
    eigendecompositions).  The converged state is checked on the host: P S P = 2 P, tr(P S) = 60, F P S = S P F."""
    from paper_1303_4916_amd import uqc
    from paper_1303_4916_amd import workloads as wl

    w = wl.medium(ndens=1)
    sh = w.shells
    nat = int(np.max(sh.atom)) + 1
    R = np.array([sh.center[np.where(sh.atom == x)[0][0]] for x in range(nat)])
    Z = np.ones(nat)
    ctx = uqc.Context(0)
    B = uqc.Basis(ctx, sh)
    opts = uqc.scf_opts(fock=uqc.default_opts(tau=w.tau))
    B.scf_rhf(Z, R, nat // 2, uqc.scf_opts(max_iter=1, fock=uqc.default_opts(tau=w.tau)))  # plan and warm-up
    runs = []
    for _ in range(max(1, a.steps)):
        r = B.scf_rhf(Z, R, nat // 2, opts)
        runs.append(r)
        print("  scf: %d iterations, %.1f ms (Fock builds %.1f ms), E = %.10f, converged %s" % (
            r["iterations"], r["ms"], r["fock_ms"], r["E_total"], r["converged"]), file=sys.stderr, flush=True)
    r = min(runs, key=lambda x: x["ms"])
    S, T, V = B.one_electron(Z, R)
    P = r["P"]
    J, K, G, _ = B.fock_build(P, uqc.default_opts(tau=w.tau))
    F = T + V + G
    out = {"metric": METRIC, "value": r["iterations"] * r["quartets"] / (r["ms"] * 1e-3), "unit": "shell quartets/s",
           "n_gpus": 1, "steps": len(runs), "warmup": 1, "ms_per_step": r["ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "rhf_lattice60: 60 unit charges, 30 doubly occupied orbitals, N=%d, tau=%g, "
                                  "DIIS 8" % (B.nbf, w.tau)},
           "scf_ms": r["ms"], "fock_ms": r["fock_ms"], "iterations": r["iterations"], "converged": r["converged"],
           "E_total": r["E_total"], "E_nuc": r["E_nuc"], "final_error": r["error"],
           "fock_builds_per_s": r["iterations"] / (r["ms"] * 1e-3),
           "check_PSP_minus_2P": float(np.max(np.abs(P @ S @ P - 2.0 * P))),
           "check_trace_PS": float(np.sum(P * S)),
           "check_FPS_minus_SPF": float(np.max(np.abs(F @ P @ S - S @ P @ F)))}
    print(json.dumps(out), flush=True)
    B.close()
    ctx.close()


def bench_uhf(a):
    """Unrestricted Hartree-Fock on the medium lattice (60 unit nuclear charges, 31 alpha and 29 beta electrons,
    2s1p1d basis, N = 660): the whole SCF on the GPU, each iteration one spin-density Fock build.  The converged
    state is checked on the host: P^s S P^s = P^s, tr(P^s S) = n_s, F^s P^s S = S P^s F^s."""
    from paper_1303_4916_amd import uqc
    from paper_1303_4916_amd import workloads as wl

    w = wl.medium(ndens=1)
    sh = w.shells
    nat = int(np.max(sh.atom)) + 1
    R = np.array([sh.center[np.where(sh.atom == x)[0][0]] for x in range(nat)])
    Z = np.ones(nat)
    na, nb = nat // 2 + 1, nat // 2 - 1
    ctx = uqc.Context(0)
    B = uqc.Basis(ctx, sh)
    opts = uqc.scf_opts(fock=uqc.default_opts(tau=w.tau))
    B.scf_uhf(Z, R, na, nb, uqc.scf_opts(max_iter=1, fock=uqc.default_opts(tau=w.tau)))  # plan and warm-up
    runs = []
    for _ in range(max(1, a.steps)):
        r = B.scf_uhf(Z, R, na, nb, opts)
        runs.append(r)
        print("  uhf: %d iterations, %.1f ms (Fock builds %.1f ms), E = %.10f, <S^2> = %.6f, converged %s" % (
            r["iterations"], r["ms"], r["fock_ms"], r["E_total"], r["s2"], r["converged"]), file=sys.stderr,
            flush=True)
    r = min(runs, key=lambda x: x["ms"])
    S, T, V = B.one_electron(Z, R)
    f = B.fock_build_uhf(r["Pa"], r["Pb"], uqc.default_opts(tau=w.tau), want=("Ga", "Gb"))
    checks = {}
    for sp, P, G, n in (("a", r["Pa"], f["Ga"], na), ("b", r["Pb"], f["Gb"], nb)):
        F = T + V + G
        checks["check_PSP_minus_P_" + sp] = float(np.max(np.abs(P @ S @ P - P)))
        checks["check_trace_PS_" + sp] = float(np.sum(P * S))
        checks["check_FPS_minus_SPF_" + sp] = float(np.max(np.abs(F @ P @ S - S @ P @ F)))
    out = {"metric": METRIC, "value": r["iterations"] * r["quartets"] / (r["ms"] * 1e-3), "unit": "shell quartets/s",
           "n_gpus": 1, "steps": len(runs), "warmup": 1, "ms_per_step": r["ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "uhf_lattice60: 60 unit charges, %d alpha and %d beta electrons, N=%d, tau=%g, "
                                  "DIIS 8" % (na, nb, B.nbf, w.tau)},
           "scf_ms": r["ms"], "fock_ms": r["fock_ms"], "fock_ms_per_build": r["fock_ms"] / r["iterations"],
           "iterations": r["iterations"], "converged": r["converged"], "E_total": r["E_total"], "E_nuc": r["E_nuc"],
           "S2": r["s2"], "final_error": r["error"], "fock_builds_per_s": r["iterations"] / (r["ms"] * 1e-3)}
    out.update(checks)
    print(json.dumps(out), flush=True)
    B.close()
    ctx.close()


def bench_mp2(a):
    """Closed-shell MP2 on a 20-atom lattice (unit nuclear charges, 10 doubly occupied orbitals, 2s1p1d, N = 220):
    restricted SCF on the GPU, canonical orbitals, then the timed MP2 calls (AO tensor of 220^4 doubles in HBM,
    four GEMM quarter transformations, energy).  The transformation GEMMs are the dense, matrix-core part; their
    rate is reported against the FP64 matrix peak."""
    from paper_1303_4916_amd import uqc
    from paper_1303_4916_amd import workloads as wl

    natoms = 20
    sh = wl.lattice(natoms, seed=2, ndens=1).shells
    nat = int(np.max(sh.atom)) + 1
    R = np.array([sh.center[np.where(sh.atom == x)[0][0]] for x in range(nat)])
    Z = np.ones(nat)
    nocc = natoms // 2
    ctx = uqc.Context(0)
    B = uqc.Basis(ctx, sh)
    s = B.scf_rhf(Z, R, nocc, uqc.scf_opts(e_conv=1e-11, d_conv=1e-9))
    S, T, V = B.one_electron(Z, R)
    _, _, G, _ = B.fock_build(s["P"])
    w, U = np.linalg.eigh(S)
    X = U @ np.diag(w ** -0.5) @ U.T
    eps, Cp = np.linalg.eigh(X.T @ (T + V + G) @ X)
    C = X @ Cp
    print("  scf: %d iterations, E = %.10f" % (s["iterations"], s["E_total"]), file=sys.stderr, flush=True)
    B.mp2(C, eps, nocc, tau=1e-12)  # warm-up
    runs = []
    for _ in range(max(1, a.steps)):
        m = B.mp2(C, eps, nocc, tau=1e-12)
        runs.append(m)
        print("  mp2: %.1f ms (AO %.1f, transform %.1f, energy %.1f), E2 = %.12f" % (
            m["ms"], m["ao_ms"], m["transform_ms"], m["energy_ms"], m["e2"]), file=sys.stderr, flush=True)
    m = min(runs, key=lambda x: x["ms"])
    tf = m["transform_flops"] / (m["transform_ms"] * 1e-3) / 1e12
    out = {"metric": "MP2 correlation energies per second", "value": 1e3 / m["ms"], "unit": "MP2 energies/s",
           "n_gpus": 1, "steps": len(runs), "warmup": 1, "ms_per_step": m["ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "mp2_lattice20: 20 unit charges, 10 doubly occupied orbitals, N=%d, tau=1e-12"
                                  % B.nbf},
           "e2": m["e2"], "e_os": m["e_os"], "e_ss": m["e_ss"], "E_scf": s["E_total"],
           "ao_ms": m["ao_ms"], "transform_ms": m["transform_ms"], "energy_ms": m["energy_ms"],
           "ao_quartets": m["quartets"], "transform_flops": m["transform_flops"],
           "roofline_transform": {"bound": "mfma", "achieved": tf, "peak": 78.6, "unit": "TFLOP/s",
                                  "frac": tf / 78.6,
                                  "note": "the four quarter transformations timed together: the first (k_mp2_q1, "
                                          "HBM-bound) and three rocBLAS FP64 GEMMs"}}
    print(json.dumps(out), flush=True)
    B.close()
    ctx.close()


def bench_rys(a):
    """The same ERI blocks by the Obara-Saika/HGP list kernel and by Rys quadrature, per class: 4096 shell
    quartets of each class drawn from the medium lattice's shells (seed 5); wall time of uqc_eri_blocks per method
    (the host-side bookkeeping is identical for both) and the largest difference between the two methods.  The
    kernel durations come from a rocprofv3 kernel trace of this command (k_list vs k_list_rys)."""
    from paper_1303_4916_amd import uqc
    from paper_1303_4916_amd import workloads as wl

    w = wl.medium(ndens=1)
    ctx = uqc.Context(0)
    B = uqc.Basis(ctx, w.shells)
    rng = np.random.default_rng(5)
    by_l = {l: np.where(B.l == l)[0] for l in range(3)}
    classes = [(la, lb, lc, ld) for la in range(3) for lb in range(la + 1) for lc in range(3) for ld in range(lc + 1)
               if (la, lb) >= (lc, ld)]
    res = {}
    for ls in classes:
        q = np.stack([rng.choice(by_l[l], size=4096) for l in ls], axis=1).astype(np.int32)
        B.eri_blocks(q[:64], uqc.FP64)
        B.eri_blocks(q[:64], uqc.RYS)
        t = time.perf_counter()
        x = B.eri_blocks(q, uqc.FP64)
        t1 = time.perf_counter()
        y = B.eri_blocks(q, uqc.RYS)
        t2 = time.perf_counter()
        d = max(float(np.max(np.abs(u - v))) for u, v in zip(x, y))
        m = max(float(np.max(np.abs(u))) for u in x)
        name = "(" + "".join("spd"[l] for l in ls[:2]) + "|" + "".join("spd"[l] for l in ls[2:]) + ")"
        res[name] = {"hgp_ms": (t1 - t) * 1e3, "rys_ms": (t2 - t1) * 1e3, "max_abs_diff": d, "max_abs": m}
        print("  %s hgp %.1f ms, rys %.1f ms, max |diff| %.2e" % (name, res[name]["hgp_ms"], res[name]["rys_ms"], d),
              file=sys.stderr, flush=True)
    out = {"metric": "shell quartets/s per method and class (explicit ERI blocks)", "unit": "shell quartets/s",
           "value": 4096 * len(classes) / (sum(v["rys_ms"] for v in res.values()) * 1e-3), "n_gpus": 1,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "eri_blocks_lattice60: 4096 quartets per class, both methods"}, "classes": res}
    print(json.dumps(out), flush=True)
    B.close()
    ctx.close()


def bench_oracle_c1(a):
    """The oracle alone on the host, one thread, on the 8-atom cube (16 shells, N = 32): the full ERI tensor and one
    J/K build of its density by the definition of Eq. (12), every quartet (no GPU)."""
    import oracle
    from paper_1303_4916_amd import workloads as wl
    w = wl.cube()
    oracle.set_threads(1)
    O = oracle.Basis(w.shells)
    t = time.perf_counter()
    O.eri_tensor()
    t_tensor = time.perf_counter() - t
    t = time.perf_counter()
    O.jk_direct([w.densities[0]])
    t_jk = time.perf_counter() - t
    print(json.dumps({"workload": "oracle_cube8: 16 shells, N = 32, one thread", "cpu_model": cpu_model(),
                      "eri_tensor_s": t_tensor, "jk_direct_s": t_jk}), flush=True)


def bench_copy(a):
    """Reference for hardware traffic counters: a plain device-to-device copy of exactly 1 GiB, three times."""
    import torch
    n = (1 << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / 3
    print(json.dumps({"workload": "copy 1 GiB", "bytes_read": 1 << 30, "bytes_written": 1 << 30,
                      "GBps_read_plus_write": 2 * (1 << 30) / dt / 1e9}), flush=True)


def bench_serve(a):
    """Poisson stream of Fock-build requests (mean 200 req/s, 4-120 atoms log-uniform, 8 iterations each) through
    the continuous-batching server, FP64 and mixed side by side; per-request latency = finish - submit."""
    from paper_1303_4916_amd import uqc
    from paper_1303_4916_amd import workloads as wl

    stream = wl.stream(512)[:a.nreq]
    ctx = uqc.Context(0)
    out = {"metric": METRIC, "unit": "requests/s", "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "data": "synthetic",
           "config": {"workload": "poisson%g_4to120atoms_8iter: first %d of 512 requests%s" % (
               a.rate, len(stream), "" if a.rate == 200.0 else " (arrival times of the 200 req/s stream scaled)"),
                      "budget_GiB": 64, "slots": 16}}
    legs = [("fp64", uqc.FP64), ("mixed", uqc.MIXED)]
    for prec_name, prec in legs[:1] if a.fp64_only else legs:
        srv = uqc.Server(ctx, 64 << 30, 16)
        t0 = time.perf_counter()
        tickets = []
        for r in stream:
            now = time.perf_counter() - t0
            arrive = r.arrival_s * (200.0 / a.rate)
            if arrive > now:
                time.sleep(arrive - now)
            tickets.append(srv.submit(r.shells, r.D0, n_iter=8, ncol=max(1, r.natoms // 2), eps=0.05,
                                      seed=4000 + r.rid, opts=uqc.default_opts(tau=1e-12, precision=prec,
                                                                                streams=a.streams)))
        done = {}
        last = time.perf_counter()
        while len(done) < len(tickets):
            for tk in tickets:
                if tk not in done:
                    res = srv.poll(tk, want_matrices=False)
                    if res is not None:
                        done[tk] = res
            if time.perf_counter() - last > 10:
                print("serve %s: %d of %d requests done after %.0f s" % (prec_name, len(done), len(tickets),
                                                                       time.perf_counter() - t0),
                      file=sys.stderr, flush=True)
                last = time.perf_counter()
            time.sleep(0.002)
        wall = time.perf_counter() - t0
        lat, q, iters = [], 0, 0
        for tk in tickets:
            res = done[tk]
            lat.append(res["finish_ms"] - res["submit_ms"])
            q += res["quartets"]
            iters += res["n_iter"]
        srv.close()
        out[prec_name] = {"wall_s": wall, "requests_per_s": len(stream) / wall, "fock_builds_per_s": iters / wall,
                          "quartets_per_s": q / wall, "p50_latency_ms": float(np.percentile(lat, 50)),
                          "p99_latency_ms": float(np.percentile(lat, 99))}
    out["value"] = out["fp64"]["quartets_per_s"]
    out["unit"] = "shell quartets/s"
    if "mixed" in out:
        out["mixed_speedup_vs_fp64"] = out["fp64"]["wall_s"] / out["mixed"]["wall_s"]
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()

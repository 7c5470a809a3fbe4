#!/usr/bin/env python3
"""Throughput of the fused forced lattice-Boltzmann step on one MI355X.

Workload: D3Q19 SMRT with the second-order force, 256^3 periodic box, Taylor-Green
initial field (u0 = 0.02) plus the steady body force g = 1e-6 (sin 2 pi z/256, 0, 0),
tau-hat_2 = 0.56, higher orders 1; populations stored as binary32 deviations from
w_i rho0 (FP32-shifted), binary32 arithmetic.  Inputs are synthetic and seeded and
sit in HBM before the timed region starts.

Prints one JSON line: MLUPS (whole job), the roofline of the step kernel against the
vendor HBM peak and against a measured stream copy, the time to steady state from the
warm start against the plain start on a few problems of the warm-start family, and the
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X vendor peak


STEP_SOURCES = ("lbm_tables.h", "lbm_node.h", "lbm_kernels.h", "lbm_lattice_impl.h",
                "lbm_internal.h", "lbm_d3q19.hip")


def kernel_source_hash() -> str:
    """Hash of the code the D3Q19 step kernel is compiled from (comments and blank lines
    removed, so a change of wording alone keeps it)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2212_07494_amd", "csrc")
    for f in STEP_SOURCES:
        with open(os.path.join(csrc, f)) as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        lines = [ln.split("//", 1)[0].rstrip() for ln in text.splitlines()]
        h.update(f.encode() + "\n".join(ln for ln in lines if ln).encode())
    return h.hexdigest()[:16]


MEMORY_VARIANTS = ["plain", "nt-store", "nt-load+store"]


def measured_traffic(kernel_hash: str, storage: str, memory_variant: str):
    """HBM bytes per launch of the step with the given memory-access variant, from the
    committed rocprofv3 counter summary, if it was taken on the current kernel sources
    and holds that variant (else None)."""
    path = os.path.join(ROOT, "profiles", f"step_d3q19_smrt_{storage}_256_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != kernel_hash:
        return None
    return d.get("hbm_bytes_by_memory_variant", {}).get(memory_variant)


def copy_roofline(torch, L, stream, nbytes=2 << 30, reps=10):
    """Best read+write bandwidth of the library's stream-copy probe (2 GiB -> 2 GiB, far
    beyond the last-level cache) over its variants and block sizes."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    best = (0.0, None)
    for variant in (1, 2):
        for block in (256, 512):
            L.lbm_copy_probe(src.data_ptr(), dst.data_ptr(), nbytes, 2, block, variant=variant,
                             stream=stream)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            L.lbm_copy_probe(src.data_ptr(), dst.data_ptr(), nbytes, reps, block,
                             variant=variant, stream=stream)
            e1.record(stream)
            e1.synchronize()
            gbps = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
            if gbps > best[0]:
                best = (gbps, {"variant": variant, "block": block})
    del src, dst
    torch.cuda.empty_cache()
    return best


def cpu_baseline(w, steps: int, steps_one_thread: int = 1):
    """The FP64 oracle as it stands, on the host cores, over `steps` steps of the
    same 256^3 workload; and on one thread over `steps_one_thread` steps."""
    import oracle
    from oracle import Oracle
    o = Oracle(w.lattice, w.collision, w.shape, walls=w.walls, tau=w.tau)
    f0 = o.init(w.rho, w.u, w.g)
    cores = oracle.set_threads(0)
    t0 = time.perf_counter()
    o.run(f0, w.g, steps)
    dt = time.perf_counter() - t0
    rec = {"value": w.N * steps / dt / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
           "sample": f"FP64 oracle, {steps} steps of the full {w.shape[0]}^3 D3Q19 SMRT "
                     f"workload ({dt:.1f} s)"}
    if steps_one_thread > 0:
        oracle.set_threads(1)
        t0 = time.perf_counter()
        o.run(f0, w.g, steps_one_thread)
        dt1 = time.perf_counter() - t0
        oracle.set_threads(cores)
        rec["one_thread"] = {"value": w.N * steps_one_thread / dt1 / 1e6, "unit": "MLUPS",
                             "cores": 1, "sample": f"{steps_one_thread} step(s) of the same "
                                                   f"workload ({dt1:.1f} s)"}
    rec["other_workloads"] = cpu_other_workloads(cores)
    return rec


def cpu_other_workloads(cores: int):
    """The same oracle on short windows of the two other single-domain workloads: the
    1024^2 D2Q9 SMRT Kolmogorov box and the 128^3 D3Q27 SMRT box with four Fourier
    forcing modes, on `cores` threads and on one.  The oracle's threads split the z
    axis, so the 2-D lattice runs on one thread either way."""
    import oracle
    from oracle import Oracle
    from paper_2212_07494_amd import inputs
    kol = inputs.kolmogorov_box(L=1024)
    p = inputs.warmstart_problem(2022, box=128)
    box = (128, 128, 128)
    g5 = inputs.fourier_force(box, p["modes"])
    cases = [("D2Q9 SMRT 1024^2 Kolmogorov, FP64",
              Oracle(kol.lattice, kol.collision, kol.shape, walls=kol.walls, tau=kol.tau),
              (kol.rho, kol.u, kol.g), kol.g, kol.N, 4, 1),
             ("D3Q27 SMRT 128^3, 4 Fourier forcing modes, FP64",
              Oracle("D3Q27", "smrt", box, tau=(p["tau2"], 1.0, 1.0)),
              (1.0, None, g5), g5, 128 ** 3, 4, 1)]
    out = []
    for name, o, init, g, n, steps, steps1 in cases:
        f0 = o.init(*init)
        rates = {}
        for threads, k in ((cores, steps), (1, steps1)):
            oracle.set_threads(threads)
            t0 = time.perf_counter()
            o.run(f0, g, k)
            dt = time.perf_counter() - t0
            rates[threads] = (n * k / dt / 1e6, k, dt)
        oracle.set_threads(cores)
        (v, k, dt), (v1, k1, dt1) = rates[cores], rates[1]
        out.append({"workload": name, "value": round(v, 3), "unit": "MLUPS", "cores": cores,
                    "one_thread": round(v1, 3),
                    "sample": f"{k} steps on {cores} threads ({dt:.1f} s), {k1} on one "
                              f"({dt1:.1f} s)"})
    return out


def time_to_steady(torch, L, nprob, box=128, seed=2022, tol=1e-8, check_every=20,
                   ref_tol=1e-11):
    """Steps and wall time to a per-step velocity residual below tol from the plain start
    and from the warm start, on nprob seeded problems of the warm-start family (D3Q27
    SMRT, FP64 storage, four Fourier forcing modes).  The warm start is the lattice's own
    steady state to third order in the forcing (fourth where the series converges slowly,
    warmstart.AUTO_ORDER4) (lbm_ws_lattice_waves), set as populations on the device
    (lbm_set_waves); its wall time includes computing and
    loading the start.  No network correction is applied here (the network's own gain is
    measured by the warm-start tests).  Both runs check the residual every check_every
    steps, which is the resolution of the step counts.  The errors at stop (plain_err,
    warm_err: relative L2 of the velocity) are against the same problem converged to a
    per-step residual below ref_tol."""
    from paper_2212_07494_amd import inputs
    from paper_2212_07494_amd import warmstart as W
    # validation problems beyond any training set the warm-start CLI draws by default
    probs = [inputs.warmstart_problem(seed + 1000 + i, box=box) for i in range(nprob)]
    ws = W.WarmStart(box=box, seed=seed, waves=True)
    rows = []
    try:
        for p in probs:
            # reference for the true errors: the steady state converged to a per-step
            # residual below ref_tol (untimed)
            dom = W.domain_of(p, box)
            with L.Lattice("D3Q27", "smrt", "f64", dom["shape"], dom["walls"], dom["tau"],
                           g_field=dom["g_field"]) as lat:
                ws.start(lat, p)
                W.run_to_steady(lat, ref_tol, 500)
                ref_u = lat.moments()[1]
            r = W.compare_starts(ws, p, box, tol, check_every=check_every, reference=ref_u)
            rows.append({"plain_steps": r["plain"]["steps"], "warm_steps": r["warm"]["steps"],
                         "plain_s": round(r["plain"]["wall_s"], 4),
                         "warm_s": round(r["warm"]["wall_s"], 4),
                         "start_s": round(r["warm"]["inference_s"], 4),
                         "plain_err": r["plain"]["final_err"],
                         "warm_err": r["warm"]["final_err"],
                         "warm_initial_err": r["warm"]["initial_err"]})
    finally:
        ws.close()
    def med(k1, k2):
        v = sorted(r[k1] / r[k2] for r in rows)
        m = len(v) // 2
        return round(v[m] if len(v) % 2 else 0.5 * (v[m - 1] + v[m]), 4)
    return {"workload": f"D3Q27 SMRT FP64, {box}^3 periodic, 4 seeded Fourier modes, "
                        f"resid < {tol:g}", "start": "the lattice's steady state to third order in the forcing (fourth where the "
                     "series converges slowly), as population waves (exact lattice response)",
            "check_every": check_every,
            "error_reference": f"converged to a per-step residual below {ref_tol:g}",
            "problems": rows, "median_steps_ratio": med("warm_steps", "plain_steps"),
            "median_plain_err": float(np.median([r["plain_err"] for r in rows])),
            "median_warm_err": float(np.median([r["warm_err"] for r in rows])),
            "median_wall_ratio": med("warm_s", "plain_s"),
            "total_plain_s": round(sum(r["plain_s"] for r in rows), 3),
            "total_warm_s": round(sum(r["warm_s"] for r in rows), 3)}


def time_to_steady_learned(nprob, tol=1e-8, check_every=20):
    """The learned warm start (the committed resummation network) against the same
    expansion without the network, on nprob held-out problems of the wide forcing family
    whose series converges slowly enough to matter (ratio sigma >= 1e-3): D3Q27 SMRT
    128^3, FP64 storage, steps and wall time (start computation included) to a per-step
    residual below tol, and the plain start for scale."""
    from paper_2212_07494_amd import resum as R
    res = R.evaluate(R.WEIGHTS, nprob, tol=tol, check=check_every, log=lambda s: None)
    rows = [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()
             if k in ("sigma", "Re", "plain", "waves", "learned", "plain_s", "waves_s",
                      "learned_s")} for r in res["problems"]]
    return {"workload": f"D3Q27 SMRT FP64, 128^3 periodic, 4 seeded Fourier modes of the wide "
                        f"family, series ratio >= {R.SIGMA_MIN:g}, resid < {tol:g}",
            "learned": "order-4 lattice expansion with per-order factors from the BF16 network "
                       "(paper_2212_07494_amd/weights/resum)",
            "without_network": "order-3 expansion, order 4 where the series converges slowly",
            "check_every": check_every, "problems": rows, "totals": res["totals"],
            "learned_over_without_network_total": round(res["learned_over_waves_total"], 4),
            "learned_over_without_network_median": round(res["learned_over_waves_median"], 4),
            "learned_over_plain_total": round(res["learned_over_plain_total"], 4),
            "wall_learned_over_without_network": round(res["wall_learned_over_waves"], 4),
            "wall_learned_over_plain": round(res["wall_learned_over_plain"], 4)}


def precision_vs_f64(L, w, stream, t, rho_t, u_t):
    """Error of the timed run's fields against the same workload stepped t steps in FP64
    storage: relative L2 of u (E2, the paper's error norm) and max |rho difference|."""
    lat = L.Lattice(w.lattice, w.collision, "f64", w.shape, w.walls, w.tau, rho=w.rho,
                    u=w.u, g_profile=w.g_profile, stream=stream)
    try:
        lat.step(t)
        rho, u = lat.moments()
    finally:
        lat.close()
    e2 = float(np.linalg.norm(u_t - u) / np.linalg.norm(u))
    return {"vs": "FP64 storage", "steps": int(t), "E2_u": e2,
            "max_abs_drho": float(np.max(np.abs(rho_t - rho)))}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--storage", default="f32s", choices=["f64", "f32", "f32s", "f16s"])
    ap.add_argument("--n", type=int, default=256, help="box edge (the workload is 256)")
    ap.add_argument("--cpu-steps", type=int, default=15)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-copy", action="store_true", help="skip the stream-copy roofline")
    ap.add_argument("--tuning", default=None,
                    help="fixed launch configuration bx,by,variant instead of the tuner")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the error of the timed run against FP64 storage")
    ap.add_argument("--ttss", type=int, default=6,
                    help="warm-start problems for the time-to-steady comparison (0: skip)")
    ap.add_argument("--learned", type=int, default=12,
                    help="held-out problems for the learned warm start's leg (0: skip)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: it measures the single-GPU step "
              "(--gpus 1); multi-GPU runs are not supported.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2212_07494_amd import inputs
    from paper_2212_07494_amd import lbm as L

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    L.load()
    w = inputs.taylor_green_3d(n=args.n)
    stream = torch.cuda.Stream()
    Q = L.QOF[w.lattice]
    S = L.STORAGE_BYTES[args.storage]
    lat = L.Lattice(w.lattice, w.collision, args.storage, w.shape, w.walls, w.tau, rho=w.rho,
                    u=w.u, g_profile=w.g_profile, stream=stream)
    lat.step(args.warmup)
    if args.tuning:
        bx, by, var = (int(v) for v in args.tuning.split(","))
        tuning = lat.tune(bx, by, var)
    else:
        tuning = lat.tune(autotune_steps=20)  # the library's launch-configuration tuner
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lat.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ms_step = ms / args.steps
    mlups = w.N * args.steps / (ms * 1e-3) / 1e6
    bytes_launch = 2 * Q * S * w.N
    achieved = bytes_launch / (ms_step * 1e-3) / 1e9
    m = lat.monitors()
    # one monitor pass (FP64 sums of the record, compared with the step before), outside
    # the timed steps: a call at a new time runs the pass
    lat.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.monitors()
    mon_ms = (time.perf_counter() - t0) * 1e3
    t_run = lat.time
    fields = None if (args.no_precision or args.storage == "f64") else lat.moments()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    precision = None
    if fields is not None:
        precision = precision_vs_f64(L, w, stream, t_run, *fields)
        fields = None
        torch.cuda.empty_cache()

    copy_gbps, copy_cfg = (None, None) if args.no_copy else copy_roofline(torch, L, stream)
    khash = kernel_source_hash()
    mem = MEMORY_VARIANTS[tuning[2] % 3]
    traffic = measured_traffic(khash, args.storage, mem) if args.n == 256 else None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic,
            "bytes_per_launch": bytes_launch,
            "measured_copy_GBps": None if copy_gbps is None else round(copy_gbps, 1),
            "copy_probe": copy_cfg,
            "launch": {"block": [tuning[0], tuning[1]],
                       "memory_variant": mem,
                       "addressing": "scalar-base" if (tuning[2] // 3) % 2 else "general",
                       "placement": ("xcd-contiguous" if tuning[2] % 12 >= 6
                                     else "dispatch order"),
                       "waves_per_simd_cap": [None, 5, 4, 3, 2][tuning[2] // 12]},
            "frac_of_copy": None if copy_gbps is None else round(achieved / copy_gbps, 4)}
    dtype = {"f64": "f64", "f32": "f32", "f32s": "f32", "f16s": "f32"}[args.storage]
    rec = {
        "metric": "MLUPS (D3Q19 SMRT+force 256^3)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"D3Q19 SMRT + second-order force, {args.n}^3 periodic, "
                               "Taylor-Green u0=0.02 + g=1e-6 sin(2 pi z/L) x, tau2=0.56, "
                               "tau3=tau4=1",
                   "storage": {"f64": "FP64", "f32": "FP32", "f32s": "FP32-shifted",
                               "f16s": "FP16-shifted"}[args.storage],
                   "nodes": w.N, "parallelism": "single GPU"},
        "roofline": roof,
        "monitors": {"step": m.step, "mass": m.mass, "umax": m.umax, "nonfinite": m.nonfinite,
                     "monitor_every": 0, "note": "the timed steps run no monitor pass; one "
                     "pass (read back included) takes monitor_pass_ms",
                     "monitor_pass_ms": round(mon_ms, 3)},
        "precision": precision,
        "kernel_source_hash": khash,
    }
    if args.ttss > 0:
        rec["time_to_steady"] = time_to_steady(torch, L, args.ttss)
    if args.learned > 0:
        rec["time_to_steady_learned"] = time_to_steady_learned(args.learned)
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()

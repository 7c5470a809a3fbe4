"""Throughput of the library on the named synthetic workloads (one GPU).

    python -m paper_2212_07494_amd.workloads d3q19 --storage f32s   # 256^3 Taylor-Green + force
    python -m paper_2212_07494_amd.workloads d3q27 --storage f64    # 128^3, 4 Fourier modes
    python -m paper_2212_07494_amd.workloads d2q9 --storage f32s    # 1024^2 Kolmogorov flow
    python -m paper_2212_07494_amd.workloads batch                  # 512 uneven D2Q9 domains
    python -m paper_2212_07494_amd.workloads womersley              # 50 x 200 channel, 20 periods

Each run: warm-up steps, the library's launch tuner, then timed steps bracketed by HIP
events on the library's stream.  Prints one JSON line: lattice updates per second, the
algorithmic bytes per second (2 Q S per update) and the per-step time.  `batch` also
times the same domains stepped as separate single-domain launches.  Inputs are the
seeded generators of `inputs`; torch supplies memory and the stream only.
"""
from __future__ import annotations

import argparse
import json

from . import inputs
from . import lbm as L


def _time(torch, stream, fn, reps):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps  # ms


def single(torch, stream, name, storage, steps, warmup, collision="smrt", **options):
    """One lattice workload; options (force_order, max_order, tau_bulk, tau_31) go to the
    lattice as in lbm.Lattice and are echoed in the record."""
    if name == "d3q19":
        w = inputs.taylor_green_3d(n=256)
        lat = L.Lattice(w.lattice, collision, storage, w.shape, w.walls, w.tau, rho=w.rho, u=w.u,
                        g_profile=w.g_profile, stream=stream, **options)
        desc = f"D3Q19 {collision.upper()} 256^3 periodic, Taylor-Green + sin force"
    elif name == "d3q27":
        p = inputs.warmstart_problem(2022, box=128)
        shape = (128, 128, 128)
        lat = L.Lattice("D3Q27", collision, storage, shape, (0, 0, 0), (p["tau2"], 1.0, 1.0),
                        g_field=inputs.fourier_force(shape, p["modes"]), stream=stream,
                        **options)
        desc = f"D3Q27 {collision.upper()} 128^3 periodic, 4 Fourier forcing modes"
    elif name == "d3q39":
        # the same forcing as d3q27 on the high-order lattice (c_s^2 = 2/3): tau-hat set
        # for the same viscosity, nu = (2/3)(tau - 1/2) = (tau_27 - 1/2)/3
        p = inputs.warmstart_problem(2022, box=128)
        shape = (128, 128, 128)
        tau = 0.5 + (p["tau2"] - 0.5) / 2.0
        lat = L.Lattice("D3Q39", collision, storage, shape, (0, 0, 0), (tau, 1.0, 1.0),
                        g_field=inputs.fourier_force(shape, p["modes"]), stream=stream,
                        **options)
        desc = f"D3Q39 {collision.upper()} 128^3 periodic, 4 Fourier forcing modes"
    elif name == "d2q9":
        w = inputs.kolmogorov_box(L=1024)
        lat = L.Lattice(w.lattice, collision, storage, w.shape, w.walls, w.tau, rho=w.rho, u=w.u,
                        g_profile=w.g_profile, stream=stream, **options)
        desc = f"D2Q9 {collision.upper()} 1024^2 periodic Kolmogorov flow"
    else:
        raise ValueError(name)
    with lat:
        lat.step(warmup)
        tuning = lat.tune(autotune_steps=20)
        ms = _time(torch, stream, lambda: lat.step(steps), 1) / steps
        N, Q = lat.N, lat.Q
    S = L.STORAGE_BYTES[storage]
    return {"workload": desc, "storage": storage, "options": options, "nodes": N,
            "steps": steps, "ms_per_step": round(ms, 5), "MLUPS": round(N / ms / 1e3, 1),
            "GBps": round(2 * Q * S * N / ms / 1e6, 1),
            "launch": {"block": list(tuning[:2]), "memory_variant": tuning[2]}}


def batch(torch, stream, storage, steps, warmup, n=512):
    doms = inputs.batch_domain_dicts(inputs.batch_domains(n))
    with L.Batch(doms, "D2Q9", "smrt", storage, stream=stream) as b:
        nodes = b.info()["nodes"]
        b.advance(warmup)
        tuning = b.tune(autotune_steps=20)
        ms = _time(torch, stream, lambda: b.advance(steps), 1) / steps
    singles = [L.Lattice("D2Q9", "smrt", storage, d["shape"], d["walls"], d["tau"], g=d.get("g"),
                         g_profile=d.get("g_profile"), stream=stream) for d in doms]
    try:
        for s in singles:
            s.step(2)
        ms1 = _time(torch, stream, lambda: [s.step(1) for s in singles], 20)
    finally:
        for s in singles:
            s.close()
    S = L.STORAGE_BYTES[storage]
    return {"workload": f"{n} uneven D2Q9 SMRT domains (channels and shear boxes)",
            "storage": storage, "nodes": nodes, "steps": steps,
            "ms_per_step": round(ms, 5), "MLUPS": round(nodes / ms / 1e3, 1),
            "GBps": round(2 * 9 * S * nodes / ms / 1e6, 1), "tuning": tuning,
            "single_domain_launches_ms_per_step": round(ms1, 5),
            "speedup_over_single_launches": round(ms1 / ms, 2)}


def womersley(torch, stream, storage, collision="smrt", periods=20, nx=50, ny=200, T=1200,
              nu=0.1, amp=1e-4):
    """Paper Sec. III.B: a channel (periodic x, halfway bounce-back plates in y) from rest
    under the uniform force -amp cos(2 pi t / T), one force factor per step.  Times the
    whole run and reports the velocity at its end against the continuum solution."""
    import math
    import numpy as np
    k = periods * T
    s = np.cos(2 * math.pi * np.arange(k + 1) / T)
    with L.Lattice("D2Q9", collision, storage, (nx, ny, 1), (0, 1, 0), (3 * nu + 0.5, 1.0, 1.0),
                   g=(-amp, 0.0, 0.0), stream=stream) as lat:
        tuning = lat.tune(autotune_steps=20)
        ms = _time(torch, stream, lambda: lat.step(k, g_scale=s[:k]), 1)
        _, u = lat.moments(g_scale=s[k])
    om = 2 * math.pi / T
    y = np.arange(ny) - (ny - 1) / 2.0
    kk = (1 + 1j) * math.sqrt(om / (2 * nu))
    uc = np.real(1j * amp / om * (1 - np.cosh(kk * y) / np.cosh(kk * ny / 2.0)) * np.exp(1j * om * k))
    ux = u[0].reshape(ny, nx)[:, 0]
    S = L.STORAGE_BYTES[storage]
    return {"workload": f"Womersley channel {nx} x {ny} D2Q9 {collision.upper()}, T={T}, "
                        f"nu={nu}, {periods} periods from rest",
            "storage": storage, "nodes": nx * ny, "steps": k, "seconds": round(ms / 1e3, 4),
            "ms_per_step": round(ms / k, 5), "MLUPS": round(nx * ny * k / ms / 1e3, 1),
            "GBps": round(2 * 9 * S * nx * ny * k / ms / 1e6, 1),
            "launch": {"block": list(tuning[:2]), "memory_variant": tuning[2]},
            "E2_vs_continuum_at_end": float(np.linalg.norm(ux - uc) / np.linalg.norm(uc))}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("workload", choices=["d3q19", "d3q27", "d3q39", "d2q9", "batch", "womersley"])
    ap.add_argument("--storage", default="f32s", choices=["f64", "f32", "f32s", "f16s"])
    ap.add_argument("--collision", default="smrt", choices=["bgk", "smrt", "rmrt"],
                    help="collision of the single-lattice workloads")
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--force-order", type=int, default=None, choices=[1, 3, 4],
                    help="SMRT force content (3: with the third-order term; 4: and the "
                         "fourth-order term)")
    ap.add_argument("--max-order", type=int, default=None, choices=[4, 6],
                    help="SMRT on D3Q27: carry orders 5-6 (6)")
    ap.add_argument("--tau-bulk", type=float, default=None, help="SMRT bulk rate (tau-hat)")
    ap.add_argument("--tau-31", type=float, default=None, help="SMRT third-order trace rate")
    args = ap.parse_args()
    options = {k: v for k, v in (("force_order", args.force_order),
                                 ("max_order", args.max_order), ("tau_bulk", args.tau_bulk),
                                 ("tau_31", args.tau_31)) if v is not None}
    import torch
    L.load()
    stream = torch.cuda.Stream()
    if args.workload == "batch":
        rec = batch(torch, stream, args.storage, args.steps, args.warmup)
    elif args.workload == "womersley":
        rec = womersley(torch, stream, args.storage)
    else:
        rec = single(torch, stream, args.workload, args.storage, args.steps, args.warmup,
                     args.collision, **options)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()

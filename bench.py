"""Benchmark of the fused two-species FLBE step on one MI355X.

Workload (the headline configuration): D3Q19, 256^3 periodic sites, two
species, FP32 storage and arithmetic, G = 1.2, tau = tau_d = 1, k_BT = 1e-5,
initial densities 1 + U(-0.01, 0.01) per species and site (seed 1), thermal
noise on.  A step is one full pass of the hot path (pull streaming, moments,
lattice force from the neighbours' densities, counter-based noise, collision,
store) over every site.  The metric is MLUPS: million two-species site
updates per second, with the populations resident in HBM.

Prints one JSON line.  Also reports the roofline of the step kernel (HBM
bound: algorithmic bytes = read + write of 2 Q populations per site) and the
FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = dict(lattice="d3q19", nx=256, ny=256, nz=256, tau=(1.0, 1.0), tau_d=1.0, G=1.2, kT=1e-5, seed=1)
BYTES_PER_SITE = {("d3q19", "f32"): 304, ("d3q19", "bf16"): 152, ("d3q19", "f16"): 152,
                  ("d2q9", "f32"): 144, ("d2q9", "f64"): 288}
KERNEL_SOURCES = ["collide.h", "rng.h", "fused.h", "kernels.h", "storage.h", "lattice.h"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1410_5584_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "fused_step_d3q19_f32_256cube_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def time_steps(fm, torch, storage: str, steps: int, warmup: int):
    import workloads
    p = fm.Params(storage=storage, rho_ref=(1.0, 1.0), **WORKLOAD)
    lat = fm.Lattice(p)
    shape = (p.nz, p.ny, p.nx)
    r1, r2 = workloads.initial_density(shape, "perturbed", seed=p.seed, amplitude=0.01)
    lat.init_density(r1, r2)
    del r1, r2
    lat.step(warmup)
    stream = lat.stream
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    lat.step(steps)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    sums = lat.global_sums()
    health = lat.health()
    lat.close()
    return ms, lat.nsites, sums, health


def cpu_baseline():
    """The FP64 oracle (as it stands) on one step of the full 256^3 workload."""
    import numpy as np

    import oracle
    import workloads
    shape = (WORKLOAD["nz"], WORKLOAD["ny"], WORKLOAD["nx"])
    s = oracle.Sim(oracle.Params(lattice=1, nx=WORKLOAD["nx"], ny=WORKLOAD["ny"], nz=WORKLOAD["nz"],
                                 tau=WORKLOAD["tau"], tau_d=WORKLOAD["tau_d"], G=WORKLOAD["G"],
                                 kT=WORKLOAD["kT"], seed=WORKLOAD["seed"]))
    r1, r2 = workloads.initial_density(shape, "perturbed", seed=WORKLOAD["seed"], amplitude=0.01)
    s.init_density(r1, r2)
    del r1, r2
    steps = 1
    t0 = time.perf_counter()
    s.step(steps)
    dt = time.perf_counter() - t0
    n = int(np.prod(shape))
    return {"value": n * steps / dt / 1e6, "unit": "MLUPS", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{steps} step of the full 256^3 D3Q19 workload in FP64 ({dt:.1f} s)"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU slab "
              "decomposition is a design, not built", file=sys.stderr)
        return 2

    import torch

    import paper_1410_5584_amd as fm
    fm.lib()
    torch.cuda.set_device(0)

    ms, nsites, sums, health = time_steps(fm, torch, "f32", args.steps, args.warmup)
    ms_per_step = ms / args.steps
    mlups = nsites * args.steps / (ms / 1e3) / 1e6
    bps = BYTES_PER_SITE[("d3q19", "f32")]
    achieved = bps * nsites / (ms_per_step / 1e3) / 1e9
    traffic = measured_traffic()
    rec = {
        "metric": "MLUPS (two-species site updates/s) + % HBM peak; BF16/batched vs plain FP32",
        "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "D3Q19 256^3 periodic, two species, FP32, G=1.2, tau=1, k_BT=1e-5, "
                               "rho=1+U(-0.01,0.01), seed 1", "sites": nsites, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "algorithmic_bytes_per_site": bps},
        "checks": {"mass": [float(sums[0]), float(sums[1])], "health": list(health)},
    }
    if not args.no_variants:
        var = {}
        for storage in ("bf16", "f16"):
            ms16, _, _, h16 = time_steps(fm, torch, storage, args.steps, args.warmup)
            m16 = nsites * args.steps / (ms16 / 1e3) / 1e6
            var[f"{storage}_dev"] = {"value": round(m16, 2), "unit": "MLUPS", "vs_f32": round(m16 / mlups, 3),
                                     "hbm_frac": round(BYTES_PER_SITE[("d3q19", storage)] * nsites /
                                                       (ms16 / args.steps / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        rec["variants"] = var
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline()
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

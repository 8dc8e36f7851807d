"""Benchmark of the fused two-species FLBE step on one MI355X.

Headline workload: D3Q19, 256^3 periodic sites, two species, FP32 storage and
arithmetic, G = 1.2, tau = tau_d = 1, k_BT = 1e-5, initial densities
1 + U(-0.01, 0.01) per species and site (seed 1), thermal noise on.  A step is
one full pass of the hot path (pull streaming, moments, lattice force from the
neighbours' densities, counter-based noise, collision, store) over every
site; it is one launch of the fused step kernel, so the per-step time is that
kernel's average launch duration.  The metric is MLUPS (million two-species
site updates per second) with the populations resident in HBM.

Prints one JSON line with the headline value, the roofline of the step kernel
(HBM bound; algorithmic bytes = read + write of 2 Q populations per site), the
same step with 16-bit deviation storage, the D2Q9 1024^2 lattice, the 512
batched D2Q9 replicas against one launch per replica, and the FP64 CPU oracle
timed on a bounded sample of the headline workload.

Helper modes for the rocprofv3 traffic figure:
  --copy-calibration   one plain 2 GiB device copy (known bytes), to scale the
                       FETCH_SIZE / WRITE_SIZE counters;
  --traffic-json F W CF CW   turn the four counter databases (step FETCH,
                       step WRITE, copy FETCH, copy WRITE) into
                       profiles/fused_step_d3q19_f32_256cube_traffic.json.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sqlite3
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = dict(lattice="d3q19", nx=256, ny=256, nz=256, tau=(1.0, 1.0), tau_d=1.0, G=1.2, kT=1e-5, seed=1)
C1 = dict(lattice="d2q9", nx=1024, ny=1024, nz=1, tau=(0.8, 1.2), tau_d=1.0, G=0.5, kT=1e-5, seed=1)
BYTES_PER_SITE = {("d3q19", "f32"): 304, ("d3q19", "bf16"): 152, ("d3q19", "f16"): 152,
                  ("d2q9", "f32"): 144, ("d2q9", "f64"): 288}
KERNEL_SOURCES = ["collide.h", "rng.h", "fused.h", "kernels.h", "storage.h", "lattice.h", "fused_ilp.hip"]
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "fused_step_d3q19_f32_256cube_traffic.json")
COPY_BYTES = 2 ** 31
STEP_KERNEL = "fused_step_kernel<fmlb::D3Q19, float"
COPY_KERNEL = "copyBuffer"


def kernel_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1410_5584_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    # The compiler flags of the step kernel's translation unit shape its code too.
    from paper_1410_5584_amd import build as _build
    h.update(repr((_build.FLAGS, _build.SOURCE_FLAGS.get("fused_ilp.hip"))).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources (else None)."""
    try:
        with open(TRAFFIC_JSON) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def _counter_mean(db: str, counter: str, kernel_part: str):
    con = sqlite3.connect(db)
    rows = [(k, v) for k, c, v in con.execute("select kernel_name, counter_name, value from counters_collection")
            if c == counter and kernel_part in k]
    if not rows:
        raise SystemExit(f"{db}: no {counter} for a kernel matching {kernel_part!r}")
    return sum(v for _, v in rows) / len(rows), rows[0][0], len(rows)


def write_traffic_json(fetch_db: str, write_db: str, cfetch_db: str, cwrite_db: str) -> dict:
    f, kname, launches = _counter_mean(fetch_db, "FETCH_SIZE", STEP_KERNEL)
    w, _, _ = _counter_mean(write_db, "WRITE_SIZE", STEP_KERNEL)
    cf, _, _ = _counter_mean(cfetch_db, "FETCH_SIZE", COPY_KERNEL)
    cw, _, _ = _counter_mean(cwrite_db, "WRITE_SIZE", COPY_KERNEL)
    kf, kw = COPY_BYTES / (cf * 1024.0), COPY_BYTES / (cw * 1024.0)
    read_b, write_b = f * 1024.0 * kf, w * 1024.0 * kw
    sites = WORKLOAD["nx"] * WORKLOAD["ny"] * WORKLOAD["nz"]
    rec = {"kernel": kname, "workload": "D3Q19 256^3 FP32", "launches": launches,
           "kernel_hash": kernel_hash(), "fetch_kib_per_launch": f, "write_kib_per_launch": w,
           "copy_calibration": {"bytes": COPY_BYTES, "fetch_kib": cf, "write_kib": cw,
                                "fetch_scale": kf, "write_scale": kw},
           "read_bytes_per_launch": read_b, "write_bytes_per_launch": write_b,
           "bytes_per_launch": read_b + write_b,
           "algorithmic_bytes_per_launch": BYTES_PER_SITE[("d3q19", "f32")] * sites}
    os.makedirs(os.path.dirname(TRAFFIC_JSON), exist_ok=True)
    with open(TRAFFIC_JSON, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


def copy_calibration():
    import torch
    torch.cuda.set_device(0)
    a = torch.ones(COPY_BYTES // 4, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": COPY_BYTES, "copies": 3}), flush=True)


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


REFERENCES = (("pull_copy", 0), ("read", 1), ("write", 2), ("copy16", 3))


def time_steps(fm, torch, storage: str, steps: int, warmup: int, work=WORKLOAD, windows: int = 0,
               references: bool = False):
    """K steps timed as one region on the lattice's stream (the contract),
    then `windows` more windows of K steps (their median and spread), and
    the bandwidth references (each timed over K launches)."""
    import workloads
    p = fm.Params(storage=storage, rho_ref=(1.0, 1.0), **work)
    lat = fm.Lattice(p)
    shape = (p.nz, p.ny, p.nx)
    r1, r2 = workloads.initial_density(shape, "perturbed", seed=p.seed, amplitude=0.01)
    lat.init_density(r1, r2)
    del r1, r2
    lat.step(warmup)
    stream = lat.stream
    start, end = _events(torch)
    torch.cuda.synchronize()
    start.record(stream)
    lat.step(steps)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    win = []
    for _ in range(windows):
        start.record(stream)
        lat.step(steps)
        end.record(stream)
        torch.cuda.synchronize()
        win.append(start.elapsed_time(end) / steps)
    sums = lat.global_sums()
    health = lat.health()
    refs = {}
    if references:
        for name, kind in REFERENCES:
            nbytes = lat.bandwidth_reference(kind)
            start.record(stream)
            for _ in range(steps):
                lat.bandwidth_reference(kind)
            end.record(stream)
            torch.cuda.synchronize()
            t = start.elapsed_time(end) / steps
            refs[name] = {"ms_per_launch": round(t, 4), "bytes": nbytes,
                          "frac": round(nbytes / (t / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    lat.close()
    return ms, p.nx * p.ny * p.nz, sums, health, refs, win


def batched(fm, torch, steps: int, warmup: int, plain_steps: int):
    """512 D2Q9 FP32 replicas (log-uniform sizes 32^2..256^2, per-replica
    seed, k_BT, G): one launch per step from replayed HIP graphs with the
    autotuned work list, against one launch per replica per step."""
    import workloads
    reps = workloads.replica_table(512)
    ps = [fm.Params(lattice="d2q9", storage="f32", nx=r["L"], ny=r["L"], nz=1, tau=r["tau"], tau_d=r["tau_d"],
                    G=r["G"], kT=r["kT"], seed=r["seed"]) for r in reps]
    sites = sum(p.nx * p.ny for p in ps)
    b = fm.Batch(ps)
    for r in range(len(ps)):
        b.init_density(r, 1.0, 1.0)
    tile = b.autotune(reps=5)
    b.step(max(warmup, 32), use_graph=True)
    steps = max(32, (steps // 32) * 32)
    start, end = _events(torch)
    torch.cuda.synchronize()
    start.record(b.stream)
    b.step(steps, use_graph=True)
    end.record(b.stream)
    torch.cuda.synchronize()
    ms_b = start.elapsed_time(end) / steps
    b.close()
    lats = []
    for p in ps:
        lat = fm.Lattice(p)
        lat.init_density(1.0, 1.0)
        lats.append(lat)
    for lat in lats:
        lat.step(2)
    start, end = _events(torch)
    torch.cuda.synchronize()
    start.record(lats[0].stream)
    for _ in range(plain_steps):
        for lat in lats:
            lat.step(1)
    end.record(lats[0].stream)
    torch.cuda.synchronize()
    ms_p = start.elapsed_time(end) / plain_steps
    for lat in lats:
        lat.close()
    mlups_b, mlups_p = sites / ms_b / 1e3, sites / ms_p / 1e3
    return {"value": round(mlups_b, 2), "unit": "MLUPS", "ms_per_step": round(ms_b, 4), "sites": sites,
            "replicas": len(ps), "tile": list(tile), "graph_steps": 32,
            "hbm_frac": round(BYTES_PER_SITE[("d2q9", "f32")] * sites / (ms_b / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "plain_per_replica": {"value": round(mlups_p, 2), "unit": "MLUPS", "ms_per_step": round(ms_p, 4),
                                  "steps": plain_steps},
            "vs_plain": round(mlups_b / mlups_p, 2),
            "note": "packed runs of sites per workgroup (autotuned shape in 'tile': 2 = 512 threads); "
                    "547 MB per buffer, above the 256 MB last-level cache: a real HBM fraction"}


def multi_species(fm, torch, steps: int, warmup: int, n: int = 3):
    """The N-species path (Apps. C and D) on D3Q19 256^3, FP32 deviation
    storage, three species with pair couplings 0.5 / 0.3 / 0.4."""
    import workloads
    G = ((0.0, 0.5, 0.3), (0.5, 0.0, 0.4), (0.3, 0.4, 0.0))
    p = fm.MultiParams(lattice="d3q19", storage="f32", nspecies=n, nx=256, ny=256, nz=256, tau=(1.0,) * n,
                       tau_d=1.0, G=G, kT=1e-5, rho_ref=(1.0,) * n, seed=1)
    m = fm.Multi(p)
    shape = (p.nz, p.ny, p.nx)
    m.init_density([workloads.initial_density(shape, "perturbed", seed=1 + s, amplitude=0.01)[0] for s in range(n)])
    m.step(warmup)
    start, end = _events(torch)
    torch.cuda.synchronize()
    start.record(m.stream)
    m.step(steps)
    end.record(m.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / steps
    sums = m.global_sums()
    m.close()
    nsites = 256 ** 3
    bps = 2 * n * 19 * 4
    return {"value": round(nsites / (ms / 1e3) / 1e6, 2), "unit": "MLUPS", "ms_per_step": round(ms, 4),
            "species": n, "hbm_frac": round(bps * nsites / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "algorithmic_bytes_per_site": bps, "mass": [float(x) for x in sums[:n]],
            "note": "one kernel per step (the asynchronous single pass, 64x4 tiles walking the whole z axis)"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def c1_end_to_end(fm, torch, steps: int = 10000, every: int = 100):
    """The C1 run as the workload states it: D2Q9 1024^2 FP32, 1e4 steps,
    structure factors accumulated every 100 steps, timed whole on the
    lattice's stream."""
    import workloads
    p = fm.Params(storage="f32", rho_ref=(1.0, 1.0), **C1)
    lat = fm.Lattice(p)
    r1, r2 = workloads.initial_density((1, p.ny, p.nx), "perturbed", seed=p.seed, amplitude=0.01)
    lat.init_density(r1, r2)
    lat.step(every)
    lat.sk_accumulate()
    lat.reset_accumulators()
    start, end = _events(torch)
    torch.cuda.synchronize()
    start.record(lat.stream)
    for _ in range(steps // every):
        lat.step(every)
        lat.sk_accumulate()
    end.record(lat.stream)
    torch.cuda.synchronize()
    ms_total = start.elapsed_time(end)
    start.record(lat.stream)
    lat.step(steps)
    end.record(lat.stream)
    torch.cuda.synchronize()
    ms_steps = start.elapsed_time(end)
    n = p.nx * p.ny
    lat.close()
    return {"value": round(n * steps / (ms_total / 1e3) / 1e6, 2), "unit": "MLUPS", "steps": steps,
            "sk_every": every, "ms_total": round(ms_total, 2), "ms_steps_only": round(ms_steps, 2),
            "sk_share": round(1.0 - ms_steps / ms_total, 4),
            "ms_per_sk": round((ms_total - ms_steps) / (steps // every), 4)}


def cpu_baseline(steps: int = 5):
    """The FP64 oracle (as it stands) on `steps` steps of the full 256^3 workload."""
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
    t0 = time.perf_counter()
    s.step(steps)
    dt = time.perf_counter() - t0
    n = int(np.prod(shape))
    return {"value": round(n * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": oracle.num_threads(),
            "kind": "oracle", "cpu_model": cpu_model(), "cpus_online": os.cpu_count(),
            "sample": f"{steps} steps of the full 256^3 D3Q19 workload in FP64 ({dt:.1f} s)"}


def storage16(fm, torch, storage, steps, warmup, mlups_f32=None, stochastic=False) -> dict:
    """The headline workload with BF16 or FP16 deviation storage, rounded to
    nearest or (stochastic) with stochastic rounding."""
    work = dict(WORKLOAD, flags=fm.FMLB_ROUND_STOCHASTIC) if stochastic else WORKLOAD
    ms16, nsites, _, _, _, _ = time_steps(fm, torch, storage, steps, warmup, work)
    m16 = nsites * steps / (ms16 / 1e3) / 1e6
    rec = {"value": round(m16, 2), "unit": "MLUPS", "ms_per_step": round(ms16 / steps, 4)}
    if mlups_f32:
        rec["vs_f32"] = round(m16 / mlups_f32, 3)
    rec["hbm_frac"] = round(BYTES_PER_SITE[("d3q19", storage)] * nsites / (ms16 / steps / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    return rec


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--windows", type=int, default=5,
                    help="further windows of --steps steps, timed for the median and spread")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--multi-only", action="store_true",
                    help="time only the three-species D3Q19 256^3 FP32 workload (for profiling)")
    ap.add_argument("--batch-only", action="store_true",
                    help="time only the 512 batched D2Q9 replicas against one launch per replica (for profiling)")
    ap.add_argument("--storage-only", choices=("bf16", "f16"),
                    help="time only the D3Q19 256^3 workload with this 16-bit storage (for profiling)")
    ap.add_argument("--stochastic", action="store_true", help="with --storage-only: stochastic rounding")
    ap.add_argument("--c1-only", action="store_true",
                    help="time only the D2Q9 1024^2 run with S(k) every 100 steps (for profiling)")
    ap.add_argument("--traffic-json", nargs=4, metavar=("FETCH_DB", "WRITE_DB", "COPY_FETCH_DB", "COPY_WRITE_DB"))
    args = ap.parse_args()
    if args.traffic_json:
        print(json.dumps(write_traffic_json(*args.traffic_json)), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU slab "
              "decomposition is a design, not built", file=sys.stderr)
        return 2
    if args.copy_calibration:
        copy_calibration()
        return 0

    import torch

    import paper_1410_5584_amd as fm
    fm.lib()
    torch.cuda.set_device(0)

    if args.batch_only:
        print(json.dumps({"d2q9_512_replicas_batched_f32": batched(fm, torch, args.steps, args.warmup, plain_steps=10)}),
              flush=True)
        return 0
    if args.storage_only:
        tag = "_stochastic" if args.stochastic else ""
        print(json.dumps({f"d3q19_256cube_{args.storage_only}_dev{tag}":
                          storage16(fm, torch, args.storage_only, args.steps, args.warmup,
                                    stochastic=args.stochastic)}), flush=True)
        return 0
    if args.c1_only:
        print(json.dumps({"d2q9_1024sq_f32_end_to_end": c1_end_to_end(fm, torch)}), flush=True)
        return 0
    if args.multi_only:
        print(json.dumps({"d3q19_256cube_3species_f32": multi_species(fm, torch, args.steps, args.warmup)}),
              flush=True)
        return 0

    ms, nsites, sums, health, refs, win = time_steps(fm, torch, "f32", args.steps, args.warmup,
                                                     windows=args.windows, references=True)
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
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "algorithmic_bytes_per_launch": bps * nsites,
                     "references": dict(refs, note="bandwidth references over the same buffers "
                                        "(fmlb_bandwidth_reference): pull_copy = the step's pull addresses, "
                                        "read / write = one direction only, copy16 = unshifted 16-byte copy")},
        "checks": {"mass": [float(sums[0]), float(sums[1])], "health": list(health)},
    }
    if win:
        rec["timing"] = {"windows": len(win), "steps_per_window": args.steps,
                         "median_ms_per_step": round(float(sorted(win)[len(win) // 2]), 4),
                         "min_ms_per_step": round(min(win), 4), "max_ms_per_step": round(max(win), 4)}
    if not args.no_variants:
        var = {}
        for storage in ("bf16", "f16"):
            var[f"d3q19_256cube_{storage}_dev"] = storage16(fm, torch, storage, args.steps, args.warmup, mlups)
            var[f"d3q19_256cube_{storage}_dev_stochastic"] = storage16(fm, torch, storage, args.steps, args.warmup,
                                                                     mlups, stochastic=True)
        ms1, n1, _, _, _, _ = time_steps(fm, torch, "f32", args.steps, args.warmup, work=C1)
        var["d2q9_1024sq_f32"] = {"value": round(n1 * args.steps / (ms1 / 1e3) / 1e6, 2), "unit": "MLUPS",
                                  "ms_per_step": round(ms1 / args.steps, 4),
                                  "note": "75 MB per buffer, cache-resident: HBM fraction not meaningful"}
        var["d2q9_1024sq_f32_end_to_end"] = c1_end_to_end(fm, torch)
        var["d2q9_512_replicas_batched_f32"] = batched(fm, torch, args.steps, args.warmup, plain_steps=10)
        var["d3q19_256cube_3species_f32"] = multi_species(fm, torch, args.steps, args.warmup)
        rec["variants"] = var
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline()
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

"""Throughput of the fused phase-field LB step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

One step is one pass of the whole hot path over the workload: pull streaming, phi and
psi with their LDS halo, the gradient/Laplacian/normal stencils, chemical potential,
velocity and pressure, g and f collisions with the level-set source, the FP64 volume
reductions.  The workload is timed for each storage precision (FP64, FP32 and
FP16-shifted; arithmetic in FP64 / FP32 / FP32); `value` is the FP32-storage rate, the
others are reported under `variants`.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & % HBM roofline, FP32/FP16-store vs FP64 GPU; adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0

# algorithmic HBM bytes per node update: every population read once and written once,
# the previous phi u read and written, and (shifted storage) the phi of the writing
# node written once and read once.  (lattice, coupled) -> storage -> bytes
BYTES_PER_NODE = {
    ("D2Q9", True): {"fp64": 2 * 9 * 8 * 2 + 2 * 8 * 2,
                     "fp32": 2 * 9 * 4 * 2 + 2 * 4 * 2 + 4 * 2,
                     "fp16s": 2 * 9 * 2 * 2 + 2 * 4 * 2 + 4 * 2},
    ("D2Q9", False): {"fp64": 9 * 8 * 2 + 2 * 8 * 2,
                      "fp32": 9 * 4 * 2 + 2 * 4 * 2 + 4 * 2,
                      "fp16s": 9 * 2 * 2 + 2 * 4 * 2 + 4 * 2},
    ("D3Q19", True): {"fp64": 2 * 19 * 8 * 2 + 3 * 8 * 2,
                      "fp32": 2 * 19 * 4 * 2 + 3 * 4 * 2 + 4 * 2,
                      "fp16s": 2 * 19 * 2 * 2 + 3 * 4 * 2 + 4 * 2},
}


def workload(name: str, storage: str):
    import workloads as W
    if name == "two_droplets_x32":
        p, phi0, u0 = W.two_droplets(storage, scale=32)
        return p, phi0, u0, {"workload": "two static drops, D2Q9 coupled, 4096x4096 periodic "
                                         "(the 128x128 two-drop case scaled x32: R = 768, 256), W = 4, "
                                         "density ratio 10, M = 0.1, sigma = 0.01, nu = 0.1"}
    if name == "rayleigh_plateau":
        p, phi0, u0 = W.rayleigh_plateau(storage)
        return p, phi0, u0, {"workload": "Rayleigh-Plateau column, D3Q19 coupled, 96x96x384 periodic, "
                                         "R(z) = 16 (1 + 0.1 cos(2 pi z / 384)), W = 4, density ratio 10, "
                                         "sigma = 0.005, nu = 0.05, M = 0.1"}
    raise SystemExit(f"unknown workload {name}")


def time_case(p, phi0, u0, steps: int, warmup: int, tile=None):
    import torch
    from paper_2505_10899_amd import vclb
    case = vclb.Case(p, tile=tile).init(phi0, u0)
    case.step(warmup)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    case.step(steps)
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = e0.elapsed_time(e1)
    # per-launch kernel duration: one fused kernel per step, bracketed by events
    k = min(steps, 50)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(k)]
    for a, b in evs:
        a.record(s)
        case.step(1)
        b.record(s)
    torch.cuda.synchronize()
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    obs = case.reduce()
    return dict(total_ms=total_ms, wall_s=wall, kern_ms=kern_ms, tile=case.tile(),
                sum_phi=float(np.sum(obs["sum_phi"])))


def cpu_baseline(budget_s: float = 15.0):
    """The CPU oracle on a bounded sample of the same kind of work: the two-drop
    case on a 256x256 box, as many steps as fit the budget, BLAS limited to 1 thread."""
    import workloads as W
    from oracle import Model
    try:
        from threadpoolctl import threadpool_limits
    except Exception:       # pragma: no cover
        threadpool_limits = None
    p, phi0, _ = W.two_droplets("fp64", scale=2)
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        m = Model(p).init(phi0)
        m.step(2)
        n = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            m.step(5)
            n += 5
        dt = time.perf_counter() - t0
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    return {"value": round(p.n_nodes * n / dt / 1e6, 4), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"numpy FP64 oracle, two-drop case 256x256 (D2Q9 coupled), {n} steps in {dt:.1f} s, "
                      f"single thread (BLAS limited to 1 thread); host has {os.cpu_count()} logical CPUs"}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="two_droplets_x32")
    ap.add_argument("--storages", default="fp32,fp64,fp16s")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile", default=None, help="bx,ty[,by3]: launch shape of the fused step")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="also run a plain device copy of this many MiB (a known-size reference "
                         "for the HBM byte counters)")
    a = ap.parse_args(argv)
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        return 2
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    storages = a.storages.split(",")
    res = {}
    meta = None
    for st in storages:
        p, phi0, u0, meta = workload(a.workload, st)
        print(f"[bench] {a.workload} {st}: {p.n_nodes} nodes, {a.warmup} warmup + {a.steps} timed steps",
              file=sys.stderr, flush=True)
        tile = tuple(int(v) for v in a.tile.split(",")) if a.tile else None
        r = time_case(p, phi0, u0, a.steps, a.warmup, tile)
        coupled = p.mode == "coupled"
        bpn = BYTES_PER_NODE[(p.lattice, coupled)][st]
        ms = r["total_ms"] / a.steps
        mlups = p.n_nodes / (ms * 1e-3) / 1e6
        gbs = p.n_nodes * bpn / (r["kern_ms"] * 1e-3) / 1e9
        res[st] = dict(mlups=mlups, ms_per_step=ms, kernel_ms=r["kern_ms"], bytes_per_node=bpn,
                       achieved_GBs=gbs, frac=gbs / HBM_PEAK_GBS, tile=r["tile"], nodes=p.n_nodes)
        print(f"[bench] {st}: {mlups:.0f} MLUPS, {ms:.3f} ms/step, kernel {r['kern_ms']:.3f} ms, "
              f"{gbs:.0f} GB/s ({100 * gbs / HBM_PEAK_GBS:.1f}% of HBM peak), tile {r['tile']}",
              file=sys.stderr, flush=True)
    head = "fp32" if "fp32" in res else storages[0]
    h = res[head]
    out = {
        "metric": METRIC, "value": round(h["mlups"], 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(h["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32", "data": "synthetic",
        "config": dict(meta, storage=head, nodes=h["nodes"], tile=list(h["tile"])),
        "roofline": {"bound": "hbm", "achieved": round(h["achieved_GBs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(h["frac"], 4), "traffic": None,
                     "bytes_per_node": h["bytes_per_node"], "kernel_ms": round(h["kernel_ms"], 5)},
        "variants": {st: {"MLUPS": round(v["mlups"], 1), "ms_per_step": round(v["ms_per_step"], 4),
                          "kernel_ms": round(v["kernel_ms"], 5), "achieved_GBs": round(v["achieved_GBs"], 1),
                          "frac_hbm_peak": round(v["frac"], 4), "bytes_per_node": v["bytes_per_node"],
                          "speedup_vs_fp64": (round(v["mlups"] / res["fp64"]["mlups"], 3) if "fp64" in res else None)}
                     for st, v in res.items()},
    }
    if a.copy_probe:
        nbytes = a.copy_probe << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = nbytes
    if not a.no_cpu_baseline:
        print("[bench] CPU oracle baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

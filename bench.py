"""Throughput of the phase-field LB hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--storages fp32,fp16s,fp64]
                    [--no-adjoint] [--no-single] [--no-cpu-baseline]

Headline workload: 512 independent D2Q9 coupled drop cases of uneven sizes (sides
log-uniform in [64, 512], PCG64 seed 10899), advanced together.  One step is one pass
of the whole hot path over every case: pull streaming with bounce-back/moving walls,
phi and psi with their LDS halo, the gradient/Laplacian/normal stencils, chemical
potential, velocity and pressure, g and f collisions with the level-set source, and
the per-case FP64 volume reductions, as one work-list kernel per step; a call's steps
are replayed from one hipGraph.  The tile is chosen by the library's autotuner, and the
runs of work items are then re-cut to the measured speed of each workgroup slot.  The
batch is timed for each storage precision; `value` is the FP32-storage rate (FP32
arithmetic), FP16-shifted and FP64 are under `variants`.

Also reported: the adjoint/forward time ratio on the 512x256 shear-flow case (4000
steps, a checkpoint every 200), single large cases for the fused single-case kernel,
and the CPU oracle on a sample of the batch.  Prints one JSON line on stdout.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & % HBM roofline, FP32/FP16-store vs FP64 GPU; adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_batch512.txt")

# Algorithmic HBM bytes per node update: every population read once and written once,
# the previous phi u read and written, and, for the 2-byte storage only, the FP32 phi the
# stored deviations refer to (that of the node that reads them) written once and read
# once (the 2-byte deviations cannot be decoded without it).  (lattice, coupled) -> storage -> bytes
BYTES_PER_NODE = {
    ("D2Q9", True): {"fp64": 2 * 9 * 8 * 2 + 2 * 8 * 2,                 # 320
                     "fp32": 2 * 9 * 4 * 2 + 2 * 4 * 2,                 # 160
                     "fp16s": 2 * 9 * 2 * 2 + 2 * 4 * 2 + 4 * 2},       # 96
    ("D2Q9", False): {"fp64": 9 * 8 * 2 + 2 * 8 * 2,                    # 176
                      "fp32": 9 * 4 * 2 + 2 * 4 * 2,                    # 88
                      "fp16s": 9 * 2 * 2 + 2 * 4 * 2 + 4 * 2},          # 60
    ("D3Q19", True): {"fp64": 2 * 19 * 8 * 2 + 3 * 8 * 2,               # 656
                      "fp32": 2 * 19 * 4 * 2 + 3 * 4 * 2,               # 328
                      "fp16s": 2 * 19 * 2 * 2 + 3 * 4 * 2 + 4 * 2},     # 184
}
# What the kernels of this library move per node update in their layout: FP32 storage
# also keeps g as deviations from a rest state, with the phi they refer to beside them
# (4 B written, 4 B read), to hold the total of phi to FP32 rounding.
LAYOUT_EXTRA = {"fp64": 0, "fp32": 8, "fp16s": 0}


def layout_bytes(lattice: str, coupled: bool, storage: str) -> int:
    return BYTES_PER_NODE[(lattice, coupled)][storage] + LAYOUT_EXTRA[storage]


KERNEL = {"fp64": "k_batch_step2d<StoreF64>", "fp32": "k_batch_step2d<StoreF32>",
          "fp16s": "k_batch_step2d<StoreF16S>"}

BATCH_DESC = ("512 independent D2Q9 coupled drop cases, sides log-uniform in [64, 512] (independent "
              "nx, ny), radius 0.1-0.3 of the shorter side, density ratio log-uniform in [1, 100], static "
              "periodic or shear between walls moving +-0.02 (1/2 each), W = 4, M = 0.1, sigma = 0.01, "
              "nu = 0.1; PCG64 seed 10899; one work-list kernel per step, hipGraph replay")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


BATCH_SOURCES = ("batch.hip", "flat2d.hpp", "step2d.hpp", "node.hpp", "devcase.hpp", "lattice.hpp", "launch.hpp")


def _code_only(text: str) -> str:
    """A source without its // comments, trailing blanks and empty lines (the sources hold
    no other comment form): editing a comment does not change the compiled kernel."""
    lines = (line.split("//", 1)[0].rstrip() for line in text.splitlines())
    return "\n".join(line for line in lines if line.strip())


def source_hash() -> str:
    """Fingerprint of the code of the sources the batched step kernel is built from:
    counter figures taken on other code are stale."""
    h = hashlib.sha256()
    for name in BATCH_SOURCES:
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_2505_10899_amd", "csrc", name), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def recorded_traffic(storage: str, bx: int):
    """HBM bytes per launch of the batched step from the committed rocprofv3 counter
    summary, if it was taken on the current sources and on the kernel instantiation that a
    bx-lane tile launches (workgroups of 256, 512 or 1024 lanes); else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_hash") != source_hash():
        return None
    lanes = 1024 if bx > 512 else (512 if bx > 256 else 256)
    kernel = kv.get(f"kernel_{storage}", "")
    args = kernel[kernel.find("<") + 1:kernel.rfind(">")].split(",")
    if len(args) < 3 or args[2].strip() != str(lanes):
        return None
    v = kv.get(f"traffic_bytes_per_launch_{storage}")
    return float(v) if v else None


def timer():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


# ----------------------------------------------------------------------------- batch
def run_batch(storage: str, steps: int, warmup: int, launch_steps: int, tune_steps: int, fixed=None,
              balance: bool = True):
    import torch
    import workloads as W
    from paper_2505_10899_amd import vclb
    cases, _ = W.batch_cases(512, storage=storage)
    b = vclb.Batch([p for p, _, _ in cases]).init([(phi0, u0) for _, phi0, u0 in cases])
    N = b.nodes()
    v0 = b.reduce()["sum_phi"].sum(axis=1)
    tuned = None
    if fixed:                      # (bx, ty, flat_pct) given: no tuning (profiling runs)
        b.set_tile(fixed[0], fixed[1])
        b.set_schedule(fixed[2])
    else:
        _, tuned = tune_batch(b, storage, tune_steps)
    tile = b.tile()
    sched = b.schedule()
    # re-cut the runs to the measured speed of each workgroup slot (state restored)
    gain = b.balance(rounds=3, steps=3) if balance else 1.0
    log(f"batch {storage}: {len(cases)} cases, {N} nodes, tile {tile}, flat_pct {sched}, "
        f"slot balancing: slowest slot {gain:.3f}x faster")
    b.step(warmup, graph=True)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = timer()
    t0 = time.perf_counter()
    e0.record(s)
    b.step(steps, graph=True)
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / steps
    # average duration of one step kernel: an eager run of launch_steps launches on this
    # stream (one closing fold of the reductions is included)
    e0, e1 = timer()
    e0.record(s)
    b.step(launch_steps, graph=False)
    e1.record(s)
    torch.cuda.synchronize()
    launch_ms = e0.elapsed_time(e1) / launch_steps
    v1 = b.reduce()["sum_phi"].sum(axis=1)
    t_end = b.cases[0].time()
    drift = float(np.max(np.abs(v1 - v0) / np.abs(v0)))
    bpn = BYTES_PER_NODE[("D2Q9", True)][storage]
    gbs = N * bpn / (launch_ms * 1e-3) / 1e9
    check = check_against_tested_shape(b, cases, storage, (tile[0], tile[1], sched), int(t_end))
    del b
    return dict(nodes=N, ms_per_step=ms, wall_s=wall, mlups=N / (ms * 1e-3) / 1e6, launch_ms=launch_ms,
                bytes_per_node=bpn, layout_bytes_per_node=layout_bytes("D2Q9", True, storage),
                achieved_GBs=gbs, frac=gbs / HBM_PEAK_GBS, tile=list(tile), flat_pct=sched,
                balance_gain=gain, max_rel_volume_drift=drift, drift_steps=int(t_end), tile_check=check,
                tuning_ms=tuned)


# Launch shapes (bx, ty, flat_pct) of the batched step that the full-size parity tests of
# tests/test_gpu_batch.py run all 512 cases in (the 1024-lane ones with 4-byte storage
# only).  The benchmark times the batch in the fastest of these.
BATCH_SHAPES = [(512, 1024, 100), (512, 1024, 101), (512, 64, 100), (1024, 1024, 101), (1024, 64, 100)]
# pairs of those shapes that give every case the same march (column strips or flattened
# bands) and differ only in how the cases are cut into items: their states must agree bit
# for bit.  (A strip and a band compute the same update with instructions the compiler
# schedules and contracts differently, and can differ in the last bit of a value, as on a
# near-zero f of 1e-45.)
SAME_MARCH = {(512, 1024, 100): (512, 64, 100), (512, 64, 100): (512, 1024, 100),
              (1024, 1024, 101): (1024, 64, 100), (1024, 64, 100): (1024, 1024, 101)}


def shapes_for(storage: str):
    return [s for s in BATCH_SHAPES if storage != "fp64" or s[0] <= 512]


def tune_batch(b, storage: str, steps: int):
    """The fastest of the tested launch shapes on this batch: each timed over `steps`
    steps, twice in alternation, keeping each one's best (the batch advances meanwhile)."""
    import torch
    best = {}
    s = torch.cuda.current_stream()
    for _ in range(2):
        for shape in shapes_for(storage):
            b.set_tile(shape[0], shape[1])
            b.set_schedule(shape[2])
            b.step(2, graph=True)
            e0, e1 = timer()
            e0.record(s)
            b.step(steps, graph=True)
            e1.record(s)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            best[shape] = min(best.get(shape, 1e30), ms)
    shape = min(best, key=best.get)
    b.set_tile(shape[0], shape[1])
    b.set_schedule(shape[2])
    return shape, {f"{k[0]},{k[1]},{k[2]}": round(v, 4) for k, v in best.items()}


def check_against_tested_shape(b, cases, storage: str, shape, t: int) -> str:
    """The timed batch against the same cases stepped as many times in the other tested
    launch shape with the same march for every case: every case's state (g, f, previous
    phi u, decoded to FP64 on the device) must be equal bit for bit.  Raises if it is
    not."""
    import torch
    from paper_2505_10899_amd import vclb
    other = SAME_MARCH.get(tuple(shape))
    if other is None:
        return f"the timed launch shape {tuple(shape)} is one the full-size parity tests run"
    ref = vclb.Batch([p for p, _, _ in cases]).init([(phi0, u0) for _, phi0, u0 in cases])
    ref.set_tile(other[0], other[1])
    ref.set_schedule(other[2])
    ref.set_reduce_every(0)
    ref.step(t, graph=True)
    torch.cuda.synchronize()
    for k, (ca, cb) in enumerate(zip(b.cases, ref.cases)):
        for xa, xb in zip(ca.state_device(), cb.state_device()):
            if xa is not None and not torch.equal(xa, xb):
                raise RuntimeError(f"batch {storage}: case {k} differs from launch shape {other} after {t} steps")
    del ref
    return (f"the timed launch shape {tuple(shape)} is one the full-size parity tests run; all {len(cases)} "
            f"cases bitwise equal after {t} steps to the same march cut as {other}")


# ----------------------------------------------------------------------------- adjoint
def run_adjoint(nsteps: int = 4000, every: int = 200):
    import torch
    import workloads as W
    from paper_2505_10899_amd import vclb
    p, phi0, u0 = W.shear_droplet("fp64")
    c = vclb.Case(p)
    c.set_reduce_every(0)
    s = torch.cuda.current_stream()
    c.init(phi0, u0).step(50)
    torch.cuda.synchronize()
    c.init(phi0, u0)
    e0, e1 = timer()
    e0.record(s)
    c.step(nsteps)
    e1.record(s)
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1)
    w = np.array([[0.0, 0.0, 0.0, 0.0, 1.0]])          # J = deformation D
    res = None
    for _ in range(2):                                  # the first pass allocates the store
        e0, e1 = timer()
        t0 = time.perf_counter()
        c.adjoint_record(phi0, u0, nsteps=nsteps, every=every)
        rec_s = time.perf_counter() - t0
        seed = vclb.obs_seed(c.reduce_raw(), 1, w)
        D = float(c.derived()[0, 4])
        torch.cuda.synchronize()
        e0.record(s)
        dphi, ds, dm = c.adjoint_run(seed)
        e1.record(s)
        torch.cuda.synchronize()
        res = (rec_s, e0.elapsed_time(e1), D, ds, dm, float(dphi.abs().max()))
    rec_s, bwd_ms, D, ds, dm, gmax = res
    nck = -(-nsteps // every)
    return {"workload": "drop in shear, D2Q9 FP64, 512x256, walls moving -+0.02, R = 48, Ca = 0.2, Re = 0.5, "
                        f"{nsteps} steps, a checkpoint every {every}; J = deformation D",
            "forward_ms": round(fwd_ms, 3), "record_ms": round(rec_s * 1e3, 3), "backward_ms": round(bwd_ms, 3),
            "ratio_backward_over_forward": round(bwd_ms / fwd_ms, 4),
            # the backward less its recompute, priced at the forward's own time per step:
            # the reverse sweep alone (its kernels and copies) against the forward
            "ratio_reverse_over_forward_est": round((bwd_ms - (nsteps - nck) * fwd_ms / nsteps) / fwd_ms, 4),
            "recomputed_steps": nsteps - nck,
            "D": D, "dD_dsigma": ds, "dD_dM": dm, "max_abs_dD_dphi0": gmax}


# ----------------------------------------------------------------------------- single cases
def run_single(name: str, storage: str, steps: int, warmup: int, tune: bool = True):
    import torch
    import workloads as W
    from paper_2505_10899_amd import vclb
    if name == "two_droplets_4096":
        p, phi0, u0 = W.two_droplets(storage, scale=32)
    elif name == "rayleigh_plateau_96x96x48":   # the z slab one of eight GPUs would hold
        p, phi0, u0 = W.rayleigh_plateau(storage, nz=48)
    else:
        p, phi0, u0 = W.rayleigh_plateau(storage)
    c = vclb.Case(p).init(phi0, u0)
    if tune:
        c.autotune(None, steps=3)
    c.step(warmup)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = timer()
    e0.record(s)
    c.step(steps)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    bpn = BYTES_PER_NODE[(p.lattice, p.mode == "coupled")][storage]
    gbs = p.n_nodes * bpn / (ms * 1e-3) / 1e9
    return {"nodes": p.n_nodes, "MLUPS": round(p.n_nodes / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
            "achieved_GBs": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
            "bytes_per_node": bpn, "layout_bytes_per_node": layout_bytes(p.lattice, p.mode == "coupled", storage),
            "tile": list(c.tile())}


# ----------------------------------------------------------------------------- CPU oracle
_CPU_CASES = None


def _oracle_case(k: int):
    """3 oracle steps of batch case k in a worker process: (node updates, seconds)."""
    from oracle import Model
    try:
        from threadpoolctl import threadpool_limits
        limit = threadpool_limits(limits=1)
    except Exception:   # pragma: no cover
        limit = None
    p, phi0, u0 = _CPU_CASES[k]
    m = Model(p).init(phi0, u0)
    t0 = time.perf_counter()
    m.step(3)
    dt = time.perf_counter() - t0
    if limit is not None:
        limit.__exit__(None, None, None)
    return 3 * p.n_nodes, dt


def cpu_baseline(budget_s: float = 15.0, max_workers: int = 16):
    """The CPU oracle on a bounded sample of the batch, one case per worker process over
    the host's cores (at most 16, the share of one GPU's host): the batch's cases in order,
    3 steps each after init, for about budget_s of wall time.  Each worker runs numpy with
    BLAS limited to one thread.  Must run before the process touches the GPU (the workers
    are forked from it)."""
    import multiprocessing as mp
    import workloads as W
    global _CPU_CASES
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    cases, _ = W.batch_cases(512, storage="fp64")
    _CPU_CASES = cases
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:   # pragma: no cover
        ncpu = os.cpu_count() or 1
    workers = max(1, min(max_workers, ncpu))
    updates, used, busy = 0, 0, 0.0
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        for n, dt in pool.imap(_oracle_case, range(len(cases))):
            updates += n
            busy += dt
            used += 1
            if time.perf_counter() - t0 > budget_s:
                break
        wall = time.perf_counter() - t0
        pool.terminate()
    # the rate of the workers' step() calls together: updates over the mean step time per
    # worker (their initialisations, outside step(), are not timed)
    return {"value": round(updates / (busy / workers) / 1e6, 4), "unit": "MLUPS", "cores": workers, "kind": "oracle",
            "sample": f"numpy FP64 oracle on the first {used} of the 512 batch cases, 3 steps each after init, "
                      f"one case per process on {workers} worker processes ({updates} node updates in {busy:.1f} s "
                      f"of step() time summed over the workers, {wall:.1f} s of wall time with their inits; BLAS "
                      f"limited to one thread per process); host has {ncpu} CPUs available"}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storages", default="fp32,fp16s,fp64")
    ap.add_argument("--launch-steps", type=int, default=50)
    ap.add_argument("--tune-steps", type=int, default=10)
    ap.add_argument("--batch-tile", default="",
                    help="storage=bx,ty,flat_pct[;...]: fixed batched launch shapes instead of autotuning")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--no-single-tune", action="store_true",
                    help="single cases keep their default tiles (profiling runs: one tile per kernel)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-balance", action="store_true",
                    help="keep runs of equal modelled cost (no per-slot speed balancing)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="also run a plain device copy of this many MiB (a known-size reference "
                         "for the HBM byte counters)")
    a = ap.parse_args(argv)
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        return 2
    cpu = None
    if not a.no_cpu_baseline:   # first: its worker processes fork from a process that has not touched the GPU
        log("CPU oracle baseline ...")
        cpu = cpu_baseline()
        log(f"CPU oracle baseline: {cpu['value']} MLUPS on {cpu['cores']} cores")
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    storages = a.storages.split(",")
    res = {}
    for st in storages:
        log(f"batch {st}: {a.warmup} warmup + {a.steps} timed steps")
        fixed = {}
        for item in filter(None, a.batch_tile.split(";")):
            k, v = item.split("=")
            fixed[k.strip()] = tuple(int(x) for x in v.split(","))
        r = run_batch(st, a.steps, a.warmup, a.launch_steps, a.tune_steps, fixed.get(st), balance=not a.no_balance)
        res[st] = r
        log(f"batch {st}: {r['mlups']:.0f} MLUPS, {r['ms_per_step']:.3f} ms/step, launch {r['launch_ms']:.3f} ms, "
            f"{r['achieved_GBs']:.0f} GB/s ({100 * r['frac']:.1f}% of HBM peak), drift {r['max_rel_volume_drift']:.2e}")
    head = "fp32" if "fp32" in res else storages[0]
    h = res[head]
    from paper_2505_10899_amd import vclb
    probe, probe_cfg = {}, {}
    for m in ("copy", "read", "write"):
        gbs, cfg = vclb.bandwidth_probe_best(m)
        probe[m], probe_cfg[m] = round(gbs, 1), cfg
    log(f"bandwidth probe (2 GiB, best of 32 kernel shapes): copy {probe['copy']:.0f} GB/s (read + write) "
        f"{probe_cfg['copy']}, read {probe['read']:.0f} {probe_cfg['read']}, write {probe['write']:.0f} "
        f"{probe_cfg['write']}")
    traffic = recorded_traffic(head, h["tile"][0])
    out = {
        "metric": METRIC, "value": round(h["mlups"], 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(h["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32", "data": "synthetic",
        "config": {"workload": BATCH_DESC, "storage": head, "cases": 512, "nodes": h["nodes"],
                   "tile": h["tile"], "flat_pct": h["flat_pct"]},
        "roofline": {"bound": "hbm", "achieved": round(h["achieved_GBs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(h["frac"], 4), "traffic": traffic,
                     "kernel": KERNEL[head], "bytes_per_node": h["bytes_per_node"],
                     "bytes_per_launch": h["bytes_per_node"] * h["nodes"],
                     "layout_bytes_per_node": h["layout_bytes_per_node"],
                     "launch_ms": round(h["launch_ms"], 5),
                     "achievable_copy_GBs": probe["copy"],
                     "frac_of_copy": round(h["achieved_GBs"] / probe["copy"], 4)},
        "bandwidth_probe_GBs": probe,
        "bandwidth_probe_shape": probe_cfg,
        "variants": {st: {"MLUPS": round(v["mlups"], 1), "ms_per_step": round(v["ms_per_step"], 4),
                          "launch_ms": round(v["launch_ms"], 5), "achieved_GBs": round(v["achieved_GBs"], 1),
                          "frac_hbm_peak": round(v["frac"], 4), "bytes_per_node": v["bytes_per_node"],
                          "layout_bytes_per_node": v["layout_bytes_per_node"],
                          "tile": v["tile"], "flat_pct": v["flat_pct"], "tile_check": v["tile_check"],
                          "tuning_ms_per_step": v["tuning_ms"],
                          "slot_balance_gain": round(v["balance_gain"], 4),
                          "max_rel_volume_drift": v["max_rel_volume_drift"],
                          "drift_over_steps": v["drift_steps"],
                          "speedup_vs_fp64": (round(v["mlups"] / res["fp64"]["mlups"], 3) if "fp64" in res else None)}
                     for st, v in res.items()},
    }
    if not a.no_adjoint:
        log("adjoint: 512x256 shear, 4000 steps, checkpoint every 200")
        out["adjoint"] = run_adjoint()
        log(f"adjoint: backward/forward = {out['adjoint']['ratio_backward_over_forward']}")
    if not a.no_single:
        single = {}
        for name, st in (("two_droplets_4096", "fp32"), ("two_droplets_4096", "fp64"),
                         ("two_droplets_4096", "fp16s"), ("rayleigh_plateau_96x96x384", "fp32"),
                         ("rayleigh_plateau_96x96x384", "fp16s"), ("rayleigh_plateau_96x96x384", "fp64")):
            single[f"{name}_{st}"] = run_single(name, st, min(a.steps, 100), 10, tune=not a.no_single_tune)
            log(f"single {name} {st}: {single[f'{name}_{st}']}")
        out["single_case"] = single
    if a.copy_probe:
        nbytes = a.copy_probe << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = nbytes
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

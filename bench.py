#!/usr/bin/env python3
"""Benchmark of the MTS PD/FE solver on one MI355X.

A step is one macro step of Algorithm 1 (one FE step at dt_FE, m fused PD
substeps at dt_PD, the multiplier solve of Eq. 49 and the final update of
Eq. 50, plus a rebuild of the unit-load responses when bonds inside their
support break).  The default workload is the 400 x 160 FP64 plate with m = 10
and 4000 PD steps (400 macro steps).  `value` counts directed bond slots
evaluated per PD substep (the free problem) per second over the timed macro
steps; setup (neighbour build, unit-load responses) is timed separately.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PD bond-updates/s (FP64 vs mixed) at stated error; served p50/p99 latency"
HBM_PEAK = 8.0e12


def bytes_per_launch(info, inst):
    """Algorithmic HBM bytes of one fused PD substep launch (layout of this build):
    per bond slot: the slot record the library reports (FP64: coefficient 8 B +
    neighbour offset 4 B; mixed: 4 + 4 B, or 6 B when the neighbour records are
    staged in LDS and two slots share a 12-byte record) + bond-state bit 1/8 B;
    per node: position (8 dim), u read (8 dim), v and a read+write (32 dim),
    predicted u write (8 dim), mass 8, constraint index 4, damage 8/m.
    Neighbour positions and displacements are counted once per node."""
    dim = info["dim"]
    per_bond = info["slot_bytes"] + 1.0 / 8.0
    per_node = 8.0 * dim * (1 + 1 + 4 + 1) + 8 + 4 + 8.0 / inst["m"]
    return info["nnz"] * per_bond + info["n_pd"] * per_node, per_bond, per_node


def source_digest():
    """Digest of the sources the PD substep kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for f in ("pd.hip", "device_math.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_2403_03605_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_per_launch(inst):
    """Measured HBM bytes per PD substep launch (FETCH_SIZE + WRITE_SIZE from
    two counter runs, scaled by the copy-kernel calibration), read from the
    committed counter summary; None when it is missing, was taken for another
    workload, or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "k_pd_substep_traffic.md")
    try:
        with open(path) as fh:
            text = fh.read()
        rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, ValueError, IndexError):
        return None
    w = rec.get("workloads", {}).get(inst["name"])
    if not w or rec.get("source_digest") != source_digest():
        return None
    return w["bytes_per_launch"]


def cpu_baseline(inst, seconds=15.0):
    """The oracle as it stands, single thread, on the same seeded lattice in
    pure-PD mode (the PD substep path: bond pass with breaking + Verlet)."""
    import mts_inputs as mi
    from oracle import Oracle
    sample = dict(inst)
    sample.update(mode="pure_pd", dom_lo=inst["pd_lo"], dom_hi=inst["pd_hi"], fe_n=(0, 0, 0), m=1)
    o = Oracle(sample)
    nnz = o.info()["nnz"]
    n = 0
    t0 = time.perf_counter()
    while True:
        o.advance(5)
        n += 5
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    o.close()
    return {"value": n * nnz / dt, "unit": "bond-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} PD substeps of the same {inst['pd_n'][0]}x{inst['pd_n'][1]} seeded lattice, "
                      f"pure-PD mode (bond pass with breaking + Verlet), plain C FP64, 1 thread, {dt:.1f} s"}


def serve_main(args, torch, mts, log):
    """Serving form: the seeded stream of plate solves (sizes 100x40 .. 800x320,
    m in {4, 8, 10}, mixed precision) with Poisson arrivals at 20 per second,
    admitted by device-memory budget and advanced together in the pool."""
    from paper_2403_03605_amd.serving import serve, stream_requests
    reqs = stream_requests(args.serve_requests, rate=args.serve_rate)
    free, _total = torch.cuda.mem_get_info()
    budget = int(args.serve_budget_gib * (1 << 30)) if args.serve_budget_gib > 0 else int(0.9 * free)
    log(f"serving {len(reqs)} requests, budget {budget / 2**30:.1f} GiB")
    out = serve(reqs, budget, max_slots=64, use_graphs=not args.serve_no_graphs,
                log=lambda m: log(m), builders=args.serve_builders)
    sizes = {}
    for r in reqs:
        sizes[f"{r['nx']}x{r['ny']}"] = sizes.get(f"{r['nx']}x{r['ny']}", 0) + 1
    line = {
        "metric": "served p99 latency (s), with p50 and aggregate PD bond-updates/s",
        "value": out["p99_s"], "unit": "s", "n_gpus": 1, "steps": out["pool_steps"], "warmup": 0,
        "ms_per_step": out["span_s"] * 1e3 / max(out["pool_steps"], 1), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 bond math / f64 integration", "data": "synthetic",
        "config": {"workload": f"serving stream: {len(reqs)} plate solves, Poisson {args.serve_rate:g}/s, "
                               "10 us of physical time each",
                   "budget_bytes": budget, "graphs": not args.serve_no_graphs,
                   "builders": args.serve_builders},
        "serving": {k: v for k, v in out.items() if k != "latencies_s"},
        "request_sizes": sizes,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed macro steps (default: the workload's)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", type=int, default=1, help="workload index (0..3)")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default=None,
                    help="override the workload's precision (same seeded instance)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel event timing pass")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (counter calibration)")
    ap.add_argument("--serve", action="store_true",
                    help="run the serving stream (Poisson arrivals of plate solves) through the pool instead")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-rate", type=float, default=20.0, help="Poisson arrival rate (requests/s)")
    ap.add_argument("--serve-budget-gib", type=float, default=0.0, help="pool budget (0: 90%% of free HBM)")
    ap.add_argument("--serve-no-graphs", action="store_true")
    ap.add_argument("--serve-builders", type=int, default=4, help="threads that build arrived requests")
    ap.add_argument("--profile-steps", type=int, default=100, help="macro steps of the event-timed pass")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    os.environ.setdefault("MTS_VERBOSE", "1")  # setup progress on stderr
    import torch
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 8, "reps": 5}), flush=True)
        return
    import mts_inputs as mi
    import paper_2403_03605_amd as mts

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.serve:
        return serve_main(args, torch, mts, log)
    inst = mi.config(args.config) if args.precision is None else mi.config(args.config, precision=args.precision)
    K = args.steps if args.steps is not None else inst["n_macro"]
    W = args.warmup
    stream = torch.cuda.Stream()
    sh = stream.cuda_stream
    log(f"workload {inst['name']}: {K} timed macro steps after {W} warm-up steps")

    if W > 0:  # warm-up on a throwaway solver of the same workload
        with torch.cuda.stream(stream):
            w = mts.Solver(inst, stream=sh)
            w.advance(W)
            w.sync()
            w.close()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = mts.Solver(inst, stream=sh)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    info = s.query()

    def timed(n):
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        s.advance(n)
        ev1.record(stream)
        s.sync()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gpu_ms = ev0.elapsed_time(ev1)
        return max(wall, gpu_ms / 1e3), wall, gpu_ms

    # timed region: K macro steps, no per-kernel events
    elapsed, wall, gpu_ms = timed(K)
    info = s.query()
    bond_updates = K * inst["m"] * info["nnz"]
    value = bond_updates / elapsed
    log(f"timed: {K} macro steps in {elapsed:.3f} s -> {value:.4g} bond-updates/s")

    roof = None
    if not args.no_profile:
        # second timed region on the same solver with HIP events around every
        # launch group (recorded on the solver's stream)
        Kp = min(K, args.profile_steps)
        s.profile(True)
        p_elapsed, _, _ = timed(Kp)
        n_launch, ms = s.kernel_time(mts.KT_PD_SUBSTEP)
        avg_s = ms / 1e3 / max(n_launch, 1)
        b, per_bond, per_node = bytes_per_launch(info, inst)
        achieved = b / avg_s
        roof = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": achieved / HBM_PEAK, "traffic": traffic_per_launch(inst),
                "kernel": "k_pd_substep", "launches": n_launch, "avg_launch_us": avg_s * 1e6,
                "algorithmic_bytes_per_launch": b, "bytes_per_bond": per_bond,
                "bytes_per_node": per_node,
                "kernel_bond_updates_per_s": info["nnz"] / avg_s,
                "profiled_macro_steps": Kp,
                "profiled_pass_bond_updates_per_s": Kp * inst["m"] * info["nnz"] / p_elapsed}
        other = {}
        for name, k in (("link", mts.KT_LINK), ("fe", mts.KT_FE), ("lambda", mts.KT_LAMBDA)):
            n_l, ms_l = s.kernel_time(k)
            other[name] = {"launch_groups": n_l, "total_ms": ms_l}
        # the multiplier solve streams the packed inverse once per macro step:
        # its bytes over the whole phase's time bound the GEMV's rate from below
        inv = s.query()["inverse_bytes"]
        n_l, ms_l = other["lambda"]["launch_groups"], other["lambda"]["total_ms"]
        other["lambda"]["inverse_bytes"] = inv
        other["lambda"]["inverse_GBps_over_phase"] = (inv * n_l / (ms_l * 1e-3) / 1e9) if ms_l > 0 else None
        roof["other_phases"] = other
    info = s.query()
    s.close()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(inst, args.cpu_seconds)

    dtype = "f64" if inst["precision"] == "fp64" else "f32 bond math / f64 integration"
    line = {
        "metric": METRIC, "value": value, "unit": "bond-updates/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": elapsed * 1e3 / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": inst["name"] + f", {K * inst['m']} PD steps ({K} macro steps)",
                   "pd_nodes": info["n_pd"], "bonds": info["nnz"], "m": inst["m"],
                   "fe_nodes": info["n_fe_nodes"], "constraints": info["n_constraints"],
                   "dt_pd": inst["dt_pd"], "rebuilds": info["n_rebuilds"], "setup_s": setup_s,
                   "source_digest": source_digest(),
                   "gpu_event_ms": gpu_ms, "wall_ms": wall * 1e3},
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark of the MTS PD/FE solver on one MI355X.

A step is one macro step of Algorithm 1: one FE step at dt_FE, m fused PD
substeps at dt_PD, the multiplier solve of Eq. 49 and the final update of
Eq. 50, plus a rebuild of the unit-load responses when bonds inside their
support break.  The default workload is the 1000 x 400 plate (400,000 PD nodes,
11.1 M bonds, m = 10, 5000 PD steps = 500 macro steps) in FP64: `value` is its
rate in PD bond-updates/s, i.e. directed bond slots evaluated per PD substep of
the free problem, per second, over the timed macro steps (inputs resident,
setup timed separately).  The same JSON line carries:
- the mixed form (FP32 bond arithmetic, FP64 integration and coupling) on the
  identical seeded instance: its rate, the speed-up over FP64, and its error
  against the FP64 run (displacement relative L2 up to the FP64 run's first
  break, crack-tip distance after);
- the served latency p50/p99 and aggregate rate of the seeded request stream
  (256 plate solves, Poisson arrivals at 20 per second);
- the bond pass's roofline (HBM bound) on two byte models and the counter
  traffic;
- the crack-branching plate of the paper's Sec. 4.1, MTS against pure PD;
- the per-step times of the efficiency study's plate (Table 2, every case but
  the MTS model with the implicit PD step), split as the paper splits them;
- the oracle's rate on the host's cores (one thread and all threads).

Prints one JSON line.  --serve, --branching and --glass-block (the 3D impact
block in glass run to the end, with its rebuilds timed) each print a line of
their own instead.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PD bond-updates/s (FP64 vs mixed) at stated error; served p50/p99 latency"
HBM_PEAK = 8.0e12


def reference_bytes(info, inst):
    """Algorithmic HBM bytes of one bond-pass launch in the reference layout of
    the method's data (neighbour index 4 B, stored reference bond vector xi of
    d FP64 values (FP32 in the mixed form), one state bit per bond; per node the
    row pointer 4 B, u, v, a read and written (48 d B), 1/m and alpha 16 B and
    the damage 8/m B), every neighbour's displacement counted once."""
    dim = info["dim"]
    xi = (4 if info["precision"] == 1 else 8) * dim
    per_bond = 4 + xi + 1.0 / 8.0
    per_node = 4 + 48.0 * dim + 16 + 8.0 / inst["m"]
    return info["nnz"] * per_bond + info["n_pd"] * per_node, per_bond, per_node


def layout_bytes(info, inst):
    """Algorithmic HBM bytes of one bond-pass launch in this build's layout:
    per bond slot the slot record the library reports (FP64: coefficient 8 B +
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


def host_threads():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(inst, seconds=8.0):
    """The oracle as it stands on the same seeded lattice in pure-PD mode (the
    PD substep path: bond pass with breaking + Verlet), timed on one thread and
    on all host threads (its OpenMP build: per-node loops, identical results)."""
    from oracle import Oracle
    sample = dict(inst)
    sample.update(mode="pure_pd", dom_lo=inst["pd_lo"], dom_hi=inst["pd_hi"], fe_n=(0, 0, 0), m=1)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or host_threads()
    os.environ["OMP_NUM_THREADS"] = str(threads)
    out = {}
    for omp in (False, True):
        o = Oracle(sample, openmp=omp)
        nnz = o.info()["nnz"]
        n = 0
        t0 = time.perf_counter()
        while True:
            o.advance(1)
            n += 1
            if time.perf_counter() - t0 >= seconds:
                break
        dt = time.perf_counter() - t0
        o.close()
        out[omp] = (n * nnz / dt, n, dt)
    v1, n1, t1 = out[False]
    vn, nn, tn = out[True]
    return {"value": vn, "unit": "bond-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{nn} PD substeps of the same {inst['pd_n'][0]}x{inst['pd_n'][1]} seeded lattice, pure-PD "
                      f"mode (bond pass with breaking + Verlet), plain C FP64, OpenMP over nodes on {threads} "
                      f"threads, {tn:.1f} s; one thread: {n1} substeps in {t1:.1f} s",
            "single_thread_value": v1, "cpu_model": cpu_model(), "host_threads": host_threads()}


def serve_run(args, torch, log):
    """The seeded stream of plate solves (sizes 100x40 .. 800x320, m in
    {4, 8, 10}, mixed precision) with Poisson arrivals, admitted by device-memory
    budget and advanced together in the pool."""
    from paper_2403_03605_amd.serving import serve, stream_requests
    reqs = stream_requests(args.serve_requests, rate=args.serve_rate)
    free, _total = torch.cuda.mem_get_info()
    budget = int(args.serve_budget_gib * (1 << 30)) if args.serve_budget_gib > 0 else int(0.9 * free)
    log(f"serving {len(reqs)} requests at {args.serve_rate:g}/s, budget {budget / 2**30:.1f} GiB")
    out = serve(reqs, budget, max_slots=64, use_graphs=not args.serve_no_graphs,
                log=(lambda m: log(m)) if args.serve_verbose else None, builders=args.serve_builders)
    sizes = {}
    for r in reqs:
        key = f"{r['nx']}x{r['ny']}"
        sizes[key] = sizes.get(key, 0) + 1
    out = {k: v for k, v in out.items() if k != "latencies_s"}
    out.update(rate_per_s=args.serve_rate, budget_bytes=budget, graphs=not args.serve_no_graphs,
               builders=args.serve_builders,
               stream="plate solves 100x40..800x320 (nx uniform over 100..800 step 20), m in {4, 8, 10}, "
                      "notch and height uniform in [0.2, 0.6], traction 0.5..2 MPa, 10 us of physical time each, "
                      "mixed precision")
    return out, sizes


def serve_main(args, torch, log):
    out, sizes = serve_run(args, torch, log)
    line = {
        "metric": "served p99 latency (s), with p50 and aggregate PD bond-updates/s",
        "value": out["p99_s"], "unit": "s", "n_gpus": 1, "steps": out["pool_steps"], "warmup": 0,
        "ms_per_step": out["span_s"] * 1e3 / max(out["pool_steps"], 1), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 bond math / f64 integration", "data": "synthetic",
        "config": {"workload": f"serving stream: {out['n_requests']} plate solves, Poisson {args.serve_rate:g}/s, "
                               "10 us of physical time each"},
        "serving": out, "request_sizes": sizes,
    }
    print(json.dumps(line), flush=True)


def run_form(mts, torch, inst, K, W, args, log):
    """Warm-up on a throwaway solver, then K timed macro steps on a fresh solver
    (no per-kernel events), then an event-timed pass for the bond pass's
    roofline and the other phases.  Returns the form's record."""
    stream = torch.cuda.Stream()
    sh = stream.cuda_stream
    log(f"workload {inst['name']}: {K} timed macro steps after {W} warm-up steps")
    if W > 0:
        w = mts.Solver(inst, stream=sh)
        w.advance(W)
        w.sync()
        w.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = mts.Solver(inst, stream=sh)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0

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

    elapsed, wall, gpu_ms = timed(K)
    info = s.query()
    value = K * inst["m"] * info["nnz"] / elapsed
    log(f"timed: {K} macro steps in {elapsed:.3f} s -> {value:.4g} bond-updates/s")
    rec = {"value": value, "ms_per_step": elapsed * 1e3 / K, "steps": K, "setup_s": setup_s,
           "gpu_event_ms": gpu_ms, "wall_ms": wall * 1e3, "rebuilds": info["n_rebuilds"], "info": info}
    if not args.no_profile:
        Kp = min(K, args.profile_steps)
        s.profile(True)
        p_elapsed, _, _ = timed(Kp)
        n_launch, ms = s.kernel_time(mts.KT_PD_SUBSTEP)
        avg_s = ms / 1e3 / max(n_launch, 1)
        b, per_bond, per_node = reference_bytes(info, inst)
        bl, per_bond_l, per_node_l = layout_bytes(info, inst)
        traffic = traffic_per_launch(inst)
        roof = {"bound": "hbm", "achieved": b / avg_s / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": b / avg_s / HBM_PEAK, "traffic": traffic,
                "kernel": "k_pd_substep", "launches": n_launch, "avg_launch_us": avg_s * 1e6,
                "algorithmic_bytes_per_launch": b, "bytes_per_bond": per_bond, "bytes_per_node": per_node,
                "byte_model": "reference layout: 4 B index + stored xi + state bit per bond; row pointer, "
                              "u/v/a read and write, 1/m, alpha, damage per node",
                "layout": {"achieved": bl / avg_s / 1e9, "frac": bl / avg_s / HBM_PEAK,
                           "algorithmic_bytes_per_launch": bl, "bytes_per_bond": per_bond_l,
                           "bytes_per_node": per_node_l,
                           "byte_model": "this build: slot record (coefficient + neighbour offset) + state bit "
                                         "per bond; node record [x, u], v, a, mass, constraint index per node"},
                "traffic_GBps": traffic / avg_s / 1e9 if traffic else None,
                "traffic_frac": traffic / avg_s / HBM_PEAK if traffic else None,
                "kernel_bond_updates_per_s": info["nnz"] / avg_s,
                "profiled_macro_steps": Kp,
                "profiled_pass_bond_updates_per_s": Kp * inst["m"] * info["nnz"] / p_elapsed}
        other = {}
        for name, k in (("link", mts.KT_LINK), ("fe", mts.KT_FE), ("lambda", mts.KT_LAMBDA)):
            n_l, ms_l = s.kernel_time(k)
            other[name] = {"launch_groups": n_l, "total_ms": ms_l}
        inv = s.query()["inverse_bytes"]
        n_l, ms_l = other["lambda"]["launch_groups"], other["lambda"]["total_ms"]
        other["lambda"]["inverse_bytes"] = inv
        other["lambda"]["inverse_GBps_over_phase"] = (inv * n_l / (ms_l * 1e-3) / 1e9) if ms_l > 0 else None
        other["bond_passes"] = {"launch_groups": Kp, "total_ms": ms}
        roof["phases_per_macro_step_us"] = {k: v["total_ms"] * 1e3 / max(v["launch_groups"], 1)
                                            for k, v in other.items()}
        roof["other_phases"] = other
        rec["roofline"] = roof
    s.close()
    return rec


def _tip(pos, phi, thresh=0.35):
    import numpy as np
    idx = np.where(phi >= thresh)[0]
    if idx.size == 0:
        return None
    return pos[idx[np.argmax(pos[idx, 0])]]


def mixed_error(mts, torch, inst64, inst_mx, K, chunk, log):
    """The mixed form against the FP64 run on the identical seeded instance:
    displacement relative L2 at checkpoints every `chunk` macro steps up to the
    FP64 run's first break, crack-tip distance (in dx) after it."""
    import numpy as np
    a = mts.Solver(inst64)
    b = mts.Solver(inst_mx)
    pos = inst64["pos"]
    dx = inst64["dx"]
    worst, last_pre, first_break, tip_worst, tips = 0.0, None, None, 0.0, 0
    done = 0
    while done < K:
        n = min(chunk, K - done)
        a.advance(n)
        b.advance(n)
        done += n
        broken = a.energy()["n_broken"]
        if broken == 0:
            ua, ub = a.read(mts.PD_U), b.read(mts.PD_U)
            e = float(np.sqrt(((ub - ua) ** 2).sum()) / max(np.sqrt((ua ** 2).sum()), 1e-300))
            worst = max(worst, e)
            last_pre = done
        else:
            if first_break is None:
                first_break = done
            ta, tb = _tip(pos, a.read(mts.DAMAGE)), _tip(pos, b.read(mts.DAMAGE))
            if ta is not None and tb is not None:
                tips += 1
                tip_worst = max(tip_worst, float(np.linalg.norm(ta - tb)) / dx)
    res = {"u_rel_l2_before_first_break": worst, "last_checkpoint_before_break_macro_step": last_pre,
           "fp64_first_break_by_macro_step": first_break, "tip_distance_after_break_max_dx": tip_worst,
           "tip_checkpoints": tips, "checkpoint_every_macro_steps": chunk, "macro_steps": K,
           "bound": "u rel L2 <= 1e-4 before the first break, tip within 2 dx after",
           "within_bound": bool(worst <= 1e-4 and tip_worst <= 2.0 + 1e-9)}
    log(f"mixed vs fp64: rel L2 {worst:.3g} up to macro step {last_pre}, tip <= {tip_worst:.2f} dx over {tips} checks")
    a.close()
    b.close()
    return res


def branching_run(mts, torch, log):
    """The crack-branching plate (100 x 40 mm glass, 50 mm notch, 12 MPa,
    dx = 0.25 mm, 6e-5 s): the pure-PD model of the whole plate (400 x 160
    nodes, 6000 steps of 1e-8 s) and the MTS model (220 x 120 PD nodes, Q4
    elements of 1 mm, m = 10, 600 macro steps), each timed from a resident
    state to the end of the run."""
    import mts_inputs as mi
    out = {}
    for mode in ("pure_pd", "coupled"):
        inst = mi.branching2d(400, mode)
        t0 = time.perf_counter()
        s = mts.Solver(inst)
        s.sync()
        setup = time.perf_counter() - t0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.advance(inst["n_macro"])
        s.sync()
        run = time.perf_counter() - t0
        info = s.query()
        e = s.energy()
        tip = _tip(inst["pos"], s.read(mts.DAMAGE))
        out[mode] = {"workload": inst["name"], "run_s": run, "setup_s": setup, "pd_nodes": info["n_pd"],
                     "bonds": info["nnz"], "pd_steps": info["pd_steps"], "macro_steps": info["macro_steps"],
                     "rebuilds": info["n_rebuilds"], "broken": e["n_broken"],
                     "bond_updates_per_s": info["pd_steps"] * info["nnz"] / run,
                     "tip_mm": None if tip is None else [float(tip[0] * 1e3), float(tip[1] * 1e3)]}
        log(f"branching {mode}: {run:.3f} s, {info['n_rebuilds']} rebuilds, {e['n_broken']} broken")
        s.close()
    out["mts_speedup_vs_pure_pd"] = out["pure_pd"]["run_s"] / out["coupled"]["run_s"]
    out["paper"] = "pure PD 1320 s vs MTS 863 s for the same 6e-5 s, RTX 3070, PeriFEM with implicit FE (context)"
    return out


def glass_block_run(mts, torch, log, precision="mixed", n_macro=None):
    """The 100 x 100 x 20 impact block in glass: the whole run (2000 PD
    steps, m = 8; or its first n_macro macro steps) from a resident state,
    with the rebuilds of the unit-load responses, H and its inverse that its
    breaks trigger, timed by the library's rebuild event pairs."""
    import mts_inputs as mi
    inst = mi.config(3, precision=precision, material="glass",
                     name=f"block 100x100x20 m=8 {precision} glass")
    t0 = time.perf_counter()
    s = mts.Solver(inst)
    s.sync()
    setup = time.perf_counter() - t0
    n_macro = min(n_macro or inst["n_macro"], inst["n_macro"])
    s.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, chunk = 0, 25
    while done < n_macro:
        k = min(chunk, n_macro - done)
        s.advance(k)
        s.sync()
        done += k
        log(f"glass block: {done}/{n_macro} macro steps, {time.perf_counter() - t0:.1f} s, "
            f"{s.query()['n_rebuilds']} rebuilds")
    run = time.perf_counter() - t0
    info = s.query()
    e = s.energy()
    ph = {}
    for name, kt in (("pd_substeps", mts.KT_PD_SUBSTEP), ("fe", mts.KT_FE), ("lambda", mts.KT_LAMBDA),
                     ("link", mts.KT_LINK), ("rebuild", mts.KT_REBUILD)):
        ph[name] = s.kernel_time(kt)[1]
    s.profile(False)
    s.close()
    nr = info["n_rebuilds"]
    rec = {"workload": inst["name"], "run_s": run, "setup_s": setup, "macro_steps": info["macro_steps"],
           "pd_steps": info["pd_steps"], "pd_nodes": info["n_pd"], "bonds": info["nnz"], "broken": e["n_broken"],
           "constraints": info["n_constraints"], "rebuilds": nr,
           "rebuild_ms_total": ph["rebuild"], "ms_per_rebuild": ph["rebuild"] / nr if nr else None,
           "rebuild_columns_fraction": (info["n_rebuild_columns"] / (nr * info["n_constraints"])) if nr else None,
           "phases_ms_total": ph, "bond_updates_per_s": info["pd_steps"] * info["nnz"] / run}
    log(f"glass block: {run:.1f} s, {nr} rebuilds at {rec['ms_per_rebuild'] or 0:.1f} ms, "
        f"{e['n_broken']} of {info['nnz']} bonds broken")
    return rec


# the paper's Table 2 cases: (case, dx, PD area, m, PD Newmark beta); case 2
# (MTS with the implicit PD step) is not run
TABLE2_CASES = [(1, 5e-4, 1.0, 1, 0.25), (3, 5e-4, 0.2, 2, 0.0), (4, 5e-4, 0.1, 2, 0.0), (5, 5e-4, 0.1, 5, 0.0),
                (6, 2.5e-4, 1.0, 1, 0.0), (7, 2.5e-4, 0.1, 10, 0.0)]
TABLE2_PAPER_MS = {1: (69.8, 69.8), 3: (95.9, 44.7), 4: (86.9, 41.0), 5: (208.7, 39.2), 6: (253.0, 253.0),
                   7: (552.9, 50.6)}


def table2_run(mts, torch, log, pd_steps=400):
    """The efficiency study's mode-I plate (Table 2) in its cases except the
    MTS model with the implicit PD step (case 2): per FE step and per PD step, wall time of pd_steps PD
    steps from a resident state, and the split into PD substeps (the paper's
    t^U), FE step (t^K) and multipliers with the final update (t^lambda) from
    a second, event-timed pass."""
    import mts_inputs as mi
    out = []
    for case, dx, frac, m, pd_beta in TABLE2_CASES:
        inst = mi.efficiency2d(dx, pd_frac=frac, m=m, pd_beta=pd_beta, n_macro=pd_steps // m)
        s = mts.Solver(inst)
        s.advance(max(2, 20 // m))
        s.sync()
        k = pd_steps // m
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.advance(k)
        s.sync()
        wall = (time.perf_counter() - t0) * 1e3 / k
        s.profile(True)
        s.advance(k)
        s.sync()
        ph = {}
        for name, kt in (("pd_substeps", mts.KT_PD_SUBSTEP), ("fe", mts.KT_FE), ("lambda", mts.KT_LAMBDA),
                         ("link", mts.KT_LINK)):
            n, ms = s.kernel_time(kt)
            ph[name] = ms / k
        s.profile(False)
        info = s.query()
        paper = TABLE2_PAPER_MS[case]
        rec = {"case": case, "workload": inst["name"], "dx_mm": dx * 1e3, "pd_area": frac, "m": m,
               "pd_nodes": info["n_pd"], "bonds": info["nnz"], "fe_beta": inst["fe_beta"], "pd_beta": pd_beta,
               "ms_per_fe_step": wall, "ms_per_pd_step": wall / m,
               "phases_ms_per_fe_step": {"t_U_pd_substeps": ph["pd_substeps"], "t_K_fe": ph["fe"],
                                         "t_lambda_multipliers_and_update": ph["lambda"] + ph["link"]},
               "paper_ms_per_fe_step": paper[0], "paper_ms_per_pd_step": paper[1]}
        out.append(rec)
        log(f"table 2 case {case}: {wall:.3f} ms per FE step ({wall / m:.4f} per PD step)")
        s.close()
    return {"cases": out, "paper": "Table 2 per-step times, RTX 3070, PeriFEM with an assembled stiffness "
                                   "(context, another discretisation and machine)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed macro steps (default: the workload's)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", type=int, default=2, help="workload index (1: 400x160 plate, 2: 1000x400 plate, "
                                                          "3: 100x100x20 block)")
    ap.add_argument("--fe-beta", type=float, default=0.0,
                    help="Newmark beta of the FE step: 0 explicit, 0.25 implicit (average acceleration)")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default=None,
                    help="precision of the headline run (default: fp64 on the plates, mixed on the block)")
    ap.add_argument("--no-companion", action="store_true",
                    help="skip the other precision on the same instance (and the error check)")
    ap.add_argument("--no-error-check", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving stream in the default line")
    ap.add_argument("--no-branching", action="store_true", help="skip the crack-branching comparison")
    ap.add_argument("--no-table2", action="store_true", help="skip the efficiency study's per-step times")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=8.0, help="per oracle build (one thread, all threads)")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel event timing pass")
    ap.add_argument("--profile-steps", type=int, default=100, help="macro steps of the event-timed pass")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (counter calibration)")
    ap.add_argument("--serve", action="store_true", help="only run the serving stream (its own JSON line)")
    ap.add_argument("--branching", action="store_true", help="only run the crack-branching comparison (its own line)")
    ap.add_argument("--glass-block", action="store_true",
                    help="only run the 100x100x20 block in glass to the end, with its rebuilds (its own line)")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-rate", type=float, default=20.0, help="Poisson arrival rate (requests/s)")
    ap.add_argument("--serve-budget-gib", type=float, default=0.0, help="pool budget (0: 90%% of free HBM)")
    ap.add_argument("--serve-no-graphs", action="store_true")
    ap.add_argument("--serve-builders", type=int, default=4, help="threads that build arrived requests")
    ap.add_argument("--serve-verbose", action="store_true")
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
        return serve_main(args, torch, log)
    if args.branching:
        br = branching_run(mts, torch, log)
        c = br["coupled"]
        print(json.dumps({
            "metric": "crack-branching plate: run time of the MTS model (s), with the pure-PD model beside it",
            "value": c["run_s"], "unit": "s", "n_gpus": 1, "steps": c["macro_steps"], "warmup": 0,
            "ms_per_step": c["run_s"] * 1e3 / c["macro_steps"], "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "crack-branching plate 100 x 40 mm, dx 0.25 mm, 6e-5 s"},
            "branching": br}), flush=True)
        return
    if args.glass_block:
        gb = glass_block_run(mts, torch, log, args.precision or "mixed", args.steps)
        print(json.dumps({
            "metric": "3D impact block in glass: run time to the end (s), rebuilds included",
            "value": gb["run_s"], "unit": "s", "n_gpus": 1, "steps": gb["macro_steps"], "warmup": 0,
            "ms_per_step": gb["run_s"] * 1e3 / gb["macro_steps"], "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64" if gb["workload"].endswith("fp64 glass") else "f32 bond math / f64 integration",
            "data": "synthetic", "config": {"workload": gb["workload"]}, "glass_block": gb}), flush=True)
        return
    default_prec = "mixed" if args.config == 3 else "fp64"
    prec = args.precision or default_prec
    inst = mi.config(args.config, precision=prec)
    if args.fe_beta:
        inst["fe_beta"] = args.fe_beta
        inst["name"] += f" implicit FE (beta {args.fe_beta:g})"
    other = "mixed" if prec == "fp64" else "fp64"
    K = args.steps if args.steps is not None else inst["n_macro"]
    W = args.warmup

    head = run_form(mts, torch, inst, K, W, args, log)
    info = head.pop("info")
    companion = None
    if not args.no_companion:
        inst2 = mi.config(args.config, precision=other)
        if args.fe_beta:
            inst2["fe_beta"] = args.fe_beta
            inst2["name"] += f" implicit FE (beta {args.fe_beta:g})"
        c = run_form(mts, torch, inst2, K, W, args, log)
        c.pop("info")
        fp64_rec, mx_rec = (head, c) if prec == "fp64" else (c, head)
        companion = {"precision": other, "workload": inst2["name"], **c,
                     "mixed_speedup_vs_fp64": mx_rec["value"] / fp64_rec["value"]}
        if not args.no_error_check:
            i64 = inst if prec == "fp64" else inst2
            imx = inst2 if prec == "fp64" else inst
            try:
                companion["mixed_error_vs_fp64"] = mixed_error(mts, torch, i64, imx, K, 25, log)
            except Exception as e:  # reported, not fatal to the line
                companion["mixed_error_vs_fp64"] = {"error": repr(e)}

    serving = None
    if not args.no_serving:
        try:
            serving, sizes = serve_run(args, torch, log)
            serving["request_sizes"] = sizes
        except Exception as e:  # reported, not fatal to the line
            serving = {"error": repr(e)}

    branching = None
    if not args.no_branching:
        try:
            branching = branching_run(mts, torch, log)
        except Exception as e:  # reported, not fatal to the line
            branching = {"error": repr(e)}

    table2 = None
    if not args.no_table2:
        try:
            table2 = table2_run(mts, torch, log)
        except Exception as e:  # reported, not fatal to the line
            table2 = {"error": repr(e)}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(inst, args.cpu_seconds)

    dtype = "f64" if prec == "fp64" else "f32 bond math / f64 integration"
    line = {
        "metric": METRIC, "value": head["value"], "unit": "bond-updates/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": inst["name"] + f", {K * inst['m']} PD steps ({K} macro steps)",
                   "pd_nodes": info["n_pd"], "bonds": info["nnz"], "m": inst["m"],
                   "fe_nodes": info["n_fe_nodes"], "constraints": info["n_constraints"],
                   "dt_pd": inst["dt_pd"], "rebuilds": head["rebuilds"], "setup_s": head["setup_s"],
                   "source_digest": source_digest(),
                   "gpu_event_ms": head["gpu_event_ms"], "wall_ms": head["wall_ms"]},
        "roofline": head.get("roofline"),
        "companion": companion,
        "serving": serving,
        "branching": branching,
        "table2": table2,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

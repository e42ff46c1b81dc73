"""Request loop over the serving pool (continuous batching).

Requests arrive on their own clock (Poisson arrivals, seconds); a few builder
threads take arrived requests in order and build each into the pool as soon as
a slot and device memory are free (mts_pool_submit runs the neighbour build and
the unit-load responses on a stream of its own), while the main thread keeps
issuing pool steps that advance every running request by one macro step.  Finished requests
are read back (damage and displacement) and released, which frees budget for
waiting arrivals.  Latency is completion minus arrival.
"""
from __future__ import annotations

import threading
import time
from typing import Dict, List, Optional

import numpy as np

from . import _lib


def serve(requests: List[Dict], budget_bytes: int, *, max_slots: int = 64, use_graphs: bool = True,
          stream=None, keep_results: bool = False, log=None, builders: int = 4) -> Dict:
    """Run `requests` (dicts with "arrival" in seconds and "inst", an instance
    dict with "n_macro") through a pool.

    Returns per-request latencies, percentiles, aggregate throughput and pool
    counters; with keep_results, also each request's damage and displacement."""
    pool = _lib.Pool(budget_bytes, max_slots=max_slots, dim=2,
                     precision=requests[0]["inst"].get("precision", "mixed") if requests else "mixed",
                     use_graphs=use_graphs, stream=stream)
    n = len(requests)
    order = sorted(range(n), key=lambda k: requests[k]["arrival"])
    t_admit = [None] * n
    t_done = [None] * n
    rid_of = {}
    results = {}
    freed = threading.Event()
    lock = threading.Lock()
    errors = []
    work = [0.0] * n  # bond-updates of each request (directed slots x PD substeps)
    rebuilds = [0] * n
    submit_s = [0.0]  # builder time inside mts_pool_submit (all builders)
    t0 = time.perf_counter()

    next_k = [0]

    def admission():
        """One of `builders` threads: take the next request in arrival order,
        wait for its arrival, build it into the pool (retrying while full)."""
        try:
            while True:
                with lock:
                    if next_k[0] >= n:
                        return
                    k = order[next_k[0]]
                    next_k[0] += 1
                r = requests[k]
                delay = t0 + r["arrival"] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                while True:
                    ts = time.perf_counter()
                    rid = pool.submit(r["inst"], r["inst"]["n_macro"])
                    with lock:
                        submit_s[0] += time.perf_counter() - ts
                    if rid is not None:
                        break
                    freed.wait(0.005)
                    freed.clear()
                with lock:
                    rid_of[rid] = k
                    t_admit[k] = time.perf_counter() - t0
                nnz = pool.poll(rid)[2]["nnz"]
                work[k] = float(nnz) * r["inst"]["m"] * r["inst"]["n_macro"]
        except Exception as e:  # surfaced by the main loop
            errors.append(e)

    threads = [threading.Thread(target=admission, daemon=True) for _ in range(max(1, builders))]
    for th in threads:
        th.start()
    finished = 0
    steps = 0
    step_s = 0.0  # host time inside mts_pool_step (it runs the rebuilds that the last step flagged)
    while finished < n:
        if errors:
            raise errors[0]
        ts = time.perf_counter()
        na, done = pool.step()
        step_s += time.perf_counter() - ts
        steps += 1
        for rid in done:
            while True:  # the admission thread registers the id right after submit returns
                with lock:
                    k = rid_of.get(rid)
                if k is not None:
                    break
                time.sleep(0.0001)
            inst = requests[k]["inst"]
            npd = inst["pos"].shape[0]
            phi = pool.read(rid, _lib.DAMAGE, npd)
            rebuilds[k] = pool.poll(rid)[2]["n_rebuilds"]
            t_done[k] = time.perf_counter() - t0
            if keep_results:
                results[k] = {"damage": phi, "u": pool.read(rid, _lib.PD_U, npd * 2)}
            pool.release(rid)
            freed.set()
            finished += 1
            if log:
                log(f"request {k} ({inst['name']}) done: latency {t_done[k] - requests[k]['arrival']:.3f} s")
        if na == 0 and not done:
            time.sleep(0.0005)
    for th in threads:
        th.join()
    info = pool.query()
    pool.close()
    arr = np.array([requests[k]["arrival"] for k in range(n)])
    lat = np.array(t_done) - arr
    wait = np.array(t_admit) - arr
    total = float(sum(work))
    span = max(t_done) - min(arr)
    out = {
        "n_requests": n, "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
        "mean_s": float(lat.mean()), "max_s": float(lat.max()),
        "admission_wait_p50_s": float(np.percentile(wait, 50)), "admission_wait_p99_s": float(np.percentile(wait, 99)),
        "bond_updates": total, "span_s": span, "bond_updates_per_s": total / span,
        "pool_steps": steps, "graph_captures": info["graph_captures"], "graph_replays": info["graph_replays"],
        "rebuilds": int(sum(rebuilds)), "requests_with_rebuilds": int(sum(1 for x in rebuilds if x)),
        "host_s_in_pool_step": step_s, "host_s_in_pool_submit": submit_s[0],
        "latencies_s": lat.tolist(),
    }
    if keep_results:
        out["results"] = results
    return out


def stream_requests(n: Optional[int] = None, precision: str = "mixed", **kw) -> List[Dict]:
    """The seeded serving stream as request dicts for serve()."""
    import mts_inputs as mi
    reqs = mi.serving_stream(**kw)
    if n is not None:
        reqs = reqs[:n]
    out = []
    for r in reqs:
        inst = mi.serving_instance(r, precision=precision)
        nx, ny = inst["pd_n"][0], inst["pd_n"][1]
        out.append({"arrival": r["arrival"], "inst": inst, "nx": nx, "ny": ny, "m": inst["m"]})
    return out

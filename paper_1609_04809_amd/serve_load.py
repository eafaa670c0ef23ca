"""Load generator for the solve server: replays a request trace against
mg_server_* and reports latency percentiles and throughput.

Each request's right-hand side is generated (seeded, U[-1, 1]) on a
background thread ahead of its arrival time -- for a trace whose requests
all arrive at once, all of them before the clock starts, so that the
generator does not pace the submissions; submission follows the trace's
arrival times on the wall clock; results are collected as they finish.
Latency is measured by the server from submission to the result being in
host memory.
"""

import queue
import threading
import time

import numpy as np

from . import workloads as W


def _producer(trace, out_q, stop):
    for r in trace:
        if stop.is_set():
            return
        b = W.interior_to_full(r["dim"], r["n"], W.rhs_uniform(r["dim"], r["n"], r["seed"]))
        kappa = W.kappa_lognormal(r["dim"], r["n"], r["seed"]) if r.get("kappa") else None
        out_q.put((r, b, kappa))
    out_q.put(None)


def run_trace(trace, hbm_budget_bytes, max_slots=64, tol=1e-8, precision="fp32_ir",
              smoother="rbgs", log=None):
    """Replay `trace` (see workloads.serving_trace).  Returns a summary dict."""
    from .mg import Server
    burst = all(r["t_arrival"] == 0.0 for r in trace)
    q = queue.Queue(maxsize=0 if burst else 64)
    stop = threading.Event()
    th = threading.Thread(target=_producer, args=(trace, q, stop), daemon=True)
    th.start()
    if burst:
        th.join()  # every right-hand side ready before the clock starts
    results = []
    dofs = {}
    failed = []
    with Server(hbm_budget_bytes, max_slots) as srv:
        t0 = time.perf_counter()
        last_log = t0
        while True:
            item = q.get()
            if item is None:
                break
            r, b, kappa = item
            wait = r["t_arrival"] - (time.perf_counter() - t0)
            while wait > 0:
                for d in srv.poll():
                    results.append(d)
                time.sleep(min(wait, 0.001))
                wait = r["t_arrival"] - (time.perf_counter() - t0)
            rid = srv.submit(r["dim"], r["n"], r["levels"], b, tol, kappa=kappa,
                             precision=precision, smoother=smoother)
            dofs[rid] = (r["n"] + 1) ** r["dim"]
            for d in srv.poll():
                results.append(d)
            if log and time.perf_counter() - last_log > 2.0:
                last_log = time.perf_counter()
                log(f"[serve] t={last_log - t0:.1f}s submitted {len(dofs)} done {len(results)}")
        srv.drain(600.0)
        for d in srv.poll():
            results.append(d)
        t_end = time.perf_counter()
        stats = srv.stats()
    stop.set()
    lat = np.array([d["latency_us"] for d in results if d["status"] == "ok"])
    failed = [d for d in results if d["status"] != "ok"]
    iters = np.array([d["iters"] for d in results if d["status"] == "ok"])
    total_dofs = sum(dofs[d["id"]] for d in results if d["status"] == "ok")
    wall = t_end - t0
    out = {
        "requests": len(trace),
        "completed": int(len(lat)),
        "failed": len(failed),
        "p50_ms": round(float(np.percentile(lat, 50)) / 1e3, 3) if len(lat) else None,
        "p99_ms": round(float(np.percentile(lat, 99)) / 1e3, 3) if len(lat) else None,
        "max_ms": round(float(lat.max()) / 1e3, 3) if len(lat) else None,
        "mean_ms": round(float(lat.mean()) / 1e3, 3) if len(lat) else None,
        "wall_s": round(wall, 3),
        "throughput_MDOF_per_s": round(total_dofs / wall / 1e6, 1),
        "throughput_req_per_s": round(len(lat) / wall, 1),
        "busy_s": round(stats["busy_s"], 3),
        "MDOF_per_busy_s": round(total_dofs / max(stats["busy_s"], 1e-9) / 1e6, 1),
        "mean_in_flight": round(len(lat) / wall * float(lat.mean()) / 1e6, 2) if len(lat) else 0,
        "batched_launches": int(stats["launches"]),
        "ops_per_launch": round(stats["fused_ops"] / max(stats["launches"], 1), 3),
        "hbm_budget_GB": round(hbm_budget_bytes / 1e9, 3),
        "hbm_peak_GB": round(stats["hbm_peak"] / 1e9, 3),
        "mean_cycles": round(float(iters.mean()), 2) if len(iters) else None,
        "tol": tol,
        "precision": precision,
        "kappa_requests": int(sum(1 for r in trace if r.get("kappa"))),
        "failed_status": {st: sum(1 for d in failed if d["status"] == st)
                          for st in sorted({d["status"] for d in failed})},
    }
    return out

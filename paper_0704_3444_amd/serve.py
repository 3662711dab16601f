"""Request loops over the library: continuous batching, and one run at a
time for comparison.

serve_batched: requests (phase-separation runs of their own box, N and
parameters) arrive over time; each is admitted into a live slot of one
Batch as soon as a slot and an arena range of its device-memory footprint
are free (first come, first served), so runs that arrive while others are
on the GPU join the persistent batched kernel without waiting for them.
The host keeps one launch of `chunk` steps queued ahead of the one whose
step counters it reads, retires runs that reached their step count (reading
their observables on the library's second stream) and admits the next ones.

serve_serial: the same requests one at a time, each with its own
Simulation (the fastest single-run path), in arrival order.

Both return per-request records (arrival, admission and finish times in
seconds from the start, latency = finish - arrival, the component masses
and, if asked, the densities) and the whole run's throughput.  Every step
of every run executes in the library's HIP kernels.
"""
from __future__ import annotations

import time
from collections import deque

import numpy as np

from .lb import Batch, Simulation


def _work(r) -> int:
    return int(np.prod(r["cfg"]["shape"])) * int(r["cfg"]["n_comp"]) * int(r["nsteps"])


def summarize(records: list, t_end: float, requests: list) -> dict:
    lat = np.array([x["latency"] for x in records])
    work = sum(_work(r) for r in requests)
    t_first = min(r["arrival"] for r in requests)
    return {
        "requests": len(records), "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
        "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2), "mean_ms": round(float(lat.mean()) * 1e3, 2),
        "makespan_s": round(float(t_end - t_first), 4),
        "mlups_x_comp": round(float(work / (t_end - t_first) / 1e6), 1),
    }


def serve_batched(requests: list, *, storage="f32", max_comp=3, max_slots=128, arena_bytes=8 << 30, chunk=100,
                  graph_steps=50, config=-1, keep_fields=False, clock=time.perf_counter, log=None):
    """Continuous batching of `requests` (dicts with arrival, cfg, rho0,
    nsteps, id; see lbinputs.serving_mix).  Returns (records, summary)."""
    batch = Batch(storage=storage, max_comp=max_comp, max_slots=max_slots, arena_bytes=arena_bytes,
                  config=config, graph_steps=graph_steps)
    order = sorted(requests, key=lambda r: r["arrival"])
    waiting: deque = deque()
    live: dict = {}
    records: list = []
    i, launched = 0, 0
    t0 = clock()
    try:
        while len(records) < len(order):
            now = clock() - t0
            while i < len(order) and order[i]["arrival"] <= now:
                waiting.append(order[i])
                i += 1
            while waiting:
                r = waiting[0]
                slot = batch.try_add(r["cfg"], r["rho0"], r["nsteps"])
                if slot is None:
                    if not live:
                        raise RuntimeError(f"request {r['id']} does not fit an empty batch")
                    break
                waiting.popleft()
                live[slot] = (r, clock() - t0)
            if not live:
                if i < len(order):
                    time.sleep(max(0.0, order[i]["arrival"] - (clock() - t0)))
                continue
            batch.step(chunk)
            launched += 1
            counts = batch.poll(lag=1 if launched > 1 else 0)
            for slot, (r, t_adm) in list(live.items()):
                if counts[slot] < r["nsteps"]:
                    continue
                out = batch.moments(slot, fields=keep_fields)
                batch.remove(slot)
                del live[slot]
                t_fin = clock() - t0
                rec = {"id": r["id"], "arrival": r["arrival"], "admitted": t_adm, "finished": t_fin,
                       "latency": t_fin - r["arrival"], "mass": out["mass"], "status": out["status"],
                       "step": out["step"]}
                if keep_fields:
                    rec["rho"] = out["rho"]
                records.append(rec)
                if log:
                    log(f"[serve] request {r['id']} done: latency {rec['latency'] * 1e3:.1f} ms, "
                        f"{len(live)} live, {len(waiting)} waiting")
        t_end = clock() - t0
    finally:
        batch.close()
    return records, summarize(records, t_end, order)


def serve_serial(requests: list, *, storage="f32", keep_fields=False, clock=time.perf_counter, log=None):
    """The same requests one at a time in arrival order.  Returns (records,
    summary)."""
    import torch

    order = sorted(requests, key=lambda r: r["arrival"])
    records = []
    t0 = clock()
    for r in order:
        wait = r["arrival"] - (clock() - t0)
        if wait > 0:
            time.sleep(wait)
        t_adm = clock() - t0
        sim = Simulation(r["cfg"], r["rho0"], storage=storage)
        sim.step(r["nsteps"])
        out = sim.moments(fields=keep_fields, raise_numeric=False)
        sim.close()
        torch.cuda.synchronize()
        t_fin = clock() - t0
        rec = {"id": r["id"], "arrival": r["arrival"], "admitted": t_adm, "finished": t_fin,
               "latency": t_fin - r["arrival"], "mass": out["mass"], "status": out["status"], "step": out["step"]}
        if keep_fields:
            rec["rho"] = out["rho"]
        records.append(rec)
        if log:
            log(f"[serial] request {r['id']} done: latency {rec['latency'] * 1e3:.1f} ms")
    t_end = clock() - t0
    return records, summarize(records, t_end, order)


def tune_batch(requests: list, *, storage="f32", max_comp=3, max_slots=64, arena_bytes=8 << 30, steps=20,
               graph_steps=50):
    """Autotune the batched kernel on a batch filled with `requests` (their
    runs are only used for timing): returns (best configuration, ms per step
    of every configuration)."""
    batch = Batch(storage=storage, max_comp=max_comp, max_slots=max_slots, arena_bytes=arena_bytes,
                  graph_steps=graph_steps)
    try:
        for r in requests:
            if batch.try_add(r["cfg"], r["rho0"], 1 << 40) is None:
                break
        return batch.tune(steps)
    finally:
        batch.close()

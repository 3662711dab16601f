"""Benchmark of the hot path: one time step of the symmetric free-energy
multicomponent LB method (Li & Wagner) on the ternary D2Q9 2048 x 2048
immersion-precipitation workload, FP32, one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--storage f32|f64|f16s]
                    [--workload NAME] [--no-cpu] [--calibrate-copy]

Prints one JSON line.  `value` is MLUPS x components (sites x components x
steps / second / 1e6) with the state resident in HBM; the timed region is K
lb_step calls bracketed by synchronisation and HIP events on the stream the
kernels run on.  `roofline` prices the fused step kernel against the HBM
peak: its algorithmic traffic per launch is every population read once and
written once, 2 * N * S * (rest + reference + (Q - 1) * moving slot bytes; the
reference, 2 bytes, only for shifted FP16).  `cpu_baseline` times the FP64 CPU
oracle on a bounded sample of the same workload on the host cores.

Three more objects on the same line (skipped with --no-f16s / --no-serving /
--no-phase): `f16s` times the same workload with shifted FP16 storage;
`serving` runs a Poisson mix of 256 phase-separation requests (N 2 or 3,
square boxes of side 64..512, 5000 steps each) through the
continuous-batching loop and, for comparison, one request at a time, and
reports p50/p99 latency and throughput of both, plus the batch's capacity
with all requests queued at t = 0; `phase_sweeps` times the four binodal run
sets of Sec. IV (D1Q3 lines of 128 sites, the paper's step counts) through
line groups, one launch per set, with throughput over the runs that stayed
physical.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS×components at 2048² ternary, % HBM peak; serving p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# sources of each fused kernel: a traffic summary holds for the sources it was
# taken with (their hash is in the summary)
COMMON_SOURCES = ["paper_0704_3444_amd/csrc/physics.hpp", "paper_0704_3444_amd/csrc/lattice.hpp",
                  "paper_0704_3444_amd/csrc/storage.hpp"]
KERNEL_SOURCES = {
    ("D2Q9", "sweep"): ["paper_0704_3444_amd/csrc/k_sweep2d.hip"] + COMMON_SOURCES,
    ("D2Q9", "tile"): ["paper_0704_3444_amd/csrc/k_fused2d.hip"] + COMMON_SOURCES,
    ("D3Q19", "sweep"): ["paper_0704_3444_amd/csrc/k_sweep3d.hip"] + COMMON_SOURCES,
}
KERNEL_NAMES = {("D2Q9", "sweep"): "k_sweep_d2q9", ("D2Q9", "tile"): "k_fused_d2q9",
                ("D3Q19", "sweep"): "k_sweep_d3q19"}
# bytes per site and component: (rest slot, moving slot, reference)
STORE_BYTES = {"f64": (8, 8, 0), "f32": (4, 4, 0), "f16s": (4, 2, 2)}


def kernel_source_hash(lattice, kpath) -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES.get((lattice, kpath), COMMON_SOURCES):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload(name):
    import lbinputs as LI

    table = {
        "ternary_d2q9_2048": lambda: LI.ternary_immersion(2048),
        "ternary_substrate_d2q9_2048": lambda: LI.ternary_film_on_substrate(2048),
        "binary_d2q9_1024": lambda: LI.binary_spinodal(1024, seed=1001),
        "ternary_d3q19_256": lambda: LI.ternary_d3q19(256),
        "five_d2q9_512": lambda: LI.five_component(512),
        "binary_d2q9_64": lambda: LI.binary_spinodal(64),
    }
    return table[name]()


def measured_traffic(name, storage, kpath, lattice):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel's sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{name}_{storage}_{kpath}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha") != kernel_source_hash(lattice, kpath):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(cfg, rho0, target_s=15.0):
    """FP64 oracle on the host cores: calibrate with one step, then run as
    many steps as fit in about target_s seconds (at most 50)."""
    from oracle import Oracle, OracleParams

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    o = Oracle(OracleParams(**cfg), rho0)
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter() - t0
    n = max(1, min(50, int(target_s / max(t1, 1e-6))))
    t0 = time.perf_counter()
    o.step(n)
    dt = time.perf_counter() - t0
    sites = int(cfg["shape"][0]) * int(cfg["shape"][1]) * (int(cfg["shape"][2]) if len(cfg["shape"]) > 2 else 1)
    value = sites * cfg["n_comp"] * n / dt / 1e6
    return {"value": round(value, 3), "unit": "MLUPS×components", "cores": threads, "kind": "oracle",
            "sample": f"{n} steps (after 1 warm-up step) of the full {cfg['shape'][0]}x{cfg['shape'][1]} "
                      f"N={cfg['n_comp']} workload from its initial state, FP64, {dt:.1f} s"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_ONE_CORE = """
import json, sys, time
sys.path.insert(0, {root!r})
import lbinputs as LI
from oracle import Oracle, OracleParams
cfg, rho0 = LI.ternary_immersion(2048)
o = Oracle(OracleParams(**cfg), rho0)
t0 = time.perf_counter(); o.step(1); t1 = time.perf_counter() - t0
n = min(20, int({target} / max(t1, 1e-6)))
if n < 2:
    print(json.dumps({{"steps": 1, "seconds": t1}}))
else:
    t0 = time.perf_counter(); o.step(n); dt = time.perf_counter() - t0
    print(json.dumps({{"steps": n, "seconds": dt}}))
"""


def cpu_single_core(target_s=10.0):
    """The same oracle sample on one host core (a child process with
    OMP_NUM_THREADS=1, since the thread count is fixed once OpenMP starts)."""
    import subprocess

    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", _ONE_CORE.format(root=ROOT, target=target_s)], env=env,
                         capture_output=True, text=True, timeout=600, check=True)
    r = json.loads(out.stdout.strip().splitlines()[-1])
    value = 2048 * 2048 * 3 * r["steps"] / r["seconds"] / 1e6
    return {"value": round(value, 3), "unit": "MLUPS×components", "cores": 1,
            "sample": f"{r['steps']} steps of the full 2048x2048 N=3 workload, FP64, {r['seconds']:.1f} s"}


def cpu_small_full_run():
    """The oracle over the whole small binary case (64x64, 2000 steps), all host cores."""
    from oracle import Oracle, OracleParams
    import lbinputs as LI

    cfg, rho0 = LI.binary_spinodal(64)
    o = Oracle(OracleParams(**cfg), rho0)
    t0 = time.perf_counter()
    o.step(2000)
    dt = time.perf_counter() - t0
    return {"workload": "binary_d2q9_64", "steps": 2000, "seconds": round(dt, 3),
            "value": round(64 * 64 * 2 * 2000 / dt / 1e6, 3), "unit": "MLUPS×components"}


def cpu_line_baseline(target_s=5.0):
    """FP64 oracle on one ternary D1Q3 line of the binodal experiments (one
    host core: a single row), as many steps as fit in about target_s."""
    from oracle import Oracle, OracleParams
    import lbinputs as LI

    cfg, rho0, _ = LI.binodal_runs("ternary_monomer")[9]
    o = Oracle(OracleParams(**cfg), rho0)
    t0 = time.perf_counter()
    o.step(1000)
    n = max(1000, int(target_s / max(time.perf_counter() - t0, 1e-6) * 1000))
    t0 = time.perf_counter()
    o.step(n)
    dt = time.perf_counter() - t0
    return {"value": round(cfg["shape"][0] * cfg["n_comp"] * n / dt / 1e6, 3), "unit": "MLUPS×components",
            "sample": f"{n} steps of one 128-site ternary D1Q3 line, FP64, {dt:.1f} s"}


def run_phase_sweeps():
    """The binodal run sets of Sec. IV, each stepped by one line group for the
    paper's step count; the timed region is the group's single launch."""
    import torch
    import lbinputs as LI
    from paper_0704_3444_amd import Lines, Simulation

    out = {}
    for exp, steps in (("binary_monomer", 50000), ("binary_polymer", 50000), ("ternary_monomer", 200000),
                       ("ternary_polymer", 200000)):
        runs = LI.binodal_runs(exp)
        sims = [Simulation(c, r) for c, r, _ in runs]
        group = Lines(sims)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        group.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        healthy = sum(1 for x in sims if x.moments(fields=False, raise_numeric=False)["status"] == 0)
        group.close()
        n = runs[0][0]["n_comp"]
        L = runs[0][0]["shape"][0]
        # throughput counts only the runs that stayed physical: a run whose
        # density went non-finite or non-positive produced no result
        out[exp] = {"runs": len(runs), "steps": steps, "seconds": round(dt, 4),
                    "us_per_step": round(dt / steps * 1e6, 3),
                    "value": round(healthy * L * n * steps / dt / 1e6, 1), "unit": "MLUPS×components",
                    "healthy_runs": healthy}
        for x in sims:
            x.close()
    return out


def calibrate_copy(gib=1.0, reps=5):
    """A plain device-to-device copy of known size, run under rocprofv3 --pmc
    to scale FETCH_SIZE / WRITE_SIZE (each copy reads and writes `gib` GiB)."""
    import torch

    n = int(gib * (1 << 30))
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty(n, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": n, "reps": reps}), flush=True)


def alg_bytes_per_step(N, S, Q, storage):
    rest_b, move_b, ref_b = STORE_BYTES[storage]
    return 2 * N * S * (rest_b + ref_b + (Q - 1) * move_b)


def time_steps(cfg, rho0, storage, kpath, steps, warmup, stream):
    """HIP-event time of `steps` lb_step calls after `warmup` untimed ones."""
    import numpy as np
    import torch

    from paper_0704_3444_amd import Simulation

    S = int(np.prod(cfg["shape"]))
    N = int(cfg["n_comp"])
    sim = Simulation(cfg, rho0, storage=storage, path=kpath, stream=stream)
    print(f"bench: {cfg['shape']} N={N} {storage} path={sim.path}; warmup {warmup}", file=sys.stderr, flush=True)
    sim.step(warmup)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    sim.step(steps)
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(end)
    # the state must still be physical after the timed steps
    health = sim.moments(fields=False)
    out = {"ms_per_step": ms / steps, "value": S * N * steps / (ms / 1e3) / 1e6, "wall": wall, "path": sim.path,
           "health": health, "mass_drift": float(np.max(np.abs(health["mass"] / rho0.sum(axis=1) - 1)))}
    sim.close()
    return out


def run_serving(n_req):
    """The Poisson request mix through the continuous-batching loop (after
    autotuning the batched kernel on a throwaway batch of the first 48
    requests) and one request at a time."""
    import lbinputs as LI
    from paper_0704_3444_amd import lb, serve

    print(f"bench: serving {n_req} requests", file=sys.stderr, flush=True)
    reqs = LI.serving_mix(n_req)
    best, ms = serve.tune_batch(reqs[:48], steps=10)
    info = lb.lb_batch_config_info("f32", 3, best)
    batched, bsum = serve.serve_batched(reqs, config=best, chunk=100, graph_steps=50)
    print(f"bench: serving batched {bsum}", file=sys.stderr, flush=True)
    best16, _ = serve.tune_batch(reqs[:48], storage="f16s", steps=10)
    info16 = lb.lb_batch_config_info("f16s", 3, best16)
    batched16, bsum16 = serve.serve_batched(reqs, storage="f16s", config=best16, chunk=100, graph_steps=50)
    print(f"bench: serving batched, shifted FP16 storage {bsum16}", file=sys.stderr, flush=True)
    # capacity: the same requests all queued at t = 0, so that the batch is
    # never short of work (the Poisson mix above arrives more slowly than the
    # batch serves it, and its throughput is the arrival rate)
    saturated = [dict(r, arrival=0.0) for r in reqs]
    sat, satsum = serve.serve_batched(saturated, config=best, chunk=100, graph_steps=50)
    print(f"bench: serving batched, all requests at t = 0 {satsum}", file=sys.stderr, flush=True)
    serial, ssum = serve.serve_serial(reqs)
    print(f"bench: serving one at a time {ssum}", file=sys.stderr, flush=True)
    bad = sum(x["status"] != 0 for x in batched + batched16 + sat + serial)
    return {"workload": f"poisson_mix_{n_req}", "rate_hz": 40.0, "steps_per_request": reqs[0]["nsteps"],
            "storage": "f32", "tuned_config": dict(info, index=best), "batched": bsum, "one_at_a_time": ssum,
            "speedup_throughput": round(bsum["mlups_x_comp"] / ssum["mlups_x_comp"], 3),
            "speedup_p99": round(ssum["p99_ms"] / bsum["p99_ms"], 3),
            "batched_saturated": satsum,
            "capacity_vs_one_at_a_time": round(satsum["mlups_x_comp"] / ssum["mlups_x_comp"], 3),
            "batched_f16s": dict(bsum16, tuned_config=dict(info16, index=best16)), "failed_requests": bad}


def run_batch_only(n_req, steps, warmup, storage):
    """One batch holding the first n_req requests of the serving mix, all
    live, stepped `steps` times after `warmup` (for profiling the batched
    kernel): HIP-event time per step and the algorithmic bytes of a step
    (every population of every slot read and written once)."""
    import numpy as np
    import torch
    import lbinputs as LI
    from paper_0704_3444_amd import lb

    reqs = LI.serving_mix(256)[:n_req]
    # the batch steps on the stream the events are recorded on (a stream of
    # its own: given the null stream, a batch creates a non-blocking stream)
    st = torch.cuda.Stream()
    batch = lb.Batch(storage=storage, max_comp=3, max_slots=n_req, arena_bytes=8 << 30, graph_steps=50,
                     stream=st.cuda_stream)
    alg = 0
    try:
        for r in reqs:
            batch.add(r["cfg"], r["rho0"], 1 << 40)
            alg += alg_bytes_per_step(int(r["cfg"]["n_comp"]), int(np.prod(r["cfg"]["shape"])), 9, storage)
        batch.step(warmup)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        batch.step(steps)
        b.record(st)
        torch.cuda.synchronize()
        batch.poll(0)
        ms = a.elapsed_time(b) / steps
    finally:
        batch.close()
    return {"requests": n_req, "storage": storage, "steps": steps, "ms_per_step": round(ms, 5),
            "algorithmic_bytes_per_step": alg, "hbm_frac": round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=150)
    ap.add_argument("--storage", default="f32", choices=["f32", "f64", "f16s"])
    ap.add_argument("--workload", default="ternary_d2q9_2048")
    ap.add_argument("--path", default="auto", choices=["auto", "sweep", "tile", "split"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--no-f16s", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-phase", action="store_true")
    ap.add_argument("--only-phase", action="store_true", help="time only the phase sweeps (for profiling them)")
    ap.add_argument("--only-batch", type=int, default=0,
                    help="time only one batch of this many serving requests (for profiling the batched kernel)")
    ap.add_argument("--walls", type=int, default=0, help="close axes by walls (bit a: axis a; walls on y only: the D2Q9 strip sweep, else the tile kernel or the split path)")
    ap.add_argument("--serving-requests", type=int, default=256)
    ap.add_argument("--no-substrate", action="store_true",
                    help="skip the film-on-a-substrate run (walls on y) timed beside the default workload")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one GPU only (a single lattice per device; multi-GPU "
              "slab decomposition is not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return

    import numpy as np
    import torch

    from paper_0704_3444_amd import Simulation, lb

    if not os.path.exists(lb.LIB_PATH):
        from paper_0704_3444_amd import build as gpu_build
        gpu_build.build()

    if args.only_phase:
        torch.cuda.set_device(0)
        print(json.dumps({"phase_sweeps": run_phase_sweeps()}), flush=True)
        return
    if args.only_batch:
        torch.cuda.set_device(0)
        print(json.dumps({"batch": run_batch_only(args.only_batch, args.steps, args.warmup, args.storage)}),
              flush=True)
        return

    cfg, rho0 = workload(args.workload)
    if args.walls:
        cfg = dict(cfg, walls=args.walls)
    shape = list(cfg["shape"]) + [1] * (3 - len(cfg["shape"]))
    S = int(np.prod(shape))
    N = int(cfg["n_comp"])
    Q = {"D1Q3": 3, "D2Q9": 9, "D3Q19": 19}[cfg["lattice"]]

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    # the same film cast on a substrate (walls on y), timed first so that
    # the main workload's launches are the last ones of the run
    substrate = None
    if not args.no_substrate and args.workload == "ternary_d2q9_2048" and args.storage == "f32" and not args.walls:
        scfg, srho = workload("ternary_substrate_d2q9_2048")
        h = time_steps(scfg, srho, "f32", args.path, args.steps, args.warmup, stream)
        sb = alg_bytes_per_step(N, S, Q, "f32")
        substrate = {"workload": "ternary_substrate_d2q9_2048", "walls": int(scfg["walls"]),
                     "value": round(h["value"], 1), "ms_per_step": round(h["ms_per_step"], 5), "path": h["path"],
                     "hbm_frac": round(sb / (h["ms_per_step"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                     "mass_drift": h["mass_drift"], "status": h["health"]["status"]}
        del srho

    r = time_steps(cfg, rho0, args.storage, args.path, args.steps, args.warmup, stream)
    ms_per_step, value, wall, path = r["ms_per_step"], r["value"], r["wall"], r["path"]
    health, mass_drift = r["health"], r["mass_drift"]

    kernels_per_step = 3 if path == "split" else 1
    alg_bytes = alg_bytes_per_step(N, S, Q, args.storage)
    achieved = alg_bytes / (ms_per_step / 1e3) / 1e9
    traffic = measured_traffic(args.workload, args.storage, path, cfg["lattice"])
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": KERNEL_NAMES.get((cfg["lattice"], path), "k_density+k_potential+k_collide"),
                "algorithmic_bytes_per_launch": alg_bytes, "launches_per_step": kernels_per_step,
                "avg_launch_ms": round(ms_per_step / kernels_per_step, 5)}

    f16s = None
    if not args.no_f16s and args.storage == "f32" and cfg["lattice"] in ("D2Q9", "D3Q19"):
        h = time_steps(cfg, rho0, "f16s", args.path, args.steps, args.warmup, stream)
        hb = alg_bytes_per_step(N, S, Q, "f16s")
        f16s = {"value": round(h["value"], 1), "ms_per_step": round(h["ms_per_step"], 5), "path": h["path"],
                "speedup_vs_f32": round(h["value"] / value, 3),
                "hbm_frac": round(hb / (h["ms_per_step"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                "algorithmic_bytes_per_launch": hb,
                "traffic": measured_traffic(args.workload, "f16s", h["path"], cfg["lattice"]),
                "mass_drift": h["mass_drift"], "status": h["health"]["status"]}

    serving = None
    if not args.no_serving:
        serving = run_serving(args.serving_requests)

    phase_sweeps = None
    if not args.no_phase:
        phase_sweeps = run_phase_sweeps()

    cpu = None
    if not args.no_cpu:
        print("bench: timing the CPU oracle on the same workload", file=sys.stderr, flush=True)
        cpu = cpu_baseline(cfg, rho0)
        cpu["cpu_model"] = cpu_model()
        cpu["host_cpus"] = len(os.sched_getaffinity(0))
        if args.workload == "ternary_d2q9_2048":
            cpu["single_core"] = cpu_single_core()
        cpu["small_full_run"] = cpu_small_full_run()
        if phase_sweeps is not None:
            cpu["line_run"] = cpu_line_baseline()

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "MLUPS×components", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.storage == "f64" else "f32", "data": "synthetic",
        "config": {"workload": args.workload, "lattice": cfg["lattice"], "shape": shape[: len(cfg["shape"])],
                   "n_comp": N, "storage": args.storage, "path": path, "force_form": cfg["force_form"],
                   "walls": int(cfg.get("walls", 0))},
        "hbm_frac": round(achieved / HBM_PEAK_GBS, 4),
        "wall_s": round(wall, 4), "mass_drift": mass_drift, "status": health["status"],
        "roofline": roofline, "cpu_baseline": cpu, "f16s": f16s, "substrate": substrate, "serving": serving,
        "phase_sweeps": phase_sweeps,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Shared helpers of the GPU tests: run a workload on the GPU library and on
the oracle from the same seeded input, and compare them."""
import numpy as np

from oracle import Oracle, OracleParams

# Pointwise tolerances at 200 steps: FP64 path 1e-12 relative, FP32 path
# 1e-5 relative, both against the FP64 oracle.
TOL = {"f64": 1e-12, "f32": 1e-5}


def paths_for(cfg, storage):
    """Kernel paths that support a run: split always; the tile kernel for
    D2Q9 in every storage; the strip sweep for D2Q9 in FP32 or shifted FP16
    with nx a multiple of 64 and N <= 4."""
    paths = ["split"]
    if cfg["lattice"] == "D2Q9":
        paths.append("tile")
        if storage in ("f32", "f16s") and cfg["shape"][0] % 64 == 0 and cfg["n_comp"] <= 4:
            paths.append("sweep")
    return paths


def run_gpu(cfg, rho0, steps, storage="f64", path="auto", fields=True):
    from paper_0704_3444_amd import Simulation

    sim = Simulation(cfg, rho0, storage=storage, path=path)
    sim.step(steps)
    out = sim.moments(fields=fields)
    out["path"] = sim.path
    out["f"] = sim.get_f() if fields else None
    sim.close()
    return out


def run_oracle(cfg, rho0, steps):
    o = Oracle(OracleParams(**cfg), rho0)
    o.step(steps)
    out = o.observe()
    out["f"] = o.get_f()
    return out


CS = 1.0 / np.sqrt(3.0)  # lattice speed of sound


def errors(gpu, ref, theta=1.0 / 3.0):
    """Max relative errors.
    rho: per site, |d rho^s| / rho^s.   f: relative to the largest population.
    U: relative to the lattice sound speed (U = u + A/(2 rho) nearly cancels
       near equilibrium, so its own size is no scale).
    mu: relative to its largest magnitude.
    P: relative to max|P| + theta * max(rho) / 100 (its bulk part vanishes
       identically and is a difference of O(theta rho) terms)."""
    e = {"rho": float(np.max(np.abs(gpu["rho"] - ref["rho"]) / np.abs(ref["rho"])))}
    e["U"] = float(np.abs(gpu["U"] - ref["U"]).max() / max(float(np.abs(ref["U"]).max()), CS))
    e["mu"] = float(np.abs(gpu["mu"] - ref["mu"]).max() / float(np.abs(ref["mu"]).max()))
    pscale = float(np.abs(ref["P"]).max()) + theta * float(ref["rho"].sum(0).max()) / 100
    e["P"] = float(np.abs(gpu["P"] - ref["P"]).max() / pscale)
    if gpu.get("f") is not None:
        e["f"] = float(np.abs(gpu["f"] - ref["f"]).max() / np.abs(ref["f"]).max())
    e["mass"] = float(np.max(np.abs(gpu["mass"] - ref["mass"]) / np.abs(ref["mass"])))
    return e

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
    with nx a multiple of 64 and N <= 4; the plane sweep for D3Q19 in FP32
    or shifted FP16 with nx a multiple of 64, ny a multiple of 4 and N <= 3
    (periodic boxes only)."""
    paths = ["split"]
    if cfg.get("walls", 0):
        return paths
    if cfg["lattice"] == "D2Q9":
        paths.append("tile")
        if storage in ("f32", "f16s") and cfg["shape"][0] % 64 == 0 and cfg["n_comp"] <= 4:
            paths.append("sweep")
    if cfg["lattice"] == "D3Q19" and storage in ("f32", "f16s") and cfg["shape"][0] % 64 == 0 \
            and cfg["shape"][1] % 4 == 0 and cfg["n_comp"] <= 3:
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


def oracle_observe_of(cfg, rho0, f):
    """The oracle's observables of a given state: populations f[N][Q][S]
    (e.g. the GPU's own, read back exactly in FP64).  Comparing them with the
    GPU's observables isolates the observable formulas (U, mu, P, mass,
    momentum) from the rounding of the time stepping."""
    o = Oracle(OracleParams(**cfg), rho0)
    o.set_f(np.ascontiguousarray(f))
    out = o.observe()
    out["f"] = np.array(f)
    return out


# Same-state observables: both sides evaluate them in FP64 from the same
# populations, so they differ by FP64 rounding in a different order only.
SAME_STATE_TOL = 1e-11


CS = 1.0 / np.sqrt(3.0)  # lattice speed of sound


def momentum_scale(ref, lattice):
    """Scale of the total first moment: sum over sites and components of |j|
    plus the total mass times the sound speed (the size of the first moments
    a velocity of order c_s would carry), from the oracle's populations."""
    from oracle.oracle import lattice_tables

    _, D, v, _ = lattice_tables(lattice)
    j = np.einsum("nqs,qa->nas", ref["f"], v[:, :D].astype(float))
    return float(np.abs(j).sum()) + float(ref["rho"].sum()) * CS


def errors(gpu, ref, theta=1.0 / 3.0, lattice=None):
    """Max relative errors.
    rho: per site, |d rho^s| / rho^s.   f: relative to the largest population.
    U: relative to max|U_ref| + 1e-3 c_s (the floor keeps a state at rest
       from dividing by 0).  U is a difference of populations of size
       O(rho c_s) that cancel to |U| << c_s, so after time stepping in FP32
       the state's rounding (about 1e-7 of rho) is 1e-4 of U: this
       normalisation is the bar for same-state comparisons
       (oracle_observe_of), where both sides start from the same populations.
    U_cs: |dU| relative to the lattice sound speed c_s, the bar after time
       stepping (the populations' own rounding scale).
    mu: relative to its largest magnitude.
    P: relative to max|P| + theta * max(rho) / 100 (its bulk part vanishes
       identically and is a difference of O(theta rho) terms).
    mom: total first moment (FP64 sums on both sides), relative to
       momentum_scale (needs the oracle's populations and the lattice)."""
    e = {"rho": float(np.max(np.abs(gpu["rho"] - ref["rho"]) / np.abs(ref["rho"])))}
    dU = float(np.abs(gpu["U"] - ref["U"]).max())
    e["U"] = dU / (float(np.abs(ref["U"]).max()) + 1e-3 * CS)
    e["U_cs"] = dU / CS
    e["mu"] = float(np.abs(gpu["mu"] - ref["mu"]).max() / float(np.abs(ref["mu"]).max()))
    pscale = float(np.abs(ref["P"]).max()) + theta * float(ref["rho"].sum(0).max()) / 100
    e["P"] = float(np.abs(gpu["P"] - ref["P"]).max() / pscale)
    if gpu.get("f") is not None:
        e["f"] = float(np.abs(gpu["f"] - ref["f"]).max() / np.abs(ref["f"]).max())
    e["mass"] = float(np.max(np.abs(gpu["mass"] - ref["mass"]) / np.abs(ref["mass"])))
    if lattice is not None and ref.get("f") is not None:
        e["mom"] = float(np.abs(gpu["mom"] - ref["mom"]).max()) / momentum_scale(ref, lattice)
    return e

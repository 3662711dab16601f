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
    with nx a multiple of 64, ny a multiple of 4 and N <= 3 (periodic boxes
    only)."""
    paths = ["split"]
    if cfg.get("walls", 0):
        return paths
    if cfg["lattice"] == "D2Q9":
        paths.append("tile")
        if storage in ("f32", "f16s") and cfg["shape"][0] % 64 == 0 and cfg["n_comp"] <= 4:
            paths.append("sweep")
    if cfg["lattice"] == "D3Q19" and storage == "f32" and cfg["shape"][0] % 64 == 0 \
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


# ---------------------------------------------------------------------------
# Rounding budget of shifted FP16 storage.
#
# The codec stores each moving population f*_i sent by a site as the FP16
# deviation d = f*_i / s - k_i h from the equilibrium at the site's own
# reference h = fl16(rho / (36 s)) (k_i = 36 w_i), and its rest slot absorbs
# every rounding (mass exact).  One stored value is off by at most
# u |f*_i - k_i h s| + 2^-25 s (u = 2^-11 the unit roundoff of FP16; the
# second term for deviations in FP16's subnormal range), and
# |k_i h s - w_i rho| <= u w_i rho.  So each step moves at most
#     e(r) = sum_{i>0} [u (|f_i(r) - w_i rho(r - v_i)| + u w_i rho(r - v_i)) + 2^-25 s]
# of density into site r (f_i(r) the population arriving at r, rho at its
# source before the collision; across a wall the source is r itself), that
# is e(r) / rho(r) relative to the site's own density, and changes the total
# first moment along axis a by at most the sum over sites of sum_i |v_ia| of
# the same terms.  Without amplification by the dynamics, the relative
# density errors of the stored state after K steps are then bounded by the
# sum over the K + 1 encodings (the initial state's included) of the
# per-step maxima over sites of e / rho (per component), and the momentum
# error by the sum of the per-step totals, along the oracle's trajectory.

U16 = 2.0 ** -11


def f16s_scale(rho0):
    """s^sigma of the shifted FP16 storage: twice the smallest power of two
    not below max rho0^sigma."""
    return 2.0 ** (np.ceil(np.log2(rho0.max(axis=1))) + 1.0)


def _source_sites(cfg, vi):
    """Index of the site whose slot is pulled into each site along v_i:
    r - v_i (periodic), or r itself where a wall lies between (bounce-back)."""
    dims = list(cfg["shape"]) + [1] * (3 - len(cfg["shape"]))
    walls = int(cfg.get("walls", 0))
    z, y, x = np.meshgrid(*(np.arange(n) for n in dims[::-1]), indexing="ij")
    src = []
    beyond = np.zeros(x.shape, bool)
    for a, c in enumerate((x, y, z)):
        sc = c - int(vi[a])
        if walls >> a & 1:
            beyond |= (sc < 0) | (sc >= dims[a])
        src.append(sc % dims[a])
    own = x + dims[0] * (y + dims[1] * z)
    pulled = src[0] + dims[0] * (src[1] + dims[1] * src[2])
    return np.where(beyond, own, pulled).reshape(-1)


def run_oracle_f16s_budget(cfg, rho0, steps, focus=None, scale=None):
    """The oracle's run (as run_oracle) and the FP16 rounding budget along it:
    {"rel": [N] bound on |d rho^s| / rho^s per site and component, "mom": [D]
    absolute bound on the total first moment per axis, "scale": s^sigma}.
    focus = (x, y): the density bound of that site alone, whose state after
    `steps` steps depends only on sites within 3 (steps - t) + 1 of it at
    step t (a periodic window's wrapped rim stays outside).  scale: s^sigma
    of the run being bounded when rho0 is only a window of its input (s
    follows the whole input's maximum)."""
    from oracle.oracle import lattice_tables

    N = cfg["n_comp"]
    q, D, v, w = lattice_tables(cfg["lattice"])
    srcs = [_source_sites(cfg, v[i]) for i in range(q)]
    s = f16s_scale(rho0) if scale is None else np.asarray(scale, float)
    cone = None
    if focus is not None:
        dims = list(cfg["shape"]) + [1] * (3 - len(cfg["shape"]))
        z, y, x = np.meshgrid(*(np.arange(n) for n in dims[::-1]), indexing="ij")
        dist = np.maximum(np.abs(x - focus[0]), np.abs(y - focus[1])).reshape(-1)
        cone = lambda t: dist <= 3 * (steps - t) + 1
    o = Oracle(OracleParams(**cfg), rho0)
    f = o.get_f()
    rho_prev = rho0
    b_rel = np.zeros(N)
    b_mom = np.zeros(D)
    for t in range(steps + 1):
        if t > 0:
            rho_prev = f.sum(axis=1)
            o.step(1)
            f = o.get_f()
        inj = np.zeros_like(rho_prev)
        for i in range(1, q):
            src = rho_prev[:, srcs[i]]
            dev = np.abs(f[:, i] - w[i] * src) + U16 * w[i] * src
            err = U16 * dev + 2.0 ** -25 * s[:, None]
            inj += err
            tot = float(err.sum())
            for a in range(D):
                b_mom[a] += abs(int(v[i][a])) * tot
        rel = inj / np.abs(f.sum(axis=1))
        b_rel += (rel if cone is None else rel[:, cone(t)]).max(axis=1)
    out = o.observe()
    out["f"] = o.get_f()
    return out, {"rel": b_rel, "mom": b_mom, "scale": s}


def f16s_check(gpu, ref, budget, cfg, rho0, arith=1e-5):
    """Ratios of the shifted FP16 path's errors to their bars (each must stay
    below 1): the rounding budget plus the FP32 arithmetic's own relative
    error `arith` (the FP32 path's bar).  rho: |d rho^s| / rho^s per site;
    f: |d f_i^s| / rho^s per site (a population's error is part of its
    site's); mu: the density bound propagated to first order through Eq.
    (lgf) per mer minus kappa lap rho, |d mu^s| <= theta / m^s B_s
    + sum_t |chi^st| B_t rho^t_max + 12 kappa B_s rho^s_max; the total first
    moment per axis; mass: exact but for the initial rounding of rho0 onto
    the 2^-24 s grid (2^-25 s per site)."""
    b = budget["rel"] + arith
    N = cfg["n_comp"]
    rr = np.abs(ref["rho"])
    r = {}
    r["rho"] = float(np.max((np.abs(gpu["rho"] - ref["rho"]) / rr).max(axis=1) / b))
    df = (np.abs(gpu["f"] - ref["f"]) / rr[:, None, :]).max(axis=(1, 2))
    r["f"] = float(np.max(df / b))
    chi = np.abs(np.asarray(cfg["chi"], float)[:N, :N])
    m = np.asarray(cfg.get("m", [1.0] * N), float)[:N]
    rmax = rr.max(axis=1)
    mu_bar = cfg["theta"] / m * b + chi @ (b * rmax) + 12.0 * cfg["kappa"] * b * rmax
    mu_bar = mu_bar + arith * float(np.abs(ref["mu"]).max())
    r["mu"] = float(np.max(np.abs(gpu["mu"] - ref["mu"]).max(axis=1) / mu_bar))
    mscale = momentum_scale(ref, cfg["lattice"])
    D = len(budget["mom"])
    dmom = np.abs(np.asarray(gpu["mom"])[:D] - np.asarray(ref["mom"])[:D])
    r["mom"] = float(np.max(dmom / (budget["mom"] + arith * mscale)))
    S = rho0.shape[1]
    mass_bar = 2.0 ** -25 * budget["scale"] * S / rho0.sum(axis=1) + 1e-13
    r["mass"] = float(np.max(np.abs(gpu["mass"] - ref["mass"]) / np.abs(ref["mass"]) / mass_bar))
    return r

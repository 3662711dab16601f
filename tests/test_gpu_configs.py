"""The workload configurations at their full sizes and lengths, beyond the
benchmark (which tests/test_gpu_fullsize.py covers): each against the FP64
oracle where the oracle can compute the outputs, else by properties that hold
at any size (conservation, agreement of precisions, permutation symmetry).

* binary spinodal 64^2, FP64, the full 2000 steps, every path vs the oracle;
* binary spinodal 1024^2, FP32 vs FP64 over 20000 steps: mass, domain-size
  growth and the concentrations of the domain cores;
* the binary coexistence concentrations at equilibrium, on a flat
  interface (a slab), GPU vs the oracle over the same 20000 steps;
* ternary D3Q19 256^3: sampled sites vs the oracle, mass conservation, and
  the same box between walls on z (sweep vs split);
* the film cast on a substrate (walls on y), D2Q9 2048^2: sampled sites vs
  the oracle;
* five components, D2Q9 512^2: permutation symmetry and sampled sites vs
  the oracle.

Sampled sites: after K steps the state at a site depends on the initial
densities within 3K sites, so the oracle run on a periodic window of
half-width 3K + 4 around a site reproduces that site exactly."""
import numpy as np
import pytest

import lbinputs as LI
from gpu_helpers import TOL, errors, paths_for, run_gpu, run_oracle
from oracle import Oracle, OracleParams

pytestmark = pytest.mark.gpu


def window_oracle(cfg, rho0, site, steps):
    """Oracle rho, mu and U at one site (x, y[, z]) after `steps`, from a
    window of half-width 3 steps + 4 around it: periodic along open axes;
    along an axis closed by walls the window is cut at the box's walls and
    closed by walls where it ends inside the box, at least the half-width
    from the site, which that wall (like a periodic window's wrap) cannot
    reach within the steps."""
    R = 3 * steps + 4
    shape = cfg["shape"]
    walls = int(cfg.get("walls", 0))
    n = cfg["n_comp"]
    idx, centre = [], []
    for a, (c, s) in enumerate(zip(site, shape)):
        if walls >> a & 1:
            lo, hi = max(0, c - R), min(s, c + R + 1)
            idx.append(np.arange(lo, hi))
            centre.append(c - lo)
        else:
            idx.append(np.arange(c - R, c + R + 1) % s)
            centre.append(R)
    g = rho0.reshape((n,) + tuple(reversed(shape)))  # [n][z][y][x] or [n][y][x]
    if len(shape) == 2:
        g = g[:, idx[1]][:, :, idx[0]]
    else:
        g = g[:, idx[2]][:, :, idx[1]][:, :, :, idx[0]]
    wshape = tuple(len(i) for i in idx)
    o = Oracle(OracleParams(**dict(cfg, shape=wshape)), np.ascontiguousarray(g.reshape(n, -1)))
    o.step(steps)
    ob = o.observe()
    c = site_index(centre, wshape)  # the site within the window
    return ob["rho"][:, c], ob["mu"][:, c], ob["U"][:, c]


def site_index(site, shape):
    s, stride = 0, 1
    for c, n in zip(site, shape):
        s += c * stride
        stride *= n
    return s


def check_sampled(cfg, rho0, out, sites, steps, tol):
    for site in sites:
        r, mu, U = window_oracle(cfg, rho0, site, steps)
        k = site_index(site, cfg["shape"])
        e_rho = float(np.max(np.abs(out["rho"][:, k] - r) / r))
        e_mu = float(np.max(np.abs(out["mu"][:, k] - mu)) / max(float(np.abs(out["mu"]).max()), 1e-30))
        e_U = float(np.max(np.abs(out["U"][:, k] - U))) * np.sqrt(3.0)
        assert max(e_rho, e_mu, e_U) < tol, (site, e_rho, e_mu, e_U)


def test_binary64_full_length_matches_oracle():
    """The small binary case over its full 2000 steps.  The spinodal
    instability amplifies the rounding differences between the GPU and the
    oracle from step to step (about 1e-14 relative after 200 steps, 1e-12
    after 2000 measured on MI355X), so the bars here are 1e-11 for FP64 and
    1e-3 for FP32 (1e-12 and 1e-5 hold at 200 steps, tests/test_gpu_parity.py)."""
    cfg, rho0 = LI.binary_spinodal(64)
    o = run_oracle(cfg, rho0, 2000)
    for storage, tol in (("f64", 1e-11), ("f32", 1e-3)):
        for path in paths_for(cfg, storage):
            g = run_gpu(cfg, rho0, 2000, storage=storage, path=path)
            e = errors(g, o, cfg["theta"])
            print(f"[configs] binary 64^2 2000 steps {storage} {path}: {e}", flush=True)
            for k in ("rho", "f", "U_cs", "mu"):
                assert e[k] < tol, (storage, path, k, e)
            assert e["mass"] < (1e-12 if storage == "f64" else 1e-6), (storage, path, e)


def domain_size(phi, n):
    """2 pi / <k> of the structure factor of phi (n x n, periodic)."""
    d = phi.reshape(n, n) - phi.mean()
    S = np.abs(np.fft.fft2(d)) ** 2
    k = 2 * np.pi * np.fft.fftfreq(n)
    km = np.sqrt(k[None, :] ** 2 + k[:, None] ** 2)
    S[0, 0] = 0.0
    return float(2 * np.pi * S.sum() / (km * S).sum())


def test_binary1024_spinodal_fp32_vs_fp64():
    """Spinodal decomposition of the binary mixture, 1024^2, 20000 steps, in
    FP32 (sweep kernel) and FP64 (tile kernel).  The two runs start from the
    same densities but their patterns decorrelate (the instability amplifies
    rounding), so they are compared by statistics: the domain size must grow
    and agree within 1%; the concentrations of the domain cores (1st and 99th
    percentiles of phi^A, with domains about 14 sites wide most sites sit in
    interfaces) within 2e-3, which allows for the curvature of the different
    patterns (the flat-interface test below holds the coexistence
    concentrations to 1e-3); mass within 1e-6 (FP32) and 1e-13 (FP64)."""
    from paper_0704_3444_amd import Simulation

    n = 1024
    cfg, rho0 = LI.binary_spinodal(n)
    m0 = rho0.sum(axis=1)
    marks = (1000, 2000, 5000, 10000, 20000)
    stats = {}
    for storage, path, mass_bar in (("f32", "sweep", 1e-6), ("f64", "tile", 1e-13)):
        sim = Simulation(cfg, rho0, storage=storage, path=path)
        done, L = 0, []
        for t in marks:
            sim.step(t - done)
            done = t
            out = sim.moments(fields=True)
            phi = out["rho"][0] / out["rho"].sum(axis=0)
            L.append(domain_size(phi, n))
            drift = float(np.max(np.abs(out["mass"] / m0 - 1)))
            assert drift < mass_bar, (storage, t, drift)
        sim.close()
        stats[storage] = (np.array(L), np.percentile(phi, 1), np.percentile(phi, 99))
        print(f"[configs] binary 1024^2 {storage}: domain size {np.round(L, 2).tolist()} at steps {list(marks)}, "
              f"core phi^A {stats[storage][1]:.5f} / {stats[storage][2]:.5f}", flush=True)
    L32, lo32, hi32 = stats["f32"]
    L64, lo64, hi64 = stats["f64"]
    assert np.all(np.diff(L32) > 0) and np.all(np.diff(L64) > 0)
    assert np.max(np.abs(L32 / L64 - 1)) < 1e-2
    assert abs(lo32 - lo64) < 2e-3 and abs(hi32 - hi64) < 2e-3


def slab(nx=256, ny=8, chi=2.4):
    """Binary D2Q9 slab: phi^A = 0.8 for x < nx/2, 0.2 elsewhere (periodic),
    total density 1, both faces smoothed over a few sites."""
    cfg = LI.params("D2Q9", 2, (nx, ny), kappa=0.01, chi=np.array([[0.0, chi], [chi, 0.0]]))
    prof = LI.film_profile(nx, 2.0)  # 1 on [0, nx/2), 0 on [nx/2, nx), tanh faces
    phi = 0.2 + 0.6 * prof
    phi2 = np.tile(phi, ny)
    return cfg, np.ascontiguousarray(np.stack([phi2, 1.0 - phi2]))


def test_slab_coexistence_matches_oracle():
    """Flat interfaces relax to the coexisting concentrations of the scheme;
    after 20000 steps the core concentrations of both phases agree with the
    oracle's run within 1e-3 (FP64 and FP32 alike; they agree to rounding),
    and the whole FP64 state still matches the oracle site by site within
    1e-10: the relaxation is stable, so the rounding differences between GPU
    and oracle only accumulate, about 1e-15 per step (1.1e-11 measured after
    20000 steps), instead of growing exponentially as in spinodal
    decomposition.  The scheme's coexistence concentrations differ from the
    binodal of Eq. (lgf) by about 1e-2 at this quench (documented finding,
    printed here, not asserted)."""
    from oracle import theory as T

    cfg, rho0 = slab()
    nx, ny = cfg["shape"]
    steps = 20000
    o = run_oracle(cfg, rho0, steps)
    phio = (o["rho"][0] / o["rho"].sum(axis=0)).reshape(ny, nx)
    core_o = (phio[:, nx // 4].mean(), phio[:, 3 * nx // 4].mean())
    for storage in ("f64", "f32"):
        g = run_gpu(cfg, rho0, steps, storage=storage, path="auto")
        phig = (g["rho"][0] / g["rho"].sum(axis=0)).reshape(ny, nx)
        core_g = (phig[:, nx // 4].mean(), phig[:, 3 * nx // 4].mean())
        e = errors(g, o, cfg["theta"])
        lo, hi = T.binary_binodal(1, 1, 2.4)
        print(f"[configs] slab {nx}x{ny} {steps} steps {storage} path={g['path']}: cores GPU "
              f"{core_g[0]:.6f} / {core_g[1]:.6f}, oracle {core_o[0]:.6f} / {core_o[1]:.6f}, "
              f"binodal {hi:.6f} / {lo:.6f}; errors {e}", flush=True)
        assert abs(core_g[0] - core_o[0]) < 1e-3 and abs(core_g[1] - core_o[1]) < 1e-3
        if storage == "f64":
            assert e["rho"] < 1e-10 and e["f"] < 1e-10, e


def test_ternary_d3q19_256_sampled_sites_and_mass():
    """Ternary D3Q19 at 256^3, FP32, on the path lb_step takes (the plane
    sweep): sampled sites after 2 steps against the oracle at the FP32 bar,
    every site bit for bit equal to the split path after 6 steps (the
    sweep's z-segments and pencil edges at the real launch configuration),
    and mass over 50 steps."""
    from paper_0704_3444_amd import Simulation

    cfg, rho0 = LI.ternary_d3q19(256)
    sim = Simulation(cfg, rho0, storage="f32", path="auto")
    assert sim.path == "sweep"
    sim.step(2)
    out = sim.moments(fields=True)
    sites = [(0, 0, 0), (255, 255, 255), (63, 64, 65), (128, 0, 255), (1, 254, 127), (200, 31, 7)]
    print(f"[configs] D3Q19 256^3 path={sim.path}: {len(sites)} sampled sites after 2 steps", flush=True)
    check_sampled(cfg, rho0, out, sites, 2, TOL["f32"])
    del out
    sim.step(4)
    ref = Simulation(cfg, rho0, storage="f32", path="split")
    ref.step(6)
    a = sim.moments(fields=True)
    b = ref.moments(fields=True)
    ref.close()
    print("[configs] D3Q19 256^3 sweep vs split after 6 steps", flush=True)
    assert np.array_equal(a["rho"], b["rho"]) and np.array_equal(a["U"], b["U"])
    del a, b
    sim.step(44)
    m = sim.moments(fields=False)["mass"]
    sim.close()
    drift = float(np.max(np.abs(m / rho0.sum(axis=1) - 1)))
    print(f"[configs] D3Q19 256^3 mass drift after 50 steps {drift:.2e}", flush=True)
    assert drift < 1e-6


def test_ternary_d3q19_256_walls_on_z():
    """The same box closed by walls on z: sampled sites after 4 steps
    against the oracle (windows cut at the walls), the plane sweep (auto) bit
    for bit equal to the split path after 6 steps at the real launch
    configuration (z-segments starting and ending at the walls), and mass
    kept over 50 steps."""
    from paper_0704_3444_amd import Simulation

    cfg, rho0 = LI.ternary_d3q19(256)
    cfg = dict(cfg, walls=0b100)
    sim = Simulation(cfg, rho0, storage="f32", path="auto")
    assert sim.path == "sweep"
    sim.step(4)
    out = sim.moments(fields=True)
    # next to both walls, one plane in, a segment's first planes and the middle
    sites = [(0, 0, 0), (255, 255, 255), (63, 64, 1), (128, 3, 254), (5, 200, 32), (200, 31, 128)]
    print(f"[configs] D3Q19 256^3 walls on z: {len(sites)} sampled sites after 4 steps", flush=True)
    check_sampled(cfg, rho0, out, sites, 4, TOL["f32"])
    del out
    sim.step(2)
    ref = Simulation(cfg, rho0, storage="f32", path="split")
    ref.step(6)
    a = sim.moments(fields=True)
    b = ref.moments(fields=True)
    ref.close()
    print("[configs] D3Q19 256^3 walls on z: sweep vs split after 6 steps", flush=True)
    assert np.array_equal(a["rho"], b["rho"]) and np.array_equal(a["U"], b["U"])
    del a, b
    sim.step(44)
    m = sim.moments(fields=False)
    sim.close()
    assert m["status"] == 0
    drift = float(np.max(np.abs(m["mass"] / rho0.sum(axis=1) - 1)))
    print(f"[configs] D3Q19 256^3 walls on z: mass drift after 50 steps {drift:.2e}", flush=True)
    assert drift < 1e-6


def test_film_on_substrate_2048_sampled_sites():
    """The film cast on a substrate at 2048^2 (walls on y, the FP32 strip
    sweep at its tuned launch configuration): sampled sites after 4 steps
    against the oracle (windows cut at the walls) next to both walls, at
    the film's free face and in the bulk."""
    from paper_0704_3444_amd import Simulation

    cfg, rho0 = LI.ternary_film_on_substrate(2048)
    sim = Simulation(cfg, rho0, storage="f32", path="auto")
    assert sim.path == "sweep"
    sim.step(4)
    out = sim.moments(fields=True)
    sim.close()
    sites = [(0, 0), (2047, 2047), (100, 1), (1500, 2046), (7, 1023), (64, 1024), (1023, 1025), (300, 500),
             (1777, 1600)]
    print(f"[configs] film on a substrate 2048^2: {len(sites)} sampled sites after 4 steps", flush=True)
    check_sampled(cfg, rho0, out, sites, 4, TOL["f32"])


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_five_components_512_permutation_and_sampled_sites(storage, tol):
    """N = 5 at 512^2 with a random symmetric interaction matrix: relabelling
    the components (densities, chi rows and columns) relabels the result,
    up to the rounding of sums taken in another order; sampled sites match
    the oracle."""
    cfg, rho0 = LI.five_component(512)
    steps = 100
    perm = np.array([3, 0, 4, 1, 2])
    cfg_p = dict(cfg, chi=np.asarray(cfg["chi"])[np.ix_(perm, perm)])
    for path in paths_for(cfg, storage):
        a = run_gpu(cfg, rho0, steps, storage=storage, path=path, fields=True)
        b = run_gpu(cfg_p, np.ascontiguousarray(rho0[perm]), steps, storage=storage, path=path, fields=True)
        e = float(np.max(np.abs(b["rho"] - a["rho"][perm]) / a["rho"][perm]))
        print(f"[configs] five components 512^2 {storage} {path}: permutation error {e:.2e}", flush=True)
        assert e < tol, (path, e)
    a = run_gpu(cfg, rho0, 2, storage=storage, path="auto", fields=True)
    check_sampled(cfg, rho0, a, [(0, 0), (511, 511), (100, 300), (256, 17)], 2, tol)

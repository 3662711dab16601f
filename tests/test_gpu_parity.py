"""GPU library vs the FP64 oracle, element by element, on seeded inputs.

Every case runs the HIP path through the C ABI (via the ctypes binding) and
the oracle from the same initial densities, then compares densities,
macroscopic velocity, chemical potentials, pressure tensor and all
populations site by site.  Bars: FP64 path 1e-12 relative, FP32 path 1e-5
relative (both against the FP64 oracle).

Shifted FP16 storage (f16s) rounds each stored deviation from the
equilibrium at the sending site's own density to 11 bits.  Its bars are the
rounding budget summed along the oracle's trajectory (f16s_check: 2^-11 of
each stored deviation per step, without amplification by the dynamics, plus
the FP32 arithmetic's own 1e-5) for densities, populations, chemical
potentials, the total first moment and the mass (exact but for the initial
rounding of rho0 onto the storage grid); the other observables are checked
on the GPU's own state, where they must agree to FP64 rounding.
"""
import numpy as np
import pytest

import lbinputs as LI
from gpu_helpers import (SAME_STATE_TOL, TOL, errors, f16s_check, f16s_scale, oracle_observe_of, paths_for, run_gpu,
                         run_oracle, run_oracle_f16s_budget)

pytestmark = pytest.mark.gpu


def _cases():
    cases = []
    p, r = LI.binary_spinodal(64)
    cases.append(("binary64_spinodal", p, r, 200))
    p, r = LI.binary_spinodal(64, chi=1.6)
    cases.append(("binary64_stable", p, r, 200))
    p, r = LI.ternary_immersion(96, ny=80)
    cases.append(("ternary_immersion_96x80", p, r, 200))
    p, r = LI.ternary_immersion(128, ny=77)
    cases.append(("ternary_immersion_128x77", p, r, 200))
    p, r = LI.binary_spinodal(130, lattice="D1Q3", chi=0.94, kappa=0.0)
    p["m"] = [10.0, 1.0]
    r = LI.sine_profile(p, [0.24, 0.76], amp=0.1)
    cases.append(("d1q3_polymer_130", p, r, 300))
    p, r = LI.ternary_d3q19(12, chi=3.0)
    p["shape"] = (12, 10, 9)
    r = LI.noisy_uniform(p, [1 / 3] * 3, 0.01, 1003)
    cases.append(("d3q19_ternary_12x10x9", p, r, 100))
    p, r = LI.five_component(40, chi_base=4.0)
    cases.append(("five_40", p, r, 100))
    # D3Q19 boxes the plane sweep takes (nx a multiple of 64, ny of 4)
    p, _ = LI.ternary_d3q19(12, chi=3.0)
    p["shape"] = (64, 12, 10)
    r = LI.noisy_uniform(p, [1 / 3] * 3, 0.01, 1013)
    cases.append(("d3q19_ternary_64x12x10", p, r, 200))
    p, _ = LI.binary_spinodal(8)
    p = dict(LI.params("D3Q19", 2, (128, 8, 6), kappa=0.01, chi=p["chi"]))
    r = LI.noisy_uniform(p, [0.5, 0.5], 0.01, 1014)
    cases.append(("d3q19_binary_128x8x6", p, r, 200))
    return cases


CASES = _cases()

@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("name,cfg,rho0,steps", CASES, ids=[c[0] for c in CASES])
def test_gpu_matches_oracle(name, cfg, rho0, steps, storage):
    """Every kernel path that supports the run against the oracle."""
    if storage == "f16s":
        o, budget = run_oracle_f16s_budget(cfg, rho0, steps)
    else:
        o = run_oracle(cfg, rho0, steps)
    for path in paths_for(cfg, storage):
        print(f"[parity] {name} storage={storage} path={path} steps={steps} shape={cfg['shape']}", flush=True)
        g = run_gpu(cfg, rho0, steps, storage=storage, path=path)
        assert g["path"] == path
        e = errors(g, o, cfg["theta"], lattice=cfg["lattice"])
        print(f"[parity] {name} {storage} {path} errors {e}", flush=True)
        if storage == "f16s":
            r = f16s_check(g, o, budget, cfg, rho0)
            print(f"[parity] {name} f16s {path} error / rounding bar {r} (relative density budget {budget['rel']})",
                  flush=True)
            for k, v in r.items():
                assert v < 1.0, (path, k, r)
        else:
            for k in ("rho", "f", "U_cs", "mu", "P", "mom"):
                assert e[k] < TOL[storage], (path, k, e)
        # the observables of the GPU's own final state, by the oracle's formulas
        es = errors(g, oracle_observe_of(cfg, rho0, g["f"]), cfg["theta"], lattice=cfg["lattice"])
        print(f"[parity] {name} {storage} {path} same-state observables {es}", flush=True)
        for k in ("rho", "U", "mu", "P", "mom", "mass"):
            assert es[k] < SAME_STATE_TOL, (path, "same-state", k, es)
        if storage != "f16s":
            assert e["mass"] < (1e-13 if storage == "f64" else 1e-6), (path, e)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
def test_fused_paths_equal_split(storage):
    """The fused kernels perform the split path's operations in the same
    order, so all paths agree bit for bit."""
    cfg, rho0 = LI.ternary_immersion(192, ny=70)
    a = run_gpu(cfg, rho0, 40, storage=storage, path="split")
    for path in paths_for(cfg, storage)[1:]:
        b = run_gpu(cfg, rho0, 40, storage=storage, path=path)
        d = np.abs(a["f"] - b["f"]).max() / np.abs(a["f"]).max()
        print(f"[fused-vs-split] {storage} {path} max rel diff {d:.3e}", flush=True)
        assert d == 0.0, (path, d)


D3Q19_SWEEP_BOXES = [((64, 4, 1), 3), ((64, 4, 3), 3), ((64, 8, 2), 2), ((128, 8, 5), 3), ((64, 12, 7), 1),
                     ((192, 4, 9), 2), ((64, 16, 33), 3)]


@pytest.mark.parametrize("storage", ["f32"])
@pytest.mark.parametrize("shape,n", D3Q19_SWEEP_BOXES, ids=[f"{s[0]}x{s[1]}x{s[2]}-N{n}" for s, n in D3Q19_SWEEP_BOXES])
def test_d3q19_sweep_equals_split(shape, n, storage):
    """The D3Q19 plane sweep against the split path, bit for bit, on boxes
    where the halo rows, halo columns and the ring of z-planes wrap onto the
    pencil itself (ny = 4, nx = 64, nz = 1 .. 3), a single z-plane, several
    pencils and segments, N = 1 .. 3."""
    chi = np.full((n, n), 1.5 if n > 1 else 0.0)
    np.fill_diagonal(chi, 0.0)
    p = LI.params("D3Q19", n, shape, kappa=0.02, chi=chi, m=[1.0 + (k == 1) for k in range(n)])
    r = LI.noisy_uniform(p, [1.0 / n] * n, 0.02 / n, 17 + n)
    a = run_gpu(p, r, 13, storage=storage, path="split")
    b = run_gpu(p, r, 13, storage=storage, path="sweep")
    assert b["path"] == "sweep"
    print(f"[d3q19-sweep] {shape} N={n} {storage}: max |df| {np.abs(a['f'] - b['f']).max():.3e}", flush=True)
    assert np.array_equal(a["f"], b["f"])


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_expanded_force_form_matches_oracle(storage):
    cfg, rho0 = LI.binary_spinodal(64)
    cfg["force_form"] = "expanded"
    o = run_oracle(cfg, rho0, 200)
    for path in paths_for(cfg, storage):
        g = run_gpu(cfg, rho0, 200, storage=storage, path=path)
        e = errors(g, o)
        tol = TOL[storage]
        assert e["rho"] < tol and e["f"] < tol and e["mu"] < tol, (path, e)


@pytest.mark.parametrize("shape", [(1, 1), (2, 3), (3, 1), (5, 2), (65, 17), (130, 33), (64, 1), (64, 3),
                                   (128, 5), (192, 77)])
def test_degenerate_and_ragged_boxes(shape):
    """Boxes smaller than the stencil (every neighbour wraps onto itself),
    boxes that leave partial tiles on both axes, and strips with ragged
    segments for the sweep kernel."""
    p, _ = LI.binary_spinodal(4)
    p["shape"] = shape
    S = shape[0] * shape[1]
    r = LI.noisy_uniform(p, [0.5, 0.5], 0.01, 7)
    o, budget = run_oracle_f16s_budget(p, r, 20)
    for storage in ("f64", "f32", "f16s"):
        for path in paths_for(p, storage):
            g = run_gpu(p, r, 20, storage=storage, path=path)
            if storage == "f16s":
                rr = f16s_check(g, o, budget, p, r)
                assert max(rr.values()) < 1.0, (shape, S, storage, path, rr)
                continue
            tol = TOL[storage]
            e = errors(g, o, lattice=p["lattice"])
            assert e["rho"] < tol and e["f"] < 2 * tol and e["mom"] < 10 * tol, (shape, S, storage, path, e)


@pytest.mark.parametrize("n", [1, 2, 4, 6, 8])
def test_component_counts(n):
    """N = 1 (pure fluid) up to the maximum N = 8, every path, both precisions."""
    p = LI.params("D2Q9", n, (128, 20), kappa=0.01, m=[1.0 + (k % 3 == 1) for k in range(n)])
    chi = np.full((n, n), 1.0)
    np.fill_diagonal(chi, 0.0)
    p["chi"] = chi
    r = LI.noisy_uniform(p, [1.0 / n] * n, 0.005 / n, 11)
    o, budget = run_oracle_f16s_budget(p, r, 50)
    for storage in ("f64", "f32", "f16s"):
        for path in paths_for(p, storage):
            g = run_gpu(p, r, 50, storage=storage, path=path)
            if storage == "f16s":
                rr = f16s_check(g, o, budget, p, r)
                print(f"[components] n={n} f16s {path} error / rounding bar {rr}", flush=True)
                assert max(rr.values()) < 1.0, (n, storage, path, rr)
                continue
            e = errors(g, o)
            tol = TOL[storage]
            print(f"[components] n={n} {storage} {path} {e}", flush=True)
            assert e["rho"] < tol and e["f"] < 2 * tol and e["mu"] < tol, (n, storage, path, e)


@pytest.mark.parametrize("path", ["split", "tile"])
def test_zero_steps_is_rest_equilibrium(path):
    cfg, rho0 = LI.ternary_immersion(40, ny=33)
    g = run_gpu(cfg, rho0, 0, path=path)
    assert g["step"] == 0
    assert np.abs(g["rho"] - rho0).max() < 1e-15
    assert np.abs(g["U"]).max() < 1  # forces exist at t = 0; U includes half of them
    _, _, _, w = __import__("paper_0704_3444_amd").lb_lattice_tables("D2Q9")
    assert np.abs(g["f"] - w[None, :, None] * rho0[:, None, :]).max() == 0.0


def test_f16s_accuracy_on_the_immersion_film():
    """The accuracy stated for shifted FP16 storage: on the phase-separated
    immersion film, where the non-solvent sits at 0.01 inside the film and at
    0.98 in the bath, every component density within 2e-3 (relative, per
    site) of the FP64 oracle after 200 steps, on every path."""
    cfg, rho0 = LI.ternary_immersion(128, ny=77)
    o = run_oracle(cfg, rho0, 200)
    for path in paths_for(cfg, "f16s"):
        g = run_gpu(cfg, rho0, 200, storage="f16s", path=path)
        e = float(np.max(np.abs(g["rho"] - o["rho"]) / o["rho"]))
        print(f"[f16s-film] {path}: max relative density error {e:.2e}", flush=True)
        assert e < 2e-3, (path, e)


def test_f16s_mass_exact_and_zero_steps():
    """Shifted FP16 storage keeps every component's mass exactly: the FP64
    sums of the stored values do not change over 2000 steps (up to the FP64
    rounding of the sum itself).  At t = 0 the stored densities equal rho0
    to 2^-25 s per site (the grid of the stored totals)."""
    from paper_0704_3444_amd import Simulation

    cfg, rho0 = LI.ternary_immersion(128, ny=64)
    for path in paths_for(cfg, "f16s"):
        s = Simulation(cfg, rho0, storage="f16s", path=path)
        m = s.moments()
        assert (np.abs(m["rho"] - rho0).max(axis=1) <= 2.0 ** -25 * f16s_scale(rho0) + 1e-16).all()
        m0 = m["mass"]
        s.step(2000)
        m1 = s.moments(fields=False)["mass"]
        s.close()
        drift = np.abs(m1 / m0 - 1).max()
        print(f"[f16s-mass] {path} drift over 2000 steps {drift:.3e}", flush=True)
        assert drift < 1e-14, (path, drift)


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
def test_mirror_symmetric_start_keeps_momentum_zero(lattice, storage):
    """A start that is mirror symmetric along every axis (rho0(r) = rho0(-r),
    periodic) stays so; the total first moment then vanishes on each axis
    (Sec. III first moments).  The GPU's FP64 sum must stay at rounding level
    relative to the total mass times c_s, on every path, while the oracle's
    does the same.  Each step's rounding is not mirror symmetric, so the
    bars follow from its random accumulation, about
    sqrt(steps S N Q) u max(f) / (M c_s) with u the storage's rounding unit
    (FP32: 2e-8 on the 64 x 48 binary box; shifted FP16: 2^-11 of the
    stored deviations, about 4e-7), with a 10x margin.  A kernel that breaks
    the mirror symmetry gives an O(1e-3) or larger value."""
    from gpu_helpers import CS

    if lattice == "D2Q9":
        p, _ = LI.binary_spinodal(64, chi=1.6)
        p["shape"] = (64, 48)
    else:
        p, _ = LI.ternary_d3q19(12, chi=2.0)
        p["shape"] = (12, 10, 8)
    dims = list(p["shape"]) + [1] * (3 - len(p["shape"]))
    r = LI.noisy_uniform(p, [1.0 / p["n_comp"]] * p["n_comp"], 0.01, 21)
    r = r.reshape(p["n_comp"], dims[2], dims[1], dims[0])
    for ax in (1, 2, 3):  # symmetrise: average with the mirror image x -> -x (mod n) along each axis
        r = 0.5 * (r + np.roll(np.flip(r, axis=ax), 1, axis=ax))
    r = np.ascontiguousarray(r.reshape(p["n_comp"], -1))
    steps = 200
    o = run_oracle(p, r, steps)
    scale = float(r.sum()) * CS
    bar = {"f64": 1e-13, "f32": 2e-7, "f16s": 4e-6}[storage]
    assert np.abs(o["mom"]).max() / scale < 1e-13
    for path in paths_for(p, storage):
        g = run_gpu(p, r, steps, storage=storage, path=path, fields=False)
        rel = np.abs(g["mom"]).max() / scale
        print(f"[mirror] {lattice} {storage} {path}: |Pi|/(M c_s) = {rel:.3e} (oracle "
              f"{np.abs(o['mom']).max() / scale:.3e})", flush=True)
        assert rel < bar, (path, g["mom"])

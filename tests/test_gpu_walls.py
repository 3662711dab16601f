"""Walls (not in the paper; lb_params.walls) on the split path and the D2Q9
tile kernel against the oracle's walls, every lattice and storage, the D2Q9
tile kernel and strip sweep (walls on y) and the D3Q19 plane sweep (walls on
z) against the split path bit for bit,
and the paths and groups that refuse them.  The oracle's walls are pinned by
tests/test_oracle_walls.py."""
import numpy as np
import pytest

import lbinputs as LI
from gpu_helpers import (SAME_STATE_TOL, TOL, errors, f16s_check, oracle_observe_of, run_gpu, run_oracle,
                         run_oracle_f16s_budget)

pytestmark = pytest.mark.gpu

CASES = [
    ("D1Q3", (70,), 0b001, 2),
    ("D2Q9", (40, 28), 0b010, 3),
    ("D2Q9", (37, 23), 0b011, 2),
    ("D3Q19", (12, 10, 9), 0b100, 3),
    ("D3Q19", (9, 8, 7), 0b111, 2),
]


def walled(lattice, shape, walls, n, seed):
    chi = np.full((n, n), 1.6) - 1.6 * np.eye(n)
    cfg = LI.params(lattice, n, shape, tau=0.9, kappa=0.03, chi=chi) | {"walls": walls}
    return cfg, LI.noisy_uniform(cfg, [1.0 / n] * n, 0.1 / n, seed)


# (case, path): the split path everywhere, the tile kernel on D2Q9
PATH_CASES = [(k, "split") for k in range(len(CASES))] + [(k, "tile") for k, c in enumerate(CASES) if c[0] == "D2Q9"]


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("case,path", PATH_CASES, ids=[f"{CASES[k][0]}-{k}-{pth}" for k, pth in PATH_CASES])
def test_walls_match_oracle(case, path, storage):
    lattice, shape, walls, n = CASES[case]
    cfg, rho0 = walled(lattice, shape, walls, n, 40 + case)
    g = run_gpu(cfg, rho0, 200, storage=storage, path=path)
    assert g["path"] == path
    o = run_oracle(cfg, rho0, 200)
    e = errors(g, o, cfg["theta"], lattice=lattice)
    print(f"[walls] {lattice} {shape} walls={walls:03b} {storage} {path}: {e}", flush=True)
    for k in ("rho", "f", "U_cs", "mu", "mom"):
        assert e[k] < TOL[storage], (k, e)
    assert e["mass"] < (1e-13 if storage == "f64" else 1e-6), e
    es = errors(g, oracle_observe_of(cfg, rho0, g["f"]), cfg["theta"], lattice=lattice)
    print(f"[walls] {lattice} {shape} walls={walls:03b} {storage} {path} same-state observables: {es}", flush=True)
    for k in ("rho", "U", "mu", "P", "mom", "mass"):
        assert es[k] < SAME_STATE_TOL, (k, es)


@pytest.mark.parametrize("case", [1, 2, 4])
def test_walls_shifted_fp16_match_oracle(case):
    """Shifted FP16 storage with walls: a bounced population is the sending
    site's own stored value, decoded with that site's reference, so the
    rounding budget is that of the periodic box with the bounce-back
    sources (f16s_check)."""
    lattice, shape, walls, n = CASES[case]
    cfg, rho0 = walled(lattice, shape, walls, n, 40 + case)
    g = run_gpu(cfg, rho0, 200, storage="f16s", path="auto")
    o, budget = run_oracle_f16s_budget(cfg, rho0, 200)
    r = f16s_check(g, o, budget, cfg, rho0)
    print(f"[walls] {lattice} {shape} walls={walls:03b} f16s error / rounding bar: {r}", flush=True)
    for k, v in r.items():
        assert v < 1.0, (k, r)


# D2Q9 boxes for the tile kernel with walls: several tiles with ragged
# edges, a box smaller than one tile, tile-multiple sides, each wall set
TILE_WALL_BOXES = [((150, 40), 0b11, 3), ((37, 23), 0b11, 2), ((64, 32), 0b10, 3), ((130, 70), 0b01, 2),
                   ((128, 48), 0b11, 1), ((2, 19), 0b01, 2), ((70, 30), 0b11, 5)]


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("shape,walls,n", TILE_WALL_BOXES,
                         ids=[f"{s[0]}x{s[1]}-w{w:02b}-N{n}" for s, w, n in TILE_WALL_BOXES])
def test_walls_tile_equals_split(shape, walls, n, storage):
    """The tile kernel with walls against the split path, bit for bit: the
    bounce-back pulls, the mirrored density ring and the potential one layer
    beyond a wall (taken from the layer next to it) give the split path's
    values in the same order."""
    cfg, rho0 = walled("D2Q9", shape, walls, n, 70 + n + walls)
    a = run_gpu(cfg, rho0, 37, storage=storage, path="split")
    b = run_gpu(cfg, rho0, 37, storage=storage, path="tile")
    print(f"[walls-tile] {shape} walls={walls:02b} N={n} {storage}: max |df| {np.abs(a['f'] - b['f']).max():.3e}",
          flush=True)
    assert np.array_equal(a["f"], b["f"])


# D2Q9 boxes for the strip sweep with walls on y: one strip and several,
# segments of four rows with a ragged last one, a box of two rows (both next
# to a wall; a segment of fewer than four rows), segments of two rounds,
# N = 1 .. 4
SWEEP_WALL_BOXES = [((128, 40), 3), ((64, 37), 2), ((192, 23), 4), ((64, 2), 1), ((128, 5), 3), ((64, 3101), 3)]


@pytest.mark.parametrize("storage", ["f32", "f16s"])
@pytest.mark.parametrize("shape,n", SWEEP_WALL_BOXES, ids=[f"{s[0]}x{s[1]}-N{n}" for s, n in SWEEP_WALL_BOXES])
def test_walls_sweep_equals_split(shape, n, storage):
    """The strip sweep with walls on y against the split path, bit for bit:
    the rows next to a wall stage their bounced group from their own
    opposite runs, and the density and potential stencils take the row next
    to the wall for the row beyond it; auto picks the sweep."""
    cfg, rho0 = walled("D2Q9", shape, 0b10, n, 90 + n)
    a = run_gpu(cfg, rho0, 37, storage=storage, path="split")
    b = run_gpu(cfg, rho0, 37, storage=storage, path="auto")
    assert b["path"] == "sweep"
    print(f"[walls-sweep] {shape} N={n} {storage}: max |df| {np.abs(a['f'] - b['f']).max():.3e}", flush=True)
    assert np.array_equal(a["f"], b["f"])


# D3Q19 boxes for the plane sweep with walls on z: two planes (both next to
# a wall), one pencil and several, segments of one plane and of four,
# N = 1 .. 3
D3Q19_SWEEP_WALL_BOXES = [((64, 4, 2), 3), ((64, 8, 5), 2), ((128, 8, 9), 3), ((64, 12, 7), 1), ((64, 16, 33), 3),
                          ((256, 48, 24), 3)]


@pytest.mark.parametrize("shape,n", D3Q19_SWEEP_WALL_BOXES,
                         ids=[f"{s[0]}x{s[1]}x{s[2]}-N{n}" for s, n in D3Q19_SWEEP_WALL_BOXES])
def test_walls_d3q19_sweep_equals_split(shape, n):
    """The D3Q19 plane sweep with walls on z against the split path, bit for
    bit: at a plane next to a wall the bounced directions are loaded from the
    site's own row and plane, run -v_i (own unit, halo-row unit and
    halo-column pieces alike), and the density and potential stencils take
    that plane for the one beyond the wall; auto picks the sweep."""
    cfg, rho0 = walled("D3Q19", shape, 0b100, n, 110 + n)
    a = run_gpu(cfg, rho0, 13, storage="f32", path="split")
    b = run_gpu(cfg, rho0, 13, storage="f32", path="auto")
    assert b["path"] == "sweep"
    print(f"[walls-sweep3d] {shape} N={n}: max |df| {np.abs(a['f'] - b['f']).max():.3e}", flush=True)
    assert np.array_equal(a["f"], b["f"])


def test_walls_keep_mass_in_shifted_fp16():
    cfg, rho0 = walled("D2Q9", (48, 32), 0b011, 3, 50)
    g = run_gpu(cfg, rho0, 500, storage="f16s", path="auto", fields=True)
    drift = float(np.max(np.abs(g["mass"] / rho0.sum(axis=1) - 1)))
    assert drift < 1e-6, drift


def test_walls_refused_where_not_built():
    from paper_0704_3444_amd import Batch, LBError, Lines, Simulation
    from paper_0704_3444_amd.lb import LB_EINVAL, LB_ENOTSUP

    cfg, rho0 = walled("D2Q9", (64, 32), 0b010, 2, 60)
    for walls in (0b001, 0b011):  # the sweep takes walls on y only
        with pytest.raises(LBError) as ei:
            Simulation(dict(cfg, walls=walls), rho0, storage="f32", path="sweep")
        assert ei.value.code == LB_ENOTSUP
    c3, r3 = walled("D3Q19", (64, 8, 6), 0b100, 2, 61)
    with pytest.raises(LBError) as ei:
        Simulation(c3, r3, storage="f32", path="tile")
    assert ei.value.code == LB_ENOTSUP
    for walls in (0b001, 0b010, 0b101):  # the D3Q19 sweep takes walls on z only
        with pytest.raises(LBError) as ei:
            Simulation(dict(c3, walls=walls), r3, storage="f32", path="sweep")
        assert ei.value.code == LB_ENOTSUP
    with pytest.raises(LBError) as ei:
        Simulation(dict(cfg, walls=0b100), rho0)  # D2Q9 has no z axis
    assert ei.value.code == LB_EINVAL
    b = Batch(storage="f32", max_comp=2, max_slots=2, arena_bytes=16 << 20)
    with pytest.raises(LBError) as ei:
        b.add(cfg, rho0, 10)
    assert ei.value.code == LB_ENOTSUP
    b.close()
    lc, lr, _ = LI.binodal_runs("binary_monomer")[0]
    s = Simulation(dict(lc, walls=1), lr)
    with pytest.raises(LBError) as ei:
        Lines([s])
    assert ei.value.code == LB_ENOTSUP
    s.close()


def test_immersion_film_on_a_wall():
    """The immersion geometry with a substrate: the ternary film of the
    benchmark workload (x < nx/2) against a wall at x = 0 and the bath
    closed by a wall at x = nx - 1.  Against the oracle after 100 steps
    (FP32 bar); healthy, with every component's mass kept, after 3000."""
    from paper_0704_3444_amd import Simulation

    cfg, rho0 = LI.ternary_immersion(128, ny=32)
    cfg = dict(cfg, walls=0b001)
    g = run_gpu(cfg, rho0, 100, storage="f32", path="auto")
    assert g["path"] == "tile"
    o = run_oracle(cfg, rho0, 100)
    e = errors(g, o, cfg["theta"])
    print(f"[walls] immersion film on a wall, 100 steps, f32: {e}", flush=True)
    for k in ("rho", "f", "U_cs", "mu"):
        assert e[k] < TOL["f32"], (k, e)
    sim = Simulation(cfg, rho0, storage="f32")
    sim.step(3000)
    m = sim.moments(fields=False)
    sim.close()
    assert m["status"] == 0
    assert float(np.max(np.abs(m["mass"] / rho0.sum(axis=1) - 1))) < 1e-6


def test_film_on_substrate_sweep():
    """The immersion film cast on a substrate (film normal along y, walls on
    y) runs on the strip sweep: against the oracle after 100 steps (FP32
    bar, and shifted FP16 within its rounding budget); healthy, with every
    component's mass kept, after 3000 steps."""
    from paper_0704_3444_amd import Simulation

    cfg, rho0 = LI.ternary_film_on_substrate(128, ny=64)
    g = run_gpu(cfg, rho0, 100, storage="f32", path="auto")
    assert g["path"] == "sweep"
    o, budget = run_oracle_f16s_budget(cfg, rho0, 100)
    e = errors(g, o, cfg["theta"], lattice="D2Q9")
    print(f"[walls] film on a substrate, 100 steps, f32 sweep: {e}", flush=True)
    for k in ("rho", "f", "U_cs", "mu", "mom"):
        assert e[k] < TOL["f32"], (k, e)
    h = run_gpu(cfg, rho0, 100, storage="f16s", path="auto")
    assert h["path"] == "sweep"
    r = f16s_check(h, o, budget, cfg, rho0)
    print(f"[walls] film on a substrate, 100 steps, f16s sweep error / rounding bar: {r}", flush=True)
    for k, v in r.items():
        assert v < 1.0, (k, r)
    for storage in ("f32", "f16s"):
        sim = Simulation(cfg, rho0, storage=storage)
        sim.step(3000)
        m = sim.moments(fields=False)
        sim.close()
        assert m["status"] == 0, storage
        assert float(np.max(np.abs(m["mass"] / rho0.sum(axis=1) - 1))) < 1e-6, storage


@pytest.mark.parametrize("case", ["d2q9-substrate", "d3q19-z"])
def test_walls_sweeps_long_runs(case):
    """Long runs on the sweeps with walls: the film on a substrate (512^2,
    20 000 steps, FP32 and shifted FP16) and a ternary D3Q19 box between
    walls on z (128 x 32 x 64, 3000 steps, FP32): healthy, every
    component's mass kept, and the FP32 state bit for bit the split path's."""
    from paper_0704_3444_amd import Simulation

    if case == "d2q9-substrate":
        cfg, rho0 = LI.ternary_film_on_substrate(512)
        steps, storages = 20000, ("f32", "f16s")
    else:
        cfg, _ = LI.ternary_d3q19(8)
        cfg = dict(cfg, shape=(128, 32, 64), walls=0b100)
        rho0 = LI.noisy_uniform(cfg, [0.3, 0.3, 0.4], 0.02, 1031)
        steps, storages = 3000, ("f32",)
    for storage in storages:
        sim = Simulation(cfg, rho0, storage=storage, path="auto")
        assert sim.path == "sweep"
        sim.step(steps)
        m = sim.moments(fields=storage == "f32")
        f = sim.get_f() if storage == "f32" else None
        sim.close()
        drift = float(np.max(np.abs(m["mass"] / rho0.sum(axis=1) - 1)))
        print(f"[walls-long] {case} {storage} {steps} steps: status {m['status']}, mass drift {drift:.2e}", flush=True)
        assert m["status"] == 0 and drift < 1e-6, (storage, m["status"], drift)
        if storage == "f32":
            ref = Simulation(cfg, rho0, storage="f32", path="split")
            ref.step(steps)
            g = ref.get_f()
            ref.close()
            assert np.array_equal(f, g)

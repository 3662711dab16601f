"""GPU runtime behaviour of the C ABI: determinism, checkpoint/resume,
translation equivariance across tile boundaries, conservation, and error
reporting (all numeric-failure cases produce NaN arithmetic only; no kernel
is made to fault)."""
import numpy as np
import pytest

import lbinputs as LI

pytestmark = pytest.mark.gpu

PATHS = ["split", "tile", "sweep"]


def storages(path):
    return {"sweep": ["f32", "f16s"], "tile": ["f64", "f32", "f16s"], "split": ["f64", "f32", "f16s"]}[path]


def sim(cfg, rho0, **kw):
    from paper_0704_3444_amd import Simulation

    return Simulation(cfg, rho0, **kw)


@pytest.mark.parametrize("path", PATHS)
def test_bitwise_deterministic(path):
    for storage in storages(path):
        cfg, rho0 = LI.ternary_immersion(128 if path == "sweep" else 70, ny=37)
        a = sim(cfg, rho0, storage=storage, path=path)
        b = sim(cfg, rho0, storage=storage, path=path)
        a.step(60)
        b.step(60)
        assert a.get_state() == b.get_state(), storage
        a.close()
        b.close()


@pytest.mark.parametrize("path", PATHS)
def test_checkpoint_resume_bitwise(path):
    """Resume from a checkpoint, also into a context created from other
    initial densities (the blob carries the shifted-storage reference)."""
    cfg, rho0 = LI.binary_spinodal(64 if path == "sweep" else 48)
    other = 0.9 * rho0[:, ::-1].copy()
    for storage in [s for s in storages(path) if s != "f64"]:
        a = sim(cfg, rho0, storage=storage, path=path)
        a.step(40)
        snap = a.get_state()
        a.step(40)
        ref = a.get_state()
        for start in (rho0, other):
            b = sim(cfg, start, storage=storage, path=path)
            b.set_state(snap)
            b.step(40)
            assert b.get_state() == ref, storage
            assert b.moments(fields=False)["step"] == 80
            b.close()
        a.close()


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
def test_translation_equivariance_bitwise(path, storage):
    """Shifting the initial state by (dx, dy) shifts the result exactly;
    shifts straddle the tiles, strips and segments of the fused kernels
    (a shift keeps the maximum of rho0, hence the f16s scale)."""
    if storage not in storages(path):
        pytest.skip(f"the {path} path does not take {storage} storage")
    nx, ny = (128 if path == "sweep" else 150), 77
    cfg, rho0 = LI.ternary_immersion(nx, ny=ny)
    g = rho0.reshape(3, ny, nx)
    for dx, dy in ((37, 11), (64, 16), (1, 76)):
        rolled = np.roll(g, (dy, dx), axis=(1, 2)).reshape(3, -1)
        a = sim(cfg, rho0, storage=storage, path=path)
        b = sim(cfg, rolled, storage=storage, path=path)
        a.step(25)
        b.step(25)
        fa = a.get_f().reshape(3, -1, ny, nx)
        fb = b.get_f().reshape(3, -1, ny, nx)
        assert np.array_equal(np.roll(fa, (dy, dx), axis=(2, 3)), fb), (dx, dy)
        a.close()
        b.close()


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("storage,bar", [("f64", 1e-13), ("f32", 1e-6), ("f16s", None)])
def test_mass_conserved_long_run(path, storage, bar):
    """Mass drift against rho0 after 3000 steps (f16s: exact after the
    initial rounding of rho0 into storage, at most 2^-25 s per site, so
    2^-25 s / mean(rho0) relative)."""
    from gpu_helpers import f16s_scale

    if storage not in storages(path):
        pytest.skip(f"the {path} path does not take {storage} storage")
    cfg, rho0 = LI.binary_spinodal(128, seed=77)
    if bar is None:
        bar = float(np.max(2.0 ** -25 * f16s_scale(rho0) / rho0.mean(axis=1))) + 1e-13
    s = sim(cfg, rho0, storage=storage, path=path)
    m0 = rho0.sum(axis=1)
    s.step(3000)
    m = s.moments(fields=False)["mass"]
    assert np.abs(m / m0 - 1).max() < bar, m / m0 - 1
    s.close()


def test_invalid_inputs_rejected():
    from paper_0704_3444_amd import LBError

    cfg, rho0 = LI.binary_spinodal(16)
    bad = rho0.copy()
    bad[1, 5] = 0.0
    with pytest.raises(LBError) as ei:
        sim(cfg, bad)
    assert ei.value.code == -1
    bad[1, 5] = np.nan
    with pytest.raises(LBError):
        sim(cfg, bad)
    with pytest.raises(LBError):
        sim(dict(cfg, chi=np.array([[0.0, 2.4], [2.3, 0.0]])), rho0)
    with pytest.raises(LBError):
        sim(dict(cfg, chi=np.array([[0.1, 2.4], [2.4, 0.0]])), rho0)
    with pytest.raises(LBError):
        sim(dict(cfg, tau=0.5), rho0)
    with pytest.raises(LBError):
        sim(dict(cfg, theta=0.0), rho0)


def test_workspace_too_small_rejected():
    import torch
    from paper_0704_3444_amd import lb

    cfg, rho0 = LI.binary_spinodal(16)
    p = lb.make_params(cfg, stream=torch.cuda.current_stream().cuda_stream)
    need = lb.lb_workspace_bytes(p)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    with pytest.raises(lb.LBError) as ei:
        lb.lb_init(p, rho0, ws.data_ptr(), need - 1024)
    assert ei.value.code == -2


@pytest.mark.parametrize("check_every", [0, 5])
def test_numeric_failure_reported(check_every):
    """A quench far beyond the scheme's stability (chi = 8 chi_c) drives a
    density negative; lb_moments reports LB_ENUMERIC."""
    from paper_0704_3444_amd import LBError

    cfg, rho0 = LI.binary_spinodal(32, chi=16.0)
    s = sim(cfg, rho0, check_every=check_every)
    s.step(300)
    with pytest.raises(LBError) as ei:
        s.moments(fields=False)
    assert ei.value.code == -5
    s.close()


def test_healthy_run_with_checks_reports_ok():
    cfg, rho0 = LI.binary_spinodal(32)
    s = sim(cfg, rho0, check_every=10)
    s.step(100)
    out = s.moments(fields=False)
    assert out["status"] == 0 and out["step"] == 100
    s.close()


def test_sweep_steps_captured_in_a_hip_graph():
    """lb_step enqueued under stream capture records only kernels; every
    replay of the graph must equal the same steps run eagerly (1024^2 sites:
    large enough for lb_init to choose a segment length)."""
    import torch

    cfg, rho0 = LI.ternary_immersion(1024)
    s = torch.cuda.Stream()
    g_sim = sim(cfg, rho0, storage="f32", path="sweep", stream=s)
    eager = sim(cfg, rho0, storage="f32", path="sweep")
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        g_sim.step(40)  # an even count: the graph leaves the state in the same copy
    for k in range(3):
        graph.replay()
        x = torch.ones(1000, device="cuda").cumsum(0)  # unrelated eager work between replays
        torch.cuda.synchronize()
        assert float(x[-1]) == 1000.0
        eager.step(40)
        a = g_sim.moments(fields=True)["rho"]
        b = eager.moments(fields=True)["rho"]
        print(f"[graph] replay {k}: {40 * (k + 1)} steps", flush=True)
        assert np.array_equal(a, b), k
    g_sim.close()
    eager.close()


# bytes per site of one component: (rest slot, moving slot, reference)
SLOT_BYTES = {"f64": (8, 8, 0), "f32": (4, 4, 0), "f16s": (4, 2, 2)}


def copy_bytes(cfg, storage):
    """Bytes of one population copy in the block layout (x padded to 64)."""
    shape = list(cfg["shape"]) + [1] * (3 - len(cfg["shape"]))
    Q = {"D1Q3": 3, "D2Q9": 9, "D3Q19": 19}[cfg["lattice"]]
    rest, move, ref = SLOT_BYTES[storage]
    return shape[1] * shape[2] * ((shape[0] + 63) // 64) * cfg["n_comp"] * 64 * (rest + ref + (Q - 1) * move)


def poison_copy(s, cfg, storage, which):
    """Fill population copy `which` of a Simulation's workspace with 0xFF
    bytes (NaN in FP64, FP32 and FP16)."""
    base = s.workspace.data_ptr()
    off = (base + 255) // 256 * 256 - base
    n = copy_bytes(cfg, storage)
    start = off + which * ((n + 255) // 256 * 256)
    s.workspace[start:start + n].fill_(255)


@pytest.mark.parametrize("case", ["d2q9", "ragged", "d3q19", "lines", "walls", "walls_y", "walls_z"])
def test_every_slot_written_each_step(case):
    """The copy a step writes is filled with NaN before the step; after three
    steps the state equals that of an unpoisoned run bit for bit, so every
    population slot is written by every step of every path (no slot left
    from an earlier step, none read before it is written)."""
    from paper_0704_3444_amd import Lines, Simulation

    if case == "d2q9":
        cfg, rho0 = LI.ternary_immersion(128, ny=64)
        combos = [(p, st) for p in PATHS for st in storages(p)]
    elif case == "ragged":
        cfg, rho0 = LI.ternary_immersion(100, ny=37)
        combos = [(p, st) for p in ("split", "tile") for st in storages(p)]
    elif case == "d3q19":
        cfg, rho0 = LI.ternary_d3q19(24)
        combos = [("split", st) for st in storages("split")]
    elif case == "walls":
        cfg, rho0 = LI.ternary_immersion(37, ny=23)
        cfg = dict(cfg, walls=0b011)
        combos = [(p, st) for p in ("split", "tile") for st in storages(p)]
    elif case == "walls_z":
        cfg, _ = LI.ternary_d3q19(8)
        cfg = dict(cfg, shape=(64, 8, 6), walls=0b100)
        rho0 = LI.noisy_uniform(cfg, [1 / 3] * 3, 0.01, 1021)
        combos = [("split", st) for st in storages("split")] + [("sweep", "f32")]
    elif case == "walls_y":
        cfg, rho0 = LI.ternary_immersion(128, ny=37)
        cfg = dict(cfg, walls=0b010)
        combos = [(p, st) for p in PATHS for st in storages(p)]
    else:
        cfg, rho0, _ = LI.binodal_runs("ternary_monomer")[9]
        combos = [("lines", "f64"), ("lines", "f32")]
    for path, storage in combos:
        kw = {"storage": storage} if path == "lines" else {"storage": storage, "path": path}
        ref, pois = Simulation(cfg, rho0, **kw), Simulation(cfg, rho0, **kw)
        group = Lines([pois]) if path == "lines" else None
        for k in range(3):
            poison_copy(pois, cfg, storage, 1 - k % 2)  # the copy this step writes
            ref.step(1)
            if group:
                group.step(1)
            else:
                pois.step(1)
        a, b = ref.get_f(), pois.get_f()
        assert np.all(np.isfinite(b)), (case, path, storage)
        assert np.array_equal(a, b), (case, path, storage)
        if group:
            group.close()
        ref.close()
        pois.close()

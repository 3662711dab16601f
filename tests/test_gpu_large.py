"""Runs at the 4 GiB boundary of one population copy (four components,
D2Q9, FP32).

The fused kernels address one copy with 32-bit byte offsets.  At 6144 x 5120
(4.53e9 bytes per copy) a run takes the split path, which computes 64-bit
offsets, and asking for the fused paths is refused; sampled sites whose
populations lie beyond the first 4 GiB of the copy (rows above 4854) are
compared with the oracle, and every component's mass is checked.  At
6144 x 4800 (4.247e9 bytes, just under 4 GiB) the fused paths take it, with
offsets that reach the end of the copy: sampled sites of the last rows
against the oracle, and the sweep and tile kernels bit for bit.

Sampled sites: after K steps a site depends on the initial densities within
3K sites, so the oracle run on a periodic window around it reproduces it."""
import numpy as np
import pytest

import lbinputs as LI
from oracle import Oracle, OracleParams

pytestmark = pytest.mark.gpu

NX, NY, N, K = 6144, 5120, 4, 2


def window_oracle(cfg, rho0, x, y, steps):
    nx, ny = cfg["shape"]
    R = 3 * steps + 4
    W = 2 * R + 1
    xs = np.arange(x - R, x + R + 1) % nx
    ys = np.arange(y - R, y + R + 1) % ny
    g = rho0.reshape(N, ny, nx)[:, ys][:, :, xs].reshape(N, -1)
    o = Oracle(OracleParams(**dict(cfg, shape=(W, W))), np.ascontiguousarray(g))
    o.step(steps)
    ob = o.observe()
    c = R * W + R
    return ob["rho"][:, c], ob["mu"][:, c], ob["U"][:, c]


def sampled_errors(cfg, rho0, out, sites):
    """Largest errors against the oracle over `sites`: rho relative, mu
    relative to the site's largest |mu|, U in units of the sound speed."""
    nx = cfg["shape"][0]
    cs = 1 / np.sqrt(3)
    worst = {"rho": 0.0, "mu": 0.0, "U": 0.0}
    for x, y in sites:
        r, mu, U = window_oracle(cfg, rho0, x, y, K)
        s = y * nx + x
        worst["rho"] = max(worst["rho"], float(np.max(np.abs(out["rho"][:, s] - r) / r)))
        worst["mu"] = max(worst["mu"], float(np.max(np.abs(out["mu"][:, s] - mu) / np.abs(mu).max())))
        worst["U"] = max(worst["U"], float(np.max(np.abs(out["U"][:, s] - U)) / cs))
    return worst


def test_copy_above_4gib_takes_split_path_and_matches_oracle():
    from paper_0704_3444_amd import LBError, Simulation
    from paper_0704_3444_amd.lb import LB_ENOTSUP

    chi = np.full((N, N), 1.4)
    np.fill_diagonal(chi, 0.0)
    cfg = LI.params("D2Q9", N, (NX, NY), tau=1.0, kappa=0.01, chi=chi)
    rho0 = LI.noisy_uniform(cfg, [0.25] * N, 0.01, 11)
    assert N * 9 * 4 * NX * NY > 2 ** 32
    for forced in ("sweep", "tile"):
        with pytest.raises(LBError) as ei:
            Simulation(cfg, rho0, storage="f32", path=forced)
        assert ei.value.code == LB_ENOTSUP
    sim = Simulation(cfg, rho0, storage="f32", path="auto")
    print(f"[large] D2Q9 {NX}x{NY} N={N} f32 path={sim.path}, {K} steps", flush=True)
    assert sim.path == "split"
    sim.step(K)
    out = sim.moments()
    sim.close()
    drift = float(np.max(np.abs(out["mass"] / rho0.sum(axis=1) - 1)))
    assert drift < 1e-6, drift
    worst = sampled_errors(cfg, rho0, out, [(0, 0), (NX - 1, NY - 1), (0, NY - 1), (NX - 1, 4855), (3071, 5000),
                                            (64, 4900), (5000, 5119)])
    print(f"[large] mass drift {drift:.1e}, worst errors {worst}", flush=True)
    for k, v in worst.items():
        assert v < 1e-5, (k, worst)


def test_copy_just_below_4gib_takes_fused_paths():
    """6144 x 4800, four components, FP32: 4.247e9 bytes per copy, just
    under 4 GiB, so the fused paths take it with 32-bit offsets that reach
    up to the end of the copy.  The sweep kernel (auto) against the oracle on
    sampled sites of the last rows; the tile kernel gives the same bits."""
    from paper_0704_3444_amd import Simulation

    ny = 4800
    chi = np.full((N, N), 1.4)
    np.fill_diagonal(chi, 0.0)
    cfg = LI.params("D2Q9", N, (NX, ny), tau=1.0, kappa=0.01, chi=chi)
    rho0 = LI.noisy_uniform(cfg, [0.25] * N, 0.01, 12)
    assert N * 9 * 4 * NX * ny < 2 ** 32
    outs = {}
    for path in ("auto", "tile"):
        sim = Simulation(cfg, rho0, storage="f32", path=path)
        print(f"[large] D2Q9 {NX}x{ny} N={N} f32 path={sim.path}, {K} steps", flush=True)
        assert sim.path == ("sweep" if path == "auto" else "tile")
        sim.step(K)
        outs[sim.path] = sim.moments()
        sim.close()
    assert np.array_equal(outs["sweep"]["rho"], outs["tile"]["rho"])
    assert np.array_equal(outs["sweep"]["U"], outs["tile"]["U"])
    out = outs["sweep"]
    worst = sampled_errors(cfg, rho0, out, [(NX - 1, ny - 1), (0, ny - 1), (6080, ny - 2), (63, ny - 1),
                                            (3000, ny - 3), (0, 0)])
    print(f"[large] below 4 GiB: worst errors {worst}", flush=True)
    for k, v in worst.items():
        assert v < 1e-5, (k, worst)

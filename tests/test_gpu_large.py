"""A run whose population copy exceeds 4 GiB (four components, D2Q9
6144 x 5120, FP32: 4.53e9 bytes per copy).

The fused kernels address one copy with 32-bit byte offsets, so such a run
takes the split path, which computes 64-bit offsets, and asking for the
fused paths is refused.  Sampled sites whose populations lie beyond the
first 4 GiB of the copy (rows above 4854) are compared with the oracle run
on a periodic window around each site (after K steps a site depends on the
initial densities within 3K sites), and every component's mass is checked
over the whole box."""
import numpy as np
import pytest

import lbinputs as LI
from oracle import Oracle, OracleParams

pytestmark = pytest.mark.gpu

NX, NY, N, K = 6144, 5120, 4, 2


def window_oracle(cfg, rho0, x, y, steps):
    R = 3 * steps + 4
    W = 2 * R + 1
    xs = np.arange(x - R, x + R + 1) % NX
    ys = np.arange(y - R, y + R + 1) % NY
    g = rho0.reshape(N, NY, NX)[:, ys][:, :, xs].reshape(N, -1)
    o = Oracle(OracleParams(**dict(cfg, shape=(W, W))), np.ascontiguousarray(g))
    o.step(steps)
    ob = o.observe()
    c = R * W + R
    return ob["rho"][:, c], ob["mu"][:, c], ob["U"][:, c]


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
    cs = 1 / np.sqrt(3)
    sites = [(0, 0), (NX - 1, NY - 1), (0, NY - 1), (NX - 1, 4855), (3071, 5000), (64, 4900), (5000, 5119)]
    worst = {"rho": 0.0, "mu": 0.0, "U": 0.0}
    for x, y in sites:
        r, mu, U = window_oracle(cfg, rho0, x, y, K)
        s = y * NX + x
        worst["rho"] = max(worst["rho"], float(np.max(np.abs(out["rho"][:, s] - r) / r)))
        worst["mu"] = max(worst["mu"], float(np.max(np.abs(out["mu"][:, s] - mu) / np.abs(mu).max())))
        worst["U"] = max(worst["U"], float(np.max(np.abs(out["U"][:, s] - U)) / cs))
    print(f"[large] mass drift {drift:.1e}, worst errors {worst}", flush=True)
    for k, v in worst.items():
        assert v < 1e-5, (k, worst)

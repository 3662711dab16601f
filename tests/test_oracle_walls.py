"""Walls in the oracle (not in the paper: its boxes are periodic).

A wall sits half a site beyond the first and last layer of a closed axis;
populations that would cross it bounce back to their site reversed, and the
stencils mirror the layer next to the wall.  Pins:

* mirror images: a closed box whose state is uniform along every open axis
  evolves like the periodic box of twice the length along the closed axis
  with mirrored contents (the walls then sit on its mirror planes, where a
  symmetric state reflects every population), for D1Q3, D2Q9 and D3Q19;
* every component's mass is kept to rounding in a closed box with
  arbitrary contents and walls on several axes;
* a uniform mixture at rest in a closed box stays uniform and at rest."""
import numpy as np
import pytest

import lbinputs as LI
from oracle import Oracle, OracleParams


def binary(lattice, shape, walls, chi=1.8, kappa=0.05, tau=0.9):
    return LI.params(lattice, 2, shape, tau=tau, kappa=kappa, chi=np.array([[0.0, chi], [chi, 0.0]]),
                     force_form="log") | {"walls": walls}


def run(cfg, rho0, steps):
    o = Oracle(OracleParams(**cfg), rho0)
    o.step(steps)
    return o.observe()


@pytest.mark.parametrize("lattice,shape,axis", [("D1Q3", (48,), 0), ("D2Q9", (6, 40), 1), ("D3Q19", (4, 5, 24), 2)])
def test_closed_box_is_half_of_a_mirrored_periodic_box(lattice, shape, axis):
    rng = np.random.default_rng(7)
    n = shape[axis]
    prof = np.stack([0.5 + 0.1 * rng.uniform(-1, 1, n), 0.5 + 0.1 * rng.uniform(-1, 1, n)])
    big = list(shape)
    big[axis] = 2 * n
    def fill(shp, prof_axis):
        idx = np.indices(tuple(reversed(shp)))[::-1][axis].reshape(-1)
        return np.ascontiguousarray(prof_axis[:, idx])
    closed = binary(lattice, shape, 1 << axis)
    periodic = binary(lattice, tuple(big), 0)
    mirrored = np.concatenate([prof, prof[:, ::-1]], axis=1)
    a = run(closed, fill(shape, prof), 300)
    b = run(periodic, fill(tuple(big), mirrored), 300)
    # the first n layers of the periodic box
    bidx = np.indices(tuple(reversed(big)))[::-1]
    keep = (bidx[axis].reshape(-1) < n)
    e = float(np.max(np.abs(a["rho"] - b["rho"][:, keep]) / b["rho"][:, keep]))
    moved = float(np.max(np.abs(a["rho"] - fill(shape, prof))))
    assert moved > 1e-3  # the state did evolve
    assert e < 1e-12, e


def test_mass_kept_in_a_closed_box():
    cfg = binary("D2Q9", (24, 20), 0b011, chi=2.4, kappa=0.02)
    rho0 = LI.noisy_uniform(cfg, [0.5, 0.5], 0.05, 31)
    o = Oracle(OracleParams(**cfg), rho0)
    o.step(400)
    m = o.observe()["rho"].sum(axis=1)
    assert np.max(np.abs(m / rho0.sum(axis=1) - 1)) < 1e-13
    cfg3 = LI.params("D3Q19", 3, (8, 7, 6), kappa=0.02,
                     chi=np.array([[0, 2.0, 1.0], [2.0, 0, 1.5], [1.0, 1.5, 0]])) | {"walls": 0b111}
    rho3 = LI.noisy_uniform(cfg3, [0.3, 0.3, 0.4], 0.05, 32)
    o3 = Oracle(OracleParams(**cfg3), rho3)
    o3.step(100)
    m3 = o3.observe()["rho"].sum(axis=1)
    assert np.max(np.abs(m3 / rho3.sum(axis=1) - 1)) < 1e-13


def test_uniform_mixture_at_rest_stays_at_rest():
    cfg = binary("D2Q9", (10, 12), 0b011, chi=2.4)
    rho0 = np.stack([np.full(120, 0.3), np.full(120, 0.7)])
    ob = run(cfg, rho0, 50)
    assert np.max(np.abs(ob["rho"] - rho0)) < 1e-15
    assert np.max(np.abs(ob["U"])) < 1e-15

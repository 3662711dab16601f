"""Pins of the oracle's time stepping against closed forms and invariants.

Linear theory (from Eq. (woche) with the Flory-Huggins potentials of Eq.
(lgf)): for a binary mixture at total density 1 and composition phi, a small
sine perturbation of phi^A with wave number k changes at the rate
    gamma = -w phi (1 - phi) k^2 [theta f''(phi) + 2 kappa k^2],
    f''(phi) = 1/(m_A phi) + 1/(m_B (1 - phi)) - 2 chi,   w = tau - 1/2.
With chi = 0 and m = 1 this is pure diffusion with D = w theta at any
amplitude.  A dropped 1/m, chi or kappa term, or a wrong sign in the force,
changes gamma at leading order.
"""
import numpy as np
import pytest

from oracle import Oracle, OracleParams
from oracle import theory as T
import lbinputs as LI


def binary(lattice, shape, *, tau=1.0, theta=1 / 3, kappa=0.0, m=(1, 1), chi=0.0, form="expanded"):
    return LI.params(lattice, 2, shape, tau=tau, theta=theta, kappa=kappa, m=m,
                     chi=np.array([[0.0, chi], [chi, 0.0]]), force_form=form)


def sine_amplitude(o, k, coord):
    ob = o.observe()
    phi = ob["rho"][0] / ob["rho"].sum(0)
    return 2 * np.mean(phi * np.sin(k * coord))


def measure_rate(p, phi0, eps, axis_coord, k, t0, t1):
    rho0 = np.vstack([phi0 + eps * np.sin(k * axis_coord), 1 - phi0 - eps * np.sin(k * axis_coord)])
    o = Oracle(OracleParams(**p), rho0)
    o.step(t0)
    a0 = sine_amplitude(o, k, axis_coord)
    o.step(t1 - t0)
    a1 = sine_amplitude(o, k, axis_coord)
    return np.log(a1 / a0) / (t1 - t0)


def predicted_rate(phi, k, tau, theta, kappa, m, chi):
    fpp = 1 / (m[0] * phi) + 1 / (m[1] * (1 - phi)) - 2 * chi
    k2_stencil = 2 * (1 - np.cos(k))          # symbol of the lattice Laplacian on an axis
    return -(tau - 0.5) * phi * (1 - phi) * k * k * (theta * fpp + 2 * kappa * k2_stencil)


@pytest.mark.parametrize("tau,theta,form", [(1.0, 1 / 3, "expanded"), (1 / 0.7, 1 / 3, "log"),
                                            (1 / 0.9, 0.1, "expanded"), (2.0, 0.5, "log")])
def test_diffusion_constant_large_amplitude(tau, theta, form):
    """chi = 0, m = 1: phi^A obeys d_t phi = w theta lap phi exactly at the
    order of the expansion, for the paper's amplitude 0.1 (Sec. IV)."""
    L = 256
    p = binary("D1Q3", (L,), tau=tau, theta=theta, form=form)
    x = np.arange(L)
    k = 2 * np.pi / L
    g = measure_rate(p, 0.5, 0.1, x, k, 2000, 8000)
    D = -g / k ** 2
    assert abs(D / ((tau - 0.5) * theta) - 1) < 1e-3


@pytest.mark.parametrize("m,chi,phi", [((1, 1), 1.5, 0.5), ((10, 1), 0.5, 0.3), ((10, 1), 1.0, 0.24),
                                       ((1, 10), 0.7, 0.6), ((1, 1), 2.4, 0.5), ((2, 1), 0.3, 0.15)])
def test_linear_rate_flory_huggins(m, chi, phi):
    """Decay below and growth above the spinodal at the rate of linear
    theory (tau = 0.8, theta = 1/3, kappa = 0)."""
    L, tau, theta = 256, 0.8, 1 / 3
    p = binary("D1Q3", (L,), tau=tau, theta=theta, m=m, chi=chi)
    x = np.arange(L)
    k = 2 * np.pi / L
    g = measure_rate(p, phi, 1e-6, x, k, 300, 3300)
    ref = predicted_rate(phi, k, tau, theta, 0.0, m, chi)
    # lattice corrections are O(k^2) of the diffusive (ideal-mixing) scale
    ideal = (tau - 0.5) * phi * (1 - phi) * k * k * theta * (1 / (m[0] * phi) + 1 / (m[1] * (1 - phi)))
    assert np.sign(g) == np.sign(ref)
    assert abs(g - ref) < 1.5e-3 * ideal, (g, ref)


def test_linear_rate_kappa_term_on_spinodal():
    """At the spinodal (f'' = 0) the bulk term vanishes.  What remains is the
    square-gradient term plus the scheme's own k^4 damping (the intrinsic
    surface tension from higher-order terms that Sec. IV mentions), which
    does not depend on kappa.  The change of rate between two kappa values
    is w phi(1-phi) k^2 2 (kappa_2 - kappa_1) k_s^2, and the intrinsic part is
    stabilising and scales as k^4."""
    tau, theta = 1.0, 1 / 3
    rates = {}
    for L in (32, 64):
        for kappa in (0.1, 0.3):
            p = binary("D1Q3", (L,), tau=tau, theta=theta, kappa=kappa, chi=2.0)
            k = 2 * np.pi / L
            rates[L, kappa] = measure_rate(p, 0.5, 1e-6, np.arange(L), k, 200, 4200)
    k = 2 * np.pi / 64
    d = rates[64, 0.3] - rates[64, 0.1]
    dref = predicted_rate(0.5, k, tau, theta, 0.3, (1, 1), 2.0) - predicted_rate(0.5, k, tau, theta, 0.1, (1, 1), 2.0)
    assert d < 0 and abs(d / dref - 1) < 1e-2, (d, dref)
    intrinsic = {L: rates[L, 0.1] - predicted_rate(0.5, 2 * np.pi / L, tau, theta, 0.1, (1, 1), 2.0) for L in (32, 64)}
    assert intrinsic[32] < 0 and intrinsic[64] < 0
    assert abs(intrinsic[32] / intrinsic[64] / 16 - 1) < 5e-2


def test_d2q9_isotropic_diffusion():
    """D2Q9: the same diffusion constant along an axis and along a diagonal."""
    L = 32
    p = binary("D2Q9", (L, L), tau=1.0, theta=1 / 3)
    s = np.arange(L * L)
    x, y = s % L, s // L
    k = 2 * np.pi / L
    g_axis = measure_rate(p, 0.5, 0.05, x, k, 100, 600)
    g_diag = measure_rate(p, 0.5, 0.05, x + y, k, 100, 600)
    D = 0.5 / 3
    assert abs(-g_axis / k ** 2 / D - 1) < 1e-2
    assert abs(-g_diag / (2 * k ** 2) / D - 1) < 2e-2


def test_d3q19_diffusion():
    L = 32
    s = np.arange(L * 16)
    z = s // 16
    p = LI.params("D3Q19", 2, (4, 4, L), tau=1.2, theta=1 / 3)
    k = 2 * np.pi / L
    g = measure_rate(p, 0.5, 0.05, z, k, 200, 1200)
    D = 0.7 / 3
    assert abs(-g / k ** 2 / D - 1) < 1e-2


@pytest.mark.parametrize("lattice,direction", [("D2Q9", "y"), ("D2Q9", "x+y"), ("D2Q9", "x-y"), ("D3Q19", "z"),
                                               ("D3Q19", "y+z")])
@pytest.mark.parametrize("form", ["log", "expanded"])
def test_diffusion_constant_off_axis_both_forms(lattice, direction, form):
    """D = w theta (Eq. (woche)) along y, z and diagonals, for both lines of
    Eq. (definef), at theta = 0.2.  At theta = 1/3 the ideal-mixing part of
    the log-form potential cancels (1/3) ln rho^s and the force vanishes for
    a binary at uniform total density, so the component gradients of the
    force would go untested; at theta = 0.2 the force carries
    -(1 - theta/c_s^2) of the lattice's own diffusion, and a force that
    misses its y or z component diffuses at w/3 instead of w theta."""
    L, tau, theta = 32, 1.0, 0.2
    shape = (L, L) if lattice == "D2Q9" else (4, L, L)
    S = int(np.prod(shape))
    s = np.arange(S)
    x, y = s % shape[0], (s // shape[0]) % shape[1]
    z = s // (shape[0] * shape[1]) if lattice == "D3Q19" else 0 * s
    coord = {"y": y, "z": z, "x+y": x + y, "x-y": x - y, "y+z": y + z}[direction]
    nk2 = 1 if direction in ("y", "z") else 2  # |wave vector|^2 / k^2
    p = binary(lattice, shape, tau=tau, theta=theta, form=form)
    k = 2 * np.pi / L
    g = measure_rate(p, 0.5, 0.05, coord, k, 100, 600)
    D = (tau - 0.5) * theta
    assert abs(-g / (nk2 * k ** 2) / D - 1) < 2e-2, (-g / (nk2 * k ** 2), D)


def spinodal_case(lattice="D2Q9", shape=(24, 20), n=2, seed=5):
    if n == 2:
        p = binary(lattice, shape, kappa=0.01, chi=2.4)
        S = int(np.prod(shape))
        rho0 = np.vstack([0.5 + 0.01 * (2 * LI.uniform(seed, c, S) - 1) for c in range(2)])
        return p, rho0
    # sub-critical multicomponent mixture with a polymer component: the noise
    # relaxes under non-trivial forces without forming sharp interfaces
    # (a pair of m = 1 and m = 2 components separates above chi = 1.457)
    chi = np.full((n, n), 1.2)
    np.fill_diagonal(chi, 0)
    p = LI.params(lattice, n, shape, kappa=0.01, chi=chi, m=[1.0 + (c == 1) for c in range(n)])
    return p, LI.noisy_uniform(p, [1 / n] * n, 0.01, seed)


@pytest.mark.parametrize("lattice,shape,n", [("D2Q9", (24, 20), 2), ("D2Q9", (16, 12), 3),
                                             ("D3Q19", (8, 6, 5), 3), ("D1Q3", (40,), 2)])
def test_mass_conserved_and_momentum_bookkeeping(lattice, shape, n):
    p, rho0 = spinodal_case(lattice, shape, n)
    o = Oracle(OracleParams(**p), rho0)
    m0 = rho0.sum(axis=1)
    for _ in range(5):
        ob = o.observe()
        o.step(1)
        ob1 = o.observe()
        dA = ob["A"].sum(axis=(0, 2))
        # round-off of summing O(1) populations over all sites, plus a bar
        # relative to the force itself
        bar = 1e-15 * ob["mass"].sum() + 1e-12 * np.abs(ob["A"]).sum()
        assert np.abs(ob1["mom"] - ob["mom"] - dA).max() < bar
        o.step(200)
    assert np.abs(o.observe()["mass"] / m0 - 1).max() < 1e-13


def test_scale_equivariance_bitwise():
    """rho0 -> 2^k rho0 with kappa -> kappa / 2^k scales the state by 2^k
    exactly (expanded force form): phi, u, u^sigma and mu are unchanged."""
    p, rho0 = spinodal_case("D2Q9", (12, 10), 3)
    p["force_form"] = "expanded"
    a = Oracle(OracleParams(**p), rho0)
    q = dict(p)
    q["kappa"] = p["kappa"] / 8
    b = Oracle(OracleParams(**q), rho0 * 8)
    a.step(30)
    b.step(30)
    assert np.array_equal(a.get_f() * 8, b.get_f())


@pytest.mark.parametrize("lattice,shape,shift", [("D2Q9", (12, 10), (5, 3)), ("D3Q19", (6, 5, 7), (2, 4, 3)),
                                                 ("D1Q3", (17,), (6,))])
def test_translation_equivariance_bitwise(lattice, shape, shift):
    p, rho0 = spinodal_case(lattice, shape, 3)
    n = p["n_comp"]
    grid = rho0.reshape((n,) + tuple(shape[::-1]))
    rolled = np.roll(grid, shift=tuple(shift[::-1]), axis=tuple(range(1, len(shape) + 1))).reshape(n, -1)
    a = Oracle(OracleParams(**p), rho0)
    b = Oracle(OracleParams(**p), rolled)
    a.step(20)
    b.step(20)
    ra = a.observe()["rho"].reshape(grid.shape)
    rb = b.observe()["rho"].reshape(grid.shape)
    assert np.array_equal(np.roll(ra, shift=tuple(shift[::-1]), axis=tuple(range(1, len(shape) + 1))), rb)


def test_permutation_of_components():
    p, rho0 = spinodal_case("D2Q9", (12, 10), 3)
    chi = np.array([[0, 2.0, 3.0], [2.0, 0, 2.5], [3.0, 2.5, 0]])
    p["chi"], p["m"] = chi, [1.0, 2.0, 1.0]
    perm = [2, 0, 1]
    q = dict(p)
    q["chi"] = chi[np.ix_(perm, perm)]
    q["m"] = [p["m"][i] for i in perm]
    a = Oracle(OracleParams(**p), rho0)
    b = Oracle(OracleParams(**q), rho0[perm])
    a.step(50)
    b.step(50)
    ra, rb = a.observe()["rho"], b.observe()["rho"]
    assert np.abs(ra[perm] - rb).max() < 1e-12


def test_mirror_symmetry():
    """x -> -x (mod L) of the initial state mirrors the evolution; a
    mirror-symmetric initial state keeps zero total x-momentum."""
    L, M = 14, 9
    p, rho0 = spinodal_case("D2Q9", (L, M), 2)
    g = rho0.reshape(2, M, L)
    mir = np.roll(g[:, :, ::-1], 1, axis=2)          # x -> (L - x) mod L
    a = Oracle(OracleParams(**p), rho0)
    b = Oracle(OracleParams(**p), mir.reshape(2, -1))
    a.step(40)
    b.step(40)
    ra = a.observe()["rho"].reshape(2, M, L)
    rb = b.observe()["rho"].reshape(2, M, L)
    assert np.abs(np.roll(ra[:, :, ::-1], 1, axis=2) - rb).max() < 1e-13
    sym = 0.5 * (g + mir)
    c = Oracle(OracleParams(**p), sym.reshape(2, -1))
    for _ in range(4):
        c.step(25)
        ob = c.observe()
        assert abs(ob["mom"][0]) < 1e-14 * ob["mass"].sum()

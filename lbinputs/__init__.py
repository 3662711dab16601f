"""Seeded synthetic inputs for the multicomponent LB workloads.

This module is the only code that the GPU-side tests/bench and the oracle
side both use.  It holds no arithmetic of the method: it only produces the
physical parameters of a run (lattice, box, tau, theta, m, chi, kappa) and
its initial component densities rho0[N][S] from a counter-based generator.

Random numbers: SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).  The uniform deviate for
(seed, component sigma, site s) is
    x = seed * 2^48 + sigma * 2^40 + s           (s < 2^40)
    z = mix64(x * 0x9E3779B97F4A7C15 + 0x9E3779B97F4A7C15)
    U = (z >> 11) * 2^-53                          in [0, 1)
with mix64 the SplitMix64 output function.

Noise recipe of every run: rho^sigma = base^sigma + amp * (2U - 1).

Parameter choices for the named workloads (theta = 1/3, m = 1, tau = 1,
interaction strengths as multiples of the mean-field critical value of the
Flory-Huggins free energy) are stated in each function.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform(seed: int, comp: int, n_sites: int, start: int = 0) -> np.ndarray:
    """U[0,1) deviates for sites start .. start+n_sites-1 of one component."""
    with np.errstate(over="ignore"):
        s = np.arange(start, start + n_sites, dtype=np.uint64)
        x = np.uint64(seed) * np.uint64(1 << 48) + np.uint64(comp) * np.uint64(1 << 40) + s
        z = _mix64(x * _GOLDEN + _GOLDEN)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def _chi(n: int, pairs: dict) -> np.ndarray:
    chi = np.zeros((n, n))
    for (a, b), v in pairs.items():
        chi[a, b] = chi[b, a] = v
    return chi


def params(lattice, n_comp, shape, *, tau=1.0, theta=1.0 / 3.0, kappa=0.0, m=None, chi=None,
           force_form="log") -> dict:
    return dict(lattice=lattice, n_comp=n_comp, shape=tuple(int(x) for x in shape), tau=float(tau),
                theta=float(theta), kappa=float(kappa),
                m=[1.0] * n_comp if m is None else [float(x) for x in m],
                chi=np.zeros((n_comp, n_comp)) if chi is None else np.asarray(chi, dtype=np.float64),
                force_form=force_form)


def noisy_uniform(p: dict, base, amp: float, seed: int, noisy=None) -> np.ndarray:
    """rho0[sigma] = base[sigma] + amp (2U - 1) on the components in `noisy`
    (all by default)."""
    n, S = p["n_comp"], int(np.prod(p["shape"]))
    rho = np.empty((n, S))
    for c in range(n):
        rho[c] = base[c]
        if noisy is None or c in noisy:
            rho[c] += amp * (2.0 * uniform(seed, c, S) - 1.0)
    return rho


# --------------------------------------------------------------------------
# Named workloads.
# --------------------------------------------------------------------------

def binary_spinodal(n=64, *, chi=2.4, kappa=0.01, seed=1000, lattice="D2Q9"):
    """Binary symmetric mixture quenched into the spinodal region.

    m = (1, 1): the mean-field critical interaction is chi_c = 2, so the
    default chi = 2.4 is 1.2 chi_c (chi = 1.6 is the linearly stable twin,
    0.8 chi_c).  rho^A, rho^B = 0.5 + 0.01 (2U - 1).  The 64^2 box is the
    small parity case, 1024^2 the spinodal-decomposition run."""
    shape = (n,) if lattice == "D1Q3" else (n, n)
    p = params(lattice, 2, shape, kappa=kappa, chi=_chi(2, {(0, 1): chi}))
    return p, noisy_uniform(p, [0.5, 0.5], 0.01, seed)


def ternary_immersion(n=2048, *, seed=1002, kappa=0.01, ny=None, width=2.0):
    """Immersion-precipitation-like ternary run (polymer P, solvent S,
    non-solvent NS), D2Q9, m = 1.

    Interactions 1.0, 1.25 and 1.5 times the binary critical value 2:
    chi^{P,S} = 2.0, chi^{S,NS} = 2.5, chi^{P,NS} = 3.0.  Left half (x < nx/2):
    rho = (0.30, 0.69, 0.01) with 0.01 (2U - 1) noise on P and S.  Right half:
    the non-solvent bath, floored at (0.01, 0.01, 0.98) because every
    component must stay strictly positive.  The two faces of the film (at
    x = nx/2 and x = 0, periodic) are smoothed as 1/2 (1 + tanh(d / width)) of
    the distance d in sites; a one-site jump drives the depleted components
    negative within a few steps."""
    ny = n if ny is None else ny
    p = params("D2Q9", 3, (n, ny), kappa=kappa,
               chi=_chi(3, {(0, 1): 2.0, (1, 2): 2.5, (0, 2): 3.0}))
    S = n * ny
    film = film_profile(n, width)[np.arange(S) % n]
    left = (0.30, 0.69, 0.01)
    right = (0.01, 0.01, 0.98)
    rho = np.empty((3, S))
    for c in range(3):
        rho[c] = film * left[c] + (1 - film) * right[c]
    for c in (0, 1):
        rho[c] += film * 0.01 * (2.0 * uniform(seed, c, S) - 1.0)
    return p, rho


def ternary_film_on_substrate(n=2048, *, seed=1003, kappa=0.01, ny=None, width=2.0):
    """The immersion film of ternary_immersion cast on a substrate: the
    film's normal along y, the substrate a wall below row 0 and the bath
    closed by a wall above row ny - 1 (walls = 0b10; x periodic).  Rows
    y < ny/2: (0.30, 0.69, 0.01) with 0.01 (2U - 1) noise on P and S; rows
    above: the bath (0.01, 0.01, 0.98).  Only the film's free face is smoothed
    (1/2 (1 + tanh(d / width)), d the distance to y = ny/2): the film meets
    the substrate as it is."""
    ny = n if ny is None else ny
    p = params("D2Q9", 3, (n, ny), kappa=kappa,
               chi=_chi(3, {(0, 1): 2.0, (1, 2): 2.5, (0, 2): 3.0})) | {"walls": 0b10}
    S = n * ny
    yc = np.arange(ny) + 0.5
    d = ny // 2 - yc
    prof = 0.5 * (1.0 + np.tanh(d / width)) if width > 0 else (d > 0).astype(float)
    film = prof[np.arange(S) // n]
    left = (0.30, 0.69, 0.01)
    right = (0.01, 0.01, 0.98)
    rho = np.empty((3, S))
    for c in range(3):
        rho[c] = film * left[c] + (1 - film) * right[c]
    for c in (0, 1):
        rho[c] += film * 0.01 * (2.0 * uniform(seed, c, S) - 1.0)
    return p, rho


def film_profile(n: int, width: float) -> np.ndarray:
    """Film fraction along x for a periodic box of length n: 1 on [0, n/2),
    0 on [n/2, n); with width > 0 both faces are smoothed as
    1/2 (1 + tanh(d / width)), d the signed distance of the cell centre to
    the nearest face (positive inside the film)."""
    xc = np.arange(n) + 0.5
    half = n // 2
    if width <= 0:
        return (xc < half).astype(float)
    inside = xc < half
    d = np.where(inside, np.minimum(xc, half - xc), -np.minimum(xc - half, n - xc))
    return 0.5 * (1.0 + np.tanh(d / width))


def ternary_d3q19(n=256, *, seed=1003, kappa=0.01, chi=3.15):
    """Ternary D3Q19 periodic cube at equal composition 1/3 + 0.01 (2U - 1);
    symmetric chi = 3.15 = 1.05 chi_c (chi_c = N = 3 at equal composition).
    Deeper quenches form binary-like interfaces at chi > 1.5 times the binary
    critical value 2, where the scheme is unstable at kappa = 0.01."""
    p = params("D3Q19", 3, (n, n, n), kappa=kappa,
               chi=_chi(3, {(0, 1): chi, (0, 2): chi, (1, 2): chi}))
    return p, noisy_uniform(p, [1 / 3] * 3, 0.01, seed)


def five_component(n=512, *, seed=1004, kappa=0.01, chi_base=4.0):
    """N = 5 D2Q9 box at equal composition 0.2 + 0.01 (2U - 1) with a random
    symmetric interaction matrix chi_ij = chi_base (1 + 0.1 (2U - 1)),
    chi_ii = 0.  At equal composition a uniform chi loses stability at
    chi = N = 5; the default chi_base = 4.0 (0.8 of that) keeps the mixture
    one phase, so the run exercises five coupled components without the
    strongly segregated interfaces on which the scheme is unstable."""
    u = uniform(seed + 1, 7, 25).reshape(5, 5)
    chi = np.zeros((5, 5))
    for a in range(5):
        for b in range(a + 1, 5):
            chi[a, b] = chi[b, a] = chi_base * (1.0 + 0.1 * (2.0 * u[a, b] - 1.0))
    p = params("D2Q9", 5, (n, n), kappa=kappa, chi=chi)
    return p, noisy_uniform(p, [0.2] * 5, 0.01, seed)


def sine_profile(p: dict, phi0, amp=0.1, rho_total=1.0, axis=0) -> np.ndarray:
    """Initial state of the paper's D1Q3 runs (Sec. IV): phi^A = phi0^A + dphi,
    phi^B = phi0^B - dphi, others constant, dphi = amp sin(2 pi x / L) with the
    wavelength equal to the box length L along `axis`."""
    shape = p["shape"]
    idx = np.indices(shape[::-1])[::-1]  # idx[a] has shape reversed; site = x + nx*y ...
    coord = idx[axis].reshape(-1) if len(shape) > 1 else np.arange(shape[0])
    L = shape[axis]
    dphi = amp * np.sin(2.0 * np.pi * coord / L)
    rho = np.empty((p["n_comp"], coord.size))
    for c in range(p["n_comp"]):
        rho[c] = phi0[c]
    rho[0] += dphi
    rho[1] -= dphi
    return rho * rho_total


def serving_mix(n_req=256, *, seed=1005, rate_hz=40.0, side=(64, 512), steps=5000,
                binary_chi=(2.2, 2.7), ternary_chi=(2.6, 2.9), solvent_chi=(0.3, 1.0), kappa=(0.005, 0.02),
                tau=(0.8, 1.0)):
    """Phase-separation requests arriving as a Poisson process: request k
    arrives at the sum of k + 1 exponential gaps of mean 1 / rate_hz
    seconds; N is 2 or 3 with equal odds; the box is square with side
    uniform in [side[0], side[1]]; tau, kappa and the interactions are
    uniform in the given ranges.
      binary:  rho0 = 1/2 + 0.01 (2U - 1) each, chi^{AB} 1.1 to 1.35 times
               the critical value 2;
      ternary: two demixing components and a compatible third,
               rho0 = (0.4, 0.4, 0.2) + 0.01 (2U - 1), chi^{AB} 1.04 to 1.16
               times 2.5 (where the A-B exchange mode of Eq. (lgf) loses
               stability at this composition), chi^{AC}, chi^{BC} in
               solvent_chi.
    Every pair stays below 1.5 times the binary critical value, beyond which
    the scheme's segregated interfaces are unstable.  Returns a list of
    dicts with keys arrival (s), cfg, rho0, nsteps, id."""
    u = uniform(seed, 99, 8 * n_req).reshape(n_req, 8)
    t = 0.0
    out = []
    for k in range(n_req):
        t += -np.log1p(-u[k, 0]) / rate_hz
        n = 2 if u[k, 1] < 0.5 else 3
        L = min(int(side[0] + np.floor(u[k, 2] * (side[1] - side[0] + 1))), side[1])
        ta = tau[0] + (tau[1] - tau[0]) * u[k, 3]
        ka = kappa[0] + (kappa[1] - kappa[0]) * u[k, 4]
        if n == 2:
            chi = _chi(2, {(0, 1): binary_chi[0] + (binary_chi[1] - binary_chi[0]) * u[k, 5]})
            base = [0.5, 0.5]
        else:
            v = uniform(seed + 1, k, 3)
            lo, hi = solvent_chi
            chi = _chi(3, {(0, 1): ternary_chi[0] + (ternary_chi[1] - ternary_chi[0]) * v[0],
                           (0, 2): lo + (hi - lo) * v[1], (1, 2): lo + (hi - lo) * v[2]})
            base = [0.4, 0.4, 0.2]
        p = params("D2Q9", n, (L, L), tau=ta, kappa=ka, chi=chi)
        rho0 = noisy_uniform(p, base, 0.01, seed + 10 + k)
        out.append({"arrival": t, "cfg": p, "rho0": rho0, "nsteps": int(steps), "id": k})
    return out


WORKLOADS = {
    "binary_d2q9_64": lambda: binary_spinodal(64),
    "binary_d2q9_64_stable": lambda: binary_spinodal(64, chi=1.6),
    "binary_d2q9_1024": lambda: binary_spinodal(1024, seed=1001),
    "ternary_d2q9_2048": lambda: ternary_immersion(2048),
    "ternary_substrate_d2q9_2048": lambda: ternary_film_on_substrate(2048),
    "ternary_d3q19_256": lambda: ternary_d3q19(256),
    "five_d2q9_512": lambda: five_component(512),
}


# --------------------------------------------------------------------------
# Phase-equilibrium experiments of Sec. IV: periodic D1Q3 lines.
# --------------------------------------------------------------------------

LINE_SITES = 128  # the paper does not give the line length; any L = 64 P works
# Plait points of the ternary systems of Fig. 3 (chi^AB = 3, chi^AC = 0.5,
# chi^BC = 0.2) for m = (1, 1, 1) and (10, 1, 1), rounded to 1e-4; computed
# with the Flory-Huggins theory tools of the test suite, which check them.
PLAIT_MONOMER = (0.3568, 0.3078, 0.3354)
PLAIT_POLYMER = (0.1659, 0.0752, 0.7589)


LINE_NOISE = 1e-6  # seeded noise on every line's start, see binodal_runs


def _line(n_comp, m, chi, inv_tau, phi0, L=LINE_SITES, theta=1.0 / 3.0, amp=0.1, seed=1010):
    p = params("D1Q3", n_comp, (L,), tau=1.0 / inv_tau, theta=theta, kappa=0.0, m=m, chi=chi)
    r = sine_profile(p, phi0, amp=amp)
    for c in range(n_comp):
        r[c] += LINE_NOISE * (2.0 * uniform(seed, c, L) - 1.0)
    return p, r


def binodal_runs(experiment: str, L: int = LINE_SITES, theta: float = 1.0 / 3.0):
    """Run sets of the binodal experiments of Sec. IV (Figs. 1 and 3): each
    entry is (cfg, rho0, label).  kappa = 0, total density 1 (the paper's
    100; with kappa = 0 the update is homogeneous of degree one in f),
    theta = 1/3 unless given (the paper does not state it), the sine
    perturbation of amplitude 0.1 over the line, plus seeded noise of
    amplitude 1e-6 on every component (seed 1010 + the run's index): on
    these lines modes of a few sites outgrow the sine, and without the noise
    they would grow from the rounding of the arithmetic, so that the domain
    pattern would depend on the order of operations of each implementation.

    binary_monomer   m = (1, 1), phi0 = (1/2, 1/2), 1/tau = 0.7 and 0.9,
                     chi^AB = 2.05 ... 3.50 (critical value 2)
    binary_polymer   m = (10, 1), phi0 = (0.24, 0.76), 1/tau = 0.9,
                     chi^AB = 0.88 ... 1.50 (critical value 0.866)
    ternary_monomer  m = (1, 1, 1), chi^AB = 3, chi^AC = 0.5, chi^BC = 0.2,
                     1/tau = 0.9, phi0 on the segment from the critical point
                     the paper quotes, (0.32, 0.32, 0.36), towards
                     (0.5, 0.5, 0): phi0 = c + s ((0.5, 0.5, 0) - c),
                     s = 0.05 ... 0.95
    ternary_polymer  m = (10, 1, 1), same chi, segment from (0.14, 0.11, 0.75)
    ternary_monomer_plait, ternary_polymer_plait
                     the same segments started from the plait points of
                     Eq. (lgf) for these chi (PLAIT_MONOMER, PLAIT_POLYMER;
                     the quoted critical points lie a few 1e-2 away), with a
                     perturbation of amplitude 0.05 (0.1 would make phi^B
                     negative next to the polymer plait point)
    """
    runs = []
    if experiment == "binary_monomer":
        for inv_tau in (0.7, 0.9):
            for chi in np.round(np.arange(2.05, 3.5001, 0.05), 2):
                p, r = _line(2, (1, 1), _chi(2, {(0, 1): chi}), inv_tau, (0.5, 0.5), L, theta,
                             seed=1010 + len(runs))
                runs.append((p, r, f"1/tau={inv_tau} chi={chi:.2f}"))
    elif experiment == "binary_polymer":
        for chi in np.round(np.arange(0.88, 1.5001, 0.02), 2):
            p, r = _line(2, (10, 1), _chi(2, {(0, 1): chi}), 0.9, (0.24, 0.76), L, theta, seed=1010 + len(runs))
            runs.append((p, r, f"chi={chi:.2f}"))
    elif experiment.startswith(("ternary_monomer", "ternary_polymer")):
        polymer = experiment.startswith("ternary_polymer")
        m = (10, 1, 1) if polymer else (1, 1, 1)
        if experiment.endswith("_plait"):
            crit = np.array(PLAIT_POLYMER if polymer else PLAIT_MONOMER)
            amp = 0.05
        else:
            crit = np.array((0.14, 0.11, 0.75) if polymer else (0.32, 0.32, 0.36))
            amp = 0.1
        end = np.array((0.5, 0.5, 0.0))
        chi = _chi(3, {(0, 1): 3.0, (0, 2): 0.5, (1, 2): 0.2})
        for s in np.round(np.arange(0.05, 0.9501, 0.05), 2):
            phi0 = crit + s * (end - crit)
            p, r = _line(3, m, chi, 0.9, phi0, L, theta, amp=amp, seed=1010 + len(runs))
            runs.append((p, r, f"s={s:.2f}"))
    else:
        raise ValueError(f"unknown experiment {experiment!r}")
    return runs


def profile_run(experiment: str, L: int = LINE_SITES):
    """The single runs behind the profile figures of Sec. IV: binary polymer
    m = (10, 1), chi^AB = 0.94 from phi0 = (0.24, 0.76) (Fig. 2); ternary
    polymer m = (10, 1, 1) with the chi of Fig. 3 from phi0 =
    (0.14, 0.11, 0.75) (Fig. 4); 1/tau = 0.9, kappa = 0."""
    if experiment == "binary_polymer_profile":
        return _line(2, (10, 1), _chi(2, {(0, 1): 0.94}), 0.9, (0.24, 0.76), L)
    if experiment == "ternary_polymer_profile":
        return _line(3, (10, 1, 1), _chi(3, {(0, 1): 3.0, (0, 2): 0.5, (1, 2): 0.2}), 0.9, (0.14, 0.11, 0.75), L)
    raise ValueError(f"unknown experiment {experiment!r}")

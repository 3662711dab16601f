"""Brute-force pin of one whole oracle step on tiny periodic lattices.

The reference here is built differently from the oracle at every point where
it can be:
  * f^e and F are obtained by SOLVING the moment conditions of Sec. III and
    Eqs. (ff1)-(ff3) as a linear system (D1Q3: three conditions, unique;
    D2Q9: the conditions up to third order plus the stated fourth moment
    sum f v_x^2 v_y^2), not from the closed polynomials;
  * mu^sigma is the complex-step derivative of the free energy Eq. (lgf)
    (per mer) plus -kappa times a literal neighbour-sum Laplacian;
  * the force is Eq. (definef) with literal neighbour-sum gradients;
  * collision and streaming follow Eq. (ssLB) on a dict keyed by coordinates.
Lattice velocities are written out here from the standard D1Q3/D2Q9 sets.
"""
import numpy as np
import pytest

from oracle import Oracle, OracleParams
from oracle import theory as T

VEL = {
    "D1Q3": [(0, 0), (1, 0), (-1, 0)],
    "D2Q9": [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)],
}
WGT = {
    "D1Q3": [2 / 3, 1 / 6, 1 / 6],
    "D2Q9": [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4,
}


def moment_rows(lat):
    v = np.array(VEL[lat], float)
    vx, vy = v[:, 0], v[:, 1]
    if lat == "D1Q3":
        return np.vstack([np.ones(3), vx, vx * vx])
    return np.vstack([np.ones(9), vx, vy, vx * vx, vx * vy, vy * vy, vx * vx * vy, vx * vy * vy,
                      vx * vx * vy * vy])


def feq_by_moments(lat, rho, u):
    ux, uy = u
    if lat == "D1Q3":
        rhs = [rho, rho * ux, rho / 3 + rho * ux * ux]
    else:
        rhs = [rho, rho * ux, rho * uy, rho / 3 + rho * ux * ux, rho * ux * uy, rho / 3 + rho * uy * uy,
               rho * uy / 3, rho * ux / 3, rho * (1 / 9 + (ux * ux + uy * uy) / 3)]
    return np.linalg.solve(moment_rows(lat), rhs)


def forcing_by_moments(lat, A, us):
    Ax, Ay = A
    ux, uy = us
    if lat == "D1Q3":
        rhs = [0.0, Ax, 2 * Ax * ux]
    else:
        rhs = [0.0, Ax, Ay, 2 * Ax * ux, Ax * uy + Ay * ux, 2 * Ay * uy, Ay / 3, Ax / 3,
               2 / 3 * (Ax * ux + Ay * uy)]
    return np.linalg.solve(moment_rows(lat), rhs)


def brute_step(lat, nx, ny, f, prm):
    """f: dict (x, y) -> array [N][Q] of post-streaming populations."""
    vel, wgt = VEL[lat], WGT[lat]
    N = prm["n_comp"]
    wrap = lambda x, y: (x % nx, y % ny)
    sites = list(f.keys())
    rho = {s: f[s].sum(axis=1) for s in sites}
    lap = {s: 6 * sum(wgt[i] * (rho[wrap(s[0] + vx, s[1] + vy)] - rho[s]) for i, (vx, vy) in enumerate(vel))
           for s in sites}
    mu = {s: T.mu_per_mer(rho[s], prm["m"], prm["chi"], prm["theta"]) - prm["kappa"] * lap[s] for s in sites}
    c = 1 - 1 / (2 * prm["tau"])

    def grad(field, s, k):
        g = np.zeros(2)
        for i, (vx, vy) in enumerate(vel):
            g += 3 * wgt[i] * np.array([vx, vy], float) * field[wrap(s[0] + vx, s[1] + vy)][k]
        return g

    new = {s: np.zeros_like(f[s]) for s in sites}
    for s in sites:
        v = np.array(vel, float)
        j = f[s] @ v                       # [N][2]
        u = j.sum(axis=0) / rho[s].sum()
        for k in range(N):
            A = -c * (rho[s][k] * grad(mu, s, k) - grad(rho, s, k) / 3)
            fe = feq_by_moments(lat, rho[s][k], u)
            F = forcing_by_moments(lat, A, j[k] / rho[s][k])
            post = f[s][k] + (fe - f[s][k]) / prm["tau"] + F
            for i, (vx, vy) in enumerate(vel):
                new[wrap(s[0] + vx, s[1] + vy)][k][i] = post[i]
    return new


CASES = [
    ("D1Q3", 5, 1, 2), ("D1Q3", 4, 1, 3), ("D2Q9", 4, 3, 2), ("D2Q9", 3, 5, 3),
]


@pytest.mark.parametrize("lat,nx,ny,N", CASES)
def test_one_and_five_steps_match_brute_force(lat, nx, ny, N):
    rng = np.random.default_rng(nx * 100 + ny * 10 + N)
    chi = rng.uniform(1.0, 3.0, (N, N))
    chi = 0.5 * (chi + chi.T)
    np.fill_diagonal(chi, 0)
    m = list(rng.choice([1.0, 10.0], N))
    prm = dict(n_comp=N, tau=rng.uniform(0.7, 1.6), theta=rng.uniform(0.2, 0.5), kappa=0.03,
               m=m, chi=chi)
    shape = (nx,) if lat == "D1Q3" else (nx, ny)
    rho0 = rng.uniform(0.2, 0.8, (N, nx * ny))
    o = Oracle(OracleParams(lattice=lat, shape=shape, **prm), rho0)
    Q = len(VEL[lat])
    # start from a non-equilibrium state so that every moment is exercised
    f0 = o.get_f() * rng.uniform(0.9, 1.1, (N, Q, nx * ny))
    o.set_f(f0)
    f = {(s % nx, s // nx): f0[:, :, s].copy() for s in range(nx * ny)}
    for nsteps in (1, 4):
        o.step(nsteps)
        for _ in range(nsteps):
            f = brute_step(lat, nx, ny, f, prm)
        got = o.get_f()
        ref = np.stack([f[(s % nx, s // nx)] for s in range(nx * ny)], axis=-1)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err < 1e-13, err

"""Brute-force pin of whole oracle steps on tiny periodic lattices, for both
lines of Eq. (definef) on D1Q3, D2Q9 and D3Q19.

The reference here is built differently from the oracle at every point where
it can be:
  * f^e and F are obtained by SOLVING the moment conditions of Sec. III and
    Eqs. (ff1)-(ff3) as a linear system (D1Q3: three conditions, unique;
    D2Q9 and D3Q19: the conditions up to third order plus the fourth moments
    sum f v_a^2 v_b^2 stated below), not from the closed polynomials;
  * mu^sigma is the complex-step derivative of the free energy Eq. (lgf)
    (per mer) plus -kappa times a literal neighbour-sum Laplacian;
  * the force is Eq. (definef), first line (log form)
        A = -c rho^s(r) grad[mu^s - (1/3) ln rho^s](r)
    or second line (expanded form)
        A = -c [rho^s(r) grad mu^s(r) - (1/3) grad rho^s(r)],
    with each gradient a literal sum over the neighbours r + v_i written per
    Cartesian axis;
  * collision and streaming follow Eq. (ssLB) on a dict keyed by coordinates.
Lattice velocities and weights are written out here from the standard
D1Q3/D2Q9/D3Q19 sets.

Fourth moments (free in the paper, fixed by the second-order polynomials the
method uses; derived by hand from those polynomials for the edge velocities
(+-1, +-1, 0) and their permutations, weight 1/36):
    sum_i f^e_i v_a^2 v_b^2 = rho [1/9 + (u_a^2 + u_b^2)/3 - u_c^2/6]
    sum_i F_i   v_a^2 v_b^2 = (2/3)(A_a us_a + A_b us_b) - A_c us_c / 3
with c the third axis (on D2Q9 u_c = A_c = 0).
"""
import itertools

import numpy as np
import pytest

from oracle import Oracle, OracleParams
from oracle import theory as T

VEL = {
    "D1Q3": [(0, 0, 0), (1, 0, 0), (-1, 0, 0)],
    "D2Q9": [(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0), (1, 1, 0), (-1, 1, 0), (-1, -1, 0),
             (1, -1, 0)],
    # rest, the six axis velocities, the twelve edge velocities
    "D3Q19": [(0, 0, 0)] + [v for v in itertools.product((-1, 0, 1), repeat=3) if sum(map(abs, v)) == 1]
             + [v for v in itertools.product((-1, 0, 1), repeat=3) if sum(map(abs, v)) == 2],
}
WGT = {
    "D1Q3": [2 / 3, 1 / 6, 1 / 6],
    "D2Q9": [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4,
    "D3Q19": [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12,
}
DIM = {"D1Q3": 1, "D2Q9": 2, "D3Q19": 3}
PAIRS = [(0, 1, 2), (0, 2, 1), (1, 2, 0)]  # (a, b, c) for the fourth moments v_a^2 v_b^2


def moment_rows(lat):
    """Rows of the moment conditions: 1, v_a, v_a v_b (a <= b), v_a^2 v_b
    (a != b), v_a^2 v_b^2 (a < b), restricted to the lattice's axes."""
    v = np.array(VEL[lat], float)
    D = DIM[lat]
    rows = [np.ones(len(v))]
    rows += [v[:, a] for a in range(D)]
    rows += [v[:, a] * v[:, b] for a in range(D) for b in range(a, D)]
    rows += [v[:, a] ** 2 * v[:, b] for a in range(D) for b in range(D) if a != b]
    rows += [v[:, a] ** 2 * v[:, b] ** 2 for (a, b, _) in PAIRS if a < D and b < D]
    M = np.vstack(rows)
    assert M.shape == (len(v), len(v)) and np.linalg.matrix_rank(M) == len(v)
    return M


def feq_by_moments(lat, rho, u):
    D = DIM[lat]
    rhs = [rho]
    rhs += [rho * u[a] for a in range(D)]
    rhs += [rho / 3 * (a == b) + rho * u[a] * u[b] for a in range(D) for b in range(a, D)]
    rhs += [rho * u[b] / 3 for a in range(D) for b in range(D) if a != b]  # (rho/3)(u_a d_ab + u_a d_ab + u_b d_aa)
    rhs += [rho * (1 / 9 + (u[a] ** 2 + u[b] ** 2) / 3 - u[c] ** 2 / 6) for (a, b, c) in PAIRS if a < D and b < D]
    return np.linalg.solve(moment_rows(lat), rhs)


def forcing_by_moments(lat, A, us):
    D = DIM[lat]
    rhs = [0.0]
    rhs += [A[a] for a in range(D)]
    rhs += [A[a] * us[b] + A[b] * us[a] for a in range(D) for b in range(a, D)]
    rhs += [A[b] / 3 for a in range(D) for b in range(D) if a != b]
    rhs += [2 / 3 * (A[a] * us[a] + A[b] * us[b]) - A[c] * us[c] / 3 for (a, b, c) in PAIRS if a < D and b < D]
    return np.linalg.solve(moment_rows(lat), rhs)


def brute_step(lat, dims, f, prm):
    """f: dict (x, y, z) -> array [N][Q] of post-streaming populations."""
    vel, wgt = VEL[lat], WGT[lat]
    N = prm["n_comp"]
    wrap = lambda s, v: tuple((s[a] + v[a]) % dims[a] for a in range(3))
    sites = list(f.keys())
    rho = {s: f[s].sum(axis=1) for s in sites}
    lap = {s: 6 * sum(wgt[i] * (rho[wrap(s, v)] - rho[s]) for i, v in enumerate(vel)) for s in sites}
    mu = {s: T.mu_per_mer(rho[s], prm["m"], prm["chi"], prm["theta"]) - prm["kappa"] * lap[s] for s in sites}
    c = 1 - 1 / (2 * prm["tau"])

    def grad(g, s):
        """grad g(r) = 3 sum_i w_i v_i g(r + v_i), per axis; g: site -> value."""
        return np.array([3 * sum(wgt[i] * v[a] * g(wrap(s, v)) for i, v in enumerate(vel)) for a in range(3)])

    new = {s: np.zeros_like(f[s]) for s in sites}
    v = np.array(vel, float)
    for s in sites:
        j = f[s] @ v                       # [N][3]
        u = j.sum(axis=0) / rho[s].sum()
        for k in range(N):
            if prm["force_form"] == "log":
                A = -c * rho[s][k] * grad(lambda r: mu[r][k] - np.log(rho[r][k]) / 3, s)
            else:
                A = -c * (rho[s][k] * grad(lambda r: mu[r][k], s) - grad(lambda r: rho[r][k], s) / 3)
            fe = feq_by_moments(lat, rho[s][k], u)
            F = forcing_by_moments(lat, A, j[k] / rho[s][k])
            post = f[s][k] + (fe - f[s][k]) / prm["tau"] + F
            for i, vi in enumerate(vel):
                new[wrap(s, vi)][k][i] = post[i]
    return new


CASES = [
    ("D1Q3", (5, 1, 1), 2, "expanded"), ("D1Q3", (4, 1, 1), 3, "log"),
    ("D2Q9", (4, 3, 1), 2, "expanded"), ("D2Q9", (3, 5, 1), 3, "expanded"),
    ("D2Q9", (4, 3, 1), 2, "log"), ("D2Q9", (3, 5, 1), 3, "log"),
    ("D3Q19", (3, 4, 3), 2, "expanded"), ("D3Q19", (3, 3, 4), 3, "log"), ("D3Q19", (4, 3, 3), 2, "log"),
]


@pytest.mark.parametrize("lat,dims,N,form", CASES)
def test_one_and_five_steps_match_brute_force(lat, dims, N, form):
    """A state far from equilibrium with densities that vary along every
    axis, so that each Cartesian component of every gradient and each
    moment takes part; theta != 1/3, so that the ideal-mixing term of the
    potential does not cancel the (1/3) ln rho^s of the log form."""
    nx, ny, nz = dims
    S = nx * ny * nz
    rng = np.random.default_rng(nx * 1000 + ny * 100 + nz * 10 + N + (form == "log"))
    chi = rng.uniform(1.0, 3.0, (N, N))
    chi = 0.5 * (chi + chi.T)
    np.fill_diagonal(chi, 0)
    m = list(rng.choice([1.0, 10.0], N))
    prm = dict(n_comp=N, tau=rng.uniform(0.7, 1.6), theta=rng.uniform(0.15, 0.3), kappa=0.03,
               m=m, chi=chi, force_form=form)
    shape = dims[:DIM[lat]]
    rho0 = rng.uniform(0.2, 0.8, (N, S))
    o = Oracle(OracleParams(lattice=lat, shape=shape, **prm), rho0)
    Q = len(VEL[lat])
    perm = oracle_order(lat)  # the oracle's slot j holds velocity VEL[lat][perm[j]]
    # start from a non-equilibrium state so that every moment is exercised
    f0 = o.get_f() * rng.uniform(0.9, 1.1, (N, Q, S))
    o.set_f(f0)
    coord = lambda s: (s % nx, (s // nx) % ny, s // (nx * ny))
    mine = np.empty_like(f0)
    mine[:, perm, :] = f0
    f = {coord(s): mine[:, :, s].copy() for s in range(S)}
    for nsteps in (1, 4):
        o.step(nsteps)
        for _ in range(nsteps):
            f = brute_step(lat, dims, f, prm)
        got = o.get_f()
        ref = np.stack([f[coord(s)] for s in range(S)], axis=-1)[:, perm, :]
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err < 1e-13, err


def oracle_order(lat):
    """Index into the sets written out here of each of the oracle's
    velocities; also checks that both sets hold the same velocities with the
    same weights."""
    from oracle.oracle import lattice_tables

    q, _, v, w = lattice_tables(lat)
    assert q == len(VEL[lat])
    perm = [VEL[lat].index(tuple(int(c) for c in x)) for x in v]
    assert sorted(perm) == list(range(q)), lat
    assert np.array_equal(w, np.array(WGT[lat])[perm]), lat
    return perm


def test_velocity_tables_match_the_oracle():
    for lat in VEL:
        oracle_order(lat)

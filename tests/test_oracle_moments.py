"""Pins of the oracle's single-site formulas against the paper's moment
definitions (Sec. III: equilibrium moments and forcing moments Eqs.
(ff1)-(ff3)), with the reading that the garbled third-moment deltas are the
fully symmetric combination.  A wrong weight, sign or dropped term in the
equilibrium or forcing polynomial breaks one of these identities."""
import numpy as np
import pytest

from oracle import oracle as O

LATTICES = ["D1Q3", "D2Q9", "D3Q19"]


def moments(lattice, f):
    Q, D, v, w = O.lattice_tables(lattice)
    v = v[:, :D].astype(float)
    m0 = f.sum()
    m1 = np.einsum("i,ia->a", f, v)
    m2 = np.einsum("i,ia,ib->ab", f, v, v)
    m3 = np.einsum("i,ia,ib,ic->abc", f, v, v, v)
    return m0, m1, m2, m3


def sym3(x, D):
    d = np.eye(D)
    return (np.einsum("a,bc->abc", x, d) + np.einsum("b,ac->abc", x, d)
            + np.einsum("c,ab->abc", x, d))


@pytest.mark.parametrize("lattice", LATTICES)
def test_lattice_tables(lattice):
    Q, D, v, w = O.lattice_tables(lattice)
    assert {"D1Q3": 3, "D2Q9": 9, "D3Q19": 19}[lattice] == Q
    assert abs(w.sum() - 1.0) < 1e-15
    vv = v[:, :D].astype(float)
    assert np.allclose(np.einsum("i,ia->a", w, vv), 0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, vv, vv), np.eye(D) / 3, atol=1e-16)
    # every velocity has its opposite
    vs = {tuple(x) for x in v}
    assert all(tuple(-x) in vs for x in v)
    assert len(vs) == Q


@pytest.mark.parametrize("lattice", LATTICES)
def test_equilibrium_moments(lattice):
    rng = np.random.default_rng(11)
    Q, D, v, w = O.lattice_tables(lattice)
    for _ in range(20):
        rho = rng.uniform(0.1, 2.0)
        u = rng.uniform(-0.1, 0.1, D)
        f = O.feq(lattice, rho, u)
        m0, m1, m2, m3 = moments(lattice, f)
        tol = 1e-15 * 4
        assert abs(m0 - rho) < tol * rho
        assert np.allclose(m1, rho * u, atol=tol * rho, rtol=0)
        assert np.allclose(m2, rho / 3 * np.eye(D) + rho * np.outer(u, u), atol=tol * rho, rtol=0)
        # third moment: (rho/3)(u_a d_bc + u_b d_ac + u_c d_ab)
        assert np.allclose(m3, rho / 3 * sym3(u, D), atol=tol * rho, rtol=0)


@pytest.mark.parametrize("lattice", LATTICES)
def test_forcing_moments(lattice):
    rng = np.random.default_rng(12)
    Q, D, v, w = O.lattice_tables(lattice)
    for _ in range(20):
        A = rng.uniform(-0.01, 0.01, D)
        us = rng.uniform(-0.1, 0.1, D)
        F = O.forcing(lattice, A, us)
        m0, m1, m2, m3 = moments(lattice, F)
        tol = 1e-17
        assert abs(m0) < tol
        assert np.allclose(m1, A, atol=tol, rtol=0)                       # Eq. (ff2)
        assert np.allclose(m2, np.outer(A, us) + np.outer(us, A), atol=tol, rtol=0)  # Eq. (ff3)
        assert np.allclose(m3, sym3(A, D) / 3, atol=tol, rtol=0)


def test_d1q3_equilibrium_is_unique():
    """On D1Q3 the three moment conditions fix f^e uniquely: solving them
    reproduces the polynomial."""
    Q, D, v, w = O.lattice_tables("D1Q3")
    vx = v[:, 0].astype(float)
    M = np.vstack([np.ones(3), vx, vx ** 2])
    for rho, u in [(1.0, 0.05), (0.3, -0.08), (2.0, 0.0)]:
        f = np.linalg.solve(M, [rho, rho * u, rho / 3 + rho * u * u])
        assert np.allclose(O.feq("D1Q3", rho, [u]), f, rtol=0, atol=4e-16 * rho)
        A, us = 0.003, -0.07
        F = np.linalg.solve(M, [0.0, A, 2 * A * us])
        assert np.allclose(O.forcing("D1Q3", [A], [us]), F, rtol=0, atol=1e-18)


def test_d2q9_fourth_moments_stated():
    """D2Q9: the moments up to third order leave one fourth moment free
    (sum f v_x^2 v_y^2).  The chosen polynomials give rho (1/9 + |u|^2/3)
    and (2/3) A.u^sigma; stated here so a change of choice is visible."""
    rng = np.random.default_rng(13)
    Q, D, v, w = O.lattice_tables("D2Q9")
    vx, vy = v[:, 0].astype(float), v[:, 1].astype(float)
    for _ in range(5):
        rho, u = rng.uniform(0.2, 2), rng.uniform(-0.1, 0.1, 2)
        f = O.feq("D2Q9", rho, u)
        assert abs((f * vx ** 2 * vy ** 2).sum() - rho * (1 / 9 + (u @ u) / 3)) < 1e-15
        A, us = rng.uniform(-0.01, 0.01, 2), rng.uniform(-0.1, 0.1, 2)
        F = O.forcing("D2Q9", A, us)
        assert abs((F * vx ** 2 * vy ** 2).sum() - 2 / 3 * (A @ us)) < 1e-17


def test_mass_and_momentum_of_collision():
    """BGK with these f^e and F leaves each component's mass unchanged and
    changes the component momentum by tau^-1 (rho^s u - j^s) + A^s."""
    rng = np.random.default_rng(14)
    for lattice in LATTICES:
        Q, D, v, w = O.lattice_tables(lattice)
        vv = v[:, :D].astype(float)
        f = w * rng.uniform(0.5, 1.5, Q)
        rho = f.sum()
        j = f @ vv
        u = rng.uniform(-0.05, 0.05, D)
        A = rng.uniform(-0.01, 0.01, D)
        tau = 0.9
        post = f + (O.feq(lattice, rho, u) - f) / tau + O.forcing(lattice, A, j / rho)
        assert abs(post.sum() - rho) < 1e-15
        assert np.allclose(post @ vv, j + (rho * u - j) / tau + A, atol=1e-16)


def test_equilibrium_rotates_with_velocity():
    """Rotating u by 90 degrees permutes the D2Q9 equilibrium populations the
    same way (isotropy of the table and of the polynomial)."""
    Q, D, v, w = O.lattice_tables("D2Q9")
    f = O.feq("D2Q9", 1.0, [0.03, -0.02])
    g = O.feq("D2Q9", 1.0, [0.02, 0.03])
    rot = {tuple(v[i, :2]): i for i in range(Q)}
    for i in range(Q):
        vx, vy = v[i, 0], v[i, 1]
        assert abs(g[rot[(-vy, vx)]] - f[i]) < 1e-16

"""Pins of the oracle's thermodynamics (Sec. IV, Eq. (lgf); Eq. (ppp)).

The oracle evaluates a closed form of the per-mer chemical potential; here it
is checked against the free energy itself, differentiated by complex step,
and against textbook Flory-Huggins results."""
import numpy as np
import pytest

from oracle import OracleParams, mu_site, psi_site
from oracle import theory as T


def rand_chi(rng, n, scale=3.0):
    c = rng.uniform(0, scale, (n, n))
    c = 0.5 * (c + c.T)
    np.fill_diagonal(c, 0.0)
    return c


@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_mu_is_derivative_of_psi(n):
    rng = np.random.default_rng(100 + n)
    for trial in range(10):
        m = rng.choice([1.0, 2.0, 10.0], n)
        chi = rand_chi(rng, n)
        theta = rng.uniform(0.05, 1.0)
        rho = rng.uniform(0.01, 2.0, n)
        p = OracleParams(lattice="D2Q9", n_comp=n, m=list(m), chi=chi, theta=theta, kappa=0.0)
        mu = mu_site(p, rho)
        ref = T.mu_per_mer(rho, m, chi, theta)
        assert np.allclose(mu, ref, rtol=1e-12, atol=1e-13), (mu, ref)
        # free-energy density agrees with Eq. (lgf) written in number densities
        assert abs(psi_site(p, rho) - np.real(T.psi(rho, m, chi, theta))) < 1e-13 * (1 + abs(psi_site(p, rho)))


def test_kappa_term_enters_mu_linearly():
    rng = np.random.default_rng(7)
    p0 = OracleParams(lattice="D2Q9", n_comp=3, m=[1, 1, 1], chi=rand_chi(rng, 3), kappa=0.0)
    p1 = OracleParams(lattice="D2Q9", n_comp=3, m=[1, 1, 1], chi=p0.chi, kappa=0.25)
    rho, lap = rng.uniform(0.1, 1, 3), rng.uniform(-0.2, 0.2, 3)
    assert np.allclose(mu_site(p1, rho, lap), mu_site(p0, rho) - 0.25 * lap, rtol=0, atol=1e-15)


def test_bulk_pressure_vanishes():
    """psi is homogeneous of degree one in the number densities, so the bulk
    pressure of Eq. (ppp) is identically zero."""
    rng = np.random.default_rng(8)
    for n in (2, 3, 5):
        m = rng.choice([1.0, 10.0], n)
        chi = rand_chi(rng, n)
        p = OracleParams(lattice="D2Q9", n_comp=n, m=list(m), chi=chi, theta=0.4)
        for _ in range(5):
            rho = rng.uniform(0.05, 3, n)
            psi = psi_site(p, rho)
            pres = np.dot(rho, mu_site(p, rho)) - psi
            assert abs(pres) < 1e-14 * max(1.0, abs(psi))


def test_mu_permutation_covariant():
    rng = np.random.default_rng(9)
    n = 4
    m = np.array([1.0, 10.0, 2.0, 1.0])
    chi = rand_chi(rng, n)
    rho = rng.uniform(0.1, 1, n)
    perm = np.array([2, 0, 3, 1])
    p = OracleParams(lattice="D2Q9", n_comp=n, m=list(m), chi=chi)
    q = OracleParams(lattice="D2Q9", n_comp=n, m=list(m[perm]), chi=chi[np.ix_(perm, perm)])
    assert np.allclose(mu_site(q, rho[perm]), mu_site(p, rho)[perm], rtol=1e-14, atol=1e-15)


def test_binary_textbook_binodal_and_critical_point():
    """The theory tools used as long-run targets: symmetric binodal
    ln(phi/(1-phi)) = chi (2 phi - 1); critical points quoted in Sec. IV:
    phi_c = 0.5 for m = (1, 1) and 0.24 for m = (10, 1)."""
    lo, hi = T.binary_binodal(1, 1, 2.4)
    assert abs(np.log(lo / (1 - lo)) - 2.4 * (2 * lo - 1)) < 1e-13
    assert abs(lo + hi - 1) < 1e-14
    assert abs(lo - 0.1707152) < 1e-7
    phi_c, chi_c = T.binary_critical(1, 1)
    assert phi_c == 0.5 and abs(chi_c - 2.0) < 1e-15
    phi_c, chi_c = T.binary_critical(10, 1)
    assert abs(phi_c - 0.24) < 0.001 and abs(chi_c - 0.866228) < 1e-6
    lo, hi = T.binary_binodal(10, 1, 0.94)
    assert abs(lo - 0.0746177) < 1e-7 and abs(hi - 0.4783912) < 1e-7
    # both phases have equal exchange potential per the full N-component free energy
    chi = np.array([[0, 0.94], [0.94, 0]])
    d = T.mu_per_mer([lo, 1 - lo], [10, 1], chi) - T.mu_per_mer([hi, 1 - hi], [10, 1], chi)
    assert np.abs(d).max() < 1e-10


def test_symmetric_ncomponent_critical_interaction():
    """At equal composition 1/N with a uniform chi, the mixture loses
    stability at chi = N (the Hessian of psi/rho in the simplex vanishes)."""
    for n in (2, 3, 5):
        def hess_min_eig(chi_val):
            chi = chi_val * (np.ones((n, n)) - np.eye(n))
            # second derivative of psi along simplex directions e_a - e_b by finite differences of mu
            phi = np.full(n, 1.0 / n)
            H = np.zeros((n - 1, n - 1))
            for a in range(n - 1):
                d = np.zeros(n)
                d[a], d[-1] = 1, -1
                h = 1e-6
                dmu = (T.mu_per_mer(phi + h * d, [1] * n, chi) - T.mu_per_mer(phi - h * d, [1] * n, chi)) / (2 * h)
                for b in range(n - 1):
                    e = np.zeros(n)
                    e[b], e[-1] = 1, -1
                    H[a, b] = dmu @ e
            return np.linalg.eigvalsh(0.5 * (H + H.T)).min()
        assert hess_min_eig(0.98 * n) > 0
        assert hess_min_eig(1.02 * n) < 0


def test_ternary_plait_point():
    """Critical point of three components: closed form for a neutral third
    component (chi^AC = chi^BC = 0, m = 1): the exchange mode of A and B at
    phi_A = phi_B = x has f_AA - f_AB = 1/x - chi, so the plait point is
    (1/chi, 1/chi, 1 - 2/chi).  For the systems of Fig. 3 the point must lie
    on the spinodal of the complex-step chemical potentials (an independent
    route to the Hessian) and differ from the quoted critical points by a
    few 1e-2 (reading R16)."""
    for chi in (2.5, 3.0, 4.0):
        c = np.array([[0, chi, 0], [chi, 0, 0], [0, 0, 0.0]])
        p = T.ternary_plait_point((1, 1, 1), c, (0.3, 0.35))
        assert np.abs(p - [1 / chi, 1 / chi, 1 - 2 / chi]).max() < 1e-10
    chi3 = np.array([[0, 3.0, 0.5], [3.0, 0, 0.2], [0.5, 0.2, 0]])
    for m, quoted in (((1, 1, 1), (0.32, 0.32, 0.36)), ((10, 1, 1), (0.14, 0.11, 0.75))):
        p = T.ternary_plait_point(m, chi3, quoted)
        H = np.zeros((2, 2))
        h = 1e-6
        for a in range(2):
            d = np.zeros(3)
            d[a], d[2] = 1, -1
            dmu = (T.mu_per_mer(p + h * d, m, chi3) - T.mu_per_mer(p - h * d, m, chi3)) / (2 * h)
            for b in range(2):
                e = np.zeros(3)
                e[b], e[2] = 1, -1
                H[a, b] = dmu @ e / (1.0 / 3.0)  # mu carries theta = 1/3
        eig = np.linalg.eigvalsh(0.5 * (H + H.T))
        assert abs(eig[0]) < 1e-6 * abs(eig[1]), eig
        assert 0.01 < np.abs(p - quoted).max() < 0.06


def test_plait_points_of_the_inputs():
    """The starting points of the plait-point run sets in lbinputs are the
    plait points of the theory tools, to their stated rounding."""
    import lbinputs as LI

    chi3 = np.array([[0, 3.0, 0.5], [3.0, 0, 0.2], [0.5, 0.2, 0]])
    for m, stored in (((1, 1, 1), LI.PLAIT_MONOMER), ((10, 1, 1), LI.PLAIT_POLYMER)):
        p = T.ternary_plait_point(m, chi3, stored)
        assert np.abs(p - stored).max() < 6e-5

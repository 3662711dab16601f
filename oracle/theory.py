"""Equilibrium thermodynamics of the Flory-Huggins free energy, Eq. (lgf).

TEST INFRASTRUCTURE ONLY.  These routines give the values that the lattice
Boltzmann runs must reach (binodals, critical points, spinodals) and are
written from the free energy itself, not from the oracle's closed-form
chemical potential:

* ``psi`` is Eq. (lgf) written out in number densities n^sigma = rho^sigma/m^sigma.
* ``mu_per_mer`` differentiates ``psi`` by the complex-step method
  (Squire & Trapp, SIAM Review 40, 1998), which is exact to rounding for
  an analytic function, and divides by m^sigma.
* ``binary_*`` use the textbook two-component Flory-Huggins mixing free energy
  per lattice site, f(phi) = phi ln(phi)/m_A + (1-phi) ln(1-phi)/m_B + chi phi (1-phi),
  and the common-tangent construction.
* ``coexistence`` solves equal chemical potentials of every component in two
  phases plus the lever rule; the bulk pressure of Eq. (ppp) vanishes
  identically for this free energy (it is homogeneous of degree one in n),
  so equal pressure adds no condition.
"""
from __future__ import annotations

import numpy as np
from scipy import optimize


def psi(rho, m, chi, theta=1.0 / 3.0):
    """Free-energy density of Eq. (lgf) for mer densities rho[N] (may be complex)."""
    rho = np.asarray(rho)
    m = np.asarray(m, dtype=float)
    chi = np.asarray(chi, dtype=float)
    n = rho / m
    phi = (m * n) / np.sum(m * n)
    out = -theta * np.sum(n * m) + theta * np.sum(n * np.log(phi))
    out = out + 0.5 * theta * np.sum(chi * np.outer(m * n, phi))
    return out


def mu_per_mer(rho, m, chi, theta=1.0 / 3.0, h=1e-30):
    """mu^sigma = (1/m^sigma) d psi / d n^sigma by complex step."""
    rho = np.asarray(rho, dtype=float)
    m = np.asarray(m, dtype=float)
    out = np.empty_like(rho)
    n = rho / m
    for s in range(rho.size):
        nz = n.astype(complex)
        nz[s] += 1j * h
        out[s] = np.imag(psi(nz * m, m, chi, theta)) / h / m[s]
    return out


def bulk_pressure(rho, m, chi, theta=1.0 / 3.0):
    """p = sum_sigma n^sigma mu_n^sigma - psi, Eq. (ppp)."""
    rho = np.asarray(rho, dtype=float)
    return float(np.sum(rho * mu_per_mer(rho, m, chi, theta)) - np.real(psi(rho, m, chi, theta)))


# ---------------------------------------------------------------- binary ----

def binary_critical(mA, mB):
    """Critical point of the binary Flory-Huggins mixture: (phi_c, chi_c)."""
    phi_c = np.sqrt(mB) / (np.sqrt(mA) + np.sqrt(mB))
    chi_c = 0.5 * (1.0 / np.sqrt(mA) + 1.0 / np.sqrt(mB)) ** 2
    return float(phi_c), float(chi_c)


def binary_spinodal_chi(phi, mA, mB):
    """chi on the spinodal, where f''(phi) = 0."""
    return 0.5 * (1.0 / (mA * phi) + 1.0 / (mB * (1.0 - phi)))


def _f(phi, mA, mB, chi):
    return phi * np.log(phi) / mA + (1 - phi) * np.log(1 - phi) / mB + chi * phi * (1 - phi)


def _fp(phi, mA, mB, chi):
    return (np.log(phi) + 1) / mA - (np.log(1 - phi) + 1) / mB + chi * (1 - 2 * phi)


def binary_binodal(mA, mB, chi):
    """Coexisting volume fractions (phi_1 < phi_2) of component A by the
    common-tangent construction on f(phi)."""
    if mA == mB:
        # symmetric: ln(phi/(1-phi)) = mA chi (2 phi - 1), phi in (0, 1/2)
        g = lambda x: np.log(x / (1 - x)) / mA - chi * (2 * x - 1)
        lo = optimize.brentq(g, 1e-15, 0.5 - 1e-12 if chi * mA > 2.0 else 0.5, xtol=1e-15)
        return lo, 1.0 - lo

    phi_c, chi_c = binary_critical(mA, mB)
    if chi <= chi_c:
        raise ValueError("no phase separation below the critical interaction")
    fp = lambda x: _fp(x, mA, mB, chi)
    icpt = lambda x: _f(x, mA, mB, chi) - x * _fp(x, mA, mB, chi)
    # spinodal points s1 < phi_c < s2: f' rises on (0, s1), falls on (s1, s2)
    # and rises again on (s2, 1).  A tangent slope lies in (f'(s2), f'(s1)).
    disc = lambda x: binary_spinodal_chi(x, mA, mB) - chi
    s1 = optimize.brentq(disc, 1e-14, phi_c, xtol=1e-16)
    s2 = optimize.brentq(disc, phi_c, 1 - 1e-14, xtol=1e-16)
    a_min = optimize.brentq(lambda x: fp(x) - fp(s2), 1e-300, s1, xtol=1e-300)

    def partner(a):  # b in (s2, 1) with the same slope as a
        return optimize.brentq(lambda x: fp(x) - fp(a), s2, 1 - 1e-16, xtol=1e-16)

    g = lambda a: icpt(a) - icpt(partner(a))
    a = optimize.brentq(g, a_min * (1 + 1e-9), s1 * (1 - 1e-9), xtol=1e-16)
    return float(a), float(partner(a))


# ------------------------------------------------------- N components ----

def coexistence(phi_mean, m, chi, guess_a, guess_b, theta=1.0 / 3.0):
    """Two coexisting phases of total mer density 1 whose lever-rule mixture
    is phi_mean: equal mu^sigma for every sigma.  Returns (phi_a, phi_b,
    fraction of phase a)."""
    phi_mean = np.asarray(phi_mean, float)
    N = phi_mean.size

    def unpack(x):
        pa = np.append(x[: N - 1], 1 - np.sum(x[: N - 1]))
        pb = np.append(x[N - 1: 2 * N - 2], 1 - np.sum(x[N - 1: 2 * N - 2]))
        return pa, pb, x[-1]

    def eqs(x):
        pa, pb, lam = unpack(x)
        if np.any(pa <= 0) or np.any(pb <= 0):
            return np.full(2 * N - 1, 1e3)
        dmu = mu_per_mer(pa, m, chi, theta) - mu_per_mer(pb, m, chi, theta)
        lever = lam * pa[: N - 1] + (1 - lam) * pb[: N - 1] - phi_mean[: N - 1]
        return np.concatenate([dmu, lever])

    ga, gb = np.asarray(guess_a, float), np.asarray(guess_b, float)
    lam0 = float(np.clip(np.dot(phi_mean - gb, ga - gb) / np.dot(ga - gb, ga - gb), 0.05, 0.95))
    x0 = np.concatenate([ga[: N - 1], gb[: N - 1], [lam0]])
    sol, info, ier, msg = optimize.fsolve(eqs, x0, full_output=True, xtol=1e-13)
    if ier != 1:
        raise RuntimeError(msg)
    pa, pb, lam = unpack(sol)
    return pa, pb, float(lam)


# ---------------------------------------------------- three components ----

def _ternary_hessian(pa, pb, m, chi):
    """Hessian of the mixing free energy per site, f = sum_s phi_s ln(phi_s)/m_s
    + sum_{s<t} chi^{st} phi_s phi_t (Eq. (lgf) divided by the total mer
    density; theta and the terms linear in phi drop out of phase behaviour),
    in the independent fractions (phi_A, phi_B), phi_C = 1 - phi_A - phi_B."""
    pc = 1.0 - pa - pb
    mA, mB, mC = m
    g = 1.0 / (mC * pc)
    haa = 1.0 / (mA * pa) + g - 2.0 * chi[0][2]
    hbb = 1.0 / (mB * pb) + g - 2.0 * chi[1][2]
    hab = g + chi[0][1] - chi[0][2] - chi[1][2]
    return haa, hab, hbb


def _ternary_critical_residual(x, m, chi):
    pa, pb = x
    pc = 1.0 - pa - pb
    if pa <= 0 or pb <= 0 or pc <= 0:
        return [1e3, 1e3]
    haa, hab, hbb = _ternary_hessian(pa, pb, m, chi)
    det = haa * hbb - hab * hab
    # null direction of the Hessian on the spinodal
    va, vb = (-hab, haa) if abs(haa) >= abs(hbb) else (hbb, -hab)
    nrm = np.hypot(va, vb)
    va, vb = va / nrm, vb / nrm
    mA, mB, mC = m
    gc = 1.0 / (mC * pc * pc)
    faaa = -1.0 / (mA * pa * pa) + gc
    fbbb = -1.0 / (mB * pb * pb) + gc
    third = faaa * va ** 3 + 3.0 * gc * va * va * vb + 3.0 * gc * va * vb * vb + fbbb * vb ** 3
    return [det, third]


def ternary_plait_point(m, chi, guess):
    """Critical (plait) point of a three-component Flory-Huggins mixture:
    the spinodal det H = 0 where the third derivative of f along the null
    direction of H also vanishes.  Returns (phi_A, phi_B, phi_C)."""
    chi = np.asarray(chi, float)
    sol, info, ier, msg = optimize.fsolve(_ternary_critical_residual, np.asarray(guess[:2], float),
                                          args=(tuple(m), chi), full_output=True, xtol=1e-12)
    r = _ternary_critical_residual(sol, tuple(m), chi)
    if max(abs(r[0]), abs(r[1])) > 1e-8:
        raise RuntimeError(f"plait point residual {r}")
    return np.array([sol[0], sol[1], 1.0 - sol[0] - sol[1]])

"""One step of the oracle about a uniform state at rest, against the exact
discrete linearisation of Eq. (ssLB) built here mode by mode.

About f_i = w_i rho^s (uniform, at rest; a fixed point of the step) a small
perturbation  df_i(r) = Re[a_i exp(i k.r)]  of a single lattice wave vector k
goes after one step into  Re[b_i exp(i k.r)]  with b = M(k) a, where M(k)
follows from linearising each piece of Sec. III at the uniform state:
  * moments: d rho^s = sum_i a^s_i, d j^s = sum_i v_i a^s_i,
    du = sum_s d j^s / rho (the barycentric velocity; j = 0 at rest);
  * lap rho -> Lambda(k) d rho with Lambda = 6 sum_i w_i (e^{i k.v_i} - 1), and
    grad g -> G(k) dg with G = 3 sum_i w_i v_i e^{i k.v_i};
  * d mu^s = sum_t (d mu^s / d rho^t) d rho^t - kappa Lambda d rho^s, the
    derivatives of Eq. (lgf) per mer taken numerically from the complex-step
    potentials of oracle/theory.py;
  * d A^s = -c G (rho^s d mu^s - d rho^s / 3) (both lines of Eq. (definef)
    reduce to this at linear order);
  * d f^e_i = w_i (d rho^s + 3 rho^s v_i.du), d F_i = 3 w_i v_i.dA^s (the
    second-order terms of the equilibrium and forcing polynomials vanish);
  * BGK: a + (d f^e - a)/tau + dF; pull streaming: b_i = e^{-i k.v_i} (...)_i.
The perturbation is a general one (every population of every component
perturbed independently), and k points obliquely, so every Cartesian
component of the gradients, the velocity terms of the equilibrium, the
forcing term, the weights and the streaming direction take part.  The
oracle's response, (f(t+1) - f_bar)/eps, must equal Re[b e^{i k.r}] to the
linearisation error O(eps) plus rounding.  Nonlinear terms are pinned by
the brute-force test; this pin checks the whole step's linear part,
including the log-form force along y and z, independently of it.
"""
import numpy as np
import pytest

from oracle import Oracle, OracleParams
from oracle import theory as T
from test_oracle_bruteforce import DIM, VEL, WGT, oracle_order


def mu_jacobian(rho, m, chi, theta, h=1e-6):
    """d mu^s / d rho^t by central differences of the complex-step potentials."""
    N = len(rho)
    J = np.empty((N, N))
    for t in range(N):
        up, dn = np.array(rho, float), np.array(rho, float)
        up[t] += h
        dn[t] -= h
        J[:, t] = (T.mu_per_mer(up, m, chi, theta) - T.mu_per_mer(dn, m, chi, theta)) / (2 * h)
    return J


def step_matrix(lat, k, rho_bar, prm):
    """M(k) acting on a[N][Q] (in the velocity order of VEL[lat])."""
    v = np.array(VEL[lat], float)
    w = np.array(WGT[lat])
    N, Q = len(rho_bar), len(w)
    E = np.exp(1j * (v @ k))
    Lam = 6 * np.sum(w * (E - 1))
    G = 3 * (w * E) @ v  # vector
    J = mu_jacobian(rho_bar, prm["m"], prm["chi"], prm["theta"])
    c = 1 - 1 / (2 * prm["tau"])
    rt = np.sum(rho_bar)

    def apply(a):
        drho = a.sum(axis=1)
        dj = a @ v  # [N][3]
        du = dj.sum(axis=0) / rt
        dmu = J @ drho - prm["kappa"] * Lam * drho
        b = np.empty_like(a)
        for s in range(N):
            dA = -c * G * (rho_bar[s] * dmu[s] - drho[s] / 3)
            dfe = w * (drho[s] + 3 * rho_bar[s] * (v @ du))
            dF = 3 * w * (v @ dA)
            post = a[s] + (dfe - a[s]) / prm["tau"] + dF
            b[s] = np.conj(E) * post
        return b

    return apply


CASES = [
    ("D2Q9", (16, 12, 1), (1, 2, 0), 2, "log", 0.2),
    ("D2Q9", (16, 12, 1), (3, -1, 0), 3, "log", 1 / 3),
    ("D2Q9", (10, 14, 1), (2, 3, 0), 2, "expanded", 0.25),
    ("D3Q19", (8, 6, 10), (1, 1, 2), 2, "log", 0.2),
    ("D3Q19", (6, 8, 6), (1, -2, 1), 3, "expanded", 0.3),
    ("D1Q3", (20, 1, 1), (3, 0, 0), 3, "log", 0.2),
]


@pytest.mark.parametrize("lat,dims,kn,N,form,theta", CASES)
def test_one_step_matches_the_discrete_linearisation(lat, dims, kn, N, form, theta):
    rng = np.random.default_rng(sum(dims) * 10 + N)
    chi = rng.uniform(0.3, 1.2, (N, N))
    chi = 0.5 * (chi + chi.T)
    np.fill_diagonal(chi, 0)
    m = list(rng.choice([1.0, 2.0, 10.0], N))
    prm = dict(n_comp=N, tau=float(rng.uniform(0.7, 1.5)), theta=theta, kappa=0.02, m=m, chi=chi, force_form=form)
    shape = dims[:DIM[lat]]
    S = int(np.prod(dims))
    rho_bar = rng.uniform(0.2, 0.6, N)
    o = Oracle(OracleParams(lattice=lat, shape=shape, **prm), np.repeat(rho_bar[:, None], S, axis=1))
    perm = oracle_order(lat)  # oracle slot j holds velocity VEL[lat][perm[j]]
    Q = len(perm)
    w = np.array(WGT[lat])
    k = 2 * np.pi * np.array(kn, float) / np.array(dims, float)
    s = np.arange(S)
    r = np.stack([s % dims[0], (s // dims[0]) % dims[1], s // (dims[0] * dims[1])], axis=1).astype(float)
    phase = np.exp(1j * (r @ k))  # [S]
    a = (rng.normal(size=(N, Q)) + 1j * rng.normal(size=(N, Q))) * rho_bar[:, None] * w[None, :]
    eps = 1e-7
    f_bar = w[None, :, None] * rho_bar[:, None, None]  # in VEL order
    df = np.real(a[:, :, None] * phase[None, None, :])
    f0 = f_bar + eps * df
    o.set_f(f0[:, perm, :])
    o.step(1)
    got = (o.get_f() - f_bar[:, perm, :]) / eps
    b = step_matrix(lat, k, rho_bar, prm)(a)
    want = np.real(b[:, :, None] * phase[None, None, :])[:, perm, :]
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err < 1e-6, err

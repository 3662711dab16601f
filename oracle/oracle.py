"""ctypes binding of the FP64 CPU oracle (``lb_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Arrays are numpy float64, component-major:
densities ``rho[N][S]``, populations ``f[N][Q][S]``, with the site index
``s = x + nx*(y + ny*z)``.  Physical parameters follow the paper's statement
of the problem (Sec. III and IV): relaxation time tau, temperature theta,
polymerisations m^sigma, interaction matrix chi^{sigma sigma'} and the
square-gradient coefficient kappa.
"""
import ctypes as C
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

from .build import ensure_built

MAX_COMP = 8
LATTICES = {"D1Q3": 1, "D2Q9": 2, "D3Q19": 3}
FORCE_FORMS = {"expanded": 0, "log": 1}


class _Params(C.Structure):
    _fields_ = [
        ("lattice", C.c_int32), ("n_comp", C.c_int32), ("force_form", C.c_int32),
        ("walls", C.c_int32),
        ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
        ("tau", C.c_double), ("theta", C.c_double), ("kappa", C.c_double),
        ("m", C.c_double * MAX_COMP), ("chi", C.c_double * (MAX_COMP * MAX_COMP)),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = C.CDLL(ensure_built())
        dp = C.POINTER(C.c_double)
        lib.orc_lattice.argtypes = [C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32), dp]
        lib.orc_lattice.restype = C.c_int
        lib.orc_feq.argtypes = [C.c_int32, C.c_double, dp, dp]
        lib.orc_forcing.argtypes = [C.c_int32, dp, dp, dp]
        lib.orc_mu_site.argtypes = [C.POINTER(_Params), dp, dp, dp]
        lib.orc_psi_site.argtypes = [C.POINTER(_Params), dp]
        lib.orc_psi_site.restype = C.c_double
        lib.orc_create.argtypes = [C.POINTER(_Params), dp]
        lib.orc_create.restype = C.c_void_p
        lib.orc_destroy.argtypes = [C.c_void_p]
        lib.orc_step.argtypes = [C.c_void_p, C.c_int64]
        lib.orc_time.argtypes = [C.c_void_p]
        lib.orc_time.restype = C.c_int64
        lib.orc_get_f.argtypes = [C.c_void_p, dp]
        lib.orc_set_f.argtypes = [C.c_void_p, dp]
        lib.orc_observe.argtypes = [C.c_void_p] + [dp] * 7
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class OracleParams:
    lattice: str = "D2Q9"
    n_comp: int = 2
    shape: Sequence[int] = (64, 64)          # (nx,), (nx, ny) or (nx, ny, nz)
    tau: float = 1.0
    theta: float = 1.0 / 3.0
    kappa: float = 0.0
    m: Sequence[float] = field(default_factory=lambda: [1.0, 1.0])
    chi: Optional[np.ndarray] = None         # N x N symmetric, zero diagonal
    force_form: str = "expanded"
    walls: int = 0                            # bit a: axis a closed by walls (not in the paper)

    def to_c(self) -> _Params:
        p = _Params()
        p.lattice = LATTICES[self.lattice]
        p.n_comp = self.n_comp
        p.force_form = FORCE_FORMS[self.force_form]
        p.walls = int(self.walls)
        dims = list(self.shape) + [1] * (3 - len(self.shape))
        p.nx, p.ny, p.nz = dims
        p.tau, p.theta, p.kappa = self.tau, self.theta, self.kappa
        for s in range(self.n_comp):
            p.m[s] = self.m[s]
        chi = np.zeros((self.n_comp, self.n_comp)) if self.chi is None else np.asarray(self.chi, float)
        for s in range(self.n_comp):
            for t in range(self.n_comp):
                p.chi[s * MAX_COMP + t] = chi[s, t]
        return p

    @property
    def sites(self) -> int:
        return int(np.prod(self.shape))


def lattice_tables(lattice: str):
    lib = _load()
    Q, D = C.c_int32(), C.c_int32()
    v = (C.c_int32 * (19 * 3))()
    w = (C.c_double * 19)()
    if lib.orc_lattice(LATTICES[lattice], C.byref(Q), C.byref(D), v, w) != 0:
        raise ValueError(lattice)
    q = Q.value
    return q, D.value, np.array(v[: 3 * q]).reshape(q, 3), np.array(w[:q])


def feq(lattice: str, rho: float, u) -> np.ndarray:
    q = lattice_tables(lattice)[0]
    out = np.zeros(q)
    uu = np.zeros(3)
    uu[: len(u)] = u
    _load().orc_feq(LATTICES[lattice], rho, _ptr(uu), _ptr(out))
    return out


def forcing(lattice: str, A, usig) -> np.ndarray:
    q = lattice_tables(lattice)[0]
    out = np.zeros(q)
    a3, u3 = np.zeros(3), np.zeros(3)
    a3[: len(A)] = A
    u3[: len(usig)] = usig
    _load().orc_forcing(LATTICES[lattice], _ptr(a3), _ptr(u3), _ptr(out))
    return out


def mu_site(params: OracleParams, rho, lap=None) -> np.ndarray:
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    lap = None if lap is None else np.ascontiguousarray(lap, dtype=np.float64)
    out = np.zeros(params.n_comp)
    p = params.to_c()
    _load().orc_mu_site(C.byref(p), _ptr(rho), _ptr(lap), _ptr(out))
    return out


def psi_site(params: OracleParams, rho) -> float:
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    p = params.to_c()
    return _load().orc_psi_site(C.byref(p), _ptr(rho))


class Oracle:
    """A periodic lattice stepped by the FP64 oracle."""

    def __init__(self, params: OracleParams, rho0: np.ndarray):
        self.params = params
        self.Q, self.D, self.v, self.w = lattice_tables(params.lattice)
        self.N, self.S = params.n_comp, params.sites
        rho0 = np.ascontiguousarray(np.asarray(rho0, dtype=np.float64).reshape(self.N, self.S))
        self._p = params.to_c()
        self._lib = _load()
        self._h = self._lib.orc_create(C.byref(self._p), _ptr(rho0))
        if not self._h:
            raise ValueError("oracle: bad parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    def step(self, n: int = 1) -> None:
        self._lib.orc_step(self._h, int(n))

    @property
    def time(self) -> int:
        return int(self._lib.orc_time(self._h))

    def get_f(self) -> np.ndarray:
        f = np.zeros((self.N, self.Q, self.S))
        self._lib.orc_get_f(self._h, _ptr(f))
        return f

    def set_f(self, f: np.ndarray) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.N, self.Q, self.S)
        self._lib.orc_set_f(self._h, _ptr(f))

    def observe(self):
        """Return a dict with rho[N,S], U[D,S], mu[N,S], P[D(D+1)/2,S],
        A[N,D,S], mass[N], mom[D] at the current time."""
        N, D, S = self.N, self.D, self.S
        out = dict(
            rho=np.zeros((N, S)), U=np.zeros((D, S)), mu=np.zeros((N, S)),
            P=np.zeros((D * (D + 1) // 2, S)), A=np.zeros((N, D, S)),
            mass=np.zeros(N), mom=np.zeros(D),
        )
        self._lib.orc_observe(self._h, *(_ptr(out[k]) for k in ("rho", "U", "mu", "P", "A", "mass", "mom")))
        return out

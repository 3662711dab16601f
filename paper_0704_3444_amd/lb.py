"""ctypes binding of the C ABI in include/lb.h (argument marshalling only).

Every function here has the name of the C entry point it wraps and does no
arithmetic of the method: each step runs in the HIP kernels of liblbm.so.
PyTorch supplies device memory (the workspace) and the stream.  If the
library is not built, loading fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")
MAX_COMP = 8

LB_OK, LB_EINVAL, LB_ENOMEM, LB_ENOTSUP, LB_EDEVICE, LB_ENUMERIC = 0, -1, -2, -3, -4, -5
LATTICE = {"D1Q3": 1, "D2Q9": 2, "D3Q19": 3}
STORAGE = {"f64": 0, "f32": 1, "f16s": 2}
FORCE_FORM = {"log": 0, "expanded": 1}
PATH = {"auto": 0, "tile": 1, "split": 2, "sweep": 3}

EXPORTS = [
    "lb_workspace_bytes", "lb_init", "lb_step", "lb_moments", "lb_get_f", "lb_state_bytes",
    "lb_get_state", "lb_set_state", "lb_lattice_tables", "lb_path_in_use", "lb_free",
    "lb_strerror", "lb_last_error",
]


class lb_params(C.Structure):
    _fields_ = [
        ("n_comp", C.c_int32), ("lattice", C.c_int32), ("storage", C.c_int32), ("force_form", C.c_int32),
        ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
        ("tau", C.c_double * MAX_COMP), ("theta", C.c_double), ("kappa", C.c_double),
        ("m", C.c_double * MAX_COMP), ("chi", C.c_double * (MAX_COMP * MAX_COMP)),
        ("path", C.c_int32), ("check_every", C.c_int32), ("stream", C.c_void_p),
    ]


class LBError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def load() -> C.CDLL:
    """Load liblbm.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_0704_3444_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    dp, vp = C.POINTER(C.c_double), C.c_void_p
    P = C.POINTER(lb_params)
    lib.lb_workspace_bytes.argtypes = [P]
    lib.lb_workspace_bytes.restype = C.c_size_t
    lib.lb_init.argtypes = [P, dp, vp, C.c_size_t, C.POINTER(vp)]
    lib.lb_step.argtypes = [vp, C.c_int64]
    lib.lb_moments.argtypes = [vp, dp, dp, dp, dp, dp, dp, C.POINTER(C.c_int64)]
    lib.lb_get_f.argtypes = [vp, dp]
    lib.lb_state_bytes.argtypes = [vp]
    lib.lb_state_bytes.restype = C.c_size_t
    lib.lb_get_state.argtypes = [vp, vp, C.c_size_t]
    lib.lb_set_state.argtypes = [vp, vp, C.c_size_t]
    lib.lb_lattice_tables.argtypes = [C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), dp]
    lib.lb_path_in_use.argtypes = [vp]
    lib.lb_free.argtypes = [vp]
    lib.lb_free.restype = None
    lib.lb_strerror.argtypes = [C.c_int]
    lib.lb_strerror.restype = C.c_char_p
    lib.lb_last_error.argtypes = []
    lib.lb_last_error.restype = C.c_char_p
    for name in ("lb_init", "lb_step", "lb_moments", "lb_get_f", "lb_get_state", "lb_set_state",
                 "lb_lattice_tables", "lb_path_in_use"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(rc: int) -> int:
    if rc < 0:
        lib = load()
        raise LBError(rc, f"{lib.lb_strerror(rc).decode()}: {lib.lb_last_error().decode()}")
    return rc


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(cfg: dict, *, storage="f64", path="auto", check_every=0, stream=None) -> lb_params:
    """lb_params from a workload dict (keys lattice, n_comp, shape, tau,
    theta, kappa, m, chi, force_form)."""
    p = lb_params()
    n = int(cfg["n_comp"])
    shape = list(cfg["shape"]) + [1] * (3 - len(cfg["shape"]))
    p.n_comp, p.lattice = n, LATTICE[cfg["lattice"]]
    p.storage, p.force_form = STORAGE[storage], FORCE_FORM[cfg.get("force_form", "log")]
    p.nx, p.ny, p.nz = (int(x) for x in shape)
    tau = cfg["tau"]
    for k in range(n):
        p.tau[k] = float(tau[k] if np.ndim(tau) else tau)
        p.m[k] = float(cfg["m"][k])
    p.theta, p.kappa = float(cfg["theta"]), float(cfg["kappa"])
    chi = np.asarray(cfg["chi"], dtype=np.float64)
    for a in range(n):
        for b in range(n):
            p.chi[a * MAX_COMP + b] = chi[a, b]
    p.path, p.check_every = PATH[path], int(check_every)
    p.stream = stream
    return p


def lb_workspace_bytes(p: lb_params) -> int:
    n = load().lb_workspace_bytes(C.byref(p))
    if n == 0:
        raise LBError(LB_EINVAL, load().lb_last_error().decode())
    return int(n)


def lb_init(p: lb_params, rho0: np.ndarray, workspace_ptr: int = 0, workspace_bytes: int = 0) -> int:
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
    h = C.c_void_p()
    _check(load().lb_init(C.byref(p), _dptr(rho0), C.c_void_p(workspace_ptr or None),
                          C.c_size_t(workspace_bytes), C.byref(h)))
    return h.value


def lb_step(ctx: int, nsteps: int) -> None:
    _check(load().lb_step(C.c_void_p(ctx), C.c_int64(nsteps)))


def lb_moments(ctx: int, n_comp: int, dim: int, sites: int, fields=True, raise_numeric=True) -> dict:
    out = {"mass": np.zeros(n_comp), "mom": np.zeros(dim)}
    if fields:
        out.update(rho=np.zeros((n_comp, sites)), U=np.zeros((dim, sites)), mu=np.zeros((n_comp, sites)),
                   P=np.zeros((dim * (dim + 1) // 2, sites)))
    step = C.c_int64()
    rc = load().lb_moments(C.c_void_p(ctx), _dptr(out.get("rho")), _dptr(out.get("U")), _dptr(out.get("mu")),
                           _dptr(out.get("P")), _dptr(out["mass"]), _dptr(out["mom"]), C.byref(step))
    out["step"] = step.value
    out["status"] = rc
    if rc != LB_ENUMERIC or raise_numeric:
        _check(rc)
    return out


def lb_get_f(ctx: int, n_comp: int, Q: int, sites: int) -> np.ndarray:
    f = np.zeros((n_comp, Q, sites))
    _check(load().lb_get_f(C.c_void_p(ctx), _dptr(f)))
    return f


def lb_state_bytes(ctx: int) -> int:
    return int(load().lb_state_bytes(C.c_void_p(ctx)))


def lb_get_state(ctx: int) -> bytes:
    n = lb_state_bytes(ctx)
    buf = (C.c_char * n)()
    _check(load().lb_get_state(C.c_void_p(ctx), buf, C.c_size_t(n)))
    return bytes(buf)


def lb_set_state(ctx: int, state: bytes) -> None:
    buf = (C.c_char * len(state)).from_buffer_copy(state)
    _check(load().lb_set_state(C.c_void_p(ctx), buf, C.c_size_t(len(state))))


def lb_lattice_tables(lattice: str):
    Q, D = C.c_int32(), C.c_int32()
    v = (C.c_int32 * 57)()
    w = (C.c_double * 19)()
    _check(load().lb_lattice_tables(LATTICE[lattice], C.byref(Q), C.byref(D), v, w))
    q = Q.value
    return q, D.value, np.array(v[: 3 * q]).reshape(q, 3), np.array(w[:q])


def lb_path_in_use(ctx: int) -> str:
    r = _check(load().lb_path_in_use(C.c_void_p(ctx)))
    return {1: "tile", 2: "split", 3: "sweep"}[r]


def lb_free(ctx: int) -> None:
    if ctx:
        load().lb_free(C.c_void_p(ctx))


class Simulation:
    """One lattice on the current CUDA/HIP device: the workspace is a torch
    uint8 tensor and the stream is torch's current stream."""

    def __init__(self, cfg: dict, rho0: np.ndarray, *, storage="f64", path="auto", check_every=0,
                 device="cuda", stream=None):
        import torch

        self.cfg = cfg
        self.n = int(cfg["n_comp"])
        self.sites = int(np.prod(cfg["shape"]))
        self.Q, self.D, _, _ = lb_lattice_tables(cfg["lattice"])
        dev = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.params = make_params(cfg, storage=storage, path=path, check_every=check_every,
                                  stream=self.stream.cuda_stream)
        nbytes = lb_workspace_bytes(self.params)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.ctx = lb_init(self.params, rho0, aligned, nbytes)

    def step(self, n: int = 1) -> None:
        lb_step(self.ctx, n)

    def moments(self, fields=True, raise_numeric=True) -> dict:
        return lb_moments(self.ctx, self.n, self.D, self.sites, fields=fields, raise_numeric=raise_numeric)

    def get_f(self) -> np.ndarray:
        return lb_get_f(self.ctx, self.n, self.Q, self.sites)

    def get_state(self) -> bytes:
        return lb_get_state(self.ctx)

    def set_state(self, s: bytes) -> None:
        lb_set_state(self.ctx, s)

    @property
    def path(self) -> str:
        return lb_path_in_use(self.ctx)

    def close(self) -> None:
        if getattr(self, "ctx", None):
            lb_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

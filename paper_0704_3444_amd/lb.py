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
    "lb_workspace_bytes", "lb_init", "lb_step", "lb_moments", "lb_moments_noalloc", "lb_get_f", "lb_state_bytes",
    "lb_get_state", "lb_set_state", "lb_lattice_tables", "lb_path_in_use", "lb_free",
    "lb_strerror", "lb_last_error",
    "lb_batch_create", "lb_batch_footprint", "lb_batch_add", "lb_batch_step", "lb_batch_poll",
    "lb_batch_moments", "lb_batch_remove", "lb_batch_config_count", "lb_batch_config_info",
    "lb_batch_set_config", "lb_batch_tune", "lb_batch_free",
    "lb_lines_create", "lb_lines_step", "lb_lines_free",
]


class lb_params(C.Structure):
    _fields_ = [
        ("n_comp", C.c_int32), ("lattice", C.c_int32), ("storage", C.c_int32), ("force_form", C.c_int32),
        ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
        ("tau", C.c_double * MAX_COMP), ("theta", C.c_double), ("kappa", C.c_double),
        ("m", C.c_double * MAX_COMP), ("chi", C.c_double * (MAX_COMP * MAX_COMP)),
        ("path", C.c_int32), ("check_every", C.c_int32), ("stream", C.c_void_p),
        ("walls", C.c_int32), ("reserved", C.c_int32),
    ]


class lb_batch_params(C.Structure):
    _fields_ = [
        ("storage", C.c_int32), ("max_comp", C.c_int32), ("max_slots", C.c_int32), ("config", C.c_int32),
        ("graph_steps", C.c_int32), ("reserved", C.c_int32), ("arena_bytes", C.c_size_t), ("stream", C.c_void_p),
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
    # PyTorch ships its own HIP runtime (soname libamdhip64.so.7).  Loading it
    # first makes liblbm.so bind to that same runtime; loading liblbm.so first
    # would bring in a second HIP runtime, after which PyTorch finds no GPU.
    import torch  # noqa: F401

    lib = C.CDLL(LIB_PATH)
    dp, vp = C.POINTER(C.c_double), C.c_void_p
    P = C.POINTER(lb_params)
    lib.lb_workspace_bytes.argtypes = [P]
    lib.lb_workspace_bytes.restype = C.c_size_t
    lib.lb_init.argtypes = [P, dp, vp, C.c_size_t, C.POINTER(vp)]
    lib.lb_step.argtypes = [vp, C.c_int64]
    lib.lb_moments.argtypes = [vp, dp, dp, dp, dp, dp, dp, C.POINTER(C.c_int64)]
    lib.lb_moments_noalloc.argtypes = [vp, dp, dp, dp, dp, dp, dp, C.POINTER(C.c_int64)]
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
    BP, bp = C.POINTER(lb_batch_params), C.c_void_p
    i32p, i64p = C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    lib.lb_batch_create.argtypes = [BP, C.POINTER(bp)]
    lib.lb_batch_footprint.argtypes = [bp, P]
    lib.lb_batch_footprint.restype = C.c_size_t
    lib.lb_batch_add.argtypes = [bp, P, dp, C.c_int64, i32p]
    lib.lb_batch_step.argtypes = [bp, C.c_int64]
    lib.lb_batch_poll.argtypes = [bp, C.c_int32, i64p]
    lib.lb_batch_moments.argtypes = [bp, C.c_int32, dp, dp, dp, dp, dp, dp, i64p]
    lib.lb_batch_remove.argtypes = [bp, C.c_int32]
    lib.lb_batch_config_count.argtypes = [C.c_int32, C.c_int32]
    lib.lb_batch_config_info.argtypes = [C.c_int32, C.c_int32, C.c_int32, i32p, i32p, i32p, i32p]
    lib.lb_batch_set_config.argtypes = [bp, C.c_int32]
    lib.lb_batch_tune.argtypes = [bp, C.c_int32, dp, i32p]
    lib.lb_batch_free.argtypes = [bp]
    lib.lb_batch_free.restype = None
    lib.lb_lines_create.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(vp)]
    lib.lb_lines_step.argtypes = [vp, C.c_int64]
    lib.lb_lines_free.argtypes = [vp]
    lib.lb_lines_free.restype = None
    for name in ("lb_init", "lb_step", "lb_moments", "lb_moments_noalloc", "lb_get_f", "lb_get_state", "lb_set_state",
                 "lb_lattice_tables", "lb_path_in_use", "lb_batch_create", "lb_batch_add", "lb_batch_step",
                 "lb_batch_poll", "lb_batch_moments", "lb_batch_remove", "lb_batch_config_count",
                 "lb_batch_config_info", "lb_batch_set_config", "lb_batch_tune", "lb_lines_create",
                 "lb_lines_step"):
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
    theta, kappa, m, chi, force_form, and optionally walls)."""
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
    p.walls = int(cfg.get("walls", 0))
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


def lb_moments(ctx: int, n_comp: int, dim: int, sites: int, fields=True, raise_numeric=True,
               noalloc=False) -> dict:
    """lb_moments, or lb_moments_noalloc with noalloc=True."""
    out = {"mass": np.zeros(n_comp), "mom": np.zeros(dim)}
    if fields:
        out.update(rho=np.zeros((n_comp, sites)), U=np.zeros((dim, sites)), mu=np.zeros((n_comp, sites)),
                   P=np.zeros((dim * (dim + 1) // 2, sites)))
    step = C.c_int64()
    fn = load().lb_moments_noalloc if noalloc else load().lb_moments
    rc = fn(C.c_void_p(ctx), _dptr(out.get("rho")), _dptr(out.get("U")), _dptr(out.get("mu")),
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

    def moments(self, fields=True, raise_numeric=True, noalloc=False) -> dict:
        return lb_moments(self.ctx, self.n, self.D, self.sites, fields=fields, raise_numeric=raise_numeric,
                          noalloc=noalloc)

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


# ------------------------------------------------------------------ batches
def lb_batch_config_count(storage: str, max_comp: int) -> int:
    return _check(load().lb_batch_config_count(STORAGE[storage], max_comp))


def lb_batch_config_info(storage: str, max_comp: int, config: int) -> dict:
    v = [C.c_int32() for _ in range(4)]
    _check(load().lb_batch_config_info(STORAGE[storage], max_comp, config, *[C.byref(x) for x in v]))
    return {"tile": (v[0].value, v[1].value), "threads": v[2].value, "groups_per_cu": v[3].value}


class Batch:
    """Many independent D2Q9 runs stepped together by the persistent batched
    kernel (lb_batch_* of the C ABI).  Slots join with add() and leave with
    remove(); step() advances every live slot; poll() returns the step
    counters; moments() reads a finished slot's observables."""

    def __init__(self, *, storage="f32", max_comp=3, max_slots=64, arena_bytes=4 << 30, config=-1,
                 graph_steps=16, stream=None):
        bp = lb_batch_params()
        bp.storage, bp.max_comp, bp.max_slots = STORAGE[storage], int(max_comp), int(max_slots)
        bp.config, bp.graph_steps, bp.arena_bytes = int(config), int(graph_steps), int(arena_bytes)
        bp.stream = stream
        self.storage, self.max_slots, self.max_comp = storage, int(max_slots), int(max_comp)
        h = C.c_void_p()
        _check(load().lb_batch_create(C.byref(bp), C.byref(h)))
        self.h = h.value
        self.meta = {}

    def footprint(self, cfg: dict) -> int:
        p = make_params(cfg, storage=self.storage)
        return int(load().lb_batch_footprint(C.c_void_p(self.h), C.byref(p)))

    def add(self, cfg: dict, rho0: np.ndarray, nsteps: int) -> int:
        p = make_params(cfg, storage=self.storage)
        rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
        slot = C.c_int32()
        _check(load().lb_batch_add(C.c_void_p(self.h), C.byref(p), _dptr(rho0), C.c_int64(nsteps), C.byref(slot)))
        self.meta[slot.value] = (int(cfg["n_comp"]), int(np.prod(cfg["shape"])))
        return slot.value

    def try_add(self, cfg: dict, rho0: np.ndarray, nsteps: int) -> Optional[int]:
        """add(), or None when the batch has no free slot or arena range."""
        try:
            return self.add(cfg, rho0, nsteps)
        except LBError as e:
            if e.code == LB_ENOMEM:
                return None
            raise

    def step(self, n: int) -> None:
        _check(load().lb_batch_step(C.c_void_p(self.h), C.c_int64(n)))

    def poll(self, lag: int = 0) -> np.ndarray:
        out = np.zeros(self.max_slots, dtype=np.int64)
        _check(load().lb_batch_poll(C.c_void_p(self.h), lag, out.ctypes.data_as(C.POINTER(C.c_int64))))
        return out

    def moments(self, slot: int, fields=True) -> dict:
        n, sites = self.meta[slot]
        out = {"mass": np.zeros(n), "mom": np.zeros(2)}
        if fields:
            out.update(rho=np.zeros((n, sites)), U=np.zeros((2, sites)), mu=np.zeros((n, sites)),
                       P=np.zeros((3, sites)))
        step = C.c_int64()
        rc = load().lb_batch_moments(C.c_void_p(self.h), slot, _dptr(out.get("rho")), _dptr(out.get("U")),
                                     _dptr(out.get("mu")), _dptr(out.get("P")), _dptr(out["mass"]),
                                     _dptr(out["mom"]), C.byref(step))
        out["step"], out["status"] = step.value, rc
        if rc != LB_ENUMERIC:
            _check(rc)
        return out

    def remove(self, slot: int) -> None:
        _check(load().lb_batch_remove(C.c_void_p(self.h), slot))
        self.meta.pop(slot, None)

    def set_config(self, config: int) -> None:
        _check(load().lb_batch_set_config(C.c_void_p(self.h), config))

    def tune(self, steps: int = 20):
        """Time every kernel configuration on the live slots and keep the
        fastest: returns (index, ms per step of each configuration)."""
        ms = np.zeros(lb_batch_config_count(self.storage, self.max_comp))
        best = C.c_int32()
        _check(load().lb_batch_tune(C.c_void_p(self.h), steps, _dptr(ms), C.byref(best)))
        return best.value, ms

    def close(self) -> None:
        if getattr(self, "h", None):
            load().lb_batch_free(C.c_void_p(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ line groups
def lb_lines_create(ctxs) -> int:
    arr = (C.c_void_p * len(ctxs))(*ctxs)
    out = C.c_void_p()
    _check(load().lb_lines_create(arr, len(ctxs), C.byref(out)))
    return out.value


def lb_lines_step(group: int, nsteps: int) -> None:
    _check(load().lb_lines_step(C.c_void_p(group), nsteps))


def lb_lines_free(group: int) -> None:
    if group:
        load().lb_lines_free(C.c_void_p(group))


class Lines:
    """Several D1Q3 Simulations stepped together (lb_lines_* of the C ABI):
    one wavefront per run holds the whole line in registers for all the
    steps of a call.  The Simulations stay usable for moments(), get_f()
    and checkpoints, and must outlive the group."""

    def __init__(self, sims):
        self.sims = list(sims)
        self.group = lb_lines_create([s.ctx for s in self.sims])

    def step(self, n: int) -> None:
        lb_lines_step(self.group, n)

    def close(self) -> None:
        if getattr(self, "group", None):
            lb_lines_free(self.group)
            self.group = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""The C-ABI library loads and exports every function include/lb.h declares
(no device call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lb.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(lb_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("lb_init", "lb_step", "lb_moments", "lb_free", "lb_workspace_bytes", "lb_get_state",
                 "lb_set_state", "lb_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_0704_3444_amd import lb

    lib = ctypes.CDLL(lb.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(lb.EXPORTS) == declared_functions()


def test_host_side_validation_without_device():
    """Parameter validation and the workspace size are host-only calls."""
    import numpy as np
    import lbinputs as LI
    from paper_0704_3444_amd import lb

    cfg, _ = LI.binary_spinodal(16)
    p = lb.make_params(cfg, storage="f32")
    n = lb.lb_workspace_bytes(p)
    # two FP32 population copies of 2 x 9 x 256 plus scratch
    assert n >= 2 * 2 * 9 * 256 * 4
    bad = lb.make_params(dict(cfg, chi=np.array([[0, 2.4], [2.0, 0]])))
    with pytest.raises(lb.LBError):
        lb.lb_workspace_bytes(bad)
    bad = lb.make_params(dict(cfg, tau=0.5))
    with pytest.raises(lb.LBError):
        lb.lb_workspace_bytes(bad)
    p = lb.make_params(cfg)
    p.tau[1] = 1.2
    with pytest.raises(lb.LBError):
        lb.lb_workspace_bytes(p)
    assert lb.load().lb_strerror(-5).decode().startswith("non-finite")


def test_lattice_tables_match_isotropy():
    import numpy as np
    from paper_0704_3444_amd import lb

    for name, q in (("D1Q3", 3), ("D2Q9", 9), ("D3Q19", 19)):
        Q, D, v, w = lb.lb_lattice_tables(name)
        assert Q == q
        vv = v[:, :D].astype(float)
        assert abs(w.sum() - 1) < 1e-15
        assert np.allclose(np.einsum("i,ia,ib->ab", w, vv, vv), np.eye(D) / 3, atol=1e-16)

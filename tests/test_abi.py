"""The C-ABI library loads and exports every entry point include/*.h declares (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header=None):
    inc = os.path.join(ROOT, "include")
    names = set()
    for h in sorted(os.listdir(inc)) if header is None else [header]:
        if not h.endswith(".h"):
            continue
        src = re.sub(r"/\*.*?\*/", "", open(os.path.join(inc, h)).read(), flags=re.S)
        names |= set(re.findall(r"\b(pts_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("pts_assemble", "pts_newton_step", "pts_solve", "pts_solve_batched", "pts_workspace_bytes",
              "pts_last_error", "pts_window_bound"):
        assert n in names
    no = _declared("pts_no.h")
    for n in ("pts_no_forward", "pts_no_backward", "pts_no_adam", "pts_no_initial_iterate", "pts_no_gemm"):
        assert n in no


def test_library_exports_every_declared_symbol():
    import paper_2406_00878_amd as P
    lib = ctypes.CDLL(P.library_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_window_bound_reproduces_section7_example():
    """Section 7: N_x = 64, mu = 1e-3, c = 1, eps = 1e-16 and tau = 1/N_t give 22 levels."""
    import paper_2406_00878_amd as P
    assert P.window_bound(1.0 / 64, 1e-3, tau=0.0, c=1.0, eps=1e-16) == 22


def test_window_bound_matches_oracle_estimate():
    import paper_2406_00878_amd as P
    from oracle import condition
    for nx, mu in [(32, 1e-2), (64, 1e-3), (128, 5e-4)]:
        assert P.window_bound(1.0 / nx, mu) == condition.max_levels_eq_cond(nx, mu)


def test_workspace_and_validation_on_host():
    import paper_2406_00878_amd as P
    import workloads as W
    p = W.heat32()
    st = P.make_problem(p)
    lib = P._lib.load()
    assert lib.pts_workspace_bytes(ctypes.byref(st)) >= 2 * 8 * p.dof
    st.nx = 0
    assert lib.pts_workspace_bytes(ctypes.byref(st)) == 0
    assert b"sizes" in lib.pts_last_error()


def test_neural_config_validation_on_host():
    """Parameter count follows the documented layout; invalid widths are rejected."""
    import paper_2406_00878_amd.neural as N
    cfg = N.NOConfig(64, 64, 16, width=32, modes=8, layers=2)
    lib = N._lib()
    c = cfg.c()
    import numpy as np
    assert lib.pts_no_param_count(ctypes.byref(c)) == sum(int(np.prod(s)) for _, s in cfg.layout())
    assert lib.pts_no_workspace_bytes(ctypes.byref(c)) > 0
    bad = N.NOConfig(64, 64, 16, width=24).c()
    assert lib.pts_no_param_count(ctypes.byref(bad)) == 0


def test_solver_option_validation_on_host():
    """Out-of-range launch options are rejected before any device work (host-side checks)."""
    import paper_2406_00878_amd as P
    import workloads as W
    p = P.make_problem(W.burgers_periodic(32, 4, 5e-4, 0.01, W.fourier_u0_periodic(32, 1)))
    lib = P._lib.load()
    opts = P._options()
    opts.wave_launch = 2
    rc = lib.pts_solve(ctypes.byref(p), None, None, 1e-12, 10, None, 0, ctypes.byref(opts), None, None)
    assert rc == P._lib.PTS_ERR_INVALID_ARG and b"wave_launch" in lib.pts_last_error()
    opts = P._options(barrier_spins=-1)
    rc = lib.pts_solve(ctypes.byref(p), None, None, 1e-12, 10, None, 0, ctypes.byref(opts), None, None)
    assert rc == P._lib.PTS_ERR_INVALID_ARG and b"negative" in lib.pts_last_error()
    with pytest.raises(KeyError):
        P._options(wave_launch="persistent")


def test_coarse_workspace_bytes_validates_on_host():
    """pts_coarse_workspace_bytes is host-only: 0 for cf < 2, for fewer than 3 periodic or 1
    Dirichlet coarse nodes, and for Dirichlet data on grids cf does not divide; grids that cf
    does not divide are otherwise accepted."""
    import paper_2406_00878_amd as P
    import workloads as W
    lib = P._lib.load()
    q = W.burgers_periodic(32, 8, 5e-4, 0.01, np.zeros((32, 32)))
    p = P.make_problem(q)
    assert lib.pts_coarse_workspace_bytes(ctypes.byref(p), 4) > 0
    assert lib.pts_coarse_workspace_bytes(ctypes.byref(p), 3) > 0  # 10 coarse nodes, 3 levels
    assert lib.pts_coarse_workspace_bytes(ctypes.byref(p), 1) == 0
    assert lib.pts_coarse_workspace_bytes(ctypes.byref(p), 11) == 0  # 2 coarse nodes
    h = W.heat_dirichlet(31, 12, 1e-3, np.zeros((31, 31)))
    ph = P.make_problem(h)
    assert lib.pts_coarse_workspace_bytes(ctypes.byref(ph), 4) > 0
    assert lib.pts_coarse_workspace_bytes(ctypes.byref(ph), 5) > 0  # 5 coarse nodes
    assert lib.pts_coarse_workspace_bytes(ctypes.byref(ph), 17) == 0  # no coarse node
    ph.bdata = 256  # host check only: the address is never read
    assert lib.pts_coarse_workspace_bytes(ctypes.byref(ph), 4) > 0
    assert lib.pts_coarse_workspace_bytes(ctypes.byref(ph), 5) == 0
    assert b"Dirichlet data" in lib.pts_last_error()
    # per-instance problems of different sizes
    arr = (P.pts_problem * 2)(P.make_problem(h), P.make_problem(W.heat_dirichlet(50, 9, 1e-3, np.zeros((50, 50)))))
    assert lib.pts_coarse_workspace_bytes_batched(arr, 2, 4) > lib.pts_coarse_workspace_bytes(ctypes.byref(arr[0]), 4)


def test_binding_error_codes_match_the_header():
    """Every PTS_OK / PTS_ERR_* value of include/pts.h (PTS_ERR_NOT_DOMINANT included) is the
    binding's constant of the same name, and the codes are distinct."""
    import paper_2406_00878_amd._lib as L
    src = open(os.path.join(ROOT, "include", "pts.h")).read()
    codes = dict((n, int(v)) for n, v in re.findall(r"\b(PTS_(?:OK|ERR_[A-Z_]+))\s*=\s*(-?\d+)", src))
    assert codes["PTS_ERR_NOT_DOMINANT"] == -7 and len(codes) == 8, codes
    for n, v in codes.items():
        assert getattr(L, n, None if n != "PTS_OK" else 0) == v, n
    assert len(set(codes.values())) == len(codes)

"""The C-ABI library loads and exports every entry point include/pts.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pts.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pts_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("pts_assemble", "pts_newton_step", "pts_solve", "pts_solve_batched", "pts_workspace_bytes",
              "pts_last_error", "pts_window_bound"):
        assert n in names


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

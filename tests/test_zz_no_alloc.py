"""pts_newton_step_static (no allocation, the library's static device scratch) against
pts_newton_step with a caller workspace, through the C ABI: the same Newton steps element by
element, on two calls in a row whose second problem is smaller (the scratch keeps the first
call's contents)."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _cases():
    rng = np.random.default_rng(21)
    big = W.heat_dirichlet(72, 10, 1e-3, W.sine_u0_dirichlet(72, rng))          # 2 x 2 regions, ragged
    small = W.burgers_periodic(40, 4, 5e-4, 0.01, W.fourier_u0_periodic(40, 5))  # smaller, other kind
    return [big, small]


def test_static_step_equals_workspace_step_on_two_calls():
    import paper_2406_00878_amd as P
    dev = torch.device("cuda:0")
    for p in _cases():
        print(f"static step: kind {p.kind} {p.nx}x{p.ny}x{p.nt}", flush=True)
        u0 = torch.as_tensor(p.u0, device=dev)
        Ua = torch.as_tensor(p.plain_iterate(), device=dev)
        Ub = Ua.clone()
        for k in range(2):  # two Newton steps each way
            sa = P.newton_step(p, Ua, u0, schedule="bulk")
            sb = P.newton_step_static(p, Ub, u0, schedule="bulk")
            torch.cuda.synchronize()
            assert sa["res_inf"][0] == sb["res_inf"][0]
            a, b = Ua.cpu().numpy(), Ub.cpu().numpy()
            assert np.all(np.isfinite(b))
            err = float(np.max(np.abs(a - b)) / np.max(np.abs(a)))
            assert err <= 1e-13, (p.nx, k, err)


def test_static_step_rejects_oversized_problem():
    import paper_2406_00878_amd as P
    lib = P._lib.load()
    p = W.heat_dirichlet(512, 64, 1e-3, np.zeros((512, 512)))
    st = P.make_problem(p)
    U = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    o = P._options()
    rc = lib.pts_newton_step_static(ctypes.byref(st), ctypes.c_void_p(U.data_ptr()),
                                    ctypes.c_void_p(U.data_ptr()), ctypes.byref(o), None, None)
    assert rc == P._lib.PTS_ERR_WORKSPACE
    assert b"static" in lib.pts_last_error()

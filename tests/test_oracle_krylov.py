"""Pins of the oracle's large-level path (BiCGSTAB branch) and of its convergence checks.

Every full-size reference (levels above 128^2 nodes) goes through the BiCGSTAB branch of
sequential.linear_solve, so that branch is pinned here on its own: against the closed-form
decay of linear heat (eigenvalues of Section 7), and against an exact sparse LU of the same
level matrices (heat, stiff Dirichlet heat and periodic Burgers, 130^2-140^2 nodes).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import sequential
from oracle.discretization import level_jacobian, level_residual


def test_periodic_linear_heat_decay_through_bicgstab():
    """Periodic linear heat on 136^2 nodes (above the LU limit): cos(2 pi k.x) decays by
    1/(1 + tau mu lambda) per level, lambda = (4/h^2)(sin^2(pi kx h) + sin^2(pi ky h))."""
    n, kx, ky, mu, dt, nt = 136, 3, 5, 0.4, 1e-3, 4
    assert n * n > sequential.LU_MAX_NS
    h = 1.0 / n
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    u0 = np.cos(2 * math.pi * (kx * X + ky * Y))
    p = W.Problem(W.HEAT, W.PERIODIC, n, n, nt, h, h, dt, mu, 0.0, u0)
    lam = 4.0 / h ** 2 * (math.sin(math.pi * kx * h) ** 2 + math.sin(math.pi * ky * h) ** 2)
    U, _ = sequential.solve_sequential(p)
    for lvl in range(nt):
        np.testing.assert_allclose(U[lvl], u0 / (1.0 + dt * mu * lam) ** (lvl + 1), rtol=0, atol=1e-13)


def test_dirichlet_linear_heat_decay_through_bicgstab():
    """Zero-Dirichlet linear heat on 131^2 nodes at tau mu / h^2 = 17 (stiff): the sine mode
    decays by 1/(1 + tau mu lambda), lambda = (4/h^2)(sin^2(pi kx h/2) + sin^2(pi ky h/2))."""
    n, kx, ky, mu, dt, nt = 131, 2, 1, 1.0, 1e-3, 3
    h = 1.0 / (n + 1)
    x = (np.arange(n) + 1.0) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    u0 = np.sin(math.pi * kx * X) * np.sin(math.pi * ky * Y)
    p = W.heat_dirichlet(n, nt, dt, u0, mu_a=mu, mu_b=0.0)
    lam = 4.0 / h ** 2 * (math.sin(math.pi * kx * h / 2) ** 2 + math.sin(math.pi * ky * h / 2) ** 2)
    U, _ = sequential.solve_sequential(p)
    for lvl in range(nt):
        np.testing.assert_allclose(U[lvl], u0 / (1.0 + dt * mu * lam) ** (lvl + 1), rtol=0, atol=1e-13)


def _level(case):
    rng = np.random.default_rng(5)
    if case == "heat_stiff":  # the heat batch's blocks: k(u) = 1 + u^2, tau/h^2 = 19.6
        n = 139
        p = W.heat_dirichlet(n, 1, 1e-3, W.sine_u0_dirichlet(n, rng))
    elif case == "burgers_periodic":  # the Burgers workloads' blocks
        n = 130
        p = W.burgers_periodic(n, 1, 5e-4, 0.01, W.fourier_u0_periodic(n, 7))
    else:  # variable-viscosity heat on a periodic grid
        n = 132
        p = W.Problem(W.HEAT, W.PERIODIC, n, n, 1, 1.0 / n, 1.0 / n, 2e-4, 0.5, 1.0,
                      W.fourier_u0_periodic(n, 9, kmax=5))
    assert p.ns > sequential.LU_MAX_NS
    return p, p.u0 + 0.05 * rng.standard_normal(p.u0.shape)


@pytest.mark.parametrize("case", ["heat_stiff", "burgers_periodic", "heat_periodic_varvisc"])
def test_bicgstab_solve_equals_exact_lu(case):
    """One Newton correction of a level above the LU limit: BiCGSTAB equals the exact sparse LU
    of the same matrix to 1e-12 relative."""
    p, v = _level(case)
    G = level_residual(v, p.u0, p)
    A = level_jacobian(v, p)
    d_k = sequential.linear_solve(A, -G.ravel())  # default branch for this size: BiCGSTAB
    d_lu = sequential.linear_solve(A, -G.ravel(), method="lu")
    assert np.max(np.abs(d_k - d_lu)) <= 1e-12 * np.max(np.abs(d_lu))
    assert np.max(np.abs(A @ d_k + G.ravel())) <= 1e-12 * np.max(np.abs(G))


@pytest.mark.parametrize("case", ["heat_stiff", "burgers_periodic"])
def test_bdf1_step_same_root_on_both_branches(case):
    """A whole BDF1 level solved with BiCGSTAB corrections and with exact LU corrections reaches
    the same root (to 1e-13 relative) and meets the tolerance."""
    p, _ = _level(case)
    u_k, it_k, h_k = sequential.bdf1_step(p.u0, p, 1)
    u_lu, it_lu, h_lu = sequential.bdf1_step(p.u0, p, 1, method="lu")
    assert h_k[-1] <= 1e-13 or h_k[-1] <= sequential.roundoff_floor(u_k, p.u0, p)
    assert np.max(np.abs(u_k - u_lu)) <= 1e-13 * np.max(np.abs(u_lu))


def test_unconverged_level_raises():
    """maxit steps without reaching tol raise instead of returning the last iterate."""
    p = W.heat32(nt=1)
    with pytest.raises(sequential.OracleNotConverged):
        sequential.bdf1_step(p.u0, p, 1, tol=1e-13, maxit=1)


def test_stall_above_roundoff_raises(monkeypatch):
    """A Newton iteration that stops decreasing far above the roundoff floor raises (a planted
    mistake: the Jacobian's sign flipped, so every correction points uphill)."""
    p = W.heat32(nt=1)
    real = sequential.level_jacobian
    monkeypatch.setattr(sequential, "level_jacobian", lambda v, q, bv=None, tau=None: -real(v, q, bv, tau))
    with pytest.raises(sequential.OracleNotConverged):
        sequential.bdf1_step(p.u0, p, 1)


def test_stall_at_roundoff_is_accepted():
    """tol = 0 cannot be met; the iteration ends at the roundoff floor and is accepted."""
    p = W.heat32(nt=1)
    u, it, hist = sequential.bdf1_step(p.u0, p, 1, tol=0.0)
    assert min(hist) <= sequential.roundoff_floor(u, p.u0, p)
    u_ref, _, _ = sequential.bdf1_step(p.u0, p, 1)
    assert np.max(np.abs(u - u_ref)) <= 1e-14

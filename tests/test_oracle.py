"""Pins of the CPU oracle against facts fixed outside it.

Each test names what fixes the expected value: a number printed in the paper,
a closed form, an invariant, or a library routine applied to a special case.
"""
import dataclasses
import math
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import allatonce, condition, sequential
from oracle.discretization import (jacobian_stencil, level_jacobian, level_residual,
                                   stencil_to_sparse)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(v) for v in line.split()])
    return rows


def _round_sig(x, digits):
    return float(f"{x:.{digits - 1}e}")


# ----------------------------------------------------------- paper's tables

@pytest.mark.parametrize("row", _golden("table1_heat_linf.txt"), ids=lambda r: f"N{int(r[0])}")
def test_table1_heat_error_reproduced(row):
    """Section 8.1, Table 1: the L-inf error of sequential BDF1 to the printed 3 digits."""
    nint, expected = int(row[0]), row[1]
    p = W.heat_mms(nint)
    U, _ = sequential.solve_sequential(p, tol=1e-13)
    X, Y = p.mesh()
    err = max(np.max(np.abs(U[n] - W.heat_exact(X, Y, (n + 1) * p.dt))) for n in range(p.nt))
    assert _round_sig(err, 3) == pytest.approx(expected, rel=1e-9)


@pytest.mark.parametrize("row", [r for r in _golden("table4_burgers_l1.txt") if r[2] == 1],
                         ids=lambda r: f"N{int(r[0])}")
def test_table4_burgers_error_reproduced(row):
    """Section 8.2, Table 4 (three finest grids): L1 error within 1% on [-0.5,0.5]^2."""
    nint, expected = int(row[0]), row[1]
    p = W.burgers_mms(nint, x0=-0.5, y0=-0.5)
    U, _ = sequential.solve_sequential(p, tol=1e-13)
    X, Y = p.mesh()
    err = sum(np.sum(np.abs(U[n] - W.burgers_exact(X, Y, (n + 1) * p.dt)))
              for n in range(p.nt)) * p.hx * p.hy * p.dt
    assert err == pytest.approx(expected, rel=1e-2)


def test_condition_example_gives_22_levels():
    """Section 7: N_x = 64, mu = 1e-3, c = 1 allows at most 22 levels."""
    assert condition.max_levels_eq_cond(64, 1e-3, c=1.0, eps_rof=1e-16) == 22


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("n,kx,ky", [(7, 1, 1), (12, 2, 3), (9, 4, 1)])
def test_linear_heat_dirichlet_fourier_decay(n, kx, ky):
    """Linear heat (mu_b = 0), zero Dirichlet: sin modes decay by 1/(1 + tau mu lambda)
    per level, lambda the five-point Laplacian eigenvalue of Section 7."""
    mu, dt, nt = 0.7, 2e-3, 6
    h = 1.0 / (n + 1)
    x = (np.arange(n) + 1.0) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    u0 = np.sin(math.pi * kx * X) * np.sin(math.pi * ky * Y)
    p = W.heat_dirichlet(n, nt, dt, u0, mu_a=mu, mu_b=0.0)
    lam = 4.0 / h ** 2 * (math.sin(math.pi * kx * h / 2) ** 2 + math.sin(math.pi * ky * h / 2) ** 2)
    U, _ = sequential.solve_sequential(p)
    for lvl in range(nt):
        expect = u0 / (1.0 + dt * mu * lam) ** (lvl + 1)
        np.testing.assert_allclose(U[lvl], expect, rtol=0, atol=1e-14)


@pytest.mark.parametrize("n,kx,ky", [(8, 1, 0), (10, 2, 3)])
def test_linear_heat_periodic_fourier_decay(n, kx, ky):
    """Periodic linear heat: cos(2 pi k.x) decays by 1/(1 + tau mu lambda),
    lambda = (4/h^2)(sin^2(pi kx h) + sin^2(pi ky h))."""
    mu, dt, nt = 0.3, 1e-3, 5
    h = 1.0 / n
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    u0 = np.cos(2 * math.pi * (kx * X + ky * Y))
    p = W.Problem(W.HEAT, W.PERIODIC, n, n, nt, h, h, dt, mu, 0.0, u0)
    lam = 4.0 / h ** 2 * (math.sin(math.pi * kx * h) ** 2 + math.sin(math.pi * ky * h) ** 2)
    U, _ = sequential.solve_sequential(p)
    for lvl in range(nt):
        np.testing.assert_allclose(U[lvl], u0 / (1.0 + dt * mu * lam) ** (lvl + 1), atol=1e-14)


def test_burgers_linearized_mode():
    """Burgers about a constant state c: a small Fourier mode moves with the central-difference
    symbol, amplification 1/(1 + tau[i c (sin 2pi kx h + sin 2pi ky h)/h + nu lambda])."""
    n, nt, dt, nu, c, eps = 16, 8, 2e-3, 0.02, 0.8, 1e-7
    kx, ky = 2, 1
    h = 1.0 / n
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    theta = 2 * math.pi * (kx * X + ky * Y)
    p = W.burgers_periodic(n, nt, dt, nu, c + eps * np.cos(theta))
    lam = 4.0 / h ** 2 * (math.sin(math.pi * kx * h) ** 2 + math.sin(math.pi * ky * h) ** 2)
    sym = 1j * c * (math.sin(2 * math.pi * kx * h) + math.sin(2 * math.pi * ky * h)) / h + nu * lam
    g = 1.0 / (1.0 + dt * sym)
    U, _ = sequential.solve_sequential(p)
    for lvl in range(nt):
        expect = np.real(g ** (lvl + 1) * np.exp(1j * theta))
        np.testing.assert_allclose((U[lvl] - c) / eps, expect, atol=2e-6)


@pytest.mark.parametrize("b", [0.0, 0.37])
def test_single_node_heat_step_is_cubic_root(b):
    """One interior node with Dirichlet value b on all sides: the BDF1 equation is the cubic
    u - u_prev + 4 tau mu((u+b)/2)(u-b)/h^2 = 0, solved here with numpy.roots."""
    mu_a, mu_b, dt, h, uprev = 0.2, 1.3, 0.05, 0.5, 0.9
    p = W.Problem(W.HEAT, W.DIRICHLET, 1, 1, 1, h, h, dt, mu_a, mu_b,
                  np.array([[uprev]]), np.full((1, 4), b))
    U, _ = sequential.solve_sequential(p, tol=1e-15)
    # 4 tau/h^2 (mu_a + mu_b (u+b)^2/4)(u - b) + u - uprev as a polynomial in u
    k = 4.0 * dt / h ** 2
    poly = np.polynomial.Polynomial
    u = poly([0.0, 1.0])
    expr = k * (mu_a + mu_b * (u + b) ** 2 / 4.0) * (u - b) + u - uprev
    roots = np.roots(expr.coef[::-1])
    real = roots[np.abs(roots.imag) < 1e-12].real
    assert len(real) == 1
    assert U[0, 0, 0] == pytest.approx(real[0], abs=1e-14)


# --------------------------------------------------------------- invariants

def test_periodic_burgers_conserves_sum():
    """Central flux differences and the conservative viscous form telescope on a periodic grid."""
    p = W.burgers_periodic(12, 6, 5e-3, 0.01, W.fourier_u0_periodic(12, 7))
    U, _ = sequential.solve_sequential(p)
    s0 = p.u0.sum()
    for lvl in range(p.nt):
        assert U[lvl].sum() == pytest.approx(s0, abs=1e-12)


def test_constant_state_is_steady():
    p = W.burgers_periodic(8, 3, 1e-2, 0.01, np.full((8, 8), 0.6))
    for bc_kind in (W.BURGERS, W.HEAT):
        p.kind = bc_kind
        G = level_residual(p.u0, p.u0, p)
        assert np.max(np.abs(G)) == 0.0


def test_heat_symmetry_preserved():
    """u0 = sin(pi x) sin(pi y) is symmetric under x <-> y and x -> 1 - x; so is the solution."""
    p = W.heat32(nt=4)
    U, _ = sequential.solve_sequential(p)
    for lvl in range(p.nt):
        np.testing.assert_allclose(U[lvl], U[lvl].T, atol=1e-14)
        np.testing.assert_allclose(U[lvl], U[lvl][:, ::-1], atol=1e-14)


# --------------------------------------------------------------- Jacobian

def _complex_step_jacobian(u, uprev, p, bvals):
    ns = u.size
    Jc = np.zeros((ns, ns))
    hstep = 1e-30
    for k in range(ns):
        v = u.astype(np.complex128).ravel()
        v[k] += 1j * hstep
        G = level_residual(v.reshape(u.shape), uprev, p, bvals)
        Jc[:, k] = G.imag.ravel() / hstep
    return Jc


@pytest.mark.parametrize("case", ["heat_dirichlet", "heat_periodic", "burgers_dirichlet",
                                  "burgers_periodic", "burgers_periodic_3x5"])
def test_jacobian_matches_complex_step(case):
    """A = I + tau dF/du equals the complex-step derivative of G at every point type
    (interior, edge, corner, periodic wrap, short periodic rows with repeated neighbours)."""
    rng = np.random.default_rng(11)
    kind = W.HEAT if case.startswith("heat") else W.BURGERS
    bc = W.PERIODIC if "periodic" in case else W.DIRICHLET
    nx, ny = (3, 5) if case.endswith("3x5") else (5, 4)
    u = rng.uniform(-1, 1.5, size=(ny, nx))
    mu_b = 0.7 if kind == W.HEAT else 0.0
    p = W.Problem(kind, bc, nx, ny, 1, 0.3, 0.2, 0.05, 0.4, mu_b, u)
    bvals = rng.uniform(-1, 1, size=2 * (nx + ny)) if bc == W.DIRICHLET else None
    J = level_jacobian(u, p, bvals).toarray()
    Jc = _complex_step_jacobian(u, rng.uniform(size=u.shape), p, bvals)
    np.testing.assert_allclose(J, Jc, rtol=1e-13, atol=1e-13)


# ------------------------------------------------------ all-at-once system

def _tiny_problems():
    rng = np.random.default_rng(3)
    heat = W.heat_dirichlet(4, 5, 2e-3, rng.uniform(0, 1, (4, 4)))
    burg = W.burgers_periodic(6, 6, 4e-3, 0.02, W.fourier_u0_periodic(6, 5))
    mms = W.heat_mms(5)
    return [heat, burg, mms]


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_global_newton_step_forms_agree(idx):
    """One Newton step of Eq. (6): dense LU of the full space-time Jacobian (numpy) equals
    the sparse LU, the block inverse of Eq. (7) and Theorem 1's decoupled system (Eq. (8))."""
    p = _tiny_problems()[idx]
    rng = np.random.default_rng(idx)
    U = p.plain_iterate() + 0.05 * rng.standard_normal((p.nt, p.ny, p.nx))
    M = allatonce.global_jacobian(U, p).toarray()
    R = allatonce.global_residual(U, p)
    dense = np.linalg.solve(M, R.ravel()).reshape(U.shape)
    scale = np.max(np.abs(dense))
    for step in (allatonce.newton_step_direct, allatonce.newton_step_inverse):
        dU, _ = step(U, p)
        assert np.max(np.abs(dU - dense)) <= 1e-12 * scale
    for window in (None, 1, 2, 3):
        dU, _ = allatonce.newton_step_theorem1(U, p, window)
        assert np.max(np.abs(dU - dense)) <= 1e-10 * scale


def test_product_matrix_diagonal_count():
    """Section 5 remark: for n < N_x = N_y, P^n = A_1 ... A_n has 2n^2 + 2n + 1 nonzero diagonals."""
    n = 10
    rng = np.random.default_rng(5)
    p = W.heat_dirichlet(n, 5, 1e-3, rng.uniform(0.5, 1, (n, n)))
    P = None
    for lvl in range(1, 5):
        A = level_jacobian(rng.uniform(0.5, 1.0, (n, n)), p).toarray()
        P = A if P is None else P @ A
        rows, cols = np.nonzero(np.abs(P) > 0)
        assert len(np.unique(cols - rows)) == 2 * lvl * lvl + 2 * lvl + 1


def test_allatonce_equals_sequential_heat():
    p = W.heat_dirichlet(8, 10, 1e-3, np.zeros((8, 8)))
    X, Y = p.mesh()
    p.u0 = np.sin(math.pi * X) * np.sin(math.pi * Y) + 0.3 * np.sin(2 * math.pi * X) * np.sin(math.pi * Y)
    Us, _ = sequential.solve_sequential(p)
    Ua, rh, _ = allatonce.solve_allatonce(p, tol=1e-13)
    assert rh[-1] <= 1e-13
    assert np.max(np.abs(Ua - Us)) <= 1e-12 * np.max(np.abs(Us))


def test_allatonce_equals_sequential_burgers():
    p = W.burgers_periodic(16, 12, 5e-3, 0.01, W.fourier_u0_periodic(16, 2))
    Us, _ = sequential.solve_sequential(p)
    Ua, rh, _ = allatonce.solve_allatonce(p, tol=1e-13)
    assert np.max(np.abs(Ua - Us)) <= 1e-12 * np.max(np.abs(Us))


def test_global_newton_converges_quadratically():
    """Section 4: the all-at-once Newton keeps the quadratic rate of sequential Newton."""
    p = W.heat32(nt=16)
    _, rh, _ = allatonce.solve_allatonce(p, tol=1e-15, maxit=12)
    # ratios r_{k+1} / r_k^2 stay bounded while above the roundoff floor
    ratios = [rh[k + 1] / rh[k] ** 2 for k in range(len(rh) - 1) if rh[k + 1] > 1e-13]
    assert len(ratios) >= 2
    assert max(ratios[1:]) < 50.0
    assert rh[-1] < 1e-13


# --------------------------------------------- coarse-grid initial iterate (Section 4)
def _field_problem(bc, n, nt, dt=1e-2):
    if bc == "periodic":
        return W.burgers_periodic(n, nt, dt, 0.01, np.zeros((n, n)))
    return W.heat_dirichlet(n, nt, dt, np.zeros((n, n)))


def _sample(p, f, t):
    X, Y = p.mesh()
    return f(X, Y, t)


@pytest.mark.parametrize("bc,f", [
    ("periodic", lambda x, y, t: (1.0 + 2.0 * t) * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) + 0.3),
    ("dirichlet", lambda x, y, t: (1.0 - t) * np.sin(np.pi * x) * np.sin(np.pi * y)),
])
def test_coarse_interpolation_is_fourth_order_and_exact_at_coarse_nodes(bc, f):
    """Cubic splines: interpolation property at coarse nodes, and the error on smooth data falls
    at least 12-fold per halving of the coarse spacing (O(h^4)); data linear in t is interpolated
    in time without error, so the error is the spatial one."""
    from oracle import coarse
    errs = []
    for n in ((32, 64) if bc == "periodic" else (31, 63)):
        cf = 4
        p = _field_problem(bc, n, 8)
        p = dataclasses.replace(p, u0=_sample(p, f, 0.0))
        pc = coarse.coarse_problem(p, cf)
        Uc = np.stack([_sample(pc, f, (m + 1) * pc.dt) for m in range(pc.nt)])
        U = coarse.interpolate(p, cf, Uc)
        exact = np.stack([_sample(p, f, (n1 + 1) * p.dt) for n1 in range(p.nt)])
        # fine levels m cf hold the coarse levels at the coarse nodes exactly
        sl = (slice(None, None, cf), slice(None, None, cf)) if bc == "periodic" else \
            (slice(cf - 1, None, cf), slice(cf - 1, None, cf))
        for m in range(pc.nt):
            np.testing.assert_allclose(U[(m + 1) * cf - 1][sl][:pc.ny, :pc.nx], Uc[m], rtol=0, atol=1e-13)
        errs.append(np.max(np.abs(U - exact)))
    ratio = errs[0] / errs[1]  # about 16 for O(h^4); an O(h^2) or O(h) defect gives 4 or 2
    assert ratio > 12.0, (errs, ratio)
    assert errs[1] < 2e-4, errs


def test_coarse_problem_sizes_and_injection():
    from oracle import coarse
    rng = np.random.default_rng(3)
    p = W.heat_dirichlet(31, 12, 1e-3, W.sine_u0_dirichlet(31, rng))
    pc = coarse.coarse_problem(p, 4)
    assert (pc.nx, pc.ny, pc.nt) == (7, 7, 3) and pc.dt == 4e-3 and pc.hx == 4 * p.hx
    # coarse interior node k sits at (k + 1) 4 h: the same physical points as fine node 4(k+1) - 1
    np.testing.assert_array_equal(pc.x_nodes(), p.x_nodes()[3::4])
    np.testing.assert_array_equal(pc.u0, p.u0[3::4, 3::4])
    q = W.burgers_periodic(32, 8, 5e-4, 0.01, W.fourier_u0_periodic(32, 4, kmax=3))
    qc = coarse.coarse_problem(q, 4)
    assert (qc.nx, qc.nt) == (8, 2)
    np.testing.assert_array_equal(qc.x_nodes(), q.x_nodes()[::4])
    # grids and levels that cf does not divide: the same domain with floor(32 / 3) = 10 nodes,
    # ceil(8 / 3) = 3 levels of step 3 tau
    q3 = coarse.coarse_problem(q, 3)
    assert (q3.nx, q3.ny, q3.nt) == (10, 10, 3) and q3.dt == 3 * q.dt
    assert abs(q3.nx * q3.hx - 1.0) < 1e-15
    p5 = coarse.coarse_problem(p, 5)  # 32 / 5: 5 interior nodes spaced 1 / 6
    assert (p5.nx, p5.nt) == (5, 3) and abs(p5.hx - 1.0 / 6.0) < 1e-15
    with pytest.raises(ValueError):  # Dirichlet data need nesting grids
        coarse.coarse_problem(dataclasses.replace(p, bdata=np.zeros((12, 4 * 31))), 5)
    with pytest.raises(ValueError):
        coarse.coarse_problem(q, 11)  # fewer than 3 coarse nodes


@pytest.mark.parametrize("bc,n", [("dirichlet", 50), ("periodic", 45)])
def test_coarse_sample_is_bilinear_and_injects_on_nesting_grids(bc, n):
    """u^0 on coarse nodes that are no fine nodes: the bilinear interpolant, exact for fields
    a + b x + c y + d x y (periodic: on the nodes whose interval does not wrap); on grids that
    nest, the fine values themselves."""
    from oracle import coarse
    f = lambda x, y: 0.3 + 1.7 * x - 0.6 * y + 2.2 * x * y
    p = _field_problem(bc, n, 8)
    p = dataclasses.replace(p, u0=_sample(p, lambda x, y, t: f(x, y), 0.0))
    pc = coarse.coarse_problem(p, 4)
    Xc, Yc = pc.mesh()
    inner = Xc < (n - 1) * p.hx + 1e-12  # periodic: no wrap into x = 1
    inner &= Yc < (n - 1) * p.hy + 1e-12
    np.testing.assert_allclose(pc.u0[inner], f(Xc, Yc)[inner], rtol=0, atol=1e-14)
    m = 4 * (n // 4) - (1 if bc == "dirichlet" else 0)  # a grid that nests
    q = _field_problem(bc, m, 8)
    q = dataclasses.replace(q, u0=np.random.default_rng(1).standard_normal((m, m)))
    qc = coarse.coarse_problem(q, 4)
    sl = slice(None, None, 4) if bc == "periodic" else slice(3, None, 4)
    np.testing.assert_array_equal(qc.u0, q.u0[sl, sl][:qc.ny, :qc.nx])


def test_coarse_interpolation_on_grids_that_do_not_nest_reproduces_cubics():
    """Dirichlet grid 50^2 and 10 levels with cf = 4 (11 coarse nodes spaced 51 h / 12, three
    coarse levels reaching 12 tau): the field g(t) x(1-x)(1+x) y(1-y)(2-y), cubic in x, y and t
    and zero on the boundary, is recovered at every fine node and level (the coarse spacing,
    the edges, the t = 0 node and the coarse level past the end all enter)."""
    from oracle import coarse
    g = lambda t: 1.0 + 3.0 * t - 40.0 * t * t + 500.0 * t ** 3
    f = lambda x, y, t: g(t) * x * (1 - x) * (1 + x) * y * (1 - y) * (2 - y)
    p = _field_problem("dirichlet", 50, 10, dt=1e-2)
    p = dataclasses.replace(p, u0=_sample(p, f, 0.0))
    pc = coarse.coarse_problem(p, 4)
    assert (pc.nx, pc.nt) == (11, 3)
    Uc = np.stack([_sample(pc, f, (m + 1) * pc.dt) for m in range(pc.nt)])
    U = coarse.interpolate(p, 4, Uc)
    exact = np.stack([_sample(p, f, (k + 1) * p.dt) for k in range(p.nt)])
    np.testing.assert_allclose(U, exact, rtol=0, atol=1e-13)


def test_periodic_interpolation_on_grids_that_do_not_nest_is_fourth_order():
    """Periodic grids 45^2 and 90^2 with cf = 4 (11 and 22 coarse nodes): the spline error of a
    smooth field falls about 16-fold per halving of the coarse spacing (a misplaced coarse node
    would leave an O(h) error)."""
    from oracle import coarse
    f = lambda x, y, t: (1.0 + t) * np.sin(2 * np.pi * x + 0.3) * np.cos(2 * np.pi * y) + 0.2
    errs = []
    for n in (45, 90):
        p = _field_problem("periodic", n, 6)
        p = dataclasses.replace(p, u0=_sample(p, f, 0.0))
        pc = coarse.coarse_problem(p, 4)
        Uc = np.stack([_sample(pc, f, (m + 1) * pc.dt) for m in range(pc.nt)])
        U = coarse.interpolate(p, 4, Uc)
        exact = np.stack([_sample(p, f, (k + 1) * p.dt) for k in range(p.nt)])
        errs.append(np.max(np.abs(U - exact)))
    assert errs[0] / errs[1] > 12.0, errs


def test_coarse_initial_iterate_is_close_to_the_solution():
    """The coarse start is an approximation of the fine solution (the Newton root): on smooth
    heat its error is far below the plain start's (the paper's reason for using it)."""
    from oracle import coarse
    rng = np.random.default_rng(5)
    p = W.heat_dirichlet(31, 16, 2e-3, W.sine_u0_dirichlet(31, rng))
    Ug, _ = coarse.coarse_initial_iterate(p, 4)
    Uo, _ = sequential.solve_sequential(p)
    e_coarse = np.max(np.abs(Ug - Uo))
    e_plain = np.max(np.abs(p.plain_iterate() - Uo))
    assert e_coarse < 0.1 * e_plain, (e_coarse, e_plain)


def test_coarse_interpolation_with_dirichlet_data_reproduces_cubic_fields():
    """Not-a-knot cubic splines reproduce cubic data exactly: with u = 1 + x^3 + 2y^2 - x y + 3t
    - t^2 on the grid and its boundary, every fine node and level is recovered (the edge values
    enter the x lines from the coarse west/east data and the y lines from the fine south/north
    data; natural ends, or a dropped edge, would leave an error)."""
    from oracle import coarse
    f = lambda x, y, t: 1.0 + x ** 3 + 2.0 * y ** 2 - x * y + 3.0 * t - t ** 2
    p = W.heat_dirichlet(23, 12, 1e-2, np.zeros((23, 23)))
    X, Y = p.mesh()
    p = dataclasses.replace(p, u0=f(X, Y, 0.0),
                            bdata=W.boundary_data(p, f, [(n + 1) * p.dt for n in range(p.nt)]))
    pc = coarse.coarse_problem(p, 4)
    assert pc.bdata.shape == (3, 2 * (pc.nx + pc.ny))
    np.testing.assert_allclose(pc.bdata, W.boundary_data(pc, f, [(m + 1) * pc.dt for m in range(pc.nt)]),
                               rtol=0, atol=1e-14)
    Xc, Yc = pc.mesh()
    Uc = np.stack([f(Xc, Yc, (m + 1) * pc.dt) for m in range(pc.nt)])
    U = coarse.interpolate(p, 4, Uc)
    exact = np.stack([f(X, Y, (n + 1) * p.dt) for n in range(p.nt)])
    np.testing.assert_allclose(U, exact, rtol=0, atol=1e-12)


def test_coarse_start_of_the_heat_exact_solution_problem():
    """Section 8.1 problem (64 intervals, 8 levels, c_f = 4 as in the paper): the coarse start
    is far closer to the exact solution than the plain start."""
    from oracle import coarse
    p = W.heat_mms(64)
    p = dataclasses.replace(p, nt=8, dt=1.0 / 8, bdata=W.boundary_data(
        p, lambda x, y, t: W.heat_exact(x, y, t), [(n + 1) / 8 for n in range(8)]))
    Ug, _ = coarse.coarse_initial_iterate(p, 4)
    X, Y = p.mesh()
    exact = np.stack([W.heat_exact(X, Y, (n + 1) * p.dt) for n in range(p.nt)])
    e_coarse = np.max(np.abs(Ug - exact))
    e_plain = np.max(np.abs(p.plain_iterate() - exact))
    assert e_coarse < 0.1 * e_plain, (e_coarse, e_plain)


# ------------------------------------------------------------ variable step sizes tau_n
def _graded_steps(nt, t_end, ratio):
    """Geometrically graded steps tau_n = tau_1 q^(n-1) summing to t_end (q = ratio^(1/(nt-1)))."""
    q = ratio ** (1.0 / (nt - 1))
    tau = q ** np.arange(nt)
    return tau * (t_end / tau.sum())


def test_linear_heat_decay_with_graded_steps():
    """Eq. (3) with tau_n = t^n - t^{n-1}: linear heat (mu_b = 0), zero Dirichlet data and a sine
    mode decay by 1/(1 + tau_n mu lambda) on level n, so u^n = prod_{m<=n} (1 + tau_m mu lambda)^-1
    u^0 (lambda from Section 7); a reading that used one step for every level, or the wrong
    level's step, fails."""
    n, kx, ky, mu, nt = 20, 2, 3, 0.7, 7
    h = 1.0 / (n + 1)
    x = (np.arange(n) + 1.0) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    u0 = np.sin(math.pi * kx * X) * np.sin(math.pi * ky * Y)
    p = W.heat_dirichlet(n, nt, 1e-3, u0, mu_a=mu, mu_b=0.0)
    p.dts = _graded_steps(nt, 0.02, 8.0)
    lam = 4.0 / h ** 2 * (math.sin(math.pi * kx * h / 2) ** 2 + math.sin(math.pi * ky * h / 2) ** 2)
    U, _ = sequential.solve_sequential(p)
    fac = 1.0
    for lvl in range(nt):
        fac /= 1.0 + p.dts[lvl] * mu * lam
        np.testing.assert_allclose(U[lvl], fac * u0, rtol=0, atol=1e-14)


def test_allatonce_equals_sequential_with_graded_steps():
    """Theorem 1's premise with variable steps: the all-at-once Newton iteration (sparse LU of the
    whole space-time matrix) reaches the sequential solution; its first step equals the Eq. (7)
    block inverse and Theorem 1's explicit products."""
    rng = np.random.default_rng(8)
    p = W.burgers_periodic(12, 6, 1e-3, 0.02, W.fourier_u0_periodic(12, 9, kmax=3))
    p.dts = _graded_steps(6, 6e-3, 0.2)
    Us, _ = sequential.solve_sequential(p)
    Ua, rh, _ = allatonce.solve_allatonce(p, tol=1e-13)
    assert rh[-1] <= 1e-13
    assert np.max(np.abs(Ua - Us)) <= 1e-12
    U = p.plain_iterate() + 0.01 * rng.standard_normal((p.nt, p.ny, p.nx))
    d1, _ = allatonce.newton_step_direct(U, p)
    d2, _ = allatonce.newton_step_inverse(U, p)
    d3, _ = allatonce.newton_step_theorem1(U, p)
    assert np.max(np.abs(d2 - d1)) <= 1e-12 * np.max(np.abs(d1))
    assert np.max(np.abs(d3 - d1)) <= 1e-10 * np.max(np.abs(d1))

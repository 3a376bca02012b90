"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances: FP64 path 1e-10 relative max error, mixed path 1e-8, both measured as
max |U - U_oracle| / max |U_oracle| over all levels and nodes.
"""
import math

import numpy as np
import pytest
import torch

import paper_2406_00878_amd as P
import workloads as W
from oracle import allatonce, sequential
from oracle.discretization import jacobian_stencil, level_bvals

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def gpu_solve(p, tol=1e-12, precision="fp64", U0=None, **opts):
    U = dev(p.plain_iterate() if U0 is None else U0)
    u0 = dev(p.u0)
    bd = dev(p.bdata) if p.bdata is not None else None
    print(f"[gpu_solve] {p.name} {p.nx}x{p.ny}x{p.nt} bc={p.bc} {precision}", flush=True)
    st = P.solve(p, U, u0, tol=tol, max_iter=60, bdata=bd, precision=precision, **opts)
    return host(U), st


def _rand_problem(case, rng):
    if case == "heat_dirichlet_bdata":
        p = W.heat_dirichlet(37, 3, 2e-4, rng.uniform(0, 1, (37, 37)))
        p.ny = 23
        p.u0 = rng.uniform(0, 1, (23, 37))
        p.hy = 1.0 / 24
        p.bdata = rng.uniform(-1, 1, (3, 2 * (37 + 23)))
        return p
    if case == "burgers_periodic_ragged":
        p = W.burgers_periodic(70, 2, 5e-4, 0.01, rng.uniform(-1, 1, (70, 70)))
        p.ny, p.hy, p.u0 = 45, 1.0 / 45, rng.uniform(-1, 1, (45, 70))
        return p
    if case == "burgers_dirichlet_tiled":
        p = W.Problem(W.BURGERS, W.DIRICHLET, 100, 67, 2, 0.01, 0.012, 1e-3, 0.02, 0.0,
                      rng.uniform(-1, 1, (67, 100)), rng.uniform(-1, 1, (2, 2 * 167)))
        return p
    if case == "heat_paper_mms":
        return W.heat_mms(12)
    if case == "single_node":
        return W.Problem(W.HEAT, W.DIRICHLET, 1, 1, 2, 0.5, 0.5, 0.05, 0.2, 1.3, np.array([[0.9]]),
                         rng.uniform(0, 1, (2, 4)))
    if case == "periodic_3x3":
        return W.Problem(W.BURGERS, W.PERIODIC, 3, 3, 2, 1 / 3, 1 / 3, 1e-2, 0.05, 0.0,
                         rng.uniform(-1, 1, (3, 3)))
    raise KeyError(case)


CASES = ["heat_dirichlet_bdata", "burgers_periodic_ragged", "burgers_dirichlet_tiled", "heat_paper_mms",
         "single_node", "periodic_3x3"]


@pytest.mark.parametrize("case", CASES)
def test_assemble_matches_oracle(case):
    rng = np.random.default_rng(CASES.index(case))
    p = _rand_problem(case, rng)
    U = p.plain_iterate() + 0.1 * rng.standard_normal((p.nt, p.ny, p.nx))
    bd = dev(p.bdata) if p.bdata is not None else None
    R, cf, rinf = P.assemble(p, dev(U), dev(p.u0), bdata=bd, coef=True)
    R, cf, rinf = host(R), host(cf), float(host(rinf))
    Ro = allatonce.global_residual(U, p)
    scale = max(1.0, np.max(np.abs(Ro)))
    np.testing.assert_allclose(R, Ro, rtol=0, atol=1e-13 * scale)
    assert rinf == pytest.approx(np.max(np.abs(Ro)), rel=1e-12)
    for n in range(p.nt):
        co = jacobian_stencil(U[n], p, level_bvals(p, n + 1))
        cscale = max(1.0, max(np.max(np.abs(c)) for c in co))
        for k in range(5):
            np.testing.assert_allclose(cf[n, k], co[k], rtol=0, atol=1e-13 * cscale)


@pytest.mark.parametrize("case", ["heat_dirichlet_bdata", "burgers_periodic_ragged", "burgers_dirichlet_tiled",
                                  "heat_paper_mms"])
def test_newton_step_matches_sparse_direct_step(case):
    """One Newton step of Eq. (6) equals the sparse-LU step of the whole space-time matrix."""
    rng = np.random.default_rng(7)
    p = _rand_problem(case, rng)
    p.nt = 5
    if p.bdata is not None:
        p.bdata = p.bdata[:5] if p.bdata.shape[0] >= 5 else rng.uniform(-1, 1, (5, p.bdata.shape[1]))
    U = p.plain_iterate() + 0.01 * rng.standard_normal((p.nt, p.ny, p.nx))
    dU, _ = allatonce.newton_step_direct(U, p)
    Ud = dev(U)
    bd = dev(p.bdata) if p.bdata is not None else None
    st = P.newton_step(p, Ud, dev(p.u0), bdata=bd, lin_tol=1e-14)
    assert st["iterations"] == 1
    got = host(Ud) - U
    assert np.max(np.abs(got - dU)) <= 1e-10 * np.max(np.abs(dU))


def test_solve_heat32_matches_oracle():
    """Nonlinear heat k(u) = 1 + u^2, 32x32, 64 levels, dt = 1e-3 (the small workload)."""
    p = W.heat32()
    Us, _ = sequential.solve_sequential(p)
    U, st = gpu_solve(p, tol=1e-12)
    assert st["converged"] and st["iterations"] <= 10
    assert relerr(U, Us) <= 1e-10


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-8)])
def test_solve_burgers_periodic_ragged_tiles(precision, tol):
    """Periodic Burgers on a grid that is not a multiple of the tile (several tiles + ragged tail)."""
    n1, n2 = 80, 72
    p = W.burgers_periodic(n1, 40, 5e-4, 0.01, W.fourier_u0_periodic(n1, 2406002)[:n2, :])
    p.ny, p.hy = n2, 1.0 / n2
    Us, _ = sequential.solve_sequential(p)
    U, st = gpu_solve(p, tol=1e-12, precision=precision)
    assert st["converged"]
    assert relerr(U, Us) <= tol


def test_solve_paper_heat_mms_with_boundary_data():
    p = W.heat_mms(24)
    Us, _ = sequential.solve_sequential(p)
    U, st = gpu_solve(p, tol=1e-11)
    assert st["converged"]
    assert relerr(U, Us) <= 1e-10


def test_solve_dirichlet_tiled_ragged():
    rng = np.random.default_rng(4)
    n = 90
    p = W.heat_dirichlet(n, 12, 1e-3, W.sine_u0_dirichlet(n, rng))
    Us, _ = sequential.solve_sequential(p)
    U, st = gpu_solve(p, tol=1e-12)
    assert relerr(U, Us) <= 1e-10


@pytest.mark.parametrize("case", ["single_node", "periodic_3x3"])
def test_solve_degenerate_grids(case):
    p = _rand_problem(case, np.random.default_rng(1))
    Us, _ = sequential.solve_sequential(p)
    U, st = gpu_solve(p, tol=1e-13)
    assert relerr(U, Us) <= 1e-10


def test_single_level():
    p = W.burgers_periodic(64, 1, 5e-4, 0.01, W.fourier_u0_periodic(64, 3))
    Us, _ = sequential.solve_sequential(p)
    U, st = gpu_solve(p)
    assert relerr(U, Us) <= 1e-10


def test_full_size_burgers256_sampled():
    """Full-size periodic Burgers 256^2 x 512 levels in the benchmark's configuration:
    the first levels against the sequential oracle, and the oracle's residual of the
    GPU result at sampled levels."""
    p = W.burgers256()
    U, st = gpu_solve(p, tol=1e-12)
    assert st["converged"]
    L = 4
    Us, _ = sequential.solve_sequential(p, levels=L)
    assert relerr(U[:L], Us) <= 1e-10
    from oracle.discretization import level_residual
    for n in (1, 2, 100, 255, 256, 511, 512):
        prev = p.u0 if n == 1 else U[n - 2]
        assert np.max(np.abs(level_residual(U[n - 1], prev, p))) <= 1e-11


def test_nonfinite_input_is_reported():
    p = W.heat32(nt=4)
    u0 = p.u0.copy()
    u0[3, 5] = np.nan
    U = dev(p.plain_iterate())
    with pytest.raises(P.PTSError) as e:
        P.solve(p, U, dev(u0))
    assert e.value.code == P._lib.PTS_ERR_NONFINITE


def test_small_workspace_is_rejected():
    p = W.heat32(nt=4)
    ws = P.workspace(p)[:100]
    with pytest.raises(P.PTSError) as e:
        P.solve(p, dev(p.plain_iterate()), dev(p.u0), ws=ws)
    assert e.value.code == P._lib.PTS_ERR_WORKSPACE


def test_not_converged_leaves_last_iterate_and_resumes():
    p = W.heat32(nt=16)
    Ua = dev(p.plain_iterate())
    st = P.solve(p, Ua, dev(p.u0), tol=1e-12, max_iter=2, raise_on_error=False, schedule="bulk")
    assert st["rc"] == P._lib.PTS_ERR_NOT_CONVERGED and st["iterations"] == 2
    Ub = dev(p.plain_iterate())
    P.newton_step(p, Ub, dev(p.u0))
    P.newton_step(p, Ub, dev(p.u0))
    assert relerr(host(Ua), host(Ub)) <= 1e-12
    st2 = P.solve(p, Ua, dev(p.u0), tol=1e-12)
    Us, _ = sequential.solve_sequential(p)
    assert st2["converged"] and relerr(host(Ua), Us) <= 1e-10


def test_repeat_runs_are_bitwise_identical():
    """Deterministic kernels and fixed-order reductions: the same solve twice gives the same bits."""
    p = W.burgers_periodic(96, 16, 5e-4, 0.01, W.fourier_u0_periodic(96, 9))
    U1, _ = gpu_solve(p, stages=6)
    U2, _ = gpu_solve(p, stages=6)
    assert np.array_equal(U1, U2)


def test_quadratic_convergence_history():
    """Section 4: the all-at-once Newton on the GPU keeps the quadratic rate (smooth heat)."""
    p = W.heat32()
    _, st = gpu_solve(p, tol=1e-14, lin_tol=1e-13)
    r = st["res_inf"]
    ratios = [r[k + 1] / r[k] ** 2 for k in range(len(r) - 1) if r[k + 1] > 1e-12]
    assert len(ratios) >= 2 and max(ratios[1:]) < 100.0


# ------------------------------------------------------------- wavefront schedule

def test_wavefront_matches_bulk():
    """The wavefront schedule overlaps Newton iterations of the same all-at-once Newton
    method; both schedules reach the same root."""
    n1, n2 = 80, 72
    p = W.burgers_periodic(n1, 24, 5e-4, 0.01, W.fourier_u0_periodic(n1, 11)[:n2, :])
    p.ny, p.hy = n2, 1.0 / n2
    Ub, sb = gpu_solve(p, tol=1e-13, schedule="bulk")
    Uw, sw = gpu_solve(p, tol=1e-13, schedule="pipeline")
    assert sw["schedule"] == P.PTS_SCHED_PIPELINE and sb["schedule"] == P.PTS_SCHED_BULK
    assert relerr(Uw, Ub) <= 1e-12


@pytest.mark.parametrize("stages", [1, 2, 3, 7])
def test_wavefront_stage_counts(stages):
    p = W.burgers_periodic(64, 30, 5e-4, 0.01, W.fourier_u0_periodic(64, 5))
    Us, _ = sequential.solve_sequential(p)
    U, st = gpu_solve(p, tol=1e-12, schedule="pipeline", stages=stages)
    assert st["converged"] and st["schedule"] == P.PTS_SCHED_PIPELINE
    assert relerr(U, Us) <= 1e-10


@pytest.mark.parametrize("case", ["mms_whole", "dirichlet_tiled_bdata"])
def test_wavefront_dirichlet_boundary_data(case):
    """The next-iterate residual formed inside the wavefront kernel reads the Dirichlet data."""
    if case == "mms_whole":
        p = W.heat_mms(20)
    else:
        rng = np.random.default_rng(9)
        p = W.Problem(W.BURGERS, W.DIRICHLET, 75, 70, 6, 1 / 76, 1 / 71, 1e-3, 0.02, 0.0,
                      0.5 * rng.uniform(-1, 1, (70, 75)), 0.5 * rng.uniform(-1, 1, (6, 2 * 145)))
    Us, _ = sequential.solve_sequential(p)
    U, st = gpu_solve(p, tol=1e-12, schedule="pipeline")
    assert st["converged"]
    assert relerr(U, Us) <= 1e-10


def test_wavefront_mixed_precision():
    p = W.burgers_periodic(96, 32, 2.5e-4, 1e-3, W.disc_u0_periodic(96, 2406003))
    Us, _ = sequential.solve_sequential(p)
    U, st = gpu_solve(p, tol=1e-12, precision="mixed", schedule="pipeline")
    assert st["converged"] and st["schedule"] == P.PTS_SCHED_PIPELINE
    assert relerr(U, Us) <= 1e-8


def _coop_case(case):
    rng = np.random.default_rng(31)
    if case == "periodic_fp64":
        p = W.burgers_periodic(80, 24, 5e-4, 0.01, W.fourier_u0_periodic(80, 11)[:72, :])
        p.ny, p.hy = 72, 1.0 / 72
        return p, "fp64", 8
    if case == "dirichlet_bdata_fp64":
        return (W.Problem(W.BURGERS, W.DIRICHLET, 75, 70, 6, 1 / 76, 1 / 71, 1e-3, 0.02, 0.0,
                          0.5 * rng.uniform(-1, 1, (70, 75)), 0.5 * rng.uniform(-1, 1, (6, 2 * 145))), "fp64", 8)
    return W.burgers_periodic(96, 32, 2.5e-4, 1e-3, W.disc_u0_periodic(96, 2406003)), "mixed", 6


@pytest.mark.parametrize("case", ["periodic_fp64", "dirichlet_bdata_fp64", "periodic_mixed"])
def test_cooperative_sequence_matches_per_diagonal_launches(case):
    """One cooperative launch per wavefront sequence (grid barrier between anti-diagonals) and
    one launch per anti-diagonal run the same pairs in the same order: bit-identical iterates
    for a fixed plan, and both match the oracle."""
    p, prec, sweeps = _coop_case(case)
    plan = dict(schedule="pipeline", stages=4, sweeps=sweeps, refine=0 if prec == "fp64" else 1)
    Uc, sc = gpu_solve(p, tol=1e-12, precision=prec, wave_launch="sequence", **plan)
    Ud, sd = gpu_solve(p, tol=1e-12, precision=prec, wave_launch="diagonal", **plan)
    assert sc["converged"] and sd["converged"] and sc["iterations"] == sd["iterations"]
    assert np.array_equal(Uc, Ud)
    # the cooperative form issues a couple of launches per sequence instead of one per anti-diagonal
    assert sc["launches"] < sd["launches"] or sd["launches"] <= 4 * sd["iterations"]
    Us, _ = sequential.solve_sequential(p)
    assert relerr(Uc, Us) <= (1e-10 if prec == "fp64" else 1e-8)


def test_cooperative_barrier_poll_limit_reports_error_and_recovers():
    """A grid-barrier wait that exceeds its poll limit (forced from the host with a limit of one
    poll: work-groups of later stages wait at the first barrier while stage 0 works) abandons
    the sequence with an error, every work-group having left; the next solve on the same
    workspace is unaffected."""
    p = W.burgers_periodic(64, 30, 5e-4, 0.01, W.fourier_u0_periodic(64, 5))
    ws = P.workspace(p, "fp64")
    u0 = dev(p.u0)
    U = dev(p.plain_iterate())
    print("[coop] poll limit 1", flush=True)
    st = P.solve(p, U, u0, tol=1e-12, ws=ws, schedule="pipeline", stages=4, sweeps=8, refine=0,
                 wave_launch="sequence", barrier_spins=1, raise_on_error=False)
    assert st["rc"] == P.PTS_ERR_HIP and "grid-barrier" in st["error"], st.get("error")
    U = dev(p.plain_iterate())
    st = P.solve(p, U, u0, tol=1e-12, ws=ws, schedule="pipeline", stages=4, sweeps=8, refine=0,
                 wave_launch="sequence")
    assert st["converged"]
    Us, _ = sequential.solve_sequential(p)
    assert relerr(host(U), Us) <= 1e-10


def test_autotune_restores_iterate_and_tuned_solve_matches_oracle():
    p = W.burgers_periodic(64, 40, 5e-4, 0.01, W.fourier_u0_periodic(64, 21))
    U = dev(p.plain_iterate())
    u0 = dev(p.u0)
    before = host(U).copy()
    tuned = P.autotune(p, U, u0, tol=1e-12)
    assert np.array_equal(host(U), before)
    assert tuned["sweeps"] >= 1 and tuned["newton_steps"] >= 1
    st = P.solve(p, U, u0, tol=1e-12)
    assert st["converged"] and st["sweeps"] == tuned["sweeps"]
    Us, _ = sequential.solve_sequential(p)
    assert relerr(host(U), Us) <= 1e-10


# --------------------------------------------------- 512^2 x 1024 disc, mixed precision

def test_full_size_burgers512_disc_mixed_sampled():
    """Periodic Burgers 512^2 x 1024 levels, nu = 1e-3, discontinuous disc initial condition,
    FP32 inner solves with FP64 residuals. Plain Newton over the whole domain diverges here;
    the safeguard solves slabs of levels all-at-once. Checked against the sequential oracle on
    the first levels and by the oracle's residual at sampled levels."""
    p = W.burgers512_disc()
    U, st = gpu_solve(p, tol=1e-12, precision="mixed")
    assert st["converged"] and st["slab"] < p.nt
    L = 3
    Us, _ = sequential.solve_sequential(p, levels=L)
    assert relerr(U[:L], Us) <= 1e-8
    from oracle.discretization import level_residual
    for n in (1, 127, 128, 129, 130, 700, 1024):
        prev = p.u0 if n == 1 else U[n - 2]
        assert np.max(np.abs(level_residual(U[n - 1], prev, p))) <= 1e-11


# ------------------------------------------------------------------ Theorem-1 windows

@pytest.mark.parametrize("case", ["heat_paper_mms", "burgers_periodic_ragged", "heat_dirichlet_bdata"])
def test_newton_step_theorem1_full_window_matches_oracle(case):
    """Theorem 1 with one window over all levels (the paper's fully decoupled form,
    Eq. (8)) gives the Newton step of Eq. (6) when the products are well conditioned."""
    rng = np.random.default_rng(17)
    p = _rand_problem(case, rng)
    p.nt = 5
    if p.bdata is not None:
        p.bdata = p.bdata[:5] if p.bdata.shape[0] >= 5 else rng.uniform(-1, 1, (5, p.bdata.shape[1]))
    U = p.plain_iterate() + 0.01 * rng.standard_normal((p.nt, p.ny, p.nx))
    dU_direct, _ = allatonce.newton_step_direct(U, p)
    dU_thm1, _ = allatonce.newton_step_theorem1(U, p, window=None)
    assert np.max(np.abs(dU_thm1 - dU_direct)) <= 1e-9 * np.max(np.abs(dU_direct))
    Ud = dev(U)
    bd = dev(p.bdata) if p.bdata is not None else None
    st = P.newton_step(p, Ud, dev(p.u0), bdata=bd, lin_tol=1e-14, window=5)
    assert st["window"] == 5
    got = host(Ud) - U
    assert np.max(np.abs(got - dU_direct)) <= 1e-8 * np.max(np.abs(dU_direct))


@pytest.mark.parametrize("which", ["heat32", "burgers_periodic"])
def test_solve_with_condition_bounded_window(which):
    """Windows chosen by the Section 7 estimate (Eq. (cond)) reach the same root."""
    if which == "heat32":
        p = W.heat32()
        mu_max = 2.0
    else:
        p = W.burgers_periodic(80, 40, 5e-4, 0.01, W.fourier_u0_periodic(80, 2406002))
        mu_max = 0.01
    w = P.window_bound(p.hx, mu_max, tau=p.dt, c=1.0, eps=1e-16, wmax=min(64, p.nt))
    assert w >= 2
    Us, _ = sequential.solve_sequential(p)
    U, st = gpu_solve(p, tol=1e-12, window=w, schedule="bulk")
    assert st["converged"] and st["window"] == w
    assert relerr(U, Us) <= 1e-10


# ------------------------------------------------------------- the paper's printed errors
def _golden(name):
    import os
    rows = []
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(v) for v in line.split()])
    return rows


@pytest.mark.parametrize("row", _golden("table1_heat_linf.txt"), ids=lambda r: f"N{int(r[0])}")
def test_gpu_reproduces_table1_heat_errors(row):
    """Section 8.1, Table 1: the all-at-once GPU solve of the heat test (N_t = N_x = N_y
    intervals, mu = 1e-6 u^2) has the printed L-inf error to three digits."""
    nint, expected = int(row[0]), row[1]
    p = W.heat_mms(nint)
    U, st = gpu_solve(p, tol=1e-12)
    assert st["converged"]
    X, Y = p.mesh()
    err = max(np.max(np.abs(U[n] - W.heat_exact(X, Y, (n + 1) * p.dt))) for n in range(p.nt))
    assert float(f"{err:.2e}") == pytest.approx(expected, rel=1e-9), err


@pytest.mark.parametrize("row", [r for r in _golden("table4_burgers_l1.txt") if r[2] == 1],
                         ids=lambda r: f"N{int(r[0])}")
def test_gpu_reproduces_table4_burgers_errors(row):
    """Section 8.2, Table 4 (three finest grids): the all-at-once GPU solve of the viscous-shock
    Burgers test has the printed L1 space-time error within 1% (domain [-0.5, 0.5]^2, reading
    of the unstated domain). At these step sizes (cell Peclet numbers near 28) the blocks have
    complex Jacobi spectra at the edge of diagonal dominance: the level solves are the banded
    LU without pivoting the paper uses."""
    nint, expected = int(row[0]), row[1]
    p = W.burgers_mms(nint, x0=-0.5, y0=-0.5)
    U, st = gpu_solve(p, tol=1e-12)
    assert st["converged"] and st["schedule"] == P.PTS_SCHED_BULK and st["sweeps"] == 0, st
    X, Y = p.mesh()
    err = sum(np.sum(np.abs(U[n] - W.burgers_exact(X, Y, (n + 1) * p.dt))) for n in range(p.nt)) * p.hx * p.hy * p.dt
    print(f"Table 4 N = {nint}: L1 error {err:.4e} (printed {expected:.2e})")
    assert err == pytest.approx(expected, rel=1e-2), err


@pytest.mark.parametrize("nint", [7, 13])
def test_banded_level_solves_match_the_dense_newton_step(nint):
    """One Newton step with the banded LU level solves (Section 8.2 problem, non-dominant blocks)
    equals the oracle's step by sparse LU of the whole space-time Jacobian, element by element;
    the converged solve equals the sequential oracle."""
    p = W.burgers_mms(nint, x0=-0.5, y0=-0.5)
    U = p.plain_iterate()
    dU_ref, _ = allatonce.newton_step_direct(U, p)
    Ud = dev(U)
    st = P.newton_step(p, Ud, dev(p.u0), bdata=dev(p.bdata))
    assert st["sweeps"] == 0, st  # banded path
    got = host(Ud) - U
    assert np.max(np.abs(got - dU_ref)) <= 1e-12 * np.max(np.abs(dU_ref))
    Uo, _ = sequential.solve_sequential(p)
    Ug, st = gpu_solve(p, tol=1e-12)
    assert st["converged"] and relerr(Ug, Uo) <= 1e-10, relerr(Ug, Uo)


def test_not_dominant_periodic_problem_is_reported():
    """A periodic Burgers problem at cell Peclet numbers above 2 with a Gershgorin radius above
    0.7: no level solve with a convergence bound applies (the banded LU is for Dirichlet grids),
    and the solve says so up front instead of diverging."""
    p = W.burgers_periodic(32, 4, 0.05, 1e-4, W.fourier_u0_periodic(32, 5))
    with pytest.raises(P.PTSError) as e:
        gpu_solve(p, tol=1e-12)
    assert e.value.code in (P._lib.PTS_ERR_NOT_DOMINANT,), e.value


# ------------------------------------------------------------ variable step sizes tau_n
def _graded(nt, t_end, ratio):
    q = ratio ** (1.0 / max(nt - 1, 1))
    tau = q ** np.arange(nt)
    return tau * (t_end / tau.sum())


@pytest.mark.parametrize("case", ["heat_dirichlet", "burgers_periodic", "heat_dirichlet_window"])
def test_graded_steps_match_oracle(case):
    """Eq. (3) with tau_n = t^n - t^{n-1} varying from level to level (geometric grading): the
    all-at-once GPU solve (bulk schedule; Theorem-1 windows of 3 levels in one case) equals the
    sequential oracle stepping with the same tau_n."""
    rng = np.random.default_rng(23)
    if case.startswith("heat"):
        p = W.heat_dirichlet(45, 10, 1e-3, W.sine_u0_dirichlet(45, rng))
        p.dts = _graded(10, 0.02, 10.0)
    else:
        p = W.burgers_periodic(48, 9, 5e-4, 0.01, W.fourier_u0_periodic(48, 24, kmax=4))
        p.dts = _graded(9, 9e-3, 0.1)
    Us, _ = sequential.solve_sequential(p)
    opts = {"window": 3, "schedule": "bulk"} if case.endswith("window") else {}
    U, st = gpu_solve(p, tol=1e-12, **opts)
    assert st["converged"] and st["schedule"] == P.PTS_SCHED_BULK, st
    assert relerr(U, Us) <= 1e-10, relerr(U, Us)


def test_graded_steps_mms_first_order_in_time():
    """Section 8.1 heat test with graded steps (tau_{n+1}/tau_n fixed, 4:1 over the run) on
    N = N_t = 8, 16, 32 intervals: the L-inf space-time error against the exact solution falls
    at least 1.6-fold per refinement (BDF1 is first order in tau, the scheme second order in h)."""
    import dataclasses
    errs = []
    for nint in (8, 16, 32):
        p = W.heat_mms(nint)
        dts = _graded(nint, 1.0, 4.0)
        ts = np.cumsum(dts)
        p = dataclasses.replace(p, dts=dts, bdata=W.boundary_data(p, lambda x, y, t: W.heat_exact(x, y, t), ts))
        U, st = gpu_solve(p, tol=1e-12)
        assert st["converged"], st
        X, Y = p.mesh()
        errs.append(max(np.max(np.abs(U[n] - W.heat_exact(X, Y, ts[n]))) for n in range(p.nt)))
    print("graded-step MMS errors", errs)
    assert errs[0] / errs[1] >= 1.6 and errs[1] / errs[2] >= 1.6, errs

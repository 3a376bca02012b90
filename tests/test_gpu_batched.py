"""Batched solves against the time-stepping oracle: independent instances with uneven grids and
level counts (one launch per level and inner launch over every instance's tiles), and instances
of one problem with different initial conditions (batched wavefront sequences)."""
import numpy as np
import pytest
import torch

import paper_2406_00878_amd as P
import workloads as W
from oracle import sequential

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _heat_batch(seed, sizes, dt=1e-3):
    rng = np.random.default_rng(seed)
    return [W.heat_dirichlet(n, L, dt, W.sine_u0_dirichlet(n, rng), name=f"h{n}x{L}") for n, L in sizes]


@pytest.mark.parametrize("precision,tol,bar", [("fp64", 1e-12, 1e-10), ("mixed", 1e-12, 1e-8)])
def test_uneven_heat_batch_matches_oracle(precision, tol, bar):
    # sizes span one whole-domain region (<= 64), several tiles, ragged tiles, and level counts
    probs = _heat_batch(5, [(20, 6), (64, 3), (37, 9), (70, 5), (100, 2)])
    Us = [dev(p.plain_iterate()) for p in probs]
    u0s = [dev(p.u0) for p in probs]
    print(f"[batched] heat {precision} {[(p.nx, p.nt) for p in probs]}", flush=True)
    sts = P.solve_batched(probs, Us, u0s, tol=tol, max_iter=40, precision=precision)
    for p, U, st in zip(probs, Us, sts):
        assert st["converged"], st
        # the 100^2 instance's blocks are stiff (radius 0.976): multigrid level solves for the
        # batch, Newton stages pipelined in shared launches
        assert st["schedule"] == P.PTS_SCHED_PIPELINE, st
        Uo, _ = sequential.solve_sequential(p)
        err = np.max(np.abs(host(U) - Uo)) / np.max(np.abs(Uo))
        assert err <= bar, (p.name, err)


def test_batch_equals_one_by_one_solves():
    probs = _heat_batch(6, [(33, 4), (65, 6), (48, 2)])
    Us = [dev(p.plain_iterate()) for p in probs]
    sts = P.solve_batched(probs, Us, [dev(p.u0) for p in probs], tol=1e-12, max_iter=40, schedule="bulk")
    for p, U, st in zip(probs, Us, sts):
        V = dev(p.plain_iterate())
        st1 = P.solve(p, V, dev(p.u0), tol=1e-12, max_iter=40, schedule="bulk")
        assert st["iterations"] == st1["iterations"]
        np.testing.assert_allclose(host(U), host(V), rtol=0, atol=1e-12 * np.max(np.abs(host(V))))


def test_periodic_burgers_batch():
    rng = np.random.default_rng(8)
    probs = [W.burgers_periodic(n, L, 5e-4, 0.01, W.fourier_u0_periodic(n, int(rng.integers(1 << 30)), kmax=4),
                                name=f"b{n}") for n, L in [(64, 4), (96, 3), (128, 2)]]
    Us = [dev(p.plain_iterate()) for p in probs]
    print("[batched] burgers periodic", flush=True)
    sts = P.solve_batched(probs, Us, [dev(p.u0) for p in probs], tol=1e-12, max_iter=40)
    for p, U, st in zip(probs, Us, sts):
        assert st["converged"]
        Uo, _ = sequential.solve_sequential(p)
        assert np.max(np.abs(host(U) - Uo)) <= 1e-10 * np.max(np.abs(Uo))


def test_mixed_boundary_kinds_fall_back_to_one_by_one():
    rng = np.random.default_rng(9)
    probs = [W.heat_dirichlet(24, 3, 1e-3, W.sine_u0_dirichlet(24, rng)),
             W.burgers_periodic(64, 2, 5e-4, 0.01, W.fourier_u0_periodic(64, 3, kmax=4))]
    Us = [dev(p.plain_iterate()) for p in probs]
    sts = P.solve_batched(probs, Us, [dev(p.u0) for p in probs], tol=1e-12, max_iter=40)
    for p, U, st in zip(probs, Us, sts):
        assert st["converged"]
        Uo, _ = sequential.solve_sequential(p)
        assert np.max(np.abs(host(U) - Uo)) <= 1e-10 * np.max(np.abs(Uo))


def test_nonconverging_instance_reports_and_others_finish():
    probs = _heat_batch(10, [(30, 4), (40, 3)])
    Us = [dev(p.plain_iterate()) for p in probs]
    with pytest.raises(P.PTSError):
        P.solve_batched(probs, Us, [dev(p.u0) for p in probs], tol=1e-30, max_iter=2)


@pytest.mark.parametrize("precision,bar,schedule", [("fp64", 1e-10, "auto"), ("mixed", 1e-8, "auto"),
                                                     ("mixed", 1e-8, "bulk")])
def test_stiff_heat_batch_multigrid_level_solves_match_oracle(precision, bar, schedule):
    """Stiff Dirichlet heat levels (Gershgorin radius >= 0.976) take the multigrid-preconditioned
    Chebyshev solve: few iterations per level, no restarted passes, same converged result; by
    default as pipelined Newton stages, with schedule="bulk" one Newton step after another."""
    probs = _heat_batch(12, [(128, 3), (100, 4), (150, 2)])
    Us = [dev(p.plain_iterate()) for p in probs]
    print(f"[batched] stiff heat {precision} {schedule}", flush=True)
    sts = P.solve_batched(probs, Us, [dev(p.u0) for p in probs], tol=1e-12, max_iter=40, precision=precision,
                          schedule=schedule)
    for p, U, st in zip(probs, Us, sts):
        assert st["converged"], st
        assert st["refine"] == 0 and st["sweeps"] <= 32, st  # spectral path: Chebyshev iterations, one pass
        assert st["schedule"] == (P.PTS_SCHED_BULK if schedule == "bulk" else P.PTS_SCHED_PIPELINE), st
        Uo, _ = sequential.solve_sequential(p)
        err = np.max(np.abs(host(U) - Uo)) / np.max(np.abs(Uo))
        print(p.name, "iterations", st["iterations"], "cheb", st["sweeps"], "err", err)
        assert err <= bar, (p.name, err)


def test_stiff_heat_batch_deep_hierarchies_match_oracle():
    """Grids whose V-cycle has three tile-kernel grids above the in-LDS part (260 -> 130 -> 65
    -> 32 ...), one odd grid (nested coarsening) and one with an even grid on the way down."""
    probs = _heat_batch(16, [(260, 2), (131, 3)])
    Us = [dev(p.plain_iterate()) for p in probs]
    print("[batched] stiff heat 260^2 x 2 + 131^2 x 3, mixed", flush=True)
    sts = P.solve_batched(probs, Us, [dev(p.u0) for p in probs], tol=1e-12, max_iter=40, precision="mixed")
    for p, U, st in zip(probs, Us, sts):
        assert st["converged"] and st["refine"] == 0 and st["sweeps"] <= 32, st
        Uo, _ = sequential.solve_sequential(p)
        err = np.max(np.abs(host(U) - Uo)) / np.max(np.abs(Uo))
        print(p.name, "iterations", st["iterations"], "cheb", st["sweeps"], "err", err, flush=True)
        assert err <= 1e-8, (p.name, err)


@pytest.mark.parametrize("stages", [0, 3])
def test_stiff_heat_batch_pipelined_stages_match_oracle(stages):
    """Pipelined Newton stages over many levels: instances with more levels than stages (the
    lanes of all stages overlap on consecutive levels) and fewer (lanes idle at the ends), the
    default stage count (7) and a short one that needs several passes over the diagonals."""
    probs = _heat_batch(21, [(128, 20), (66, 33), (100, 9), (90, 1)])
    Us = [dev(p.plain_iterate()) for p in probs]
    print(f"[batched] stiff heat pipelined, stages {stages}", flush=True)
    sts = P.solve_batched(probs, Us, [dev(p.u0) for p in probs], tol=1e-12, max_iter=40, precision="mixed",
                          stages=stages)
    for p, U, st in zip(probs, Us, sts):
        assert st["converged"] and st["schedule"] == P.PTS_SCHED_PIPELINE, st
        if stages:
            assert st["iterations"] % stages == 0, st
        Uo, _ = sequential.solve_sequential(p)
        err = np.max(np.abs(host(U) - Uo)) / np.max(np.abs(Uo))
        print(p.name, "iterations", st["iterations"], "cheb", st["sweeps"], "err", err, flush=True)
        assert err <= 1e-8, (p.name, err)


def test_stiff_heat_batch_gives_each_instance_its_own_stage_count():
    """The first solve of a batch records the Newton steps each instance needed; a second solve
    of the same batch runs each instance for its own count (an instance whose u^0 is small
    needs fewer steps than one of amplitude 1), with the same results as the oracle."""
    rng = np.random.default_rng(41)
    probs = []
    for n, L, amp in [(128, 14, 1.0), (100, 9, 1e-4), (90, 11, 0.3)]:
        probs.append(W.heat_dirichlet(n, L, 1e-3, amp * W.sine_u0_dirichlet(n, rng), name=f"h{n}x{L}a{amp:g}"))
    u0s = [dev(p.u0) for p in probs]
    print("[batched] per-instance stage counts", flush=True)
    first = P.solve_batched(probs, [dev(p.plain_iterate()) for p in probs], u0s, tol=1e-12, max_iter=40,
                            precision="mixed")
    need = [st["needed"] for st in first]
    assert len(set(need)) > 1, need  # the instances need different step counts
    Us = [dev(p.plain_iterate()) for p in probs]
    sts = P.solve_batched(probs, Us, u0s, tol=1e-12, max_iter=40, precision="mixed")
    for p, U, st, k in zip(probs, Us, sts, need):
        assert st["converged"] and st["schedule"] == P.PTS_SCHED_PIPELINE, st
        assert st["needed"] == k and st["iterations"] == k, (p.name, st["iterations"], k)
        Uo, _ = sequential.solve_sequential(p)
        err = np.max(np.abs(host(U) - Uo)) / np.max(np.abs(Uo))
        print(p.name, "needed", k, "iterations", st["iterations"], "err", err, flush=True)
        assert err <= 1e-8, (p.name, err)


def test_stiff_heat_batch_stage_cache_falls_short_then_grows():
    """The stage cache is keyed by the problem, not by u^0: a batch first solved from a small
    u^0 (few Newton steps) and then from u^0 of amplitude 1 gets too few stages from the
    cache; the solve goes on in short passes of two stages, converges to the oracle's
    solution, and the cache grows to the larger count for the next solve."""
    rng = np.random.default_rng(43)
    shape = [(120, 10), (96, 13)]
    base = [W.sine_u0_dirichlet(n, rng) for n, _ in shape]
    small = [W.heat_dirichlet(n, L, 1e-3, 1e-4 * b, name=f"s{n}") for (n, L), b in zip(shape, base)]
    full = [W.heat_dirichlet(n, L, 1e-3, b, name=f"f{n}") for (n, L), b in zip(shape, base)]
    tag = 5

    def run(probs):
        Us = [dev(p.plain_iterate()) for p in probs]
        return Us, P.solve_batched(probs, Us, [dev(p.u0) for p in probs], tol=1e-12, max_iter=40,
                                   precision="mixed", cache_tag=tag)

    print("[batched] stage cache shortfall", flush=True)
    _, st_small = run(small)
    k_small = [st["needed"] for st in st_small]
    Us, st_full = run(full)  # cache: k_small stages, too few
    k_full = [st["needed"] for st in st_full]
    assert all(a < b for a, b in zip(k_small, k_full)), (k_small, k_full)
    for p, U, st, a in zip(full, Us, st_full, k_small):
        assert st["converged"], st
        assert st["iterations"] > a and (st["iterations"] - a) % 2 == 0, (st["iterations"], a)  # passes of 2
        Uo, _ = sequential.solve_sequential(p)
        assert np.max(np.abs(host(U) - Uo)) <= 1e-8 * np.max(np.abs(Uo)), p.name
    _, st_again = run(full)  # the cache now holds the larger counts: one pass of exactly those
    assert [st["iterations"] for st in st_again] == k_full, (st_again, k_full)


def test_stiff_heat_batch_pipelined_with_boundary_data_matches_oracle():
    """Pipelined multigrid stages on stiff heat instances whose Dirichlet data vary in space and
    time (the level residuals read the data; the V-cycles solve for updates with zero data)."""
    rng = np.random.default_rng(31)
    probs = []
    for n, L in [(128, 6), (100, 11)]:
        p = W.heat_dirichlet(n, L, 1e-3, W.sine_u0_dirichlet(n, rng), name=f"hb{n}x{L}")
        g = lambda x, y, t: 0.3 * np.sin(2 * np.pi * x) * np.cos(np.pi * y) * np.exp(-t)
        p.bdata = W.boundary_data(p, g, [(k + 1) * p.dt for k in range(p.nt)])
        probs.append(p)
    Us = [dev(p.plain_iterate()) for p in probs]
    print("[batched] stiff heat with boundary data, pipelined", flush=True)
    sts = P.solve_batched(probs, Us, [dev(p.u0) for p in probs], tol=1e-12, max_iter=40, precision="mixed",
                          bdatas=[dev(p.bdata) for p in probs])
    for p, U, st in zip(probs, Us, sts):
        assert st["converged"] and st["schedule"] == P.PTS_SCHED_PIPELINE, st
        Uo, _ = sequential.solve_sequential(p)
        err = np.max(np.abs(host(U) - Uo)) / np.max(np.abs(Uo))
        print(p.name, "iterations", st["iterations"], "err", err, flush=True)
        assert err <= 1e-8, (p.name, err)


def test_stiff_heat_pipelined_limits_and_single_instance():
    """Pipelined multigrid stages at their limits: max_iter below the stage count (the pass is
    shortened, the iterate stays finite and the solve reports PTS_ERR_NOT_CONVERGED), and a
    batch of one stiff instance with one level."""
    probs = _heat_batch(33, [(128, 5), (100, 3)])
    Us = [dev(p.plain_iterate()) for p in probs]
    print("[batched] stiff heat pipelined, max_iter 3", flush=True)
    with pytest.raises(P.PTSError) as e:
        P.solve_batched(probs, Us, [dev(p.u0) for p in probs], tol=1e-30, max_iter=3, precision="mixed")
    assert e.value.code == P._lib.PTS_ERR_NOT_CONVERGED, e.value
    assert all(np.all(np.isfinite(host(U))) for U in Us)
    one = _heat_batch(34, [(150, 1)])
    U1 = [dev(one[0].plain_iterate())]
    print("[batched] stiff heat pipelined, one instance, one level", flush=True)
    st = P.solve_batched(one, U1, [dev(one[0].u0)], tol=1e-12, max_iter=40, precision="mixed")[0]
    assert st["converged"] and st["schedule"] == P.PTS_SCHED_PIPELINE, st
    Uo, _ = sequential.solve_sequential(one[0])
    assert np.max(np.abs(host(U1[0]) - Uo)) <= 1e-8 * np.max(np.abs(Uo))


@pytest.mark.parametrize("schedule", ["auto", "bulk"])
def test_stiff_batch_with_whole_vcycle_in_lds(schedule):
    """Instances of at most 64^2 nodes in a multigrid batch run their whole V-cycle in LDS,
    which applies the Chebyshev step itself (once): their level solves are as accurate as the
    others', so their Newton counts stay those of the stiff instance."""
    probs = _heat_batch(35, [(40, 12), (64, 10), (150, 3)])
    Us = [dev(p.plain_iterate()) for p in probs]
    print(f"[batched] stiff heat with LDS-only hierarchies, {schedule}", flush=True)
    sts = P.solve_batched(probs, Us, [dev(p.u0) for p in probs], tol=1e-12, max_iter=40, precision="mixed",
                          schedule=schedule)
    for p, U, st in zip(probs, Us, sts):
        Uo, _ = sequential.solve_sequential(p)
        err = np.max(np.abs(host(U) - Uo)) / np.max(np.abs(Uo))
        print(p.name, "needed", st["needed"], "iterations", st["iterations"], "err", err, flush=True)
        assert st["converged"] and err <= 1e-8, (p.name, st, err)
        assert st["needed"] is not None and st["needed"] <= 7, (p.name, st["needed"])


def test_windows_option_solves_instances_one_after_another():
    probs = _heat_batch(14, [(20, 5), (33, 4)])
    Us = [dev(p.plain_iterate()) for p in probs]
    sts = P.solve_batched(probs, Us, [dev(p.u0) for p in probs], tol=1e-12, max_iter=40, window=2)
    for p, U, st in zip(probs, Us, sts):
        assert st["converged"] and st["window"] == 2
        Uo, _ = sequential.solve_sequential(p)
        assert np.max(np.abs(host(U) - Uo)) <= 1e-10 * np.max(np.abs(Uo))


def test_single_instance_batch_and_single_levels():
    probs = _heat_batch(15, [(50, 1)])
    Us = [dev(p.plain_iterate()) for p in probs]
    sts = P.solve_batched(probs, Us, [dev(p.u0) for p in probs], tol=1e-12, max_iter=40)
    Uo, _ = sequential.solve_sequential(probs[0])
    assert sts[0]["converged"]
    assert np.max(np.abs(host(Us[0]) - Uo)) <= 1e-10 * np.max(np.abs(Uo))


# ------------------------------------------------------- one problem, many initial conditions
def _burgers_family(n, nt, seeds, nu=0.01, dt=5e-4):
    return [W.burgers_periodic(n, nt, dt, nu, W.fourier_u0_periodic(n, s, kmax=4), name=f"b{n}s{s}") for s in seeds]


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("mixed", 1e-8)])
def test_one_problem_batch_runs_batched_wavefront(precision, bar):
    """Instances that differ only in u^0 share every anti-diagonal launch (ragged tiles at 80^2,
    several sequences) and each reaches the time-stepping oracle's solution."""
    probs = _burgers_family(80, 7, [21, 22, 23])
    Us = [dev(p.plain_iterate()) for p in probs]
    print(f"[batched-wave] burgers 80x80x7 x3 {precision}", flush=True)
    sts = P.solve_batched(probs, Us, [dev(p.u0) for p in probs], tol=1e-12, max_iter=40, precision=precision,
                          stages=2)
    for p, U, st in zip(probs, Us, sts):
        assert st["converged"] and st["schedule"] == P.PTS_SCHED_PIPELINE, st
        Uo, _ = sequential.solve_sequential(p)
        err = np.max(np.abs(host(U) - Uo)) / np.max(np.abs(Uo))
        assert err <= bar, (p.name, err)


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
def test_batched_wavefront_equals_one_by_one_wavefront(bc):
    """With the plan and stage count fixed, the batched launches compute each instance's pairs
    exactly as the one-instance launches do."""
    if bc == "periodic":
        probs = _burgers_family(96, 9, [31, 32, 33, 34])
    else:
        rng = np.random.default_rng(35)
        # 100^2 Dirichlet heat at tau = 2e-5: several tiles per level, Jacobi radius ~0.6
        probs = [W.heat_dirichlet(100, 6, 2e-5, W.sine_u0_dirichlet(100, rng), name=f"h100_{k}") for k in range(3)]
    plan = dict(sweeps=8, refine=0, stages=3)
    Us = [dev(p.plain_iterate()) for p in probs]
    print(f"[batched-wave] equals one-by-one {bc}", flush=True)
    sts = P.solve_batched(probs, Us, [dev(p.u0) for p in probs], tol=1e-12, max_iter=40, **plan)
    for p, U, st in zip(probs, Us, sts):
        assert st["schedule"] == P.PTS_SCHED_PIPELINE
        V = dev(p.plain_iterate())
        st1 = P.solve(p, V, dev(p.u0), tol=1e-12, max_iter=40, schedule="pipeline", **plan)
        assert st["converged"] and st1["converged"]
        assert st["iterations"] == st1["iterations"], (st["iterations"], st1["iterations"])
        np.testing.assert_allclose(host(U), host(V), rtol=0, atol=1e-13 * np.max(np.abs(host(V))))


def test_batched_wavefront_replays_and_whole_region_heat():
    """C1-sized Dirichlet heat (one whole-domain region per level): the same batch solved twice
    (the second from cached graphs) gives the same answer, matching the oracle."""
    rng = np.random.default_rng(41)
    probs = [W.heat_dirichlet(32, 12, 1e-3, W.sine_u0_dirichlet(32, rng), name=f"h32_{k}") for k in range(5)]
    outs = []
    for rep in range(2):
        Us = [dev(p.plain_iterate()) for p in probs]
        print(f"[batched-wave] heat 32x32x12 x5 pass {rep}", flush=True)
        sts = P.solve_batched(probs, Us, [dev(p.u0) for p in probs], tol=1e-12, max_iter=40, stages=4)
        assert all(st["converged"] and st["schedule"] == P.PTS_SCHED_PIPELINE for st in sts)
        outs.append([host(U) for U in Us])
    for p, a, b in zip(probs, outs[0], outs[1]):
        assert np.array_equal(a, b)
        Uo, _ = sequential.solve_sequential(p)
        assert np.max(np.abs(a - Uo)) <= 1e-10 * np.max(np.abs(Uo)), p.name


def test_batched_wavefront_mixed_convergence_and_limit():
    """Instances that need different Newton step counts leave the batch one by one; with a step
    limit below what one needs, that one reports not converged and the others finish."""
    n = 64
    u_small = 1e-3 * W.fourier_u0_periodic(n, 51, kmax=2)
    u_big = W.fourier_u0_periodic(n, 52, kmax=4)
    probs = [W.burgers_periodic(n, 6, 5e-4, 0.01, u, name=nm) for u, nm in ((u_small, "small"), (u_big, "big"))]
    Us = [dev(p.plain_iterate()) for p in probs]
    sts = P.solve_batched(probs, Us, [dev(p.u0) for p in probs], tol=1e-12, max_iter=40, stages=1)
    assert all(st["converged"] for st in sts)
    assert sts[0]["iterations"] < sts[1]["iterations"], [st["iterations"] for st in sts]
    for p, U in zip(probs, Us):
        Uo, _ = sequential.solve_sequential(p)
        assert np.max(np.abs(host(U) - Uo)) <= 1e-10 * np.max(np.abs(Uo))
    lim = sts[0]["iterations"]
    Us = [dev(p.plain_iterate()) for p in probs]
    with pytest.raises(P.PTSError):
        P.solve_batched(probs, Us, [dev(p.u0) for p in probs], tol=1e-12, max_iter=lim, stages=1)
    Uo, _ = sequential.solve_sequential(probs[0])
    assert np.max(np.abs(host(Us[0]) - Uo)) <= 1e-10 * np.max(np.abs(Uo))


def test_batched_autotune_restores_iterates_and_sets_the_batch_plan():
    probs = _burgers_family(64, 6, [61, 62, 63])
    Us = [dev(p.plain_iterate()) for p in probs]
    before = [host(U) for U in Us]
    u0s = [dev(p.u0) for p in probs]
    print("[batched-wave] autotune 64x64x6 x3", flush=True)
    plan = P.autotune_batched(probs, Us, u0s, tol=1e-12, max_iter=40, cache_tag=5)
    assert plan["sweeps"] > 0 and plan["solve_ms"] > 0, plan
    for a, U in zip(before, Us):
        assert np.array_equal(a, host(U))
    sts = P.solve_batched(probs, Us, u0s, tol=1e-12, max_iter=40, cache_tag=5)
    for p, U, st in zip(probs, Us, sts):
        assert st["converged"] and st["sweeps"] == plan["sweeps"], (st["sweeps"], plan)
        Uo, _ = sequential.solve_sequential(p)
        assert np.max(np.abs(host(U) - Uo)) <= 1e-10 * np.max(np.abs(Uo))
    other = _heat_batch(64, [(20, 3), (24, 3)])
    with pytest.raises(P.PTSError):
        P.autotune_batched(other, [dev(p.plain_iterate()) for p in other], [dev(p.u0) for p in other])

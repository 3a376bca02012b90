"""Full-size parity: the benchmark workloads solved on the GPU at their full sizes, every level
checked against the oracle.

For each workload:
  (a) the oracle's residual G^n(U) (Eq. (5), tau-scaled) of the GPU result at EVERY level,
      below the solve tolerance plus the rounding floor of the residual's own terms
      (oracle.sequential.roundoff_floor: 64 ulps of |u^n|, |u^{n-1}| and tau times the largest
      viscous and convective terms);
  (b) the oracle's BDF1 step (sequential Newton, Section 2) re-run from the GPU's level n-1 at
      32 evenly spaced levels, compared with the GPU's level n element by element, relative to
      the largest |u| of the whole space-time solution (the relative max error of every
      result; heat levels decay by orders of magnitude, so a level's own max would measure the
      rounding floor of the stiff residual against a vanishing solution): 1e-10 for FP64
      forms, 1e-8 for mixed-precision and learned forms;
  (c) the first levels against the sequential oracle (the same bars).
The oracle runs on the host's cores: residuals on threads (NumPy releases the GIL), re-solves
in spawned worker processes, which import the oracle only.
"""
import concurrent.futures as cf
import multiprocessing as mp
import os

import numpy as np
import pytest
import torch

import oracle_pool
import paper_2406_00878_amd as P
import workloads as W
from oracle import sequential
from oracle.discretization import level_bvals, level_residual

pytestmark = pytest.mark.gpu

WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))
TOL = 1e-12


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _level_check(U, p, n0, n1, tol):
    """Largest ratio |G^n|_inf / (tol + rounding floor) over levels n0+1..n1 (1-based n)."""
    worst = 0.0
    for n in range(n0 + 1, n1 + 1):
        prev = p.u0 if n == 1 else U[n - 2]
        tau = p.tau(n)
        g = float(np.max(np.abs(level_residual(U[n - 1], prev, p, level_bvals(p, n), tau))))
        worst = max(worst, g / (tol + sequential.roundoff_floor(U[n - 1], prev, p, tau)))
    return worst


def all_level_residual_ratio(U, p, tol=TOL):
    """(a): the worst level's residual relative to its bound; <= 1 passes."""
    chunks = np.linspace(0, p.nt, min(p.nt, 4 * WORKERS) + 1).astype(int)
    with cf.ThreadPoolExecutor(WORKERS) as ex:
        return max(ex.map(lambda ab: _level_check(U, p, ab[0], ab[1], tol), zip(chunks[:-1], chunks[1:])))


def resolve_errors(jobs):
    """(b): jobs (problem, level n, GPU level n-1 (or u0), GPU level n, scale); returns the max
    differences between the oracle's step from the GPU's level n-1 and the GPU's level n,
    divided by scale (the largest |u| of that problem's space-time solution)."""
    ctx = mp.get_context("spawn")
    with cf.ProcessPoolExecutor(min(WORKERS, len(jobs)), mp_context=ctx) as ex:
        outs = list(ex.map(oracle_pool.bdf1_from, [(p, n, prev) for p, n, prev, _, _ in jobs]))
    return [float(np.max(np.abs(got - u)) / scale) for (p, n, prev, got, scale), (_, u) in zip(jobs, outs)]


def sampled_levels(nt, count=32):
    return sorted(set(int(round(x)) for x in np.linspace(1, nt, min(count, nt))))


def check_problem(p, U, bar, levels=32, prefix=2):
    """(a), (b) and (c) for one problem whose GPU result is the host array U."""
    ratio = all_level_residual_ratio(U, p)
    print(f"[fullsize] {p.name or p.kind} {p.nx}^2 x {p.nt}: worst residual / bound {ratio:.3f}", flush=True)
    assert ratio <= 1.0, ratio
    scale = float(np.max(np.abs(U)))
    jobs = [(p, n, p.u0 if n == 1 else U[n - 2], U[n - 1], scale) for n in sampled_levels(p.nt, levels)]
    errs = resolve_errors(jobs)
    print(f"[fullsize] oracle steps from the GPU's previous level at {len(jobs)} levels: max rel. diff "
          f"{max(errs):.2e}", flush=True)
    assert max(errs) <= bar, errs
    if prefix:
        Us, _ = sequential.solve_sequential(p, levels=prefix)
        e = float(np.max(np.abs(U[:prefix] - Us)) / np.max(np.abs(Us)))
        print(f"[fullsize] first {prefix} levels vs the sequential oracle: {e:.2e}", flush=True)
        assert e <= bar, e


def test_fullsize_burgers256_fp64():
    """Periodic Burgers 256^2 x 512 levels, nu = 0.01, FP64 (the wavefront schedule)."""
    p = W.burgers256()
    U = dev(p.plain_iterate())
    print("[fullsize] burgers256 fp64 solve", flush=True)
    st = P.solve(p, U, dev(p.u0), tol=TOL, max_iter=60)
    assert st["converged"], st
    check_problem(p, U.cpu().numpy(), 1e-10, prefix=4)


@pytest.mark.timeout(400)
def test_fullsize_burgers512_disc_mixed():
    """Periodic Burgers 512^2 x 1024 levels, nu = 1e-3, disc initial condition, FP32 inner solves
    with FP64 residuals (slabs of levels, the safeguard of the solve)."""
    p = W.burgers512_disc()
    U = dev(p.plain_iterate())
    print("[fullsize] burgers512 disc mixed solve", flush=True)
    st = P.solve(p, U, dev(p.u0), tol=TOL, max_iter=60, precision="mixed")
    assert st["converged"], st
    check_problem(p, U.cpu().numpy(), 1e-8, prefix=2)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("start", ["plain", "coarse"])
def test_fullsize_heat_batch_mixed(start):
    """The 64 uneven nonlinear heat instances (grids 66^2..507^2, 128..1010 levels, 3.35 G
    space-time nodes), solved as one batch with the multigrid-preconditioned FP32 level solves,
    from the plain start and from the coarse-grid start (Section 4, c_f = 4; most grids and
    level counts are no multiples of 4): (a) at every level of every instance; (b) at 32 levels
    spread over the instances (one level of every other instance, evenly spaced in its own
    level range)."""
    probs = W.heat_batch()
    u0s = [dev(p.u0) for p in probs]
    if start == "plain":
        Us = [dev(p.plain_iterate()) for p in probs]
    else:
        Us = [torch.empty((p.nt, p.ny, p.nx), dtype=torch.float64, device="cuda") for p in probs]
        print("[fullsize] heat batch coarse starts", flush=True)
        P.coarse_initial_iterate_batched(probs, Us, u0s, 4, tol=1e-10)
    print(f"[fullsize] heat batch 64 instances mixed solve ({start} start)", flush=True)
    sts = P.solve_batched(probs, Us, u0s, tol=TOL, max_iter=60, precision="mixed", cache_tag=0 if start == "plain" else 2)
    assert all(st["converged"] for st in sts)
    jobs, worst = [], 0.0
    for i, (p, Ud) in enumerate(zip(probs, Us)):
        U = Ud.cpu().numpy()
        worst = max(worst, all_level_residual_ratio(U, p))
        if i % 2 == 0:  # one level per instance, its position moving through the level range
            n = 1 + int(round((i / 2) / 31 * (p.nt - 1)))
            jobs.append((p, n, p.u0 if n == 1 else U[n - 2].copy(), U[n - 1].copy(), float(np.max(np.abs(U)))))
        del U
    print(f"[fullsize] heat batch: worst residual / bound over all levels {worst:.3f}", flush=True)
    assert worst <= 1.0, worst
    errs = resolve_errors(jobs)
    print(f"[fullsize] heat batch: oracle steps at {len(jobs)} levels: max rel. diff {max(errs):.2e}", flush=True)
    assert max(errs) <= 1e-8, errs
    i = min(range(len(probs)), key=lambda q: probs[q].dof)
    Uo, _ = sequential.solve_sequential(probs[i], levels=3)
    e = float(np.max(np.abs(Us[i][:3].cpu().numpy() - Uo)) / np.max(np.abs(Uo)))
    assert e <= 1e-8, e


@pytest.mark.timeout(400)
def test_fullsize_learned_start_burgers256x256_mixed():
    """The learned-iterate workload at its full size (Burgers nu = 0.005, 256^2 x 256 levels):
    a network of the production shape (width 32, 12 modes, 4 layers, 16 temporal modes) trained
    briefly on method-generated solves gives the start, the mixed-precision solve converges from
    it, and the result is the oracle's at every level."""
    import paper_2406_00878_amd.neural as NO
    cfg = NO.NOConfig(nx=256, ny=256, nt=256, width=32, modes=12, layers=4, tmodes=16)
    net = NO.NeuralOperator(cfg, seed=5)
    print("[fullsize] learned: generate 48 solves, train 4 epochs", flush=True)
    u0s, coefs, _ = NO.generate(net, lambda i: W.burgers256_learned(nt=256, index=i), 48)
    NO.train(net, u0s, coefs, epochs=4, lr=2e-3, batch=8)
    del u0s, coefs
    p = W.burgers256_learned(nt=256, index=2000)
    u0 = dev(p.u0)
    U = torch.empty((p.nt, p.ny, p.nx), dtype=torch.float64, device="cuda")
    j = net.initial_iterate(p, u0, U)
    print(f"[fullsize] learned: judge {j}", flush=True)
    st = P.solve(p, U, u0, tol=1e-10, max_iter=60, precision="mixed", cache_tag=1)
    assert st["converged"], st
    Uh = U.cpu().numpy()
    ratio = all_level_residual_ratio(Uh, p, tol=1e-10)
    assert ratio <= 1.0, ratio
    jobs = [(p, n, p.u0 if n == 1 else Uh[n - 2], Uh[n - 1], float(np.max(np.abs(Uh)))) for n in sampled_levels(p.nt)]
    errs = resolve_errors(jobs)
    print(f"[fullsize] learned: oracle steps at {len(jobs)} levels: max rel. diff {max(errs):.2e}", flush=True)
    assert max(errs) <= 1e-8, errs
    Us, _ = sequential.solve_sequential(p, levels=2)
    assert float(np.max(np.abs(Uh[:2] - Us)) / np.max(np.abs(Us))) <= 1e-8

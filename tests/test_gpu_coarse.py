"""The coarse-grid initial iterate (Section 4) through the C ABI against the oracle's: the same
coarse solution (all-at-once on the GPU, sequential in the oracle; equal by Theorem 1) carried to
the fine grid by the same cubic splines."""
import numpy as np
import pytest
import torch

import paper_2406_00878_amd as P
import workloads as W
from oracle import coarse, sequential

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _cases():
    rng = np.random.default_rng(71)
    return [
        ("burgers_per32_cf4", W.burgers_periodic(32, 8, 5e-4, 0.01, W.fourier_u0_periodic(32, 72, kmax=3)), 4),
        ("burgers_per96_cf3", W.burgers_periodic(96, 12, 5e-4, 0.01, W.fourier_u0_periodic(96, 73, kmax=4)), 3),
        ("heat_dir31_cf4", W.heat_dirichlet(31, 12, 1e-3, W.sine_u0_dirichlet(31, rng)), 4),
        ("heat_dir31_cf2", W.heat_dirichlet(31, 6, 1e-3, W.sine_u0_dirichlet(31, rng)), 2),
        ("heat_dir71x8_cf8", W.heat_dirichlet(71, 16, 2e-3, W.sine_u0_dirichlet(71, rng)), 8),
    ]


@pytest.mark.parametrize("name,prob,cf", _cases(), ids=lambda v: v if isinstance(v, str) else "")
def test_coarse_iterate_matches_oracle(name, prob, cf):
    U = torch.empty((prob.nt, prob.ny, prob.nx), dtype=torch.float64, device="cuda")
    print(f"[coarse] {name}", flush=True)
    st = P.coarse_initial_iterate(prob, U, dev(prob.u0), cf, tol=1e-13)
    assert st["converged"], st
    Ug, Uc = coarse.coarse_initial_iterate(prob, cf)
    err = np.max(np.abs(host(U) - Ug)) / np.max(np.abs(Ug))
    assert err <= 1e-10, (name, err)


def test_newton_from_the_coarse_iterate_reaches_the_oracle_solution():
    """Started from the coarse iterate, the all-at-once Newton iteration needs fewer steps than
    from the plain one and reaches the same root."""
    rng = np.random.default_rng(74)
    p = W.heat_dirichlet(63, 32, 1e-3, W.sine_u0_dirichlet(63, rng))
    u0 = dev(p.u0)
    U = torch.empty((p.nt, p.ny, p.nx), dtype=torch.float64, device="cuda")
    P.coarse_initial_iterate(p, U, u0, 4, tol=1e-12)
    st_c = P.solve(p, U, u0, tol=1e-12, max_iter=40, schedule="bulk")
    Uo, _ = sequential.solve_sequential(p)
    assert np.max(np.abs(host(U) - Uo)) <= 1e-10 * np.max(np.abs(Uo))
    V = dev(p.plain_iterate())
    st_p = P.solve(p, V, u0, tol=1e-12, max_iter=40, schedule="bulk")
    print("Newton steps: coarse start", st_c["iterations"], "plain start", st_p["iterations"])
    assert st_c["iterations"] < st_p["iterations"], (st_c["iterations"], st_p["iterations"])


def test_coarse_iterate_rejects_sizes_cf_does_not_divide():
    p = W.burgers_periodic(32, 8, 5e-4, 0.01, W.fourier_u0_periodic(32, 75, kmax=3))
    U = torch.empty((p.nt, p.ny, p.nx), dtype=torch.float64, device="cuda")
    with pytest.raises(P.PTSError):
        P.coarse_initial_iterate(p, U, dev(p.u0), 3)  # 3 divides neither 32 nor 8
    with pytest.raises(P.PTSError):
        P.coarse_initial_iterate(p, U, dev(p.u0), 16)  # 2 coarse nodes per direction

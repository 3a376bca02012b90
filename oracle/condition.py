"""Condition-number estimate of the decoupled system (oracle, test infrastructure only).

Section 7: for the linear heat equation with identical blocks A = I + tau mu Lap_h,
the eigenvalues of the five-point Laplacian are (4/h^2) sin^2(pi k h / 2) summed
over both directions, so one block has condition number about
    K = (1 + 8 mu tau / h^2) / (1 + 2 pi^2 mu tau)
and the product of n blocks about K^n. Requiring K^{N_t} below c h^4 / eps_rof
with tau = 1/N_t is Eq. (cond); the paper's example (N_x = N_y = 64, mu = 1e-3,
c = 1, eps_rof = 1e-16) allows at most 22 levels.

Parity: pinned to the paper's worked example (22 levels) in tests/test_oracle.py.
"""
from __future__ import annotations

import math


def block_condition(mu, tau, h):
    """K = (1 + 8 mu tau / h^2) / (1 + 2 pi^2 mu tau)."""
    return (1.0 + 8.0 * mu * tau / (h * h)) / (1.0 + 2.0 * math.pi ** 2 * mu * tau)


def max_levels_eq_cond(nx, mu, c=1.0, eps_rof=1e-16, nmax=100000):
    """Largest N_t with K(tau = 1/N_t)^{N_t} < c h^4 / eps_rof, h = 1/nx (Eq. (cond))."""
    h = 1.0 / nx
    rhs = math.log(c * h ** 4 / eps_rof)
    best = 0
    for nt in range(1, nmax + 1):
        if nt * math.log(block_condition(mu, 1.0 / nt, h)) < rhs:
            best = nt
        else:
            break
    return best

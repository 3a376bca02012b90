"""Sequential BDF1 time stepper with Newton at every step (oracle, test infrastructure only).

Section 2 (after Eq. (3)): the discrete equations are solved one time level after
another, n = 1..N_t, each by Newton's method started from the previous level.
By Theorem 1 the all-at-once Newton iteration has the same root, so this is the
reference the all-at-once HIP path is compared with.

Per step: v <- u^{n-1}; repeat G = v - u^{n-1} + tau_n F(v); A = I + tau_n dF/du(v) (tau_n =
t^n - t^{n-1}, Eq. (3));
solve A d = -G; v <- v + d; until ||G||_inf <= tol. Linear solves are exact sparse
LU for small levels and BiCGSTAB with a tight relative tolerance for large ones (the
root does not depend on the linear solver; only the Newton path does).

A level is accepted only at tol, or where the residual has stopped decreasing at the
roundoff floor of its own terms (a few ulps of |u^n|, |u^{n-1}| and the largest
viscous and convective terms of tau F). Anything else (a stall above that floor, or
maxit steps) raises OracleNotConverged: a reference that silently returns an
unconverged level would make every comparison against it meaningless.

Parity: pinned by the closed-form linear-heat decay (on both linear-solver branches:
LU below 128^2 nodes, BiCGSTAB above), the agreement of the BiCGSTAB solve with an
exact LU of the same matrix on 130^2-140^2 levels, the scalar-cubic step and the
invariants in tests/test_oracle*.py.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .discretization import level_bvals, level_jacobian, level_residual

LU_MAX_NS = 128 * 128
EPS = np.finfo(np.float64).eps


class OracleNotConverged(RuntimeError):
    """A BDF1 level whose Newton iteration ended above tol and above the roundoff floor."""


def linear_solve(A, b, rtol=1e-14, method=None):
    """Solve A x = b: sparse LU for small systems, BiCGSTAB otherwise.

    method forces "lu" or "bicgstab" (tests of each branch); None picks by size.
    """
    n = b.size
    if method is None:
        method = "lu" if n <= LU_MAX_NS else "bicgstab"
    if method == "lu":
        return spla.splu(A.tocsc()).solve(b)
    x, info = spla.bicgstab(A, b, rtol=rtol, atol=0.0, maxiter=4000)
    if info != 0:
        return spla.splu(A.tocsc()).solve(b)
    return x


def roundoff_floor(v, uprev, p, tau=None):
    """Residual level below which rounding of G's own terms dominates (64 ulps of their size)."""
    vmax = float(np.max(np.abs(v)))
    mu_max = p.mu_a + p.mu_b * vmax * vmax
    visc = 2.0 * mu_max * (2.0 / p.hx ** 2 + 2.0 / p.hy ** 2) * vmax
    conv = abs(p.cflux) * vmax * vmax * (1.0 / p.hx + 1.0 / p.hy)
    return 64.0 * EPS * (vmax + float(np.max(np.abs(uprev))) + (p.dt if tau is None else tau) * (visc + conv))


def bdf1_step(uprev, p, n, tol=1e-13, maxit=50, method=None):
    """Advance one BDF1 level by Newton's method. Returns (u^n, iterations, residual history).

    Raises OracleNotConverged when the level is not solved (see the module header).
    """
    bv = level_bvals(p, n)
    tau = p.tau(n)
    v = uprev.copy()
    hist = []
    best, stall = np.inf, 0
    for it in range(maxit):
        G = level_residual(v, uprev, p, bv, tau)
        g = float(np.max(np.abs(G)))
        hist.append(g)
        if g <= tol:
            return v, it, hist
        if not np.isfinite(g):
            raise OracleNotConverged(f"level {n}: non-finite residual at Newton step {it}")
        # stagnation: no new smallest residual over two Newton steps (a residual that
        # oscillates at the rounding level counts, not only one that rises twice in a row)
        if g < best:
            best, vbest, stall = g, v, 0
        else:
            stall += 1
            if stall >= 2:
                floor = roundoff_floor(vbest, uprev, p, tau)
                if best <= floor:
                    return vbest, it, hist
                raise OracleNotConverged(
                    f"level {n}: residual stalled at {best:.3e} (tol {tol:.1e}, roundoff floor {floor:.1e})")
        A = level_jacobian(v, p, bv, tau)
        d = linear_solve(A, -G.ravel(), method=method)
        v = v + d.reshape(v.shape)
    raise OracleNotConverged(f"level {n}: {maxit} Newton steps, residual {hist[-1]:.3e}")


def solve_sequential(p, tol=1e-13, levels=None, callback=None, method=None):
    """Sequential BDF1 solution U[n-1] = u^n for n = 1..levels (default all N_t levels)."""
    nt = p.nt if levels is None else levels
    U = np.empty((nt, p.ny, p.nx))
    iters = []
    u = np.array(p.u0, dtype=np.float64)
    for n in range(1, nt + 1):
        u, it, hist = bdf1_step(u, p, n, tol, method=method)
        U[n - 1] = u
        iters.append(it)
        if callback is not None:
            callback(n, u, it, hist)
    return U, iters

"""Sequential BDF1 time stepper with Newton at every step (oracle, test infrastructure only).

Section 2 (after Eq. (3)): the discrete equations are solved one time level after
another, n = 1..N_t, each by Newton's method started from the previous level.
By Theorem 1 the all-at-once Newton iteration has the same root, so this is the
reference the all-at-once HIP path is compared with.

Per step: v <- u^{n-1}; repeat G = v - u^{n-1} + tau F(v); A = I + tau dF/du(v);
solve A d = -G; v <- v + d; until ||G||_inf <= tol or the residual stops
decreasing. Linear solves are exact sparse LU for small levels and BiCGSTAB with
a tight relative tolerance for large ones (the root does not depend on the
linear solver; only the Newton path does).

Parity: pinned by the closed-form linear-heat decay, the scalar-cubic step and
the invariants in tests/test_oracle_*.py.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .discretization import level_bvals, level_jacobian, level_residual

LU_MAX_NS = 128 * 128


def linear_solve(A, b, rtol=1e-14):
    """Solve A x = b: sparse LU for small systems, BiCGSTAB otherwise."""
    n = b.size
    if n <= LU_MAX_NS:
        return spla.splu(A.tocsc()).solve(b)
    x, info = spla.bicgstab(A, b, rtol=rtol, atol=0.0, maxiter=4000)
    if info != 0:
        return spla.splu(A.tocsc()).solve(b)
    return x


def bdf1_step(uprev, p, n, tol=1e-13, maxit=50):
    """Advance one BDF1 level by Newton's method. Returns (u^n, iterations, residual history)."""
    bv = level_bvals(p, n)
    v = uprev.copy()
    hist = []
    stall = 0
    for it in range(maxit):
        G = level_residual(v, uprev, p, bv)
        g = float(np.max(np.abs(G)))
        hist.append(g)
        if g <= tol:
            return v, it, hist
        if len(hist) > 1 and g >= hist[-2]:
            stall += 1
            if stall >= 2:
                return v, it, hist
        else:
            stall = 0
        A = level_jacobian(v, p, bv)
        d = linear_solve(A, -G.ravel())
        v = v + d.reshape(v.shape)
    return v, maxit, hist


def solve_sequential(p, tol=1e-13, levels=None, callback=None):
    """Sequential BDF1 solution U[n-1] = u^n for n = 1..levels (default all N_t levels)."""
    nt = p.nt if levels is None else levels
    U = np.empty((nt, p.ny, p.nx))
    iters = []
    u = np.array(p.u0, dtype=np.float64)
    for n in range(1, nt + 1):
        u, it, hist = bdf1_step(u, p, n, tol)
        U[n - 1] = u
        iters.append(it)
        if callback is not None:
            callback(n, u, it, hist)
    return U, iters

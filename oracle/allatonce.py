"""All-at-once space-time Newton system (oracle, test infrastructure only).

Section 3, Eq. (4)-(6): all N_t tau-scaled BDF1 equations form one global system.
One Newton step solves the block lower-bidiagonal system

    [ A_1               ] [du^1]   [r^1]
    [ -I  A_2           ] [du^2] = [r^2] ,   A_n = I + tau dF/du(u^n_k),
    [      .    .       ] [ .. ]   [ ..]     r^n = -G^n(U_k).
    [          -I  A_Nt ] [du^N]   [r^N]

Three independent evaluations of that step are kept here:
  * newton_step_direct      sparse LU of the whole space-time matrix (the plain
                            definition of the Newton step);
  * newton_step_inverse     Eq. (7): du^n = sum_{j<=n} A_n^{-1} ... A_j^{-1} r^j,
                            the exact block lower-triangular inverse (each product
                            applied right to left as Remark 1 requires);
  * newton_step_theorem1    Theorem 1, Eq. (8): P^n du^n = rt^n with the explicit
                            products P^n = A_1 ... A_n and rt^n = sum_j P^{j-1} r^j,
                            built with the recursion of Section 5
                            (P^{n+1} = P^n A_{n+1}, rt^{n+1} = P^n r^{n+1} + rt^n),
                            optionally restarted every `window` levels, where
                            the restart carries du^{w0-1} into rt^{w0} through
                            the -I block of Eq. (6).

Parity: newton_step_direct is the definition. The other two are pinned to it on
tiny grids (they agree to roundoff while the product condition numbers are small).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .discretization import level_bvals, level_jacobian, level_residual


def global_residual(U, p):
    """R = [r^1 .. r^Nt] with r^n = -G^n(U), shape (nt, ny, nx)."""
    R = np.empty_like(U)
    prev = p.u0
    for n in range(1, p.nt + 1):
        R[n - 1] = -level_residual(U[n - 1], prev, p, level_bvals(p, n), p.tau(n))
        prev = U[n - 1]
    return R


def level_blocks(U, p):
    """[A_1 .. A_Nt] at the iterate U."""
    return [level_jacobian(U[n - 1], p, level_bvals(p, n), p.tau(n)) for n in range(1, p.nt + 1)]


def global_jacobian(U, p) -> sp.csr_matrix:
    """The block lower-bidiagonal space-time matrix of Eq. (6)."""
    A = level_blocks(U, p)
    ns = p.ns
    eye = sp.identity(ns, format="csr")
    rows = []
    for n in range(p.nt):
        row = [None] * p.nt
        row[n] = A[n]
        if n > 0:
            row[n - 1] = -eye
        rows.append(row)
    return sp.bmat(rows, format="csr")


def newton_step_direct(U, p):
    """Global Newton step dU = M^{-1} R by sparse LU of the whole space-time matrix."""
    M = global_jacobian(U, p)
    R = global_residual(U, p)
    dU = spla.splu(M.tocsc()).solve(R.ravel())
    return dU.reshape(U.shape), R


def newton_step_inverse(U, p):
    """Global Newton step by the explicit block inverse of Eq. (7).

    du^n = A_n^{-1} r^n + A_n^{-1} A_{n-1}^{-1} r^{n-1} + ... + A_n^{-1} ... A_1^{-1} r^1,
    each term evaluated right to left with independent sparse solves.
    """
    A = level_blocks(U, p)
    lu = [spla.splu(a.tocsc()) for a in A]
    R = global_residual(U, p)
    dU = np.zeros_like(U)
    for n in range(p.nt):
        acc = np.zeros(p.ns)
        for j in range(n + 1):
            v = R[j].ravel()
            for i in range(j, n + 1):  # A_j^{-1} first, A_n^{-1} last
                v = lu[i].solve(v)
            acc += v
        dU[n] = acc.reshape(p.ny, p.nx)
    return dU, R


def newton_step_theorem1(U, p, window=None):
    """Global Newton step by Theorem 1 with explicit dense products P^n (tiny grids only).

    Within each window of consecutive levels starting at w0, level w solves
    P_w du^w = rt^w with P_w = A_{w0} ... A_w and rt^w = sum_{j=w0..w} P_{j-1} b^j,
    where b^{w0} = r^{w0} + du^{w0-1} and b^j = r^j otherwise (P_{w0-1} = I).
    window = None means a single window of all N_t levels (the paper's form).
    """
    A = [a.toarray() for a in level_blocks(U, p)]
    R = global_residual(U, p)
    W = p.nt if window is None else window
    dU = np.zeros_like(U)
    prev = np.zeros(p.ns)
    for w0 in range(0, p.nt, W):
        P = np.eye(p.ns)
        rt = np.zeros(p.ns)
        for w in range(w0, min(w0 + W, p.nt)):
            b = R[w].ravel() + (prev if w == w0 else 0.0)
            rt = P @ b + rt  # rt^{w} = P^{w-1} b^w + rt^{w-1}
            P = P @ A[w]  # P^{w} = P^{w-1} A_w
            dU[w] = np.linalg.solve(P, rt).reshape(p.ny, p.nx)
        prev = dU[min(w0 + W, p.nt) - 1].ravel()
    return dU, R


def solve_allatonce(p, U0=None, tol=1e-12, maxit=60, step=newton_step_direct):
    """Global Newton iteration from U0 (default u^n = u^0) until ||R||_inf <= tol.

    Returns (U, history of ||R||_inf, history of the RMS update norm of Section 8.1).
    """
    U = p.plain_iterate() if U0 is None else np.array(U0, dtype=np.float64)
    rhist, uhist = [], []
    for _ in range(maxit):
        dU, R = step(U, p)
        r = float(np.max(np.abs(R)))
        rhist.append(r)
        if r <= tol:
            break
        U = U + dU
        uhist.append(float(np.sqrt(np.mean(dU * dU))))
    return U, rhist, uhist

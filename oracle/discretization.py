"""Spatial discretization of one time level (oracle, test infrastructure only).

Follows Section 2, Eq. (3): BDF1 in time, second-order central differences of
the inviscid fluxes, and the conservative three-point viscous operator with face
viscosities. Everything is moved to the left-hand side as in Section 3, Eq. (4),
and multiplied by the step size tau as the paper does before linearizing (Eq. (5)):

    G^n(u^n) = u^n - u^{n-1} + tau F(u^n)            (q^n = 0: no source term;
                                                     Dirichlet data enter through
                                                     the ghost ring)
    F_P = [f(u_E) - f(u_W)] / (2 hx) + [g(u_N) - g(u_S)] / (2 hy)
          - [mu_e (u_E - u_P) - mu_w (u_P - u_W)] / hx^2
          - [mu_n (u_N - u_P) - mu_s (u_P - u_S)] / hy^2

with f = g = cflux u^2 and mu(u) = mu_a + mu_b u^2. Readings taken where the
paper is silent or garbled:
  * face viscosity mu_{i+1/2} = mu((u_i + u_{i+1}) / 2), viscosity of the mean
    of the two nodal values (the paper does not define it; this reading
    reproduces the heat-equation errors of Table 1 to the printed digits, while
    the mean of the nodal viscosities misses them by a factor of 1.9);
  * the y-flux in Eq. (3) is printed with f; g is meant (f = g in both models);
  * A_n = I + tau dF/du (the paper's tau-scaled block, Eq. (6)); r^n = -G^n.

Pins (tests/test_oracle_*.py): complex-step derivatives of the residual pin the
Jacobian; the closed-form discrete Fourier decay of linear heat pins the stencil
scale, the boundary treatment and BDF1; a scalar cubic solved by numpy.roots pins
one nonlinear step; conservation and symmetry invariants pin the flux form.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

DIRICHLET = 0
PERIODIC = 1


def ghost(u: np.ndarray, bc: int, bvals=None) -> np.ndarray:
    """Level field with a one-node ghost ring: boundary data (Dirichlet) or wrap (periodic).

    bvals is the level's Dirichlet data ordered south row, north row, west
    column, east column (None = zero). Corner ghosts are never read.
    """
    ny, nx = u.shape
    g = np.zeros((ny + 2, nx + 2), dtype=u.dtype)
    g[1:-1, 1:-1] = u
    if bc == PERIODIC:
        g[0, 1:-1] = u[-1, :]
        g[-1, 1:-1] = u[0, :]
        g[1:-1, 0] = u[:, -1]
        g[1:-1, -1] = u[:, 0]
    elif bvals is not None:
        g[0, 1:-1] = bvals[0:nx]
        g[-1, 1:-1] = bvals[nx:2 * nx]
        g[1:-1, 0] = bvals[2 * nx:2 * nx + ny]
        g[1:-1, -1] = bvals[2 * nx + ny:2 * nx + 2 * ny]
    return g


def _neighbours(g):
    """Centre, west, east, south, north views of a ghosted field."""
    return g[1:-1, 1:-1], g[1:-1, :-2], g[1:-1, 2:], g[:-2, 1:-1], g[2:, 1:-1]


def viscosity(p, v):
    """mu(v) = mu_a + mu_b v^2."""
    return p.mu_a + p.mu_b * v * v


def _face_viscosities(p, uP, uW, uE, uS, uN):
    """mu at the east, west, north and south faces: mu of the mean of the two nodal values."""
    return (viscosity(p, 0.5 * (uP + uE)), viscosity(p, 0.5 * (uP + uW)),
            viscosity(p, 0.5 * (uP + uN)), viscosity(p, 0.5 * (uP + uS)))


def spatial_operator(u, p, bvals=None):
    """F(u) of Eq. (3) (inviscid minus viscous terms) at every node of one level."""
    g = ghost(u, p.bc, bvals)
    uP, uW, uE, uS, uN = _neighbours(g)
    mu_e, mu_w, mu_n, mu_s = _face_viscosities(p, uP, uW, uE, uS, uN)
    cf = p.cflux
    conv = cf * (uE * uE - uW * uW) / (2.0 * p.hx) + cf * (uN * uN - uS * uS) / (2.0 * p.hy)
    visc = (mu_e * (uE - uP) - mu_w * (uP - uW)) / p.hx ** 2 \
        + (mu_n * (uN - uP) - mu_s * (uP - uS)) / p.hy ** 2
    return conv - visc


def level_residual(u, uprev, p, bvals=None, tau=None):
    """G^n = u^n - u^{n-1} + tau_n F(u^n): the tau-scaled BDF1 equation of one level (tau_n =
    t^n - t^{n-1}, Eq. (3); default the problem's uniform step)."""
    return u - uprev + (p.dt if tau is None else tau) * spatial_operator(u, p, bvals)


def jacobian_stencil(u, p, bvals=None, tau=None):
    """Five coefficients (C, W, E, S, N) of A = I + tau dF/du at every node.

    Entry X at node P is dG_P / du_X for the neighbour X of P. For Dirichlet
    problems a neighbour on the boundary is data, so its coefficient is set to
    zero. For periodic problems the neighbour index wraps.
    """
    g = ghost(u, p.bc, bvals)
    uP, uW, uE, uS, uN = _neighbours(g)
    mu_e, mu_w, mu_n, mu_s = _face_viscosities(p, uP, uW, uE, uS, uN)
    # d mu_face / d u_node = mu'(mean) / 2 = mu_b * mean for either node of the face
    b = p.mu_b
    hx2, hy2 = p.hx ** 2, p.hy ** 2
    cf = p.cflux
    dE_ = -(mu_e + 0.5 * b * (uE * uE - uP * uP)) / hx2 + cf * uE / p.hx
    dW_ = -(mu_w - 0.5 * b * (uP * uP - uW * uW)) / hx2 - cf * uW / p.hx
    dN_ = -(mu_n + 0.5 * b * (uN * uN - uP * uP)) / hy2 + cf * uN / p.hy
    dS_ = -(mu_s - 0.5 * b * (uP * uP - uS * uS)) / hy2 - cf * uS / p.hy
    dP_ = (mu_e + mu_w - 0.5 * b * (uE * uE - uP * uP) + 0.5 * b * (uP * uP - uW * uW)) / hx2 \
        + (mu_n + mu_s - 0.5 * b * (uN * uN - uP * uP) + 0.5 * b * (uP * uP - uS * uS)) / hy2
    tau = p.dt if tau is None else tau
    C = 1.0 + tau * dP_
    W, E, S, N = tau * dW_, tau * dE_, tau * dS_, tau * dN_
    if p.bc == DIRICHLET:
        W = W.copy(); E = E.copy(); S = S.copy(); N = N.copy()
        W[:, 0] = 0.0
        E[:, -1] = 0.0
        S[0, :] = 0.0
        N[-1, :] = 0.0
    return C, W, E, S, N


def stencil_to_sparse(coef, p) -> sp.csr_matrix:
    """Assemble the N_s x N_s sparse matrix of a five-coefficient stencil (sums repeated columns)."""
    C, W, E, S, N = coef
    ny, nx = C.shape
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    row = (jj * nx + ii).ravel()
    rows, cols, vals = [row], [row], [C.ravel()]
    for arr, dj, di in ((W, 0, -1), (E, 0, 1), (S, -1, 0), (N, 1, 0)):
        j2, i2 = jj + dj, ii + di
        if p.bc == PERIODIC:
            j2 %= ny
            i2 %= nx
            keep = np.ones_like(row, dtype=bool)
        else:
            keep = ((j2 >= 0) & (j2 < ny) & (i2 >= 0) & (i2 < nx)).ravel()
        rows.append(row[keep])
        cols.append((j2 * nx + i2).ravel()[keep])
        vals.append(arr.ravel()[keep])
    n = nx * ny
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n)).tocsr()


def level_jacobian(u, p, bvals=None, tau=None) -> sp.csr_matrix:
    """A = I + tau_n dF/du at u, as a sparse matrix (Eq. (6))."""
    return stencil_to_sparse(jacobian_stencil(u, p, bvals, tau), p)


def level_bvals(p, n):
    """Dirichlet data of level n (1-based), or None for zero data / periodic problems."""
    if p.bc != DIRICHLET or p.bdata is None:
        return None
    return p.bdata[n - 1]

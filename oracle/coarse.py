"""Coarse-grid initial iterate (oracle, test infrastructure only).

Section 4 (initial guess of the all-at-once Newton iteration): the problem is solved
sequentially on a grid coarsened by the same factor c_f in each spatial direction and in
time, and the coarse solution is carried to the fine space-time grid by 1-D cubic splines.
Sections 8.1 and 8.2 use c_f = 4 (heat) and c_f = 3 (Burgers).

Readings where the paper is silent (the same on the HIP side):
  * coarse nodes are every c_f-th fine node: periodic node x_k = k c_f h_x (fine index
    k c_f, when c_f divides n_x); Dirichlet interior node k at (k + 1) c_f h_x (fine interior
    index (k + 1) c_f - 1, when c_f divides n_x + 1), the domain edges staying where they are;
    coarse step c_f tau, coarse level m at t = m c_f tau (c_f divides N_t); u^0 and the
    Dirichlet data restricted by injection (coarse level m takes the fine data of level m c_f);
  * grids that c_f does not divide (the paper's grids all nest): the coarse grid spans the
    same domain with floor(n_x / c_f) periodic nodes or floor((n_x + 1) / c_f) - 1 Dirichlet
    interior nodes, evenly spaced (h_c = domain length / coarse intervals; c_f h_x when the
    grids nest), and ceil(N_t / c_f) coarse levels of step c_f tau (the last may lie past the
    fine end time; the time spline is only evaluated up to it); u^0 at a coarse node is the
    bilinear interpolant of the fine u^0 there (the injected value when the node is a fine
    node); Dirichlet data need nesting grids and levels;
  * spatial splines: x first, then y; periodic lines close with the period, Dirichlet lines
    take the boundary values as end nodes (x lines: the coarse data of the west and east
    edges; y lines: the fine data of the south and north edges at the coarse level's time)
    with not-a-knot end conditions (the usual default of cubic-spline routines; natural ends
    would force a zero second derivative at the edges, which the Section 8.1 solution lacks);
  * time: after the spatial splines, a spline through t = 0 (the fine u^0) and the coarse
    levels at every fine node, not-a-knot end conditions.

The coarse solve is the sequential oracle itself; the splines are scipy's CubicSpline.
Parity: pinned in tests/test_oracle.py (interpolation property at coarse nodes, fourth-order
convergence on smooth periodic and Dirichlet fields, exact reproduction of cubic fields with
nonzero Dirichlet data, the coarse start of the Section 8.1 exact-solution problem close to the
exact solution; on grids that do not nest: the sampled u^0 exact for bilinear fields, cubic
fields reproduced exactly in x, y and t, fourth-order convergence of the periodic splines).
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy.interpolate import CubicSpline

from .sequential import solve_sequential

PERIODIC = 1


def _axis(n, h, cf, periodic):
    """Coarse node count and spacing of one axis with n fine nodes of spacing h."""
    if periodic:
        nc, nested = n // cf, n % cf == 0
        if nc < 3:
            raise ValueError("fewer than 3 coarse nodes")
        return nc, (cf * h if nested else n * h / nc)
    nc, nested = (n + 1) // cf - 1, (n + 1) % cf == 0
    if nc < 1:
        raise ValueError("no coarse interior node")
    return nc, (cf * h if nested else (n + 1) * h / (nc + 1))


def _sample_axis(v, n, nc, periodic, axis):
    """Linear interpolation of v along `axis` (n fine nodes) at the nc coarse node positions.
    The position of coarse node k in fine spacings is k n / nc (periodic) or
    (k + 1)(n + 1) / (nc + 1) - 1 (Dirichlet), taken as a whole part and a remainder."""
    k = np.arange(nc)
    num, den = (k * n, nc) if periodic else ((k + 1) * (n + 1), nc + 1)
    i0 = num // den - (0 if periodic else 1)
    t = (num % den) / den
    i1 = (i0 + 1) % n if periodic else np.minimum(i0 + 1, n - 1)
    v = np.moveaxis(np.asarray(v, dtype=np.float64), axis, -1)
    out = np.where(t == 0.0, v[..., i0], (1.0 - t) * v[..., i0] + t * v[..., i1])
    return np.moveaxis(out, -1, axis)


def coarse_problem(p, cf):
    """The problem on the grid coarsened by cf in x, y and t (u^0 by injection, or by bilinear
    interpolation where the grids do not nest)."""
    if cf < 2:
        raise ValueError("cf must be >= 2")
    per = p.bc == PERIODIC
    nx, hx = _axis(p.nx, p.hx, cf, per)
    ny, hy = _axis(p.ny, p.hy, cf, per)
    nested = p.nt % cf == 0 and (p.nx % cf == 0 and p.ny % cf == 0 if per
                                 else (p.nx + 1) % cf == 0 and (p.ny + 1) % cf == 0)
    u0 = _sample_axis(_sample_axis(p.u0, p.nx, nx, per, 1), p.ny, ny, per, 0)
    bdata = None
    if p.bc != PERIODIC and p.bdata is not None:
        if not nested:
            raise ValueError("Dirichlet data need grids and levels that cf divides")
        S, N, Wd, E = _edges(p)
        lv = slice(cf - 1, None, cf)  # fine level (m + 1) cf for coarse level m + 1
        ix = slice(cf - 1, None, cf)
        bdata = np.concatenate([S[lv][:, ix][:, :nx], N[lv][:, ix][:, :nx], Wd[lv][:, ix][:, :ny],
                                E[lv][:, ix][:, :ny]], axis=1)
    return dataclasses.replace(p, nx=nx, ny=ny, nt=-(-p.nt // cf), hx=hx, hy=hy, dt=cf * p.dt,
                               u0=np.ascontiguousarray(u0), bdata=bdata, name=p.name + f"/cf{cf}")


def _edges(p):
    """Dirichlet data split into its south, north, west and east parts, each [nt][n]."""
    b = np.asarray(p.bdata, dtype=np.float64)
    return (b[:, :p.nx], b[:, p.nx:2 * p.nx], b[:, 2 * p.nx:2 * p.nx + p.ny], b[:, 2 * p.nx + p.ny:])


def _spline_axis(vals, h_c, n_fine, h_fine, periodic, axis, lo=None, hi=None):
    """Cubic spline of coarse values (spacing h_c) along `axis`, evaluated at the fine nodes of
    that axis. Dirichlet lines end in the edge values lo and hi (arrays shaped like vals
    without that axis; zero when None)."""
    vals = np.moveaxis(vals, axis, -1)
    nc = vals.shape[-1]
    if periodic:
        xc = np.arange(nc + 1) * h_c
        yc = np.concatenate([vals, vals[..., :1]], axis=-1)
        s = CubicSpline(xc, yc, axis=-1, bc_type="periodic")
        xf = np.arange(n_fine) * h_fine
    else:
        xc = np.arange(nc + 2) * h_c  # edges at 0 and (nc + 1) h_c = (n_fine + 1) h
        zero = np.zeros(vals.shape[:-1])
        lo = zero if lo is None else lo
        hi = zero if hi is None else hi
        yc = np.concatenate([lo[..., None], vals, hi[..., None]], axis=-1)
        s = CubicSpline(xc, yc, axis=-1, bc_type="not-a-knot")
        xf = (np.arange(n_fine) + 1.0) * h_fine
    return np.moveaxis(s(xf), -1, axis)


def interpolate(p, cf, Uc):
    """Fine space-time iterate [nt][ny][nx] from coarse levels Uc [ceil(nt/cf)][ny_c][nx_c]."""
    per = p.bc == PERIODIC
    Uc = np.asarray(Uc, dtype=np.float64)
    hxc, hyc = _axis(p.nx, p.hx, cf, per)[1], _axis(p.ny, p.hy, cf, per)[1]
    wl = wh = sl = sh = None
    if not per and p.bdata is not None:
        S, N, Wd, E = _edges(p)
        lv, iy = slice(cf - 1, None, cf), slice(cf - 1, None, cf)
        wl, wh = Wd[lv][:, iy][:, :Uc.shape[1]], E[lv][:, iy][:, :Uc.shape[1]]  # [m][yc]
        sl, sh = S[lv], N[lv]  # [m][x] at the coarse levels' times
    V = _spline_axis(Uc, hxc, p.nx, p.hx, per, axis=2, lo=wl, hi=wh)
    V = _spline_axis(V, hyc, p.ny, p.hy, per, axis=1, lo=sl, hi=sh)
    tc = np.arange(Uc.shape[0] + 1) * cf * p.dt
    data = np.concatenate([np.asarray(p.u0, dtype=np.float64)[None], V], axis=0)
    s = CubicSpline(tc, data, axis=0, bc_type="not-a-knot")
    return s(np.arange(1, p.nt + 1) * p.dt)


def coarse_initial_iterate(p, cf, tol=1e-13):
    """Section 4's initial iterate: sequential coarse solve, then the splines."""
    pc = coarse_problem(p, cf)
    Uc, _ = solve_sequential(pc, tol=tol)
    return interpolate(p, cf, Uc), Uc

"""Seeded synthetic inputs for the space-time BDF1 problems.

This module holds only problem descriptions and input fields (grids, initial
conditions, boundary data). It contains none of the method's arithmetic: no
residuals, Jacobians or solves. Both the CPU oracle and the HIP path take their
inputs from here, so the two sides see identical data.

Problem statement (Section 2, Eq. (1)-(2)): a scalar 2-D conservation law
    u_t + f(u)_x + g(u)_y = (mu(u) u_x)_x + (mu(u) u_y)_y
with f = g = cflux * u^2 (Burgers: cflux = 1/2; heat: cflux = 0) and
mu(u) = mu_a + mu_b * u^2 (the paper's heat model is mu_a = 0, mu_b = mu_0;
the heat model k(u) = 1 + u^2 is mu_a = mu_b = 1; Burgers is mu_b = 0).

Grids count unknowns. A Dirichlet problem with nx x ny unknowns has interior
nodes x_i = x0 + (i+1) hx, i = 0..nx-1, and boundary nodes at x0 and
x0 + (nx+1) hx. A periodic problem with nx x ny unknowns has nodes
x_i = x0 + i hx with hx = Lx / nx.

Level vectors are stored x fastest, rows in y (Section 3, Eq. (4)): index
j*nx + i for node (x_i, y_j). The space-time iterate holds levels 1..nt; the
initial condition u^0 is separate.

Dirichlet boundary data for level n (1..nt) is a vector of 2(nx+ny) values in
the order: south row (y = y0, i = 0..nx-1), north row (i = 0..nx-1), west
column (x = x0, j = 0..ny-1), east column (j = 0..ny-1). None means zero.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

HEAT = 0
BURGERS = 1
DIRICHLET = 0
PERIODIC = 1


@dataclasses.dataclass
class Problem:
    """One space-time instance: model, grid, step size and data."""

    kind: int  # HEAT | BURGERS (chooses cflux)
    bc: int  # DIRICHLET | PERIODIC
    nx: int
    ny: int
    nt: int
    hx: float
    hy: float
    dt: float
    mu_a: float
    mu_b: float
    u0: np.ndarray  # (ny, nx) float64
    bdata: Optional[np.ndarray] = None  # (nt, 2*(nx+ny)) float64 or None (zero)
    dts: Optional[np.ndarray] = None  # (nt,) step sizes tau_n = t^n - t^{n-1}, or None (all dt)
    x0: float = 0.0
    y0: float = 0.0
    name: str = ""

    @property
    def cflux(self) -> float:
        return 0.5 if self.kind == BURGERS else 0.0

    def tau(self, n: int) -> float:
        """Step size of level n (1-based): tau_n = t^n - t^{n-1}."""
        return float(self.dts[n - 1]) if self.dts is not None else float(self.dt)

    def times(self) -> np.ndarray:
        """t^1 .. t^nt."""
        return np.cumsum(self.dts) if self.dts is not None else np.arange(1, self.nt + 1) * self.dt

    @property
    def ns(self) -> int:
        return self.nx * self.ny

    @property
    def dof(self) -> int:
        return self.nt * self.nx * self.ny

    def x_nodes(self) -> np.ndarray:
        i = np.arange(self.nx, dtype=np.float64)
        if self.bc == DIRICHLET:
            return self.x0 + (i + 1.0) * self.hx
        return self.x0 + i * self.hx

    def y_nodes(self) -> np.ndarray:
        j = np.arange(self.ny, dtype=np.float64)
        if self.bc == DIRICHLET:
            return self.y0 + (j + 1.0) * self.hy
        return self.y0 + j * self.hy

    def mesh(self):
        """(X, Y) arrays of shape (ny, nx)."""
        return np.meshgrid(self.x_nodes(), self.y_nodes(), indexing="xy")

    def plain_iterate(self) -> np.ndarray:
        """u^n_0 = u^0 for every level: Newton started from the initial condition."""
        return np.broadcast_to(self.u0, (self.nt, self.ny, self.nx)).copy()


def _normalize_max(u: np.ndarray) -> np.ndarray:
    m = np.max(np.abs(u))
    return u / m if m > 0 else u


def fourier_u0_periodic(n: int, seed: int, kmax: int = 8, power: float = 2.0) -> np.ndarray:
    """Random Fourier sum on the periodic unit square, max |u0| = 1.

    u0 = sum over k in a half lattice with 0 < |k| <= kmax of
         |k|^-power (a_k cos 2 pi k.x + b_k sin 2 pi k.x), a_k, b_k ~ N(0,1).
    Modes are ordered by kx then ky; all a_k are drawn first, then all b_k.
    """
    modes = [(kx, ky) for kx in range(0, kmax + 1) for ky in range(-kmax, kmax + 1)
             if (kx > 0 or ky > 0) and kx * kx + ky * ky <= kmax * kmax]
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(len(modes))
    b = rng.standard_normal(len(modes))
    # separable evaluation: cos(p + q) = cos p cos q - sin p sin q, sin(p + q) = sin p cos q + cos p sin q
    x = np.arange(n, dtype=np.float64) / n
    ks = np.arange(-kmax, kmax + 1)
    cx, sx = np.cos(2 * math.pi * np.outer(ks, x)), np.sin(2 * math.pi * np.outer(ks, x))
    A = np.zeros((2 * kmax + 1, 2 * kmax + 1))  # [ky, kx] coefficients of cos(2 pi k.x)
    B = np.zeros_like(A)  # of sin(2 pi k.x)
    for (kx, ky), ak, bk in zip(modes, a, b):
        amp = (kx * kx + ky * ky) ** (-power / 2.0)
        A[ky + kmax, kx + kmax] = amp * ak
        B[ky + kmax, kx + kmax] = amp * bk
    # u[j, i] = sum_k A (cy cx - sy sx) + B (sy cx + cy sx), rows j = y, columns i = x
    u = cx.T @ A @ cx - sx.T @ A @ sx + sx.T @ B @ cx + cx.T @ B @ sx
    return _normalize_max(u)


def sine_u0_dirichlet(n: int, rng: np.random.Generator, kmax: int = 6,
                      power: float = 3.0) -> np.ndarray:
    """Random sine series vanishing on the boundary of [0,1]^2, max |u0| = 1.

    u0 = sum_{kx,ky >= 1, |k| <= kmax} c_k |k|^-power sin(pi kx x) sin(pi ky y).
    """
    modes = [(kx, ky) for kx in range(1, kmax + 1) for ky in range(1, kmax + 1)
             if kx * kx + ky * ky <= kmax * kmax]
    c = rng.standard_normal(len(modes))
    h = 1.0 / (n + 1)
    x = (np.arange(n, dtype=np.float64) + 1.0) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    u = np.zeros((n, n))
    for (kx, ky), ck in zip(modes, c):
        amp = (kx * kx + ky * ky) ** (-power / 2.0)
        u += ck * amp * np.sin(math.pi * kx * X) * np.sin(math.pi * ky * Y)
    return _normalize_max(u)


def disc_u0_periodic(n: int, seed: int, radius: float = 0.25, noise: float = 1e-3) -> np.ndarray:
    """1 inside the disc of given radius centred at (0.5, 0.5), 0 outside, plus iid U(-noise, noise)."""
    x = np.arange(n, dtype=np.float64) / n
    X, Y = np.meshgrid(x, x, indexing="xy")
    u = ((X - 0.5) ** 2 + (Y - 0.5) ** 2 < radius * radius).astype(np.float64)
    rng = np.random.default_rng(seed)
    return u + rng.uniform(-noise, noise, size=(n, n))


# ---------------------------------------------------------------- workloads

def heat_dirichlet(n: int, nt: int, dt: float, u0: np.ndarray, mu_a=1.0, mu_b=1.0,
                   name="") -> Problem:
    h = 1.0 / (n + 1)
    return Problem(HEAT, DIRICHLET, n, n, nt, h, h, dt, mu_a, mu_b, u0, None, name=name)


def burgers_periodic(n: int, nt: int, dt: float, nu: float, u0: np.ndarray, name="") -> Problem:
    h = 1.0 / n
    return Problem(BURGERS, PERIODIC, n, n, nt, h, h, dt, nu, 0.0, u0, None, name=name)


def heat32(nt: int = 64) -> Problem:
    """Nonlinear heat k(u) = 1 + u^2, 32x32 interior, zero Dirichlet, dt = 1e-3,
    u0 = sin(pi x) sin(pi y)."""
    n = 32
    h = 1.0 / (n + 1)
    x = (np.arange(n) + 1.0) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    u0 = np.sin(math.pi * X) * np.sin(math.pi * Y)
    return heat_dirichlet(n, nt, 1e-3, u0, name=f"heat32_nt{nt}")


def burgers256(nt: int = 512, seed: int = 2406002) -> Problem:
    """Viscous Burgers nu = 0.01, periodic 256^2, dt = 5e-4, random Fourier u0 (|k| <= 8, |k|^-2)."""
    return burgers_periodic(256, nt, 5e-4, 0.01, fourier_u0_periodic(256, seed),
                            name=f"burgers256_nt{nt}")


def burgers512_disc(nt: int = 1024, seed: int = 2406003) -> Problem:
    """Viscous Burgers nu = 1e-3, periodic 512^2, dt = 2.5e-4, disc + 1e-3 noise."""
    return burgers_periodic(512, nt, 2.5e-4, 1e-3, disc_u0_periodic(512, seed),
                            name=f"burgers512disc_nt{nt}")


def burgers256_learned(nt: int = 256, seed: int = 2406055, index: int = 0) -> Problem:
    """Viscous Burgers nu = 0.005, periodic 256^2, dt = 5e-4 (learned-iterate workload)."""
    s = np.random.SeedSequence(seed, spawn_key=(index,))  # child `index` of SeedSequence(seed).spawn
    u0 = fourier_u0_periodic(256, int(s.generate_state(1)[0]))
    return burgers_periodic(256, nt, 5e-4, 0.005, u0, name=f"burgers256nu005_nt{nt}_{index}")


def heat_batch(count: int = 64, seed: int = 2406004, nmin=64, nmax=512, lmin=128, lmax=1024,
               dt: float = 1e-3):
    """Batch of heat instances k(u) = 1 + u^2 with uneven square grids and level counts."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=count)
    ls = rng.integers(lmin, lmax + 1, size=count)
    out = []
    for i in range(count):
        u0 = sine_u0_dirichlet(int(ns[i]), rng)
        out.append(heat_dirichlet(int(ns[i]), int(ls[i]), dt, u0, name=f"heat_b{i}"))
    return out


# ------------------------------------------------- exact-solution problems

def heat_exact(x, y, t, mu0=1e-6, alpha=1.0):
    """Exact solution of the nonlinear heat model mu = mu0 u^2 (Section 8.1)."""
    return np.sqrt(np.sqrt(alpha / mu0) * (x + y) + alpha * t + 1.0)


def burgers_exact(x, y, t, v=0.5, mu=1e-3):
    """Viscous-shock exact solution of the 2-D Burgers model (Section 8.2)."""
    return 0.5 * v * (1.0 - np.tanh(v * (x + y - v * t) / (4.0 * mu)))


def boundary_data(p: Problem, exact, times) -> np.ndarray:
    """Dirichlet data of an exact solution on the boundary nodes for each level time."""
    xs = p.x_nodes()
    ys = p.y_nodes()
    xl, xr = p.x0, p.x0 + (p.nx + 1) * p.hx
    yl, yr = p.y0, p.y0 + (p.ny + 1) * p.hy
    out = np.empty((len(times), 2 * (p.nx + p.ny)))
    for n, t in enumerate(times):
        out[n, 0:p.nx] = exact(xs, yl, t)
        out[n, p.nx:2 * p.nx] = exact(xs, yr, t)
        out[n, 2 * p.nx:2 * p.nx + p.ny] = exact(xl, ys, t)
        out[n, 2 * p.nx + p.ny:] = exact(xr, ys, t)
    return out


def heat_mms(nint: int, mu0=1e-6, alpha=1.0) -> Problem:
    """Paper's heat test (Section 8.1): [0.1,1.1]^2, t in [0,1], N_t = N_x = N_y = nint
    grid intervals, mu = mu0 u^2; Dirichlet data and u0 from the exact solution."""
    h = 1.0 / nint
    n = nint - 1
    p = Problem(HEAT, DIRICHLET, n, n, nint, h, h, 1.0 / nint, 0.0, mu0,
                np.zeros((n, n)), None, x0=0.1, y0=0.1, name=f"heat_mms{nint}")
    X, Y = p.mesh()
    p.u0 = heat_exact(X, Y, 0.0, mu0, alpha)
    p.bdata = boundary_data(p, lambda x, y, t: heat_exact(x, y, t, mu0, alpha),
                            [(n_ + 1) * p.dt for n_ in range(p.nt)])
    return p


def burgers_mms(nint: int, v=0.5, mu=1e-3, x0=0.0, y0=0.0) -> Problem:
    """Paper's Burgers test (Section 8.2) on [x0, x0+1]^2 (the domain is not stated in the
    paper), t in [0,1], N_t = N_x = N_y = nint intervals, constant mu."""
    h = 1.0 / nint
    n = nint - 1
    p = Problem(BURGERS, DIRICHLET, n, n, nint, h, h, 1.0 / nint, mu, 0.0,
                np.zeros((n, n)), None, x0=x0, y0=y0, name=f"burgers_mms{nint}")
    X, Y = p.mesh()
    p.u0 = burgers_exact(X, Y, 0.0, v, mu)
    p.bdata = boundary_data(p, lambda x, y, t: burgers_exact(x, y, t, v, mu),
                            [(n_ + 1) * p.dt for n_ in range(p.nt)])
    return p

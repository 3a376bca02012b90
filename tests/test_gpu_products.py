"""The paper's explicit-product form of Theorem 1 (Section 4, Eq. (8); Section 5, Eq. (9),
Algorithm 1; Section 7 diagonal preconditioner; banded LU without pivoting) through the C ABI:
the products against the oracle's dense products entry by entry (and the 2n^2 + 2n + 1
diagonals of the Section 5 remark), the Newton step against the oracle's Theorem-1 step and
the definition (sparse LU of the whole space-time matrix), and the paper's Tables 1 and 3
replayed with this form."""
import numpy as np
import pytest
import torch

import paper_2406_00878_amd as P
import workloads as W
from oracle import allatonce, coarse, sequential

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _small(kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "heat":
        p = W.heat_dirichlet(9, 5, 2e-3, W.sine_u0_dirichlet(9, rng))
        p = W.Problem(p.kind, p.bc, 9, 7, 5, p.hx, p.hx * 9 / 7, 2e-3, 1.0, 1.0, rng.uniform(-1, 1, (7, 9)),
                      rng.uniform(-0.5, 0.5, (5, 2 * (9 + 7))), name="heat9x7")
    else:
        p = W.burgers_mms(12, x0=-0.5, y0=-0.5)
        p.nt, p.dt, p.bdata = 4, 0.05, p.bdata[:4]
    U = p.plain_iterate() + 0.02 * rng.standard_normal((p.nt, p.ny, p.nx))
    return p, U


@pytest.mark.parametrize("kind", ["heat", "burgers"])
def test_product_diamonds_equal_dense_products(kind):
    """P^n = A_1 ... A_n: every diamond entry equals the dense product's entry, and the dense
    product has no entry outside the 2n^2 + 2n + 1 diagonals."""
    p, U = _small(kind, 3)
    A = [a.toarray() for a in allatonce.level_blocks(U, p)]
    Pd = np.eye(p.ns)
    for n in range(1, p.nt + 1):
        Pd = Pd @ A[n - 1]
        D = host(P.product_diamond(p, dev(U), dev(p.u0), n, bdata=dev(p.bdata)))
        assert D.shape[0] == 2 * n * n + 2 * n + 1
        got = np.zeros_like(Pd)
        e = 0
        for a in range(-n, n + 1):
            for b in range(-(n - abs(a)), n - abs(a) + 1):
                for y in range(p.ny):
                    for x in range(p.nx):
                        if 0 <= x + b < p.nx and 0 <= y + a < p.ny:
                            got[y * p.nx + x, (y + a) * p.nx + x + b] = D[e, y, x]
                e += 1
        assert np.max(np.abs(got - Pd)) <= 1e-12 * np.max(np.abs(Pd)), n


@pytest.mark.parametrize("kind", ["heat", "burgers"])
def test_products_newton_step_equals_theorem1_and_definition(kind):
    """The explicit-product step equals the oracle's Theorem-1 step (dense products) and the
    definition (sparse LU of the space-time matrix) while the products are well conditioned."""
    p, U = _small(kind, 5)
    d_def, _ = allatonce.newton_step_direct(U, p)
    d_thm, _ = allatonce.newton_step_theorem1(U, p)
    Ud = dev(U)
    st = P.newton_step_products(p, Ud, dev(p.u0), bdata=dev(p.bdata))
    got = host(Ud) - U
    scale = np.max(np.abs(d_def))
    print(f"{kind}: |products - definition| {np.max(np.abs(got - d_def)) / scale:.2e}, "
          f"|oracle thm1 - definition| {np.max(np.abs(d_thm - d_def)) / scale:.2e}")
    assert np.max(np.abs(got - d_def)) <= 1e-10 * scale
    assert np.max(np.abs(got - d_thm)) <= 1e-10 * scale
    assert st["res_inf"][0] == pytest.approx(float(np.max(np.abs(allatonce.global_residual(U, p)))), rel=1e-12)


def test_products_solve_matches_sequential_oracle():
    """Newton with every step in the explicit-product form reaches the sequential solution."""
    rng = np.random.default_rng(7)
    p = W.heat_dirichlet(20, 6, 1e-3, W.sine_u0_dirichlet(20, rng))
    U = dev(p.plain_iterate())
    st = P.solve_products(p, U, dev(p.u0), tol=1e-12, max_iter=20)
    assert st["converged"], st
    Us, _ = sequential.solve_sequential(p)
    assert np.max(np.abs(host(U) - Us)) <= 1e-10 * np.max(np.abs(Us))


def _golden(name):
    import os
    rows = []
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(v) for v in line.split()])
    return rows


@pytest.mark.parametrize("row", _golden("table1_heat_linf.txt")[:3], ids=lambda r: f"N{int(r[0])}")
def test_products_reproduce_table1_heat_errors(row):
    """Section 8.1, Table 1 with the paper's own decoupled form (N_t = N_x = N_y = 8, 16, 24
    intervals): the printed L-inf error to three digits."""
    nint, expected = int(row[0]), row[1]
    p = W.heat_mms(nint)
    U = dev(p.plain_iterate())
    st = P.solve_products(p, U, dev(p.u0), tol=1e-12, max_iter=20, bdata=dev(p.bdata))
    assert st["converged"], st
    Uh = host(U)
    X, Y = p.mesh()
    err = max(np.max(np.abs(Uh[n] - W.heat_exact(X, Y, (n + 1) * p.dt))) for n in range(p.nt))
    print(f"Table 1 N = {nint}: {err:.3e} (printed {expected:.2e}), Newton steps {st['iterations']}")
    assert float(f"{err:.2e}") == pytest.approx(expected, rel=1e-9), err


def test_products_table3_newton_counts_from_the_coarse_start():
    """Section 8.1, Table 3 with the explicit-product form (64 x 64 intervals, coarse start
    c_f = 4): 2 Newton iterations at N_t = 8 and 16 bring the RMS update below a tenth of the
    discretization error, as printed."""
    import dataclasses
    counts = {}
    for nt in (8, 16):
        p = W.heat_mms(64)
        ex = lambda x, y, t: W.heat_exact(x, y, t)
        p = dataclasses.replace(p, nt=nt, dt=1.0 / nt, bdata=W.boundary_data(p, ex, [(n + 1) / nt for n in range(nt)]))
        bd, u0 = dev(p.bdata), dev(p.u0)
        U = torch.empty((p.nt, p.ny, p.nx), dtype=torch.float64, device="cuda")
        print(f"[products] table 3, N_t = {nt}", flush=True)
        P.coarse_initial_iterate(p, U, u0, 4, tol=1e-12, bdata=bd)
        st = P.solve_products(p, U, u0, tol=1e-11, max_iter=8, bdata=bd)
        X, Y = p.mesh()
        exact = np.stack([ex(X, Y, (n + 1) * p.dt) for n in range(p.nt)])
        err = np.max(np.abs(host(U) - exact))
        counts[nt] = next(k + 1 for k, r in enumerate(st["upd_rms"]) if r <= 0.1 * err)
        print(f"  RMS updates {[f'{r:.1e}' for r in st['upd_rms']]}, error {err:.2e}", flush=True)
    assert counts == {8: 2, 16: 2}, counts

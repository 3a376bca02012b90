"""Pins of the FP64 reference network: hand-derived gradients against central finite
differences of the loss, and structural facts of the trigonometric basis."""
import numpy as np
import pytest

from oracle import neural


def _setup(seed=0, nx=8, ny=6, nt=5, width=3, modes=2, layers=2, tmodes=3):
    rng = np.random.default_rng(seed)
    lay = neural.param_layout(nx, ny, nt, width, modes, layers, tmodes)
    n = sum(int(np.prod(s)) for _, s in lay)
    flat = 0.3 * rng.standard_normal(n)
    u0 = rng.uniform(-1, 1, (ny, nx))
    Ut = rng.uniform(-1, 1, (nt, ny, nx))
    return lay, flat, u0, Ut, layers, modes


def test_gradients_match_central_differences():
    lay, flat, u0, Ut, L, m = _setup()
    loss, g = neural.loss_and_grads(neural.unflatten(flat, lay), u0, Ut, L, m)
    gflat = neural.flatten(g, lay)
    h = 1e-6
    fd = np.empty_like(flat)
    for i in range(flat.size):
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        lp, _ = neural.loss_and_grads(neural.unflatten(fp, lay), u0, Ut, L, m)
        lm, _ = neural.loss_and_grads(neural.unflatten(fm, lay), u0, Ut, L, m)
        fd[i] = (lp - lm) / (2 * h)
    np.testing.assert_allclose(gflat, fd, rtol=1e-5, atol=1e-9)


def test_coefficient_loss_gradients_match_central_differences():
    lay, flat, u0, Ut, L, m = _setup(seed=4)
    ct = neural.encode(Ut, u0, 3)
    nt = Ut.shape[0]
    loss, g = neural.coef_loss_and_grads(neural.unflatten(flat, lay), u0, ct, nt, L, m)
    gflat = neural.flatten(g, lay)
    h = 1e-6
    rng = np.random.default_rng(5)
    for i in rng.choice(flat.size, 40, replace=False):
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        lp, _ = neural.coef_loss_and_grads(neural.unflatten(fp, lay), u0, ct, nt, L, m)
        lm, _ = neural.coef_loss_and_grads(neural.unflatten(fm, lay), u0, ct, nt, L, m)
        np.testing.assert_allclose(gflat[i], (lp - lm) / (2 * h), rtol=1e-5, atol=1e-9)


def test_coefficient_loss_is_the_level_loss_minus_the_projection_residual():
    """Orthonormal columns: mean((U_pred - U)^2) = |c - c_true|^2 / count + |(I - Phi Phi^T)(U - u0)|^2 / count."""
    lay, flat, u0, Ut, L, m = _setup(seed=6)
    p = neural.unflatten(flat, lay)
    nt, K = Ut.shape[0], 3
    lu, gu = neural.loss_and_grads(p, u0, Ut, L, m)
    lc, gc = neural.coef_loss_and_grads(p, u0, neural.encode(Ut, u0, K), nt, L, m)
    Phi = neural.time_basis(nt, K)
    d = (Ut - u0[None]).reshape(nt, -1)
    perp = d - Phi @ (Phi.T @ d)
    assert abs(lu - (lc + np.sum(perp * perp) / Ut.size)) < 1e-13
    # the constant does not depend on the parameters: identical gradients
    np.testing.assert_allclose(neural.flatten(gu, lay), neural.flatten(gc, lay), rtol=1e-10, atol=1e-14)


def test_time_basis_is_gram_schmidt_of_the_sine_columns():
    """Orthonormal columns, each column k in the span of the first k sines with a positive
    coefficient on sine k (what Gram-Schmidt in order produces), zero at t = 0."""
    nt, K = 40, 7
    Phi = neural.time_basis(nt, K)
    np.testing.assert_allclose(Phi.T @ Phi, np.eye(K), atol=1e-13)
    n = np.arange(1, nt + 1)[:, None]
    S = np.sin(np.pi * (np.arange(1, K + 1)[None, :] - 0.5) * n / nt)
    T = np.linalg.lstsq(S, Phi, rcond=None)[0]  # Phi = S T, T upper triangular, diag > 0
    np.testing.assert_allclose(S @ T, Phi, atol=1e-12)
    np.testing.assert_allclose(np.tril(T, -1), 0, atol=1e-10)
    assert np.all(np.diag(T) > 0)
    # first column is the normalised first sine: sin(pi n / (2 nt)) / norm
    s1 = np.sin(np.pi * 0.5 * np.arange(1, nt + 1) / nt)
    np.testing.assert_allclose(Phi[:, 0], s1 / np.linalg.norm(s1), atol=1e-14)


def test_encode_recovers_fields_in_the_span():
    """U = u0 + Phi c (any c) encodes back to c exactly."""
    rng = np.random.default_rng(8)
    nt, K = 9, 4
    u0 = rng.standard_normal((5, 6))
    c = rng.standard_normal((K, 5, 6))
    U = u0[None] + np.einsum("nk,kji->nji", neural.time_basis(nt, K), c)
    np.testing.assert_allclose(neural.encode(U, u0, K), c, atol=1e-13)


def test_basis_is_orthogonal_on_the_periodic_grid():
    """cos/sin modes below the Nyquist frequency are orthogonal with norms n (k = 0) and n/2."""
    n, m = 16, 5
    ph = neural.basis(n, m)
    G = ph.T @ ph
    expect = np.diag([n] + [n / 2] * (2 * m - 2))
    np.testing.assert_allclose(G, expect, atol=1e-12)


def test_spectral_layer_reproduces_band_limited_fields():
    """With R = identity on every mode and W = 0, b = 0, the spectral convolution of a field in
    the span of the basis is the field weighted by 1 (k = 0) or 1/2 per direction otherwise."""
    n, m = 12, 3
    ph = neural.basis(n, m)
    rng = np.random.default_rng(1)
    coef = rng.standard_normal((2 * m - 1, 2 * m - 1))
    v = ph @ coef @ ph.T  # v[j, i] = sum_ab coef[a, b] phi_a(y_j) phi_b(x_i)
    vh = np.einsum("ja,ji,ib->ab", ph, v, ph) / (n * n)
    w = np.array([1.0] + [0.5] * (2 * m - 2))
    np.testing.assert_allclose(vh, coef * np.outer(w, w), atol=1e-12)


def _one_layer_K(R, v, m):
    """(K v) for one channel-diagonal spectral layer, via the oracle's own pieces."""
    ny, nx = v.shape[1:]
    phx, phy = neural.basis(nx, m), neural.basis(ny, m)
    vh = np.einsum("ja,cji,ib->cab", phy, v, phx) / (nx * ny)
    wh = neural.spectral_mix(R, vh, m)
    return np.einsum("ja,kab,ib->kji", phy, wh, phx)


def test_spectral_layer_translates_band_limited_fields():
    """Complex weights W(k) = exp(-2 pi i k.s) / (basis norm) on every mode shift a band-limited
    field by s (FNO's mode-wise multiplication is a convolution): (K v)(x) = v(x - s). A layer
    that mixed the cosine and sine coefficients independently could not do this."""
    n, m, C = 16, 4, 2
    rng = np.random.default_rng(3)
    sx, sy = 0.23, -0.11

    def field(X, Y, amp):
        out = np.zeros_like(X)
        for (ky, kx), (a, b) in amp.items():
            out += a * np.cos(2 * np.pi * (kx * X + ky * Y)) + b * np.sin(2 * np.pi * (kx * X + ky * Y))
        return out

    amp = {(ky, kx): tuple(rng.standard_normal(2)) for ky in range(-m + 1, m) for kx in range(0, m)
           if (kx > 0 or ky >= 0)}
    x = np.arange(n) / n
    X, Y = np.meshgrid(x, x, indexing="xy")
    v = np.stack([field(X, Y, amp), 2.0 * field(X, Y, amp)])
    expect = np.stack([field(X - sx, Y - sy, amp), 2.0 * field(X - sx, Y - sy, amp)])
    R = np.zeros((2 * m - 1, 2 * m - 1, C, C))
    eye = np.eye(C)
    for ky in range(m):
        for kx in range(m):
            cy, sy_, cx, sx_ = ky, m - 1 + ky, kx, m - 1 + kx
            if kx and ky:
                wp = 4.0 * np.exp(-2j * np.pi * (kx * sx + ky * sy))  # mode kx x + ky y
                wm = 4.0 * np.exp(-2j * np.pi * (kx * sx - ky * sy))  # mode kx x - ky y
                R[cy, cx], R[cy, sx_] = wp.real * eye, wp.imag * eye
                R[sy_, cx], R[sy_, sx_] = wm.real * eye, wm.imag * eye
            elif kx:
                w = 2.0 * np.exp(-2j * np.pi * kx * sx)
                R[0, cx], R[0, sx_] = w.real * eye, w.imag * eye
            elif ky:
                w = 2.0 * np.exp(-2j * np.pi * ky * sy)
                R[cy, 0], R[sy_, 0] = w.real * eye, w.imag * eye
            else:
                R[0, 0] = eye
    np.testing.assert_allclose(_one_layer_K(R, v, m), expect, atol=1e-12)


def test_spectral_mix_adjoint_is_the_transpose():
    """<mix(R, x), y> = <x, mix_adjoint(R, ., y)>, and d<mix(R, x), y>/dR = dR of the adjoint."""
    m, C = 3, 4
    rng = np.random.default_rng(9)
    R = rng.standard_normal((2 * m - 1, 2 * m - 1, C, C))
    x = rng.standard_normal((C, 2 * m - 1, 2 * m - 1))
    y = rng.standard_normal((C, 2 * m - 1, 2 * m - 1))
    dx, dR = neural.spectral_mix_adjoint(R, x, y, m)
    assert abs(np.sum(neural.spectral_mix(R, x, m) * y) - np.sum(x * dx)) < 1e-12
    # the mix is linear in R as well: <mix(R', x), y> = <R', dR>
    R2 = rng.standard_normal(R.shape)
    assert abs(np.sum(neural.spectral_mix(R2, x, m) * y) - np.sum(R2 * dR)) < 1e-12


# ------------------------------------------------------------ the staged bfloat16 form

def test_bf16_rounding_matches_torch_conversion():
    """oracle.neural_bf16.bf16 is round-to-nearest-even to bfloat16, as torch converts."""
    import torch

    from oracle import neural_bf16 as OB
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        [0.0, -0.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 1e-40, -3e-39,
                         3.4e38, np.inf, -np.inf]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = OB.bf16(x)
    np.testing.assert_array_equal(got, ref)
    assert np.isnan(OB.bf16(np.array([np.nan], dtype=np.float32)))[0]
    # ties go to the even neighbour: 1 + 2^-8 -> 1, 1 + 3 2^-8 -> 1 + 2^-6
    assert got[20002] == 1.0 and got[20003] == 1.0 + 2.0 ** -6


def test_staged_network_without_rounding_is_the_network():
    """With exact products the staged order (x transform first, intermediates as operands)
    is the network of oracle.neural; the only difference is its float32 basis tables."""
    from oracle import neural_bf16 as OB
    lay, flat, u0, Ut, L, m = _setup(seed=9, nx=12, ny=10, nt=6, width=4, modes=3, layers=2, tmodes=3)
    p = neural.unflatten(flat, lay)
    ident = lambda a: np.asarray(a, dtype=np.float64)
    U = neural.forward(p, u0, 6, L, m)
    Us = OB.forward(p, u0, 6, L, m, rnd=ident)
    assert np.max(np.abs(Us - U)) <= 1e-6 * np.max(np.abs(U - u0[None]))
    lo, go = neural.loss_and_grads(p, u0, Ut, L, m)
    ls, gs = OB.loss_grads(p, u0, Ut, L, m, rnd=ident)
    assert abs(ls - lo) <= 1e-6 * lo
    for name, _ in lay:
        assert np.max(np.abs(gs[name] - go[name])) <= 1e-5 * np.max(np.abs(go[name])), name


def test_staged_network_rounds_at_bfloat16_size():
    """Rounded products move the output by the bfloat16 unit (2^-9) times a modest factor:
    more than float32 rounding, far less than the output."""
    from oracle import neural_bf16 as OB
    lay, flat, u0, Ut, L, m = _setup(seed=10, nx=16, ny=12, nt=6, width=8, modes=3, layers=2, tmodes=3)
    p = neural.unflatten(flat, lay)
    U = neural.forward(p, u0, 6, L, m)
    Ub = OB.forward(p, u0, 6, L, m)
    e = np.linalg.norm(Ub - U) / np.linalg.norm(U - u0[None])
    assert 1e-5 < e < 5e-2, e

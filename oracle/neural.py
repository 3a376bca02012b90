"""FP64 reference of the spectral neural operator used for the learned initial iterate
(oracle, test infrastructure only).

Network (written from its definition, independently of the HIP kernels):
    v_0 = lift_w u0 + lift_b                                        (1 -> width channels)
    v_{l+1} = GELU(W_l v_l + b_l + K_l v_l)
    c_k = sum_c proj_w[k, c] v_L[c] + proj_b[k]                      (width -> K temporal modes)
    U_pred^n = u0 + sum_k Phi[n, k] c_k                              (K modes -> nt levels)
Phi [nt, K] has orthonormal columns spanning s_k(n) = sin(pi (k - 1/2) n / nt), n = 1..nt,
k = 1..K (smooth in time, zero at t = 0): the Gram-Schmidt orthonormalisation of those
columns in order, i.e. the Q factor of S = QR with a positive diagonal of R.
K_l: the Fourier neural operator's truncated spectral convolution, which multiplies each
complex Fourier mode exp(2 pi i (kx x + ky y)), |kx|, |ky| < m, of every channel by a
complex channel-mixing matrix. A real field is held in the real trigonometric basis
    phi_k(x) = cos(2 pi k x), k = 0..m-1;   phi_{m-1+k}(x) = sin(2 pi k x), k = 1..m-1,
    vhat[c, a, b] = (1/(nx ny)) sum_{j, i} v[c, j, i] phi_a(y_j) phi_b(x_i),
and its complex amplitudes are read off the products of cosines and sines: for
kx, ky >= 1 the four coefficients A (cos y cos x), B (cos y sin x), C (sin y cos x),
D (sin y sin x) are Re[z+ e^{i(x+y)}] + Re[z- e^{i(x-y)}] with
    z+ = (A - D)/2 - i (B + C)/2,      z- = (A + D)/2 - i (B - C)/2,
a pair with one zero frequency (cos, sin in the other direction) is Re[z e^{i x}] with
z = cos-coefficient - i sin-coefficient, and the mean is real. Each amplitude is
multiplied by W = alpha + i beta (width x width), the result is expanded back into the
real basis (what) and synthesised: (K_l v)[c', j, i] = sum_{a, b} what[c', a, b] phi_a(y_j) phi_b(x_i).
The real parameters R_l[a, b] (one width x width matrix per real basis pair) hold the
complex weights: for kx, ky >= 1, alpha+ = R[cos ky, cos kx], beta+ = R[cos ky, sin kx],
alpha- = R[sin ky, cos kx], beta- = R[sin ky, sin kx]; for a zero frequency in one
direction, alpha = R at the cosine, beta = R at the sine position; the mean uses R[0, 0].
GELU(z) = z/2 (1 + tanh(sqrt(2/pi)(z + 0.044715 z^3))). Loss: mean((U_pred - U_true)^2).
Because the columns of Phi are orthonormal, the same loss splits into
|c - c_true|^2 / (nt nx ny) plus a constant, with the encoded target
c_true = Phi^T (U_true - u0) (coef_loss_and_grads, encode).

The backward pass is derived by hand and pinned by central finite differences of the
loss (tests/test_oracle_neural.py); no other reference exists for this network
(it is not from the paper).
"""
from __future__ import annotations

import math

import numpy as np


def basis(n, m):
    """phi[i, k] on the periodic nodes x_i = i / n (cos 0..m-1, then sin 1..m-1)."""
    x = np.arange(n, dtype=np.float64) / n
    ph = np.empty((n, 2 * m - 1))
    for k in range(m):
        ph[:, k] = np.cos(2 * math.pi * k * x)
    for k in range(1, m):
        ph[:, m - 1 + k] = np.sin(2 * math.pi * k * x)
    return ph


def _blocks(m):
    """Frequency blocks (ky, kx) in [0, m)^2 with their real-basis indices (row = y, column = x)."""
    out = []
    for ky in range(m):
        for kx in range(m):
            out.append((ky, kx, ky, m - 1 + ky if ky else None, kx, m - 1 + kx if kx else None))
    return out


def spectral_mix(R, vh, m):
    """what = the complex mode-wise channel mixing of vh (both [C, 2m-1, 2m-1])."""
    wh = np.zeros((R.shape[2],) + vh.shape[1:])
    for ky, kx, cy, sy, cx, sx in _blocks(m):
        if kx and ky:
            A, B, Cc, D = vh[:, cy, cx], vh[:, cy, sx], vh[:, sy, cx], vh[:, sy, sx]
            zp = 0.5 * (A - D) - 0.5j * (B + Cc)
            zm = 0.5 * (A + D) - 0.5j * (B - Cc)
            zp2 = (R[cy, cx] + 1j * R[cy, sx]) @ zp
            zm2 = (R[sy, cx] + 1j * R[sy, sx]) @ zm
            wh[:, cy, cx] = zp2.real + zm2.real
            wh[:, sy, sx] = zm2.real - zp2.real
            wh[:, cy, sx] = -(zp2.imag + zm2.imag)
            wh[:, sy, cx] = zm2.imag - zp2.imag
        elif kx or ky:
            qc, qs = ((cy, cx), (cy, sx)) if kx else ((cy, cx), (sy, cx))
            z = vh[:, qc[0], qc[1]] - 1j * vh[:, qs[0], qs[1]]
            z2 = (R[qc] + 1j * R[qs]) @ z
            wh[:, qc[0], qc[1]] = z2.real
            wh[:, qs[0], qs[1]] = -z2.imag
        else:
            wh[:, 0, 0] = R[0, 0] @ vh[:, 0, 0]
    return wh


def spectral_mix_adjoint(R, vh, dwh, m):
    """(d vh, d R) of the spectral mixing for the output gradient dwh."""
    dvh = np.zeros_like(vh)
    dR = np.zeros_like(R)
    for ky, kx, cy, sy, cx, sx in _blocks(m):
        if kx and ky:
            A, B, Cc, D = vh[:, cy, cx], vh[:, cy, sx], vh[:, sy, cx], vh[:, sy, sx]
            zp = 0.5 * (A - D) - 0.5j * (B + Cc)
            zm = 0.5 * (A + D) - 0.5j * (B - Cc)
            dA2, dB2, dC2, dD2 = dwh[:, cy, cx], dwh[:, cy, sx], dwh[:, sy, cx], dwh[:, sy, sx]
            # gradients in the convention d/dRe + i d/dIm
            gp2 = (dA2 - dD2) + 1j * (-dB2 - dC2)
            gm2 = (dA2 + dD2) + 1j * (-dB2 + dC2)
            Wp = R[cy, cx] + 1j * R[cy, sx]
            Wm = R[sy, cx] + 1j * R[sy, sx]
            gp = Wp.conj().T @ gp2
            gm = Wm.conj().T @ gm2
            gWp = np.outer(gp2, zp.conj())
            gWm = np.outer(gm2, zm.conj())
            dR[cy, cx] += gWp.real
            dR[cy, sx] += gWp.imag
            dR[sy, cx] += gWm.real
            dR[sy, sx] += gWm.imag
            dvh[:, cy, cx] = 0.5 * (gp.real + gm.real)
            dvh[:, sy, sx] = 0.5 * (gm.real - gp.real)
            dvh[:, cy, sx] = -0.5 * (gp.imag + gm.imag)
            dvh[:, sy, cx] = 0.5 * (gm.imag - gp.imag)
        elif kx or ky:
            qc, qs = ((cy, cx), (cy, sx)) if kx else ((cy, cx), (sy, cx))
            z = vh[:, qc[0], qc[1]] - 1j * vh[:, qs[0], qs[1]]
            g2 = dwh[:, qc[0], qc[1]] - 1j * dwh[:, qs[0], qs[1]]
            W = R[qc] + 1j * R[qs]
            g = W.conj().T @ g2
            gW = np.outer(g2, z.conj())
            dR[qc] += gW.real
            dR[qs] += gW.imag
            dvh[:, qc[0], qc[1]] = g.real
            dvh[:, qs[0], qs[1]] = -g.imag
        else:
            dR[0, 0] += np.outer(dwh[:, 0, 0], vh[:, 0, 0])
            dvh[:, 0, 0] = R[0, 0].T @ dwh[:, 0, 0]
    return dvh, dR


def time_basis(nt, K):
    """Phi [nt, K]: orthonormalised sin(pi (k - 1/2) n / nt), n = 1..nt, k = 1..K."""
    n = np.arange(1, nt + 1, dtype=np.float64)[:, None]
    k = np.arange(1, K + 1, dtype=np.float64)[None, :]
    S = np.sin(math.pi * (k - 0.5) * n / nt)
    Q, R = np.linalg.qr(S)
    return Q * np.sign(np.diag(R))[None, :]


def param_layout(nx, ny, nt, width, modes, layers, tmodes):
    """[(name, shape)] in the flat float32 order the library uses."""
    C = width
    out = [("lift_w", (C,)), ("lift_b", (C,))]
    for l in range(layers):
        out += [(f"W{l}", (C, C)), (f"b{l}", (C,)), (f"R{l}", (2 * modes - 1, 2 * modes - 1, C, C))]
    out += [("proj_w", (tmodes, C)), ("proj_b", (tmodes,))]
    return out


def unflatten(flat, layout):
    params, o = {}, 0
    for name, shape in layout:
        size = int(np.prod(shape))
        params[name] = np.asarray(flat[o:o + size], dtype=np.float64).reshape(shape)
        o += size
    return params


def flatten(grads, layout):
    return np.concatenate([grads[name].ravel() for name, _ in layout])


def _gelu(z):
    a = math.sqrt(2 / math.pi) * (z + 0.044715 * z ** 3)
    return 0.5 * z * (1 + np.tanh(a))


def _gelu_grad(z):
    a = math.sqrt(2 / math.pi) * (z + 0.044715 * z ** 3)
    t = np.tanh(a)
    da = math.sqrt(2 / math.pi) * (1 + 3 * 0.044715 * z * z)
    return 0.5 * (1 + t) + 0.5 * z * (1 - t * t) * da


def forward(params, u0, nt, layers, modes, cache=False):
    ny, nx = u0.shape
    Phi = time_basis(nt, params["proj_w"].shape[0])
    phx, phy = basis(nx, modes), basis(ny, modes)
    v = params["lift_w"][:, None, None] * u0[None] + params["lift_b"][:, None, None]
    store = {"v": [v], "z": [], "vh": []}
    for l in range(layers):
        vh = np.einsum("ja,cji,ib->cab", phy, v, phx) / (nx * ny)
        wh = spectral_mix(params[f"R{l}"], vh, modes)
        K = np.einsum("ja,kab,ib->kji", phy, wh, phx)
        z = K + np.einsum("kc,cji->kji", params[f"W{l}"], v) + params[f"b{l}"][:, None, None]
        v = _gelu(z)
        store["v"].append(v)
        store["z"].append(z)
        store["vh"].append(vh)
    coef = np.einsum("kc,cji->kji", params["proj_w"], v) + params["proj_b"][:, None, None]
    store["coef"] = coef
    U = u0[None] + np.einsum("nk,kji->nji", Phi, coef)
    return (U, store) if cache else U


def encode(U, u0, K):
    """c = Phi^T (U - u0): the K temporal-mode coefficients of a space-time field."""
    return np.einsum("nk,nji->kji", time_basis(U.shape[0], K), U - u0[None])


def _backward(params, st, dcoef, u0, layers, modes):
    """Gradients of a loss from its derivative with respect to the coefficient fields."""
    ny, nx = u0.shape
    phx, phy = basis(nx, modes), basis(ny, modes)
    g = {}
    vL = st["v"][-1]
    g["proj_w"] = np.einsum("kji,cji->kc", dcoef, vL)
    g["proj_b"] = dcoef.sum(axis=(1, 2))
    dv = np.einsum("kc,kji->cji", params["proj_w"], dcoef)
    for l in range(layers - 1, -1, -1):
        z, vin, vh = st["z"][l], st["v"][l], st["vh"][l]
        dz = dv * _gelu_grad(z)
        g[f"b{l}"] = dz.sum(axis=(1, 2))
        g[f"W{l}"] = np.einsum("kji,cji->kc", dz, vin)
        dv_new = np.einsum("kc,kji->cji", params[f"W{l}"], dz)
        dwh = np.einsum("ja,kji,ib->kab", phy, dz, phx)
        dvh, g[f"R{l}"] = spectral_mix_adjoint(params[f"R{l}"], vh, dwh, modes)
        dv_new += np.einsum("ja,cab,ib->cji", phy, dvh, phx) / (nx * ny)
        dv = dv_new
    g["lift_w"] = np.einsum("cji,ji->c", dv, u0)
    g["lift_b"] = dv.sum(axis=(1, 2))
    return g


def loss_and_grads(params, u0, U_true, layers, modes):
    """Loss mean((U_pred - U_true)^2) and its gradient with respect to every parameter."""
    nt = U_true.shape[0]
    U, st = forward(params, u0, nt, layers, modes, cache=True)
    e = U - U_true
    loss = float(np.mean(e * e))
    dU = 2.0 * e / e.size
    dcoef = np.einsum("nk,nji->kji", time_basis(nt, params["proj_w"].shape[0]), dU)
    return loss, _backward(params, st, dcoef, u0, layers, modes)


def coef_loss_and_grads(params, u0, coef_true, nt, layers, modes):
    """Loss |c - c_true|^2 / (nt nx ny) in the temporal-mode coefficients and its gradient."""
    _, st = forward(params, u0, nt, layers, modes, cache=True)
    d = st["coef"] - coef_true
    count = nt * u0.size
    loss = float(np.sum(d * d) / count)
    return loss, _backward(params, st, 2.0 * d / count, u0, layers, modes)

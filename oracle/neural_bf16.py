"""The spectral neural operator of oracle/neural.py with bfloat16 operands in its matrix
products (oracle, test infrastructure only).

oracle/neural.py defines the network in exact (float64) arithmetic. This module takes the
same network and states where a bfloat16 matrix engine rounds: every matrix product
sum_k a[m, k] b[k, n] rounds both operands to float32 and then to bfloat16 (round to
nearest, ties to even) and sums the exact products; everything else (the mode-wise channel
mixing, GELU, biases, the temporal synthesis) stays exact. The products are taken in this
order, each intermediate rounded again when it becomes an operand:
    spectral analysis   t1 = v phix (x direction first), vhat = (1/(nx ny)) phiy^T t1
    spectral synthesis  t2 = phiy what,                    K v = t2 phix^T
    channel mix         W v;   projection   proj_w v_L
and, in the backward pass, dW = dz v^T, dv = W^T dz, d proj_w = dcoef v_L^T,
dv = proj_w^T dcoef, the analysis of dz (adjoint of the synthesis) and
t2 = (1/(nx ny)) phiy dvhat, dv += t2 phix^T (adjoint of the analysis).
In exact arithmetic (rnd = identity) every value equals oracle/neural.py's; the tests pin
that reduction and the rounding function against torch's bfloat16 conversion.
"""
from __future__ import annotations

import numpy as np

from . import neural as N


def bf16(a):
    """a rounded to float32, then to bfloat16 (nearest, ties to even), as float64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    r = np.where(nan, ((u >> 16) | 0x40) << 16, r)
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(a))


def _exact(a):
    return np.asarray(a, dtype=np.float64)


def _tables(nx, ny, modes):
    """Trigonometric bases phi[i, k] as float32 values (the form a product reads them in)."""
    return (N.basis(nx, modes).astype(np.float32).astype(np.float64),
            N.basis(ny, modes).astype(np.float32).astype(np.float64))


def analysis(v, phx, phy, alpha, rnd):
    """alpha phiy^T v phix per channel of v [C, ny, nx], x direction first."""
    t1 = rnd(v) @ rnd(phx)                       # [C, ny, m2]
    return alpha * (rnd(phy).T @ rnd(t1))        # [C, m2, m2]


def synthesis(w, phx, phy, alpha, rnd):
    """phiy (alpha w) phix^T per channel of w [C, m2, m2]: t2 = alpha phiy w, then t2 phix^T."""
    t2 = alpha * (rnd(phy) @ rnd(w))             # [C, ny, m2]
    return rnd(t2) @ rnd(phx).T                  # [C, ny, nx]


def _chan(Wm, v, rnd):
    """sum_c Wm[k, c] v[c, :, :] as one product over the flattened grid."""
    C = v.shape[0]
    return (rnd(Wm) @ rnd(v.reshape(C, -1))).reshape((Wm.shape[0],) + v.shape[1:])


def forward(params, u0, nt, layers, modes, rnd=bf16, cache=False):
    """U_pred [nt, ny, nx] (and the stored activations with cache=True)."""
    ny, nx = u0.shape
    phx, phy = _tables(nx, ny, modes)
    Phi = N.time_basis(nt, params["proj_w"].shape[0])
    v = params["lift_w"][:, None, None] * u0[None] + params["lift_b"][:, None, None]
    st = {"v": [v], "z": [], "vh": []}
    for l in range(layers):
        vh = analysis(v, phx, phy, 1.0 / (nx * ny), rnd)
        wh = N.spectral_mix(params[f"R{l}"], vh, modes)
        z = synthesis(wh, phx, phy, 1.0, rnd) + _chan(params[f"W{l}"], v, rnd) + params[f"b{l}"][:, None, None]
        v = N._gelu(z)
        st["v"].append(v)
        st["z"].append(z)
        st["vh"].append(vh)
    coef = _chan(params["proj_w"], v, rnd)
    st["coef"] = coef
    U = u0[None] + np.einsum("nk,kji->nji", Phi, coef + params["proj_b"][:, None, None])
    return (U, st) if cache else U


def backward(params, st, dcoef, u0, layers, modes, rnd=bf16):
    """Gradients of a loss from dL/dcoef (the fields before proj_b), products rounded as above."""
    ny, nx = u0.shape
    phx, phy = _tables(nx, ny, modes)
    K, C = params["proj_w"].shape
    g = {}
    vL = st["v"][-1]
    g["proj_w"] = rnd(dcoef.reshape(K, -1)) @ rnd(vL.reshape(C, -1)).T
    g["proj_b"] = dcoef.sum(axis=(1, 2))
    dv = _chan(params["proj_w"].T, dcoef, rnd)
    for l in range(layers - 1, -1, -1):
        z, vin, vh = st["z"][l], st["v"][l], st["vh"][l]
        dz = dv * N._gelu_grad(z)
        g[f"b{l}"] = dz.sum(axis=(1, 2))
        g[f"W{l}"] = rnd(dz.reshape(C, -1)) @ rnd(vin.reshape(C, -1)).T
        dv_new = _chan(params[f"W{l}"].T, dz, rnd)
        dwh = analysis(dz, phx, phy, 1.0, rnd)
        dvh, g[f"R{l}"] = N.spectral_mix_adjoint(params[f"R{l}"], vh, dwh, modes)
        dv = dv_new + synthesis(dvh, phx, phy, 1.0 / (nx * ny), rnd)
    g["lift_w"] = np.einsum("cji,ji->c", dv, u0)
    g["lift_b"] = dv.sum(axis=(1, 2))
    return g


def loss_grads(params, u0, U_true, layers, modes, rnd=bf16):
    """mean((U_pred - U_true)^2) and its gradients, products rounded as above."""
    nt = U_true.shape[0]
    U, st = forward(params, u0, nt, layers, modes, rnd, cache=True)
    e = U - U_true
    dcoef = np.einsum("nk,nji->kji", N.time_basis(nt, params["proj_w"].shape[0]), 2.0 * e / e.size)
    return float(np.mean(e * e)), backward(params, st, dcoef, u0, layers, modes, rnd)

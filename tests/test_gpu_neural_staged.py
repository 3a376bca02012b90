"""The network on the GPU against the staged bfloat16 oracle (oracle/neural_bf16.py),
element by element, at the production grid (256 x 256, width 32, 12 modes, 16 temporal
modes).

The staged oracle rounds the operands of every matrix product to bfloat16 where the kernels
do, so the two sides differ only by float32 accumulation order and float32 elementwise
arithmetic (relative ~1e-7). A bfloat16 rounding amplifies such a difference only where an
operand lies within it of a rounding boundary: there the two sides round to neighbouring
bfloat16 values, one unit (2^-8 relative) apart. With a relative difference d entering a
product, a fraction ~2 d / 2^-8 of its operands flip, and the product then differs by about
sqrt(2 d 2^-8) (relative, worst entries); layer by layer d grows 1e-7 -> 1e-5 -> 3e-4 -> 2e-3.
The flipped entries are few, so most entries stay close: the tests bound the median and the
99th percentile of |gpu - oracle| / max|oracle| tightly and the maximum loosely. An error
of the network itself (a dropped mode band, a wrong channel, a transposed operand) moves
every entry by the size of that term, far above the median bound. The bounds are about ten
times what a float32-accumulation emulation of the same staging shows on these inputs.
"""
import numpy as np
import pytest
import torch

import paper_2406_00878_amd.neural as NO
from oracle import neural as ON
from oracle import neural_bf16 as OB

pytestmark = pytest.mark.gpu

#  layers: (median, p99, max) for U - u0, and the same for each gradient block
BOUNDS = {
    1: ((1e-6, 3e-4, 2e-2), (1e-5, 1e-4, 1e-3)),
    2: ((1e-6, 3e-3, 3e-2), (1e-5, 3e-4, 1e-3)),
    4: ((3e-4, 1e-2, 4e-2), (3e-3, 1e-2, 2e-2)),
}


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _cfg(layers, nt=64):
    return NO.NOConfig(nx=256, ny=256, nt=nt, width=32, modes=12, layers=layers, tmodes=16)


def _params(cfg, seed):
    """The library's initialisation with biases drawn and a projection of unit scale."""
    net_host = NO.NeuralOperator.__new__(NO.NeuralOperator)
    net_host.cfg = cfg
    p = net_host.init_params(seed).numpy().astype(np.float32).copy()
    rng = np.random.default_rng(seed)
    o = 0
    for name, shape in cfg.layout():
        size = int(np.prod(shape))
        if name == "proj_w":
            p[o:o + size] *= 100.0
        if name.startswith("b") or name in ("lift_b", "proj_b"):
            p[o:o + size] = 0.1 * rng.standard_normal(size)
        o += size
    return p


def _unflat(cfg, p):
    lay = ON.param_layout(cfg.nx, cfg.ny, cfg.nt, cfg.width, cfg.modes, cfg.layers, cfg.tmodes)
    return ON.unflatten(np.asarray(p, dtype=np.float32).astype(np.float64), lay), lay


def _quantiles(got, ref):
    e = np.abs(np.asarray(got) - ref).ravel() / max(float(np.max(np.abs(ref))), 1e-300)
    return np.quantile(e, [0.5, 0.99, 1.0])


def _check(q, bound, what):
    print(f"{what}: median {q[0]:.1e} p99 {q[1]:.1e} max {q[2]:.1e}", flush=True)
    assert q[0] <= bound[0] and q[1] <= bound[1] and q[2] <= bound[2], (what, q, bound)


@pytest.mark.parametrize("layers", [1, 2, 4])
def test_forward_elementwise_matches_staged_oracle(layers):
    cfg = _cfg(layers)
    net = NO.NeuralOperator(cfg)
    p = _params(cfg, 40 + layers)
    net.params.copy_(dev(p, torch.float32))
    u0 = np.random.default_rng(50 + layers).uniform(-1, 1, (cfg.ny, cfg.nx))
    print(f"[staged forward] {cfg}", flush=True)
    U = host(net.forward(dev(u0)))
    pr, _ = _unflat(cfg, p)
    Uo = OB.forward(pr, u0, cfg.nt, cfg.layers, cfg.modes)
    _check(_quantiles(U - u0[None], Uo - u0[None]), BOUNDS[layers][0], f"U - u0 ({layers} layers)")


@pytest.mark.parametrize("layers", [1, 4])
def test_backward_elementwise_matches_staged_oracle(layers):
    cfg = _cfg(layers)
    net = NO.NeuralOperator(cfg)
    p = _params(cfg, 60 + layers)
    net.params.copy_(dev(p, torch.float32))
    rng = np.random.default_rng(70 + layers)
    u0 = rng.uniform(-1, 1, (cfg.ny, cfg.nx))
    pr, lay = _unflat(cfg, p)
    Uo = OB.forward(pr, u0, cfg.nt, cfg.layers, cfg.modes)
    # a target unrelated to the prediction: the loss gradient is not a small difference
    span = float(np.max(np.abs(Uo - u0[None])))
    Ut = u0[None] + 0.5 * (Uo - u0[None]) + 0.1 * span * rng.standard_normal(Uo.shape)
    print(f"[staged backward] {cfg}", flush=True)
    du0 = dev(u0)
    Up = net.forward(du0)
    net.zero_grad()
    net.backward(du0, Up, dev(Ut))
    g = ON.unflatten(host(net.grads).astype(np.float64), lay)
    loss = float(host(net.loss)[0])
    lo, go = OB.loss_grads(pr, u0, Ut, cfg.layers, cfg.modes)
    assert abs(loss - lo) <= 1e-4 * lo, (loss, lo)
    bound = BOUNDS[layers][1]
    for name, _ in lay:
        _check(_quantiles(g[name], go[name]), bound, f"d{name} ({layers} layers)")


def test_batched_forward_elementwise_matches_staged_oracle():
    """Three samples in one batched pass (transforms over 3 x 32 channels)."""
    cfg = _cfg(2, nt=32)
    net = NO.NeuralOperator(cfg)
    p = _params(cfg, 80)
    net.params.copy_(dev(p, torch.float32))
    pr, _ = _unflat(cfg, p)
    rng = np.random.default_rng(81)
    u0s = [rng.uniform(-1, 1, (cfg.ny, cfg.nx)) for _ in range(3)]
    outs = [torch.empty((cfg.nt, cfg.ny, cfg.nx), dtype=torch.float64, device="cuda") for _ in u0s]
    print(f"[staged forward batched x3] {cfg}", flush=True)
    net.forward_batched([dev(u) for u in u0s], outs, net.workspace_batched(3))
    for b, (u0, U) in enumerate(zip(u0s, outs)):
        Uo = OB.forward(pr, u0, cfg.nt, cfg.layers, cfg.modes)
        _check(_quantiles(host(U) - u0[None], Uo - u0[None]), BOUNDS[2][0], f"sample {b}: U - u0")

"""Learned initial space-time iterate: spectral neural operator (include/pts_no.h).

Argument marshalling over the library's kernels plus the training driver: training data
are solutions the method itself computes (pts_solve from the plain iterate of random
initial conditions), the forward/backward passes and the Adam steps run in the library's
HIP kernels (BF16 MFMA products with FP32 accumulation), and the Newton residual judges
the prediction against the plain iterate before every solve.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
from typing import Callable, Optional

import torch

from . import _check, _dev_f64, _lib_checked, _ptr, _stream, make_problem, workspace


class pts_no_config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nt", C.c_int32), ("width", C.c_int32),
                ("modes", C.c_int32), ("layers", C.c_int32), ("tmodes", C.c_int32)]


JUDGES = {"residual": 0, "accumulated": 1}


_sig_done = False


def _lib():
    global _sig_done
    lib = _lib_checked()
    if not _sig_done:
        P = C.POINTER(pts_no_config)
        V, I, S, F, D, L = C.c_void_p, C.c_int, C.c_size_t, C.c_float, C.c_double, C.c_long
        sig = {
            "pts_no_param_count": (S, [P]),
            "pts_no_workspace_bytes": (S, [P]),
            "pts_no_prepare": (I, [P, V, S, V]),
            "pts_no_forward": (I, [P, V, V, V, V, S, V]),
            "pts_no_backward": (I, [P, V, V, V, V, V, V, V, S, V]),
            "pts_no_backward_coef": (I, [P, V, V, V, V, V, V, S, V]),
            "pts_no_encode": (I, [P, V, V, V, V, S, V]),
            "pts_no_adam": (I, [S, V, V, V, V, I, F, F, F, F, F, V]),
            "pts_no_initial_iterate": (I, [C.c_void_p, P, V, V, V, V, S, V, S, I, C.POINTER(I),
                                           C.POINTER(D), C.POINTER(D), V]),
            "pts_no_gemm": (I, [I, I, I, F, V, L, L, L, V, L, L, L, F, V, L, L, L, I, V]),
            "pts_no_workspace_bytes_batched": (S, [P, I]),
            "pts_no_forward_batched": (I, [P, V, I, V, V, V, S, V]),
            "pts_no_initial_iterate_batched": (I, [C.c_void_p, P, V, I, V, V, V, S, V, S, I, C.POINTER(I), V]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _sig_done = True
    return lib


@dataclasses.dataclass(frozen=True)
class NOConfig:
    nx: int
    ny: int
    nt: int
    width: int = 32
    modes: int = 12
    layers: int = 4
    tmodes: int = 16

    def c(self) -> pts_no_config:
        return pts_no_config(self.nx, self.ny, self.nt, self.width, self.modes, self.layers, self.tmodes)

    def layout(self):
        """[(name, shape)] of the flat parameter array (order of include/pts_no.h)."""
        Cw, m2 = self.width, 2 * self.modes - 1
        out = [("lift_w", (Cw,)), ("lift_b", (Cw,))]
        for l in range(self.layers):
            out += [(f"W{l}", (Cw, Cw)), (f"b{l}", (Cw,)), (f"R{l}", (m2, m2, Cw, Cw))]
        out += [("proj_w", (self.tmodes, Cw)), ("proj_b", (self.tmodes,))]
        return out


def gemm(A, B, Cout, M, N, K, sa, sb, sc, batch=1, bs=(0, 0, 0), alpha=1.0, beta=0.0, stream=None):
    """Strided batched BF16-MFMA product (testing hook of the library's GEMM)."""
    _check(_lib().pts_no_gemm(M, N, K, alpha, _ptr(A), sa[0], sa[1], bs[0], _ptr(B), sb[0], sb[1], bs[1], beta,
                              _ptr(Cout), sc[0], sc[1], bs[2], batch, _stream(stream)))


class NeuralOperator:
    """Parameters, Adam state and workspace of one network on one device."""

    def __init__(self, cfg: NOConfig, device="cuda", seed: int = 0):
        self.cfg = cfg
        self._c = cfg.c()
        lib = _lib()
        self.n_params = lib.pts_no_param_count(C.byref(self._c))
        if self.n_params == 0:
            _check(-1)
        self.ws = self.workspace(device)
        self.params = self.init_params(seed).to(device)
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self.loss = torch.zeros(1, dtype=torch.float64, device=device)

    def workspace(self, device="cuda") -> torch.Tensor:
        """A prepared network workspace (basis tables filled). Inference calls on different
        streams at once need one each."""
        lib = _lib()
        nb = lib.pts_no_workspace_bytes(C.byref(self._c))
        raw = torch.empty(nb + 256, dtype=torch.uint8, device=device)
        off = (-raw.data_ptr()) % 256
        ws = raw[off:off + nb]
        _check(lib.pts_no_prepare(C.byref(self._c), _ptr(ws), ws.numel(), _stream(None)))
        return ws

    def workspace_batched(self, batch: int, device="cuda") -> torch.Tensor:
        """A prepared workspace for forward passes of `batch` samples at once."""
        lib = _lib()
        nb = lib.pts_no_workspace_bytes_batched(C.byref(self._c), int(batch))
        if nb == 0:
            _check(-1)
        raw = torch.empty(nb + 256, dtype=torch.uint8, device=device)
        off = (-raw.data_ptr()) % 256
        ws = raw[off:off + nb]
        _check(lib.pts_no_prepare(C.byref(self._c), _ptr(ws), ws.numel(), _stream(None)))
        return ws

    def forward_batched(self, u0s, outs, ws, stream=None):
        """U_pred for several samples in one batched pass (ws from workspace_batched)."""
        cfg = self.cfg
        n = len(u0s)
        for u0, U in zip(u0s, outs):
            _dev_f64(u0, (cfg.ny, cfg.nx), "u0")
            _dev_f64(U, (cfg.nt, cfg.ny, cfg.nx), "U")
        up = (C.c_void_p * n)(*[u.data_ptr() for u in u0s])
        op = (C.c_void_p * n)(*[U.data_ptr() for U in outs])
        _check(_lib().pts_no_forward_batched(C.byref(self._c), _ptr(self.params), n, up, op, _ptr(ws), ws.numel(),
                                             _stream(stream)))
        return outs

    def init_params(self, seed: int) -> torch.Tensor:
        """Random initial weights (host generator): lift ~ N(0,1), channel mixes ~ N(0, 1/width),
        spectral weights ~ N(0, 4/width^2), projection small, biases zero."""
        g = torch.Generator().manual_seed(seed)
        Cw = self.cfg.width
        parts = []
        for name, shape in self.cfg.layout():
            if name.startswith("lift_w"):
                t = torch.randn(shape, generator=g)
            elif name.startswith("W"):
                t = torch.randn(shape, generator=g) / math.sqrt(Cw)
            elif name.startswith("R"):
                t = 2.0 * torch.randn(shape, generator=g) / Cw
            elif name == "proj_w":
                t = 0.01 * torch.randn(shape, generator=g) / math.sqrt(Cw)
            else:
                t = torch.zeros(shape)
            parts.append(t.reshape(-1))
        return torch.cat(parts).to(torch.float32).contiguous()

    def forward(self, u0: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None,
                coef_only: bool = False) -> Optional[torch.Tensor]:
        """U_pred (nt, ny, nx); with coef_only only the coefficient fields are formed."""
        cfg = self.cfg
        _dev_f64(u0, (cfg.ny, cfg.nx), "u0")
        if out is None and not coef_only:
            out = torch.empty((cfg.nt, cfg.ny, cfg.nx), dtype=torch.float64, device=u0.device)
        _check(_lib().pts_no_forward(C.byref(self._c), _ptr(self.params), _ptr(u0),
                                     None if coef_only else _ptr(out), _ptr(self.ws), self.ws.numel(),
                                     _stream(stream)))
        return None if coef_only else out

    def encode(self, u0: torch.Tensor, U: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
        """Temporal-mode coefficients (tmodes, ny, nx) float32 of a solved space-time field U."""
        cfg = self.cfg
        _dev_f64(u0, (cfg.ny, cfg.nx), "u0")
        _dev_f64(U, (cfg.nt, cfg.ny, cfg.nx), "U")
        if out is None:
            out = torch.empty((cfg.tmodes, cfg.ny, cfg.nx), dtype=torch.float32, device=U.device)
        _check(_lib().pts_no_encode(C.byref(self._c), _ptr(u0), _ptr(U), _ptr(out), _ptr(self.ws), self.ws.numel(),
                                    _stream(stream)))
        return out

    def backward_coef(self, u0, coef_true, stream=None):
        """Accumulate the coefficient-space loss and gradient (after forward on the same sample)."""
        _check(_lib().pts_no_backward_coef(C.byref(self._c), _ptr(self.params), _ptr(u0), _ptr(coef_true),
                                           _ptr(self.grads), _ptr(self.loss), _ptr(self.ws), self.ws.numel(),
                                           _stream(stream)))

    def backward(self, u0, U_pred, U_true, stream=None):
        """Accumulate the MSE loss and its gradient (after forward on the same sample)."""
        _check(_lib().pts_no_backward(C.byref(self._c), _ptr(self.params), _ptr(u0), _ptr(U_pred), _ptr(U_true),
                                      _ptr(self.grads), _ptr(self.loss), _ptr(self.ws), self.ws.numel(),
                                      _stream(stream)))

    def zero_grad(self):
        self.grads.zero_()
        self.loss.zero_()

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, grad_scale=1.0, stream=None):
        self.step += 1
        _check(_lib().pts_no_adam(self.n_params, _ptr(self.params), _ptr(self.grads), _ptr(self.m), _ptr(self.v),
                                  self.step, lr, beta1, beta2, eps, grad_scale, _stream(stream)))

    def initial_iterate(self, prob, u0, U, solver_ws=None, judge="accumulated", report=True,
                        stream=None, net_ws=None) -> Optional[dict]:
        """U <- prediction if its Newton residual beats the plain iterate's, else plain. The
        decision is taken on the device; with report=False nothing is read back (no sync).
        net_ws: a network workspace from workspace() (default: the network's own)."""
        p = make_problem(prob, "fp64")
        solver_ws = workspace(prob, "fp64", U.device) if solver_ws is None else solver_ws
        net_ws = self.ws if net_ws is None else net_ws
        ch, rp, r0 = C.c_int(0), C.c_double(0), C.c_double(0)
        refs = (C.byref(ch), C.byref(rp), C.byref(r0)) if report else (None, None, None)
        _check(_lib().pts_no_initial_iterate(C.cast(C.pointer(p), C.c_void_p), C.byref(self._c), _ptr(self.params),
                                             _ptr(u0), _ptr(U), _ptr(net_ws), net_ws.numel(), _ptr(solver_ws),
                                             solver_ws.numel(), JUDGES[judge], *refs, _stream(stream)))
        if not report:
            return None
        return {"chosen": "learned" if ch.value else "plain", "res_pred": rp.value, "res_plain": r0.value}

    def initial_iterate_batched(self, prob, u0s, Us, net_ws, solver_ws=None, judge="accumulated", report=True,
                                stream=None):
        """initial_iterate for several initial conditions of `prob`: one batched forward pass
        (net_ws from workspace_batched(len(u0s))), then each judge. Returns the choices when
        report (a synchronisation), else None."""
        p = make_problem(prob, "fp64")
        n = len(u0s)
        solver_ws = workspace(prob, "fp64", Us[0].device) if solver_ws is None else solver_ws
        for u0, U in zip(u0s, Us):
            _dev_f64(u0, (p.ny, p.nx), "u0")
            _dev_f64(U, (p.nt, p.ny, p.nx), "U")
        up = (C.c_void_p * n)(*[u.data_ptr() for u in u0s])
        op = (C.c_void_p * n)(*[U.data_ptr() for U in Us])
        ch = (C.c_int * n)()
        _check(_lib().pts_no_initial_iterate_batched(C.cast(C.pointer(p), C.c_void_p), C.byref(self._c),
                                                     _ptr(self.params), n, up, op, _ptr(net_ws), net_ws.numel(),
                                                     _ptr(solver_ws), solver_ws.numel(), JUDGES[judge],
                                                     ch if report else None, _stream(stream)))
        if not report:
            return None
        return ["learned" if c else "plain" for c in ch]


def generate(net: NeuralOperator, make_problem_fn: Callable[[int], object], samples: int,
             solver_opts: Optional[dict] = None, log: Optional[Callable[[int], None]] = None):
    """Training set from solutions the method computes: sample i is make_problem_fn(i)
    solved by all-at-once Newton from its plain iterate, stored as (u0, encoded
    coefficients) on the device. Returns (u0s [S, ny, nx] float64, coefs [S, K, ny, nx] float32,
    Newton steps per sample)."""
    from . import init_plain, solve
    dev = net.params.device
    cfg = net.cfg
    u0s = torch.empty((samples, cfg.ny, cfg.nx), dtype=torch.float64, device=dev)
    coefs = torch.empty((samples, cfg.tmodes, cfg.ny, cfg.nx), dtype=torch.float32, device=dev)
    U = torch.empty((cfg.nt, cfg.ny, cfg.nx), dtype=torch.float64, device=dev)
    ws = None
    steps = []
    for i in range(samples):
        prob = make_problem_fn(i)
        u0s[i].copy_(torch.as_tensor(prob.u0, dtype=torch.float64))
        if ws is None:
            ws = workspace(prob, "fp64", dev)
        init_plain(prob, U, u0s[i])
        st = solve(prob, U, u0s[i], tol=1e-10, max_iter=60, ws=ws, **(solver_opts or {}))
        steps.append(st["iterations"])
        net.encode(u0s[i], U, coefs[i])
        if log:
            log(i + 1)
    return u0s, coefs, steps


def train(net: NeuralOperator, u0s: torch.Tensor, coefs: torch.Tensor, epochs: int, lr: float = 1e-3,
          batch: int = 8, seed: int = 0, lr_final: Optional[float] = None,
          log: Optional[Callable[[int, float], None]] = None):
    """Adam on the coefficient-space loss over the device-resident training set; the learning
    rate decays geometrically to lr_final (default lr / 10). Returns the mean loss per epoch."""
    S = u0s.shape[0]
    g = torch.Generator().manual_seed(seed)
    steps_total = epochs * ((S + batch - 1) // batch)
    lr_final = lr / 10 if lr_final is None else lr_final
    decay = (lr_final / lr) ** (1.0 / max(steps_total - 1, 1))
    history = []
    step = 0
    for ep in range(epochs):
        order = torch.randperm(S, generator=g).tolist()
        tot = torch.zeros((), dtype=torch.float64, device=u0s.device)
        for b0 in range(0, S, batch):
            idx = order[b0:b0 + batch]
            net.zero_grad()
            for i in idx:
                net.forward(u0s[i], coef_only=True)
                net.backward_coef(u0s[i], coefs[i])
            net.adam(lr=lr * decay ** step, grad_scale=1.0 / len(idx))
            tot += net.loss[0]
            step += 1
        loss = float(tot.item()) / S
        history.append(loss)
        if log:
            log(ep + 1, loss)
    return history

"""Learned initial iterate on the GPU (include/pts_no.h) against the FP64 network oracle.

Tolerances follow from the arithmetic of the kernels:
* GEMM: operands are rounded to bfloat16 (checked exactly by rounding them the same way
  here); products of two bfloat16 values are exact in float32, so the only error is the
  float32 accumulation of K terms, bounded by K * 2^-24 * sum_k |a_mk b_kn|.
* Network forward/backward: every product rounds its operands to bfloat16 (unit roundoff
  2^-9 ~ 2e-3); a layer applies about ten such roundings in sequence (two transforms,
  their inverses, the channel mix), so with L layers the normwise relative error is of the
  order sqrt(10 L) * 2e-3 (~1.3e-2 for L = 4). The tests allow 3e-2 for the forward output
  and 6e-2 per gradient block (the backward chains twice as many products).
* Converged solutions from either initial iterate: the FP64 parity bar, 1e-10.
"""
import numpy as np
import pytest
import torch

import paper_2406_00878_amd as P
import paper_2406_00878_amd.neural as NO
import workloads as W
from oracle import allatonce
from oracle import neural as ON
from oracle import sequential

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def bf16(a):
    """Round float32 values to bfloat16 (nearest even), returned as float64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)


def strided(buf, rows, cols, sr, sc, off=0):
    idx = off + np.arange(rows)[:, None] * sr + np.arange(cols)[None, :] * sc
    return buf[idx]


GEMM_CASES = [
    # M, N, K, A (row, col) strides, B strides, batch, alpha, beta
    dict(M=64, N=64, K=16, ta=False, tb=False, batch=1, alpha=1.0, beta=0.0),
    dict(M=70, N=45, K=37, ta=False, tb=False, batch=1, alpha=1.0, beta=0.0),
    dict(M=33, N=130, K=50, ta=True, tb=False, batch=1, alpha=0.5, beta=0.0),
    dict(M=40, N=17, K=70, ta=False, tb=True, batch=3, alpha=1.0, beta=2.0),
    dict(M=16, N=200, K=1000, ta=True, tb=True, batch=2, alpha=-1.5, beta=1.0),
    dict(M=1, N=1, K=1, ta=False, tb=False, batch=1, alpha=1.0, beta=0.0),
]


@pytest.mark.parametrize("case", range(len(GEMM_CASES)))
def test_gemm_bf16_mfma_matches_rounded_reference(case):
    c = GEMM_CASES[case]
    M, N, K, B_ = c["M"], c["N"], c["K"], c["batch"]
    rng = np.random.default_rng(100 + case)
    print(f"[gemm] {c}", flush=True)
    sa = (1, M) if c["ta"] else (K, 1)
    sb = (1, K) if c["tb"] else (N, 1)
    A = rng.standard_normal(B_ * M * K).astype(np.float32)
    Bm = rng.standard_normal(B_ * K * N).astype(np.float32)
    C0 = rng.standard_normal(B_ * M * N).astype(np.float32)
    dA, dB, dC = dev(A, torch.float32), dev(Bm, torch.float32), dev(C0, torch.float32)
    NO.gemm(dA, dB, dC, M, N, K, sa, sb, (N, 1), batch=B_, bs=(M * K, K * N, M * N), alpha=c["alpha"],
           beta=c["beta"])
    got = host(dC).astype(np.float64).reshape(B_, M, N)
    for b in range(B_):
        a = bf16(strided(A, M, K, sa[0], sa[1], b * M * K))
        bb = bf16(strided(Bm, K, N, sb[0], sb[1], b * K * N))
        ref = c["alpha"] * (a @ bb) + c["beta"] * C0[b * M * N:(b + 1) * M * N].reshape(M, N).astype(np.float64)
        bound = abs(c["alpha"]) * K * 2.0 ** -24 * (np.abs(a) @ np.abs(bb)) + 2.0 ** -23 * np.abs(ref) + 1e-30
        err = np.abs(got[b] - ref)
        assert np.all(err <= 2 * bound), (b, float(np.max(err / bound)))


def test_gemm_rejects_bad_sizes():
    x = torch.zeros(4, dtype=torch.float32, device="cuda")
    with pytest.raises(P.PTSError):
        NO.gemm(x, x, x, 0, 1, 1, (1, 1), (1, 1), (1, 1))


SMALL = NO.NOConfig(nx=32, ny=24, nt=10, width=16, modes=4, layers=2, tmodes=4)


def _params(cfg, seed, proj_scale=1.0):
    net_host = NO.NeuralOperator.__new__(NO.NeuralOperator)
    net_host.cfg = cfg
    p = net_host.init_params(seed).numpy().copy()
    o = 0
    for name, shape in cfg.layout():
        size = int(np.prod(shape))
        if name == "proj_w":
            p[o:o + size] *= 100.0 * proj_scale
        if name.startswith("b") or name in ("lift_b", "proj_b"):
            p[o:o + size] = 0.1 * np.random.default_rng(seed + o).standard_normal(size)
        o += size
    return p


def _u0(cfg, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, (cfg.ny, cfg.nx))


def _layout(cfg):
    return ON.param_layout(cfg.nx, cfg.ny, cfg.nt, cfg.width, cfg.modes, cfg.layers, cfg.tmodes)


def _relnorm(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_forward_matches_oracle():
    cfg = SMALL
    net = NO.NeuralOperator(cfg)
    p = _params(cfg, 7)
    net.params.copy_(dev(p, torch.float32))
    u0 = _u0(cfg, 8)
    print(f"[forward] {cfg}", flush=True)
    U = host(net.forward(dev(u0)))
    pr = ON.unflatten(p.astype(np.float64), _layout(cfg))
    Uo = ON.forward(pr, u0, cfg.nt, cfg.layers, cfg.modes)
    e = _relnorm(U - u0[None], Uo - u0[None])
    print(f"forward normwise rel err {e:.3e}")
    assert e < 3e-2


def test_backward_matches_oracle_gradients():
    cfg = SMALL
    net = NO.NeuralOperator(cfg)
    p = _params(cfg, 11)
    net.params.copy_(dev(p, torch.float32))
    u0 = _u0(cfg, 12)
    Ut = np.random.default_rng(13).uniform(-1, 1, (cfg.nt, cfg.ny, cfg.nx))
    print(f"[backward] {cfg}", flush=True)
    du0 = dev(u0)
    Up = net.forward(du0)
    net.zero_grad()
    net.backward(du0, Up, dev(Ut))
    g = host(net.grads).astype(np.float64)
    loss = float(host(net.loss)[0])
    lay = _layout(cfg)
    pr = ON.unflatten(p.astype(np.float64), lay)
    lo, go = ON.loss_and_grads(pr, u0, Ut, cfg.layers, cfg.modes)
    assert abs(loss - lo) <= 1e-2 * lo
    gg = ON.unflatten(g, lay)
    worst = {}
    for name, _ in lay:
        worst[name] = _relnorm(gg[name], go[name])
    print("gradient normwise rel err per block:", {k: f"{v:.2e}" for k, v in worst.items()})
    assert max(worst.values()) < 6e-2, worst
    # a second backward on the same sample accumulates exactly twice the gradient
    net.backward(du0, Up, dev(Ut))
    g2 = host(net.grads).astype(np.float64)
    np.testing.assert_allclose(g2, 2 * g, rtol=1e-5, atol=1e-6 * np.max(np.abs(g)))


def test_coefficient_backward_matches_oracle_and_level_backward():
    cfg = SMALL
    net = NO.NeuralOperator(cfg)
    p = _params(cfg, 21)
    net.params.copy_(dev(p, torch.float32))
    u0 = _u0(cfg, 22)
    Ut = np.random.default_rng(23).uniform(-1, 1, (cfg.nt, cfg.ny, cfg.nx))
    print(f"[backward_coef] {cfg}", flush=True)
    du0, dUt = dev(u0), dev(Ut)
    ct = net.encode(du0, dUt)
    np.testing.assert_allclose(host(ct), ON.encode(Ut, u0, cfg.tmodes), rtol=0, atol=1e-5)
    net.forward(du0, coef_only=True)
    net.zero_grad()
    net.backward_coef(du0, ct)
    g = host(net.grads).astype(np.float64)
    loss = float(host(net.loss)[0])
    lay = _layout(cfg)
    pr = ON.unflatten(p.astype(np.float64), lay)
    lo, go = ON.coef_loss_and_grads(pr, u0, ON.encode(Ut, u0, cfg.tmodes), cfg.nt, cfg.layers, cfg.modes)
    assert abs(loss - lo) <= 1e-2 * lo
    gg = ON.unflatten(g, lay)
    worst = {name: _relnorm(gg[name], go[name]) for name, _ in lay}
    print("coef gradient normwise rel err per block:", {k: f"{v:.2e}" for k, v in worst.items()})
    assert max(worst.values()) < 6e-2, worst
    # the level-space backward has the same gradient (orthonormal temporal basis)
    Up = net.forward(du0)
    net.zero_grad()
    net.backward(du0, Up, dUt)
    g_lvl = host(net.grads).astype(np.float64)
    assert _relnorm(g_lvl, g) < 1e-3


@pytest.mark.parametrize("nt,K", [(10, 4), (256, 16), (1000, 64), (7, 7)])
def test_encode_inverts_synthesis(nt, K):
    """encode(u0 + Phi c) = c: checks the device temporal basis (orthonormal, same span)."""
    cfg = NO.NOConfig(nx=16, ny=16, nt=nt, width=16, modes=2, layers=1, tmodes=K)
    net = NO.NeuralOperator(cfg)
    rng = np.random.default_rng(nt)
    u0 = rng.uniform(-1, 1, (16, 16))
    c = rng.standard_normal((K, 16, 16))
    Phi = ON.time_basis(nt, K)
    U = u0[None] + np.einsum("nk,kji->nji", Phi, c)
    print(f"[encode] nt={nt} K={K}", flush=True)
    got = host(net.encode(dev(u0), dev(U)))
    np.testing.assert_allclose(got, c, rtol=0, atol=1e-5 * np.sqrt(nt) * np.max(np.abs(c)))


def test_adam_step_matches_formula():
    n = 1000
    rng = np.random.default_rng(3)
    p, g, m, v = (rng.standard_normal(n).astype(np.float32) for _ in range(4))
    v = np.abs(v)
    dp, dg, dm, dv = (dev(a, torch.float32) for a in (p, g, m, v))
    lib = NO._lib()
    import ctypes as C
    for step in (1, 2, 7):
        P._check(lib.pts_no_adam(n, C.c_void_p(dp.data_ptr()), C.c_void_p(dg.data_ptr()), C.c_void_p(dm.data_ptr()),
                                 C.c_void_p(dv.data_ptr()), step, 1e-2, 0.9, 0.999, 1e-8, 0.25,
                                 C.c_void_p(torch.cuda.current_stream().cuda_stream)))
        gt = 0.25 * g.astype(np.float64)
        m = 0.9 * m + 0.1 * gt
        v = 0.999 * v + 0.001 * gt * gt
        p = p - 1e-2 * (m / (1 - 0.9 ** step)) / (np.sqrt(v / (1 - 0.999 ** step)) + 1e-8)
    np.testing.assert_allclose(host(dp), p, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(host(dm), m, rtol=1e-5, atol=1e-7)


# ------------------------------------------------------------------ training + judge

TRAIN_CFG = NO.NOConfig(nx=32, ny=32, nt=16, width=16, modes=8, layers=2, tmodes=8)


def _burgers(i, seed=91):
    s = np.random.SeedSequence(seed, spawn_key=(i,))
    u0 = W.fourier_u0_periodic(32, int(s.generate_state(1)[0]))
    return W.burgers_periodic(32, 16, 5e-4, 0.005, u0, name=f"b32_{i}")


@pytest.fixture(scope="module")
def trained():
    net = NO.NeuralOperator(TRAIN_CFG, seed=5)
    print("[train] 32x32x16 Burgers, 128 samples x 30 epochs", flush=True)
    u0s, coefs, _ = NO.generate(net, _burgers, 128)
    hist = NO.train(net, u0s, coefs, epochs=30, lr=3e-3, batch=8)
    return net, hist


def test_training_reduces_loss(trained):
    _, hist = trained
    print(f"loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    assert hist[-1] < 0.1 * hist[0]


@pytest.mark.parametrize("judge", ["accumulated", "residual"])
def test_judged_iterate_converges_to_the_oracle_solution(trained, judge):
    """Whichever iterate the judge picks, Newton converges to the time-stepping solution."""
    net, _ = trained
    for i in range(2):
        p = _burgers(1000 + i)
        u0 = dev(p.u0)
        U = torch.empty((p.nt, p.ny, p.nx), dtype=torch.float64, device="cuda")
        print(f"[judge] {judge} held-out sample {i}", flush=True)
        j = net.initial_iterate(p, u0, U, judge=judge)
        print(j)
        if judge == "accumulated":
            assert j["chosen"] == "learned", j
        P.solve(p, U, u0, tol=1e-11, max_iter=60, cache_tag=1)
        Us, _ = sequential.solve_sequential(p)
        assert np.max(np.abs(host(U) - Us)) <= 1e-10 * np.max(np.abs(Us))


# the learned-iterate workload (viscous Burgers, nu = 0.005, periodic 256^2, dt = 5e-4) at 128 levels
GAIN_CFG = NO.NOConfig(nx=256, ny=256, nt=128, width=32, modes=12, layers=4, tmodes=16)


def test_trained_network_saves_newton_steps_on_the_learned_workload():
    """Train on 160 method-generated solves (15 epochs), then on held-out initial conditions:
    the judge takes the prediction, Newton from it needs fewer steps to |R| <= 1e-10 than
    from the plain iterate, and both starts converge to the same solution (the first levels
    also checked against the time-stepping oracle)."""
    net = NO.NeuralOperator(GAIN_CFG, seed=3)
    print("[gain] generate 160 solves 256^2 x 128", flush=True)
    u0s, coefs, steps = NO.generate(net, lambda i: W.burgers256_learned(nt=128, index=i), 160)
    print(f"[gain] plain Newton steps in generation: mean {np.mean(steps):.2f}; train 15 epochs", flush=True)
    hist = NO.train(net, u0s, coefs, epochs=15, lr=2e-3, batch=8)
    print(f"loss {hist[0]:.3e} -> {hist[-1]:.3e}", flush=True)
    saved = []
    for i in range(3):
        p = W.burgers256_learned(nt=128, seed=777, index=i)
        u0 = dev(p.u0)
        U = torch.empty((p.nt, p.ny, p.nx), dtype=torch.float64, device="cuda")
        j = net.initial_iterate(p, u0, U)
        assert j["chosen"] == "learned", j
        st_l = P.solve(p, U, u0, tol=1e-10, max_iter=60, cache_tag=1)
        Up = dev(p.plain_iterate())
        st_p = P.solve(p, Up, u0, tol=1e-10, max_iter=60)
        print(f"[gain] held-out {i}: judge {j}; steps needed learned {st_l['needed']} plain {st_p['needed']}",
              flush=True)
        assert st_l["needed"] <= st_p["needed"]
        saved.append(st_p["needed"] - st_l["needed"])
        Ul, Upl = host(U), host(Up)
        assert np.max(np.abs(Ul - Upl)) <= 1e-10 * np.max(np.abs(Upl))
        if i == 0:
            Us, _ = sequential.solve_sequential(p, levels=2)
            assert np.max(np.abs(Ul[:2] - Us)) <= 1e-10 * np.max(np.abs(Us))
    print("Newton steps saved per held-out sample:", saved)
    assert sum(saved) >= 2


@pytest.mark.parametrize("nt", [2, 16, 40])
@pytest.mark.parametrize("judge", ["accumulated", "residual"])
def test_judge_norms_match_the_oracle_residual(nt, judge):
    """The judge's figures are the oracle's residual norms of the two candidates: max |r^n_p|,
    or max |sum_{m<=n} r^m_p| for the accumulated judge, of the network's prediction (res_pred)
    and of the plain iterate (res_plain). nt = 16 is one chunk of the two-pass accumulated
    form, nt = 40 three with a ragged tail, nt = 2 the stored-residual form."""
    cfg = NO.NOConfig(nx=32, ny=32, nt=nt, width=16, modes=4, layers=1, tmodes=min(nt, 4))
    net = NO.NeuralOperator(cfg)
    net.params.copy_(dev(_params(cfg, 23, proj_scale=3.0), torch.float32))
    s = np.random.SeedSequence(44, spawn_key=(nt,))
    p = W.burgers_periodic(32, nt, 5e-4, 0.005, W.fourier_u0_periodic(32, int(s.generate_state(1)[0])))
    u0 = dev(p.u0)
    Upred = host(net.forward(u0))
    U = torch.empty((nt, 32, 32), dtype=torch.float64, device="cuda")
    print(f"[judge] norms nt={nt} {judge}", flush=True)
    j = net.initial_iterate(p, u0, U, judge=judge)

    def norm(V):
        R = allatonce.global_residual(V, p)
        return float(np.max(np.abs(np.cumsum(R, axis=0) if judge == "accumulated" else R)))

    scale = float(np.max(np.abs(Upred)))
    assert abs(j["res_pred"] - norm(Upred)) <= 1e-12 * (1 + nt) * scale, (j, norm(Upred))
    assert abs(j["res_plain"] - norm(p.plain_iterate())) <= 1e-12 * (1 + nt) * scale, j
    expect = "learned" if j["res_pred"] < j["res_plain"] else "plain"
    assert j["chosen"] == expect
    np.testing.assert_array_equal(host(U), Upred if expect == "learned" else p.plain_iterate())


def test_corrupted_network_falls_back_to_plain_iterate_and_matches_oracle():
    net = NO.NeuralOperator(TRAIN_CFG, seed=6)
    # noise-scale projection: the prediction is garbage, the judge must reject it
    net.params.copy_(dev(_params(TRAIN_CFG, 17, proj_scale=50.0), torch.float32))
    p = _burgers(2000)
    u0 = dev(p.u0)
    for judge in ("accumulated", "residual"):
        U = torch.empty((p.nt, p.ny, p.nx), dtype=torch.float64, device="cuda")
        print(f"[judge] corrupted network, {judge}", flush=True)
        j = net.initial_iterate(p, u0, U, judge=judge)
        assert j["chosen"] == "plain", j
        assert j["res_pred"] > j["res_plain"]
        np.testing.assert_array_equal(host(U), p.plain_iterate())
    P.solve(p, U, u0, tol=1e-11, max_iter=60)
    Us, _ = sequential.solve_sequential(p)
    assert np.max(np.abs(host(U) - Us)) <= 1e-10 * np.max(np.abs(Us))


def test_initial_iterate_rejects_mismatched_problem():
    net = NO.NeuralOperator(TRAIN_CFG)
    p = W.burgers_periodic(32, 8, 5e-4, 0.005, np.zeros((32, 32)))
    U = torch.zeros((8, 32, 32), dtype=torch.float64, device="cuda")
    with pytest.raises(P.PTSError):
        net.initial_iterate(p, dev(p.u0), U)


def test_batched_forward_equals_one_sample_forwards():
    """The batched forward (transforms over the channels of all samples, batched channel mixes)
    gives each sample's one-sample forward (the same bfloat16 products; summation order may
    differ in the split-K transforms)."""
    cfg = SMALL
    net = NO.NeuralOperator(cfg)
    net.params.copy_(dev(_params(cfg, 17), torch.float32))
    u0s = [dev(_u0(cfg, 20 + b)) for b in range(5)]
    ws = net.workspace_batched(len(u0s))
    outs = [torch.empty((cfg.nt, cfg.ny, cfg.nx), dtype=torch.float64, device="cuda") for _ in u0s]
    print("[forward] batched x5", flush=True)
    net.forward_batched(u0s, outs, ws)
    for u0, U in zip(u0s, outs):
        ref = host(net.forward(u0)) - host(u0)[None]
        assert _relnorm(host(U) - host(u0)[None], ref) < 1e-5


def test_batched_initial_iterate_matches_one_by_one(trained):
    net, _ = trained
    probs = [_burgers(2000 + i) for i in range(3)]
    u0s = [dev(p.u0) for p in probs]
    Us = [torch.empty((p.nt, p.ny, p.nx), dtype=torch.float64, device="cuda") for p in probs]
    print("[judge] batched x3", flush=True)
    chosen = net.initial_iterate_batched(probs[0], u0s, Us, net.workspace_batched(3))
    for p, u0, U, c in zip(probs, u0s, Us, chosen):
        V = torch.empty_like(U)
        j = net.initial_iterate(p, u0, V)
        assert c == j["chosen"], (c, j)
        ref = host(V) - host(u0)[None]
        assert _relnorm(host(U) - host(u0)[None], ref) < 1e-5

"""Space-time BDF1 Newton solver (ParaDIn direct-inverse method) on MI355X.

Thin Python binding of libpts.so (include/pts.h). Every step of the method runs
in the library's HIP kernels; this module only checks tensors, fills the C
structures and passes device pointers plus the current HIP stream. PyTorch
provides device memory and streams.

Arrays: float64 CUDA (HIP) tensors, contiguous. U has shape (nt, ny, nx) and
holds levels 1..nt, u0 has shape (ny, nx) (Section 3, Eq. (4) ordering, x fastest).
A problem is any object with the attributes kind, bc, nx, ny, nt, hx, hy, dt,
mu_a, mu_b (for instance workloads.Problem), plus an optional device tensor of
Dirichlet data of shape (nt, 2 (nx + ny)).
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import torch

from . import _lib
from ._lib import (PTS_BURGERS, PTS_DIRICHLET, PTS_ERR_HIP, PTS_FP64, PTS_HEAT, PTS_MIXED, PTS_PERIODIC,
                   PTS_SCHED_AUTO, PTS_SCHED_BULK, PTS_SCHED_PIPELINE, pts_options, pts_problem,
                   pts_stats)

__all__ = ["PTSError", "make_problem", "workspace", "init_plain", "assemble", "newton_step", "newton_step_static",
           "products_workspace", "newton_step_products", "solve_products", "product_diamond",
           "solve", "autotune",
           "solve_batched", "autotune_batched", "batched_workspace", "coarse_workspace", "coarse_initial_iterate",
           "coarse_workspace_batched", "coarse_initial_iterate_batched", "window_bound",
           "library_path", "version"]


class PTSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pts error {code}: {msg}")
        self.code = code


def _lib_checked():
    return _lib.load()


def library_path() -> str:
    return _lib.LIB_PATH


def version() -> str:
    return _lib_checked().pts_version().decode()


def _check(rc: int):
    if rc != 0:
        raise PTSError(rc, _lib_checked().pts_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _dev_f64(t: torch.Tensor, shape, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def make_problem(prob, precision: str = "fp64", bdata: Optional[torch.Tensor] = None,
                 dts: Optional[torch.Tensor] = None) -> pts_problem:
    """Fill a pts_problem from a problem description. Per-level step sizes come from `dts` (a
    device float64 tensor of nt entries) or, when that is None, from the description's `dts`
    array (copied to the device and kept alive with the returned structure)."""
    p = pts_problem()
    p.kind = int(prob.kind)
    p.bc = int(prob.bc)
    p.nx, p.ny, p.nt = int(prob.nx), int(prob.ny), int(prob.nt)
    p.precision = PTS_MIXED if precision == "mixed" else PTS_FP64
    p.hx, p.hy, p.dt = float(prob.hx), float(prob.hy), float(prob.dt)
    p.mu_a, p.mu_b = float(prob.mu_a), float(prob.mu_b)
    if bdata is not None:
        _dev_f64(bdata, (p.nt, 2 * (p.nx + p.ny)), "bdata")
        p.bdata = bdata.data_ptr()
    else:
        p.bdata = None
    if dts is None and getattr(prob, "dts", None) is not None:
        dts = torch.as_tensor(prob.dts, dtype=torch.float64, device="cuda").contiguous()
    if dts is not None:
        _dev_f64(dts, (p.nt,), "dts")
        p.dt_levels = dts.data_ptr()
        p._dts = dts  # keeps the device copy alive as long as the structure
    else:
        p.dt_levels = None
    return p


def _stream(stream=None) -> C.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def workspace(prob, precision: str = "fp64", device="cuda") -> torch.Tensor:
    """Allocate the device workspace pts_solve / pts_newton_step need for `prob`."""
    p = make_problem(prob, precision)
    nbytes = _lib_checked().pts_workspace_bytes(C.byref(p))
    if nbytes == 0:
        _check(_lib.PTS_ERR_INVALID_ARG)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nbytes]


def _options(window=0, schedule="auto", sweeps=0, refine=-1, lin_tol=0.0, use_graph=True, stages=0,
             profile=False, cache_tag=0, wave_launch="diagonal", barrier_spins=0):
    o = pts_options()
    o.window = int(window)
    o.schedule = {"auto": PTS_SCHED_AUTO, "bulk": PTS_SCHED_BULK, "pipeline": PTS_SCHED_PIPELINE}[schedule]
    o.sweeps = int(sweeps)
    o.refine = int(refine)
    o.lin_tol = float(lin_tol)
    o.use_graph = 1 if use_graph else 0
    o.stages = int(stages)
    o.profile = 1 if profile else 0
    o.cache_tag = int(cache_tag)
    o.wave_launch = {"diagonal": 0, "sequence": 1}[wave_launch]
    o.barrier_spins = int(barrier_spins)
    return o


def _stats_dict(st: pts_stats) -> dict:
    k = st.iterations
    n = min(st.hist if st.hist > 0 else k + 1, _lib.PTS_MAX_HIST)
    return {
        "iterations": k, "converged": bool(st.converged), "window": st.window, "sweeps": st.sweeps,
        "refine": st.refine, "schedule": st.schedule, "launches": st.launches, "slab": st.slab,
        "res_inf": list(st.res_inf[:n]), "upd_rms": list(st.upd_rms[1:n]),
        "rho_max": list(st.rho_max[:n]), "solve_ms": st.solve_ms,
        "prof_ms": list(st.prof_ms), "prof_count": list(st.prof_count),
        "level_solve_bytes": st.level_solve_bytes,
        "kern_ms": list(st.kern_ms), "kern_count": list(st.kern_count), "kern_bytes": list(st.kern_bytes),
    }


def init_plain(prob, U, u0, stream=None):
    """U <- u^0 at every level (plain Newton start), on the device."""
    p = make_problem(prob)
    _dev_f64(U, (p.nt, p.ny, p.nx), "U")
    _dev_f64(u0, (p.ny, p.nx), "u0")
    _check(_lib_checked().pts_init_plain(C.byref(p), _ptr(U), _ptr(u0), _stream(stream)))


def assemble(prob, U, u0, bdata=None, coef: bool = False, stream=None):
    """Residual r^n and (optionally) the five rows of A_n at every level.

    Returns (R, coef or None, max|R| as a 0-d device tensor)."""
    p = make_problem(prob, "fp64", bdata)
    _dev_f64(U, (p.nt, p.ny, p.nx), "U")
    _dev_f64(u0, (p.ny, p.nx), "u0")
    R = torch.empty_like(U)
    cf = torch.empty((p.nt, 5, p.ny, p.nx), dtype=torch.float64, device=U.device) if coef else None
    rinf = torch.empty((), dtype=torch.float64, device=U.device)
    _check(_lib_checked().pts_assemble(C.byref(p), _ptr(U), _ptr(u0), _ptr(R), _ptr(cf), _ptr(rinf),
                                       _stream(stream)))
    return R, cf, rinf


def newton_step(prob, U, u0, bdata=None, precision="fp64", ws=None, stream=None, **opts) -> dict:
    """One all-at-once Newton step applied to U in place; returns the statistics."""
    p = make_problem(prob, precision, bdata)
    _dev_f64(U, (p.nt, p.ny, p.nx), "U")
    _dev_f64(u0, (p.ny, p.nx), "u0")
    ws = workspace(prob, precision, U.device) if ws is None else ws
    o = _options(**opts)
    st = pts_stats()
    _check(_lib_checked().pts_newton_step(C.byref(p), _ptr(U), _ptr(u0), _ptr(ws), ws.numel(), C.byref(o),
                                          C.byref(st), _stream(stream)))
    return _stats_dict(st)


def newton_step_static(prob, U, u0, bdata=None, precision="fp64", stream=None, **opts) -> dict:
    """One all-at-once Newton step applied to U in place, with the library's static device
    scratch instead of a workspace (pts_newton_step_static: allocates nothing); returns the
    statistics."""
    p = make_problem(prob, precision, bdata)
    _dev_f64(U, (p.nt, p.ny, p.nx), "U")
    _dev_f64(u0, (p.ny, p.nx), "u0")
    o = _options(**opts)
    st = pts_stats()
    _check(_lib_checked().pts_newton_step_static(C.byref(p), _ptr(U), _ptr(u0), C.byref(o), C.byref(st),
                                                 _stream(stream)))
    return _stats_dict(st)


def products_workspace(prob, device="cuda") -> torch.Tensor:
    """Device workspace of the explicit-product form (pts_products_workspace_bytes)."""
    p = make_problem(prob)
    nbytes = _lib_checked().pts_products_workspace_bytes(C.byref(p))
    if nbytes == 0:
        _check(_lib.PTS_ERR_INVALID_ARG)
    return _aligned_bytes(nbytes, device)


def newton_step_products(prob, U, u0, bdata=None, ws=None, stream=None) -> dict:
    """One Newton step in the paper's explicit-product form (Theorem 1, Eq. (8))."""
    p = make_problem(prob, "fp64", bdata)
    _dev_f64(U, (p.nt, p.ny, p.nx), "U")
    _dev_f64(u0, (p.ny, p.nx), "u0")
    ws = products_workspace(prob, U.device) if ws is None else ws
    st = pts_stats()
    _check(_lib_checked().pts_newton_step_products(C.byref(p), _ptr(U), _ptr(u0), _ptr(ws), ws.numel(),
                                                   C.byref(st), _stream(stream)))
    return _stats_dict(st)


def solve_products(prob, U, u0, tol=1e-12, max_iter=50, bdata=None, ws=None, stream=None) -> dict:
    """Newton iteration with every step in the explicit-product form."""
    p = make_problem(prob, "fp64", bdata)
    _dev_f64(U, (p.nt, p.ny, p.nx), "U")
    _dev_f64(u0, (p.ny, p.nx), "u0")
    ws = products_workspace(prob, U.device) if ws is None else ws
    st = pts_stats()
    _check(_lib_checked().pts_solve_products(C.byref(p), _ptr(U), _ptr(u0), float(tol), int(max_iter), _ptr(ws),
                                             ws.numel(), C.byref(st), _stream(stream)))
    return _stats_dict(st)


def product_diamond(prob, U, u0, n, bdata=None, ws=None, stream=None) -> torch.Tensor:
    """P^n = A_1 ... A_n at U in diamond storage, shape (2n^2 + 2n + 1, ny, nx)."""
    p = make_problem(prob, "fp64", bdata)
    _dev_f64(U, (p.nt, p.ny, p.nx), "U")
    _dev_f64(u0, (p.ny, p.nx), "u0")
    ws = products_workspace(prob, U.device) if ws is None else ws
    out = torch.empty((2 * n * n + 2 * n + 1, p.ny, p.nx), dtype=torch.float64, device=U.device)
    _check(_lib_checked().pts_product_diamond(C.byref(p), _ptr(U), _ptr(u0), int(n), _ptr(out), _ptr(ws), ws.numel(),
                                              _stream(stream)))
    return out


def solve(prob, U, u0, tol=1e-12, max_iter=50, bdata=None, precision="fp64", ws=None, stream=None,
          raise_on_error=True, **opts) -> dict:
    """Newton iteration on U in place until max|R| <= tol; returns the statistics.

    With raise_on_error=False the return code is reported in the dict instead."""
    p = make_problem(prob, precision, bdata)
    _dev_f64(U, (p.nt, p.ny, p.nx), "U")
    _dev_f64(u0, (p.ny, p.nx), "u0")
    ws = workspace(prob, precision, U.device) if ws is None else ws
    o = _options(**opts)
    st = pts_stats()
    rc = _lib_checked().pts_solve(C.byref(p), _ptr(U), _ptr(u0), float(tol), int(max_iter), _ptr(ws),
                                  ws.numel(), C.byref(o), C.byref(st), _stream(stream))
    out = _stats_dict(st)
    out["rc"] = rc
    # Newton steps after which |R| <= tol was first reached (the pipelined schedule may
    # apply a few more in the same launch sequence)
    out["needed"] = next((k for k, r in enumerate(out["res_inf"]) if r <= tol), None)
    if rc != 0:
        out["error"] = _lib_checked().pts_last_error().decode()
        if raise_on_error:
            _check(rc)
    return out


def autotune(prob, U, u0, tol=1e-12, max_iter=50, bdata=None, precision="fp64", ws=None, stream=None,
             **opts) -> dict:
    """Pick the fastest inner plan of the wavefront schedule for this problem (U is restored)."""
    p = make_problem(prob, precision, bdata)
    _dev_f64(U, (p.nt, p.ny, p.nx), "U")
    _dev_f64(u0, (p.ny, p.nx), "u0")
    ws = workspace(prob, precision, U.device) if ws is None else ws
    o = _options(**opts)
    st = pts_stats()
    _check(_lib_checked().pts_autotune(C.byref(p), _ptr(U), _ptr(u0), float(tol), int(max_iter), _ptr(ws),
                                       ws.numel(), C.byref(o), C.byref(st), _stream(stream)))
    return {"sweeps": st.sweeps, "passes": st.refine + 1, "newton_steps": st.iterations, "ms": st.solve_ms,
            "slab": st.slab}


def _aligned_bytes(nbytes, device):
    raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % 256
    return raw[off:off + nbytes]


def batched_workspace(probs, precision="fp64", device="cuda", bdatas=None) -> torch.Tensor:
    """Device workspace of solve_batched / autotune_batched for these instances. Reusing one
    across calls keeps the captured wavefront graphs valid (they hold its address)."""
    n = len(probs)
    bdatas = bdatas or [None] * n
    arr = (pts_problem * n)(*[make_problem(q, precision, b) for q, b in zip(probs, bdatas)])
    nbytes = _lib_checked().pts_workspace_bytes_batched(arr, n)
    if nbytes == 0:
        _check(_lib.PTS_ERR_INVALID_ARG)
    return _aligned_bytes(nbytes, device)


def _batched_args(probs, Us, u0s, bdatas, precision, ws):
    n = len(probs)
    bdatas = bdatas or [None] * n
    structs = [make_problem(q, precision, b) for q, b in zip(probs, bdatas)]
    arr = (pts_problem * n)(*structs)
    arr._keep = structs  # their device copies of per-level steps stay alive with the array
    for q, U, u0 in zip(probs, Us, u0s):
        _dev_f64(U, (q.nt, q.ny, q.nx), "U")
        _dev_f64(u0, (q.ny, q.nx), "u0")
    if ws is None:
        ws = batched_workspace(probs, precision, Us[0].device, bdatas)
    uptr = (C.c_void_p * n)(*[U.data_ptr() for U in Us])
    u0ptr = (C.c_void_p * n)(*[u.data_ptr() for u in u0s])
    return arr, ws, uptr, u0ptr


def solve_batched(probs, Us, u0s, tol=1e-12, max_iter=50, bdatas=None, precision="fp64", stream=None, ws=None,
                  **opts):
    """Solve independent instances together; returns one statistics dict per instance.
    ws: a batched_workspace (allocated per call when None)."""
    n = len(probs)
    arr, ws, uptr, u0ptr = _batched_args(probs, Us, u0s, bdatas, precision, ws)
    o = _options(**opts)
    sts = (pts_stats * n)()
    rc = _lib_checked().pts_solve_batched(arr, n, uptr, u0ptr, float(tol), int(max_iter), _ptr(ws), ws.numel(),
                                          C.byref(o), sts, _stream(stream))
    _check(rc)
    out = [_stats_dict(s) for s in sts]
    for d in out:  # Newton steps after which |R| <= tol was first reached
        d["needed"] = next((k for k, r in enumerate(d["res_inf"]) if r <= tol), None)
    return out


def autotune_batched(probs, Us, u0s, tol=1e-12, max_iter=50, bdatas=None, precision="fp64", stream=None,
                     ws=None, **opts) -> dict:
    """Pick the fastest wavefront plan for batches of one problem (Us restored); returns the
    chosen plan (sweeps, refine, iterations, solve_ms). ws: as for solve_batched."""
    n = len(probs)
    arr, ws, uptr, u0ptr = _batched_args(probs, Us, u0s, bdatas, precision, ws)
    o = _options(**opts)
    sts = (pts_stats * n)()
    _check(_lib_checked().pts_autotune_batched(arr, n, uptr, u0ptr, float(tol), int(max_iter), _ptr(ws),
                                               ws.numel(), C.byref(o), sts, _stream(stream)))
    return {"sweeps": sts[0].sweeps, "refine": sts[0].refine, "iterations": sts[0].iterations,
            "solve_ms": sts[0].solve_ms}


def coarse_workspace(prob, cf, device="cuda") -> torch.Tensor:
    """Device workspace of coarse_initial_iterate for `prob` and coarsening factor cf."""
    p = make_problem(prob)
    nbytes = _lib_checked().pts_coarse_workspace_bytes(C.byref(p), int(cf))
    if nbytes == 0:
        _check(_lib.PTS_ERR_INVALID_ARG)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nbytes]


def coarse_initial_iterate(prob, U, u0, cf, tol=1e-12, max_iter=50, ws=None, bdata=None, stream=None) -> dict:
    """Section 4's initial iterate into U: solve on the grid coarsened by cf in space and time,
    cubic splines back to the fine grid. Returns the coarse solve's statistics."""
    p = make_problem(prob, "fp64", bdata)
    _dev_f64(U, (p.nt, p.ny, p.nx), "U")
    _dev_f64(u0, (p.ny, p.nx), "u0")
    ws = coarse_workspace(prob, cf, U.device) if ws is None else ws
    st = pts_stats()
    _check(_lib_checked().pts_coarse_initial_iterate(C.byref(p), int(cf), _ptr(u0), _ptr(U), float(tol),
                                                     int(max_iter), _ptr(ws), ws.numel(), C.byref(st),
                                                     _stream(stream)))
    return _stats_dict(st)


def _coarse_problems(prob, n, bdata):
    """pts_problem array of n instances: one problem for all, or a list of n problems."""
    probs = list(prob) if isinstance(prob, (list, tuple)) else [prob] * n
    if len(probs) != n:
        raise ValueError(f"{len(probs)} problems for {n} instances")
    bdatas = list(bdata) if isinstance(bdata, (list, tuple)) else [bdata] * n
    structs = [make_problem(q, "fp64", b) for q, b in zip(probs, bdatas)]
    arr = (pts_problem * n)(*structs)
    arr._keep = structs
    return probs, arr


def coarse_workspace_batched(prob, cf, n, device="cuda") -> torch.Tensor:
    """Device workspace of coarse_initial_iterate_batched for n instances of `prob` (one
    problem, or a list of n problems)."""
    _, arr = _coarse_problems(prob, n, None)
    nbytes = _lib_checked().pts_coarse_workspace_bytes_batched(arr, int(n), int(cf))
    if nbytes == 0:
        _check(_lib.PTS_ERR_INVALID_ARG)
    return _aligned_bytes(nbytes, device)


def coarse_initial_iterate_batched(prob, Us, u0s, cf, tol=1e-12, max_iter=50, bdata=None, ws=None,
                                   stream=None) -> list:
    """The coarse-grid start of several instances (prob: one problem for all, or one per
    instance; grids and level counts may differ): the coarse solves share batched launches.
    Returns the coarse solves' statistics. ws: a coarse_workspace_batched (allocated per call
    when None). bdata: one array for all, or a list."""
    n = len(Us)
    probs, arr = _coarse_problems(prob, n, bdata)
    for q, U, u0 in zip(probs, Us, u0s):
        _dev_f64(U, (q.nt, q.ny, q.nx), "U")
        _dev_f64(u0, (q.ny, q.nx), "u0")
    lib = _lib_checked()
    ws = coarse_workspace_batched(probs, cf, n, Us[0].device) if ws is None else ws
    uptr = (C.c_void_p * n)(*[U.data_ptr() for U in Us])
    u0ptr = (C.c_void_p * n)(*[u.data_ptr() for u in u0s])
    sts = (pts_stats * n)()
    _check(lib.pts_coarse_initial_iterate_batched(arr, n, int(cf), u0ptr, uptr, float(tol), int(max_iter),
                                                  _ptr(ws), ws.numel(), sts, _stream(stream)))
    return [_stats_dict(s) for s in sts]


def window_bound(h, mu, tau=0.0, c=1.0, eps=1e-16, wmax=100000) -> int:
    """Section 7, Eq. (cond): largest window W with K^W < c h^4 / eps (host only)."""
    r = _lib_checked().pts_window_bound(float(h), float(mu), float(tau), float(c), float(eps), int(wmax))
    if r < 0:
        _check(r)
    return r

"""ctypes view of libpts.so (include/pts.h). Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpts.so")

PTS_HEAT, PTS_BURGERS = 0, 1
PTS_DIRICHLET, PTS_PERIODIC = 0, 1
PTS_FP64, PTS_MIXED = 0, 1
PTS_SCHED_AUTO, PTS_SCHED_BULK, PTS_SCHED_PIPELINE = 0, 1, 2
PTS_OK = 0
PTS_ERR_INVALID_ARG = -1
PTS_ERR_HIP = -2
PTS_ERR_NONFINITE = -3
PTS_ERR_SINGULAR = -4
PTS_ERR_NOT_CONVERGED = -5
PTS_ERR_WORKSPACE = -6
PTS_ERR_NOT_DOMINANT = -7
PTS_MAX_HIST = 64


class pts_problem(C.Structure):
    _fields_ = [("kind", C.c_int32), ("bc", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("nt", C.c_int32), ("precision", C.c_int32), ("hx", C.c_double), ("hy", C.c_double),
                ("dt", C.c_double), ("mu_a", C.c_double), ("mu_b", C.c_double), ("bdata", C.c_void_p),
                ("dt_levels", C.c_void_p)]


class pts_options(C.Structure):
    _fields_ = [("window", C.c_int32), ("schedule", C.c_int32), ("sweeps", C.c_int32),
                ("refine", C.c_int32), ("lin_tol", C.c_double), ("use_graph", C.c_int32),
                ("stages", C.c_int32), ("profile", C.c_int32), ("cache_tag", C.c_int32),
                ("wave_launch", C.c_int32), ("barrier_spins", C.c_int32)]


class pts_stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("window", C.c_int32),
                ("sweeps", C.c_int32), ("refine", C.c_int32), ("schedule", C.c_int32),
                ("launches", C.c_int32), ("slab", C.c_int32), ("hist", C.c_int32), ("pad", C.c_int32),
                ("res_inf", C.c_double * PTS_MAX_HIST), ("upd_rms", C.c_double * PTS_MAX_HIST),
                ("rho_max", C.c_double * PTS_MAX_HIST), ("solve_ms", C.c_double),
                ("prof_ms", C.c_double * 4), ("prof_count", C.c_int32 * 4),
                ("level_solve_bytes", C.c_double), ("kern_ms", C.c_double * 8),
                ("kern_count", C.c_int32 * 8), ("kern_bytes", C.c_double * 8)]


_lib = None


def load():
    """Load libpts.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2406_00878_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    P, V, I, D, S = C.POINTER(pts_problem), C.c_void_p, C.c_int, C.c_double, C.c_size_t
    sig = {
        "pts_workspace_bytes": (S, [P]),
        "pts_assemble": (I, [P, V, V, V, V, V, V]),
        "pts_init_plain": (I, [P, V, V, V]),
        "pts_newton_step": (I, [P, V, V, V, S, C.POINTER(pts_options), C.POINTER(pts_stats), V]),
        "pts_newton_step_static": (I, [P, V, V, C.POINTER(pts_options), C.POINTER(pts_stats), V]),
        "pts_solve": (I, [P, V, V, D, I, V, S, C.POINTER(pts_options), C.POINTER(pts_stats), V]),
        "pts_products_workspace_bytes": (S, [P]),
        "pts_newton_step_products": (I, [P, V, V, V, S, C.POINTER(pts_stats), V]),
        "pts_solve_products": (I, [P, V, V, D, I, V, S, C.POINTER(pts_stats), V]),
        "pts_product_diamond": (I, [P, V, V, I, V, V, S, V]),
        "pts_autotune": (I, [P, V, V, D, I, V, S, C.POINTER(pts_options), C.POINTER(pts_stats), V]),
        "pts_workspace_bytes_batched": (S, [P, I]),
        "pts_solve_batched": (I, [P, I, V, V, D, I, V, S, C.POINTER(pts_options), C.POINTER(pts_stats), V]),
        "pts_autotune_batched": (I, [P, I, V, V, D, I, V, S, C.POINTER(pts_options), C.POINTER(pts_stats), V]),
        "pts_coarse_workspace_bytes": (S, [P, I]),
        "pts_coarse_initial_iterate": (I, [P, I, V, V, D, I, V, S, C.POINTER(pts_stats), V]),
        "pts_coarse_workspace_bytes_batched": (S, [P, I, I]),
        "pts_coarse_initial_iterate_batched": (I, [P, I, I, V, V, D, I, V, S, C.POINTER(pts_stats), V]),
        "pts_window_bound": (I, [D, D, D, D, D, I]),
        "pts_last_error": (C.c_char_p, []),
        "pts_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib

"""ctypes declarations of libds3.so (the C ABI in include/ds3.h). Loading fails loudly when the library
has not been built: there is no fallback path."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# DS3_LIB names another build of the library to load (the sanitizer test's host-instrumented copy)
LIB_PATH = os.environ.get("DS3_LIB") or os.path.join(HERE, "libds3.so")

F32, BF16 = 0, 1


class Image(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("px_offset", C.c_int64)]


class Edge(C.Structure):
    _fields_ = [("i", C.c_int32), ("j", C.c_int32), ("idx_offset", C.c_int64)]


class MatchParams(C.Structure):
    _fields_ = [("max_iters", C.c_int32), ("lambda0", C.c_double), ("lambda_min", C.c_double),
                ("step_tol_px", C.c_double), ("ang_tol_px", C.c_double),
                ("range_rel_tol", C.c_double), ("mutual_radius_px", C.c_int32),
                ("q_min", C.c_double), ("nu_min", C.c_double)]


class GNParams(C.Structure):
    _fields_ = [("sigma_ray", C.c_double), ("sigma_dist", C.c_double), ("huber_k", C.c_double),
                ("lam", C.c_double), ("eps0", C.c_double), ("eps_mult", C.c_double),
                ("max_attempts", C.c_int32), ("K", C.POINTER(C.c_double)), ("sigma_pix", C.c_double),
                ("sigma_logz", C.c_double)]


class TrackParams(C.Structure):
    _fields_ = [("lambda0", C.c_double), ("lambda_min", C.c_double), ("lambda_up", C.c_double),
                ("lambda_down", C.c_double), ("max_trials", C.c_int32), ("step_tol", C.c_double)]


class TrackProblem(C.Structure):
    _fields_ = [("keyframe", Image), ("frame", Image), ("idx_offset", C.c_int64)]


class DepthParams(C.Structure):
    _fields_ = [("segments_per_kf", C.c_int32), ("conf_min", C.c_double), ("min_seg_px", C.c_int32),
                ("slic_iters", C.c_int32), ("sigma_point", C.c_double), ("huber_k", C.c_double),
                ("lambda_smooth", C.c_double), ("lambda_prior", C.c_double), ("lambda_lm", C.c_double),
                ("eta_max", C.c_double)]


class FusePair(C.Structure):
    _fields_ = [("canon_off", C.c_int64), ("pred_off", C.c_int64), ("n_px", C.c_int64)]


class PlanOpts(C.Structure):
    _fields_ = [("autotune", C.c_int32), ("px_per_thread", C.c_int32), ("use_graph", C.c_int32),
                ("reduce_timer", C.c_void_p), ("unroll", C.c_int32), ("solver", C.c_int32)]


_lib = None

vp, sz, i32, i64, f32, f64 = C.c_void_p, C.c_size_t, C.c_int32, C.c_int64, C.c_float, C.c_double
P_img, P_edge, P_i32, P_i64, P_f64 = (C.POINTER(Image), C.POINTER(Edge), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int64), C.POINTER(C.c_double))

_SIGS = {
    "ds3_default_match_params": (None, [C.POINTER(MatchParams)]),
    "ds3_default_gn_params": (None, [C.POINTER(GNParams)]),
    "ds3_status_string": (C.c_char_p, [C.c_int]),
    "ds3_version": (C.c_int, []),
    "ds3_pack_xyzc": (C.c_int, [vp, vp, i64, C.c_int, vp, vp]),
    "ds3_match_workspace_bytes": (sz, [i32, i32]),
    "ds3_match_bidir_workspace_bytes": (sz, [i32, i32, i32, i32]),
    "ds3_match": (C.c_int, [vp, Image, vp, Image, C.c_int, C.POINTER(MatchParams), vp, vp, vp, vp, sz, vp]),
    "ds3_match_bidir": (C.c_int, [vp, vp, vp, vp, Image, Image, C.c_int, C.POINTER(MatchParams), vp, vp,
                                  vp, vp, vp, sz, vp]),
    "ds3_match_batch_workspace_bytes": (sz, [i32, P_img, i32, P_edge]),
    "ds3_match_batch": (C.c_int, [vp, P_img, i32, vp, P_i64, P_edge, i32, C.c_int,
                                  C.POINTER(MatchParams), vp, vp, vp, vp, vp, vp, vp, sz, vp]),
    "ds3_timer_create": (C.c_int, [C.POINTER(vp)]),
    "ds3_timer_elapsed_ms": (C.c_int, [vp, C.POINTER(C.c_float)]),
    "ds3_timer_destroy": (C.c_int, [vp]),
    "ds3_gauge_workspace_bytes": (sz, [i32]),
    "ds3_gauge_align": (C.c_int, [vp, Image, vp, Image, C.c_int, vp, vp, vp, i32, i32, i32, i32, vp, vp,
                                  vp, sz, vp]),
    "ds3_apply_gauge": (C.c_int, [vp, i32, vp, vp, vp]),
    "ds3_umeyama": (C.c_int, [P_f64, P_f64, i64, P_f64]),
    "ds3_gauge_sync": (C.c_int, [vp, i32, P_i32, vp, P_img, C.c_int, P_edge, i32, vp, vp, vp, i32, P_i32,
                                 vp, sz, vp]),
    "ds3_sim3_exp": (C.c_int, [vp, vp, i32, vp]),
    "ds3_sim3_log": (C.c_int, [vp, vp, i32, vp]),
    "ds3_sim3_update": (C.c_int, [vp, vp, vp, i32, vp]),
    "ds3_gn_workspace_bytes": (sz, [i32, P_img, i32, P_edge, C.c_int]),
    "ds3_gn_linearize": (C.c_int, [vp, i32, P_img, vp, C.c_int, P_edge, i32, vp, C.POINTER(GNParams),
                                   P_i32, i32, vp, vp, vp, vp, vp, sz, vp]),
    "ds3_sim3_gn_step": (C.c_int, [vp, i32, P_img, vp, C.c_int, P_edge, i32, vp, C.POINTER(GNParams),
                                   P_i32, i32, vp, vp, vp, vp, sz, vp]),
    "ds3_chol_workspace_bytes": (sz, [i32]),
    "ds3_chol_ladder_solve": (C.c_int, [vp, vp, i32, f64, f64, f64, i32, vp, vp, vp, sz, vp]),
    "ds3_gn_plan_create": (C.c_int, [i32, P_img, vp, C.c_int, P_edge, i32, vp, C.POINTER(GNParams), P_i32,
                                     i32, C.POINTER(PlanOpts), vp, C.POINTER(vp), vp]),
    "ds3_gn_plan_run": (C.c_int, [vp, i32, vp, vp, vp]),
    "ds3_spchol_analyse": (C.c_int, [i32, i32, P_i32, P_i32, P_i32, P_i64]),
    "ds3_spchol_create": (C.c_int, [i32, i32, P_i32, C.POINTER(vp)]),
    "ds3_spchol_info": (C.c_int, [vp, P_i64]),
    "ds3_spchol_solve": (C.c_int, [vp, vp, vp, f64, f64, f64, i32, vp, vp, vp]),
    "ds3_spchol_destroy": (None, [vp]),
    "ds3_tilechol_analyse": (C.c_int, [i32, i32, P_i32, P_i32, P_i64]),
    "ds3_tilechol_create": (C.c_int, [i32, i32, P_i32, C.POINTER(vp)]),
    "ds3_tilechol_info": (C.c_int, [vp, P_i64]),
    "ds3_tilechol_solve": (C.c_int, [vp, vp, vp, f64, f64, f64, i32, vp, vp, vp, sz, vp]),
    "ds3_tilechol_destroy": (None, [vp]),
    "ds3_gn_plan_time_reduce": (C.c_int, [vp, i32, C.POINTER(C.c_float), vp]),
    "ds3_gn_plan_info": (C.c_int, [vp, P_i64, i32]),
    "ds3_gn_plan_refresh": (C.c_int, [vp, vp]),
    "ds3_gn_plan_destroy": (C.c_int, [vp]),
    "ds3_gn_plan_set_timer": (C.c_int, [vp, vp]),
    "ds3_tune_cache_reset": (C.c_int, []),
    "ds3_gn_cost": (C.c_int, [vp, i32, P_img, vp, C.c_int, P_edge, i32, vp, C.POINTER(GNParams), vp, vp,
                              sz, vp]),
    "ds3_gn_cost_adjoint": (C.c_int, [vp, i32, P_img, vp, C.c_int, P_edge, i32, vp, C.POINTER(GNParams),
                                      f32, vp, vp, vp, vp, vp, sz, vp]),
    "ds3_adjoint_plan_create": (C.c_int, [i32, P_img, vp, C.c_int, P_edge, i32, vp, C.POINTER(GNParams),
                                          C.POINTER(vp), vp]),
    "ds3_adjoint_plan_run": (C.c_int, [vp, vp, f32, vp, vp, vp, vp, vp, vp]),
    "ds3_adjoint_plan_destroy": (C.c_int, [vp]),
    "ds3_default_track_params": (None, [C.POINTER(TrackParams)]),
    "ds3_track_workspace_bytes": (sz, [i32, C.POINTER(TrackProblem), C.c_int]),
    "ds3_track": (C.c_int, [vp, C.c_int, C.POINTER(TrackProblem), i32, vp, C.POINTER(GNParams),
                            C.POINTER(TrackParams), vp, vp, vp, vp, vp, vp, sz, vp]),
    "ds3_track_noalloc": (C.c_int, [vp, C.c_int, C.POINTER(TrackProblem), i32, vp, C.POINTER(GNParams),
                                    C.POINTER(TrackParams), vp, vp, vp, vp, vp]),
    "ds3_default_depth_params": (None, [C.POINTER(DepthParams)]),
    "ds3_depth_plan_create": (C.c_int, [i32, P_img, vp, C.c_int, P_edge, i32, vp, P_i32, i32,
                                        C.POINTER(DepthParams), C.POINTER(vp), vp]),
    "ds3_depth_plan_run": (C.c_int, [vp, vp, i32, vp, vp, vp]),
    "ds3_depth_plan_info": (C.c_int, [vp, P_i64, i32]),
    "ds3_depth_plan_get": (C.c_int, [vp, vp, vp, vp]),
    "ds3_depth_plan_set_eta": (C.c_int, [vp, vp, vp]),
    "ds3_depth_plan_apply": (C.c_int, [vp, vp, vp]),
    "ds3_depth_plan_destroy": (C.c_int, [vp]),
    "ds3_fuse_workspace_bytes": (sz, [i32]),
    "ds3_fuse": (C.c_int, [vp, i64, vp, i64, C.POINTER(FusePair), i32, vp, i32, vp, sz, vp]),
}


def load():
    """Load libds3.so and declare its signatures. Raises if the library is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_names():
    return list(_SIGS)


class DS3Error(RuntimeError):
    def __init__(self, fn: str, code: int):
        msg = load().ds3_status_string(code).decode()
        super().__init__(f"{fn} failed with {code}: {msg}")
        self.code = code


def call(name: str, *args):
    rc = getattr(load(), name)(*args)
    if rc != 0:
        raise DS3Error(name, rc)
    return rc

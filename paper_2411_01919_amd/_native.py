"""ctypes view of libpp.so (the C ABI declared in include/pp.h).

Structures mirror pp.h field for field.  Loading fails loudly when the
library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PP_LIB") or os.path.join(_HERE, "libpp.so")

c_i32, c_u64, c_f32, c_f64, c_vp = ctypes.c_int32, ctypes.c_uint64, ctypes.c_float, ctypes.c_double, ctypes.c_void_p

PP_OK, PP_PENDING = 0, 1
PP_E_INVAL, PP_E_NOMEM, PP_E_BUDGET, PP_E_HIP, PP_E_NODEVICE, PP_E_CLOSED, PP_E_UNSUPPORTED, PP_E_TIMEOUT = \
    -1, -2, -3, -4, -5, -6, -7, -8
PP_E_AGAIN = -9
PP_EDGE_EXP, PP_EDGE_RATIONAL = 0, 1
PP_DIFFUSE_EDGE4, PP_DIFFUSE_PIXEL, PP_DIFFUSE_EDGE8 = 0, 1, 2
PP_SCORE_FP32, PP_SCORE_MFMA_F32, PP_SCORE_BF16, PP_SCORE_FP16 = 0, 1, 2, 3


class Intrinsics(ctypes.Structure):
    _fields_ = [("fx", c_f32), ("fy", c_f32), ("cx", c_f32), ("cy", c_f32)]


class FrameDesc(ctypes.Structure):
    _fields_ = [("width", c_i32), ("height", c_i32), ("pitch_px", c_i32)]


class DiffuseParams(ctypes.Structure):
    _fields_ = [("iters", c_i32), ("lam", c_f32), ("kappa_mm", c_f32), ("edge_stop", c_i32), ("scheme", c_i32)]


class RansacParams(ctypes.Structure):
    _fields_ = [("max_planes", c_i32), ("hyps_per_plane", c_i32), ("min_inliers", c_i32), ("thresh_m", c_f32),
                ("seed", c_u64), ("frame_id", c_u64), ("precision", c_i32), ("recheck_band_m", c_f32)]


class Plane(ctypes.Structure):
    _fields_ = [("n", c_f64 * 3), ("d", c_f64), ("centroid", c_f64 * 3), ("inliers", c_i32), ("hyp_index", c_i32)]


class RansacDebug(ctypes.Structure):
    _fields_ = [("counts", c_vp), ("hyps", c_vp), ("triples", c_vp), ("round_info", c_vp), ("masks", c_vp),
                ("valid_list", c_vp), ("n_valid", c_vp), ("scored", c_vp)]


class RegionDebug(ctypes.Structure):
    _fields_ = [("npts", c_vp), ("triples", c_vp), ("hyps", c_vp), ("errors", c_vp), ("counts", c_vp),
                ("jstar", c_vp)]


class SegmentParams(ctypes.Structure):
    _fields_ = [("low", c_f32), ("high", c_f32), ("min_area", c_i32), ("max_regions", c_i32)]


class MapParams(ctypes.Structure):
    _fields_ = [("drift_tolerance_m", ctypes.c_double), ("sigma_p", ctypes.c_double), ("sigma_m", ctypes.c_double),
                ("max_tilt_deg", ctypes.c_double)]


class MapObservation(ctypes.Structure):
    _fields_ = [("n", ctypes.c_double * 3), ("d", ctypes.c_double), ("centroid", ctypes.c_double * 3),
                ("support", c_i32), ("n_vertices", c_i32), ("xy_px", c_vp)]


class MapFrameResult(ctypes.Structure):
    _fields_ = [("matched", c_i32), ("added", c_i32), ("skipped", c_i32), ("pad", c_i32),
                ("measurement", ctypes.c_double), ("drift", ctypes.c_double), ("variance", ctypes.c_double)]


class MapPolygonInfo(ctypes.Structure):
    _fields_ = [("height", ctypes.c_double), ("support", ctypes.c_int64), ("n_vertices", c_i32), ("pad", c_i32)]


class FrameJob(ctypes.Structure):
    _fields_ = [("depth", c_vp), ("desc", FrameDesc), ("K", Intrinsics), ("diffuse", DiffuseParams),
                ("ransac", RansacParams), ("depth_mm", c_vp), ("points", c_vp), ("normals", c_vp),
                ("valid", c_vp), ("planes", c_vp), ("n_planes", c_vp), ("labels", c_vp)]


class Tuning(ctypes.Structure):
    _fields_ = [("diffuse_tile", c_i32), ("diffuse_t", c_i32), ("score_hb", c_i32), ("score_chunk", c_i32)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("device", c_i32), ("hbm_budget_bytes", c_u64), ("max_batch", c_i32), ("lanes", c_i32),
                ("staging_frames", c_i32), ("use_graphs", c_i32), ("dry_run_us", c_i32), ("dry_run_fail_batch", c_i32)]


class Result(ctypes.Structure):
    _fields_ = [("planes", c_vp), ("n_planes", c_vp), ("labels", c_vp), ("stream_id", c_i32),
                ("frame_id", c_u64), ("latency_us", c_f64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", c_u64), ("completed", c_u64), ("rejected", c_u64), ("cancelled", c_u64),
                ("launches", c_u64), ("mean_batch", c_f64), ("p50_us", c_f64), ("p99_us", c_f64), ("max_us", c_f64),
                ("hbm_in_use", c_u64), ("hbm_peak", c_u64), ("queued", c_i32), ("in_flight", c_i32)]


# name -> (restype, argtypes); exactly the entry points pp.h declares
SIGNATURES = {
    "pp_ctx_create": (c_i32, [c_i32, ctypes.POINTER(c_vp)]),
    "pp_ctx_destroy": (c_i32, [c_vp]),
    "pp_status_string": (ctypes.c_char_p, [c_i32]),
    "pp_last_error": (ctypes.c_char_p, [c_vp]),
    "pp_diffuse": (c_i32, [c_vp, c_vp, c_vp, FrameDesc, ctypes.POINTER(DiffuseParams), c_vp]),
    "pp_normals": (c_i32, [c_vp, c_vp, FrameDesc, Intrinsics, c_vp, c_vp, c_vp, c_vp]),
    "pp_ransac_planes": (c_i32, [c_vp, c_vp, c_vp, c_vp, FrameDesc, ctypes.POINTER(RansacParams), c_vp, c_vp, c_vp, c_vp]),
    "pp_ransac_planes_noalloc": (c_i32, [c_vp, c_vp, FrameDesc, ctypes.POINTER(RansacParams), c_vp, c_vp, c_vp, c_vp]),
    "pp_ransac_planes_dbg": (c_i32, [c_vp, c_vp, c_vp, FrameDesc, ctypes.POINTER(RansacParams), c_vp, c_vp, c_vp,
                                     ctypes.POINTER(RansacDebug), c_vp]),
    "pp_map_create": (c_i32, [ctypes.POINTER(MapParams), ctypes.POINTER(c_vp)]),
    "pp_map_destroy": (c_i32, [c_vp]),
    "pp_map_integrate": (c_i32, [c_vp, Intrinsics, c_vp, c_vp, c_vp, c_i32, c_vp, ctypes.POINTER(MapFrameResult)]),
    "pp_map_size": (c_i32, [c_vp, ctypes.POINTER(c_i32)]),
    "pp_map_polygon": (c_i32, [c_vp, c_i32, ctypes.POINTER(MapPolygonInfo), c_vp, c_i32]),
    "pp_region_polygons": (c_i32, [c_vp, FrameDesc, c_i32, ctypes.c_double, c_vp, c_i32, c_vp]),
    "pp_segment": (c_i32, [c_vp, c_vp, c_vp, FrameDesc, ctypes.POINTER(SegmentParams), c_vp, c_vp, c_vp, c_vp]),
    "pp_ransac_regions_dbg": (c_i32, [c_vp, c_vp, c_vp, c_vp, FrameDesc, ctypes.POINTER(RansacParams), c_vp, c_vp,
                                      c_vp, ctypes.POINTER(RegionDebug), c_vp]),
    "pp_debug_score_triples": (c_i32, [c_vp, c_vp, c_vp, FrameDesc, c_vp, c_i32, c_f32, c_i32, c_f32, c_vp, c_vp, c_vp]),
    "pp_validate_job": (c_i32, [ctypes.POINTER(FrameJob)]),
    "pp_batch_run": (c_i32, [c_vp, c_i32, ctypes.POINTER(FrameJob), c_vp]),
    "pp_batch_run_eager": (c_i32, [c_vp, c_i32, ctypes.POINTER(FrameJob), c_vp]),
    "pp_set_tuning": (c_i32, [c_vp, ctypes.POINTER(Tuning)]),
    "pp_get_tuning": (c_i32, [c_vp, ctypes.POINTER(Tuning)]),
    "pp_tuning_space": (c_i32, [ctypes.POINTER(c_i32)] * 4),
    "pp_set_stage_timing": (c_i32, [c_vp, c_i32]),
    "pp_stage_breakdown": (c_i32, [c_vp, ctypes.POINTER(c_f32)]),
    "pp_server_create": (c_i32, [ctypes.POINTER(ServerCfg), ctypes.POINTER(c_vp)]),
    "pp_server_destroy": (c_i32, [c_vp]),
    "pp_server_last_error": (ctypes.c_char_p, [c_vp]),
    "pp_stream_open": (c_i32, [c_vp, c_i32, FrameDesc, Intrinsics, ctypes.POINTER(DiffuseParams),
                               ctypes.POINTER(RansacParams)]),
    "pp_stream_close": (c_i32, [c_vp, c_i32]),
    "pp_submit": (c_i32, [c_vp, c_i32, c_vp, c_u64, ctypes.POINTER(c_u64)]),
    "pp_poll": (c_i32, [c_vp, c_u64, ctypes.POINTER(Result), c_i32]),
    "pp_server_stats_get": (c_i32, [c_vp, ctypes.POINTER(ServerStats)]),
    "pp_server_reset": (c_i32, [c_vp]),
    "pp_stage_time": (c_i32, [c_vp, ctypes.POINTER(c_f32), ctypes.POINTER(c_i32)]),
}

_lib = None


class LibraryMissing(RuntimeError):
    pass


def lib():
    """Load libpp.so (once).  Raises LibraryMissing if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(f"{LIB_PATH} is not built: run `python -m paper_2411_01919_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


# bytes of device scratch pp_ransac_planes_noalloc holds per GPU (PP_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 << 20


def status_string(s: int) -> str:
    return lib().pp_status_string(int(s)).decode()

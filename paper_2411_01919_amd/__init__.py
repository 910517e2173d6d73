"""MI355X-native plane extraction from depth images (arXiv 2411.01919 hot path).

Python binding of libpp.so: marshals torch tensors (device memory) and torch
streams into the C ABI of include/pp.h.  Every step of the path runs in the
library's HIP kernels; this module only checks shapes and passes pointers.

    depth_mm = diffuse(depth_u16, iters=20)                     # Eq. 1 / Alg. 1
    pts, nrm, valid = normals(depth_mm, K)                      # Alg. 2 / Eq. 2
    planes, n, labels = ransac_planes(pts, valid, params)       # Alg. 2 / Eq. 3
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

from . import _native as N
from ._native import (PP_DIFFUSE_EDGE4, PP_DIFFUSE_EDGE8, PP_DIFFUSE_PIXEL, PP_EDGE_EXP,  # noqa: F401
                      PP_EDGE_RATIONAL, PP_SCORE_BF16, PP_SCORE_FP16, PP_SCORE_FP32, PP_SCORE_MFMA_F32,
                      LibraryMissing)

__all__ = [
    "PPError", "Server", "Context", "RansacConfig", "DiffuseConfig", "default_context", "diffuse", "normals",
    "ransac_planes", "ransac_planes_debug", "ransac_regions", "segment", "region_polygons", "DriftMap", "paper_chain", "score_triples", "FrameOutputs", "make_outputs", "batch_run",
    "planes_to_numpy", "PP_DIFFUSE_EDGE4", "PP_DIFFUSE_PIXEL", "PP_DIFFUSE_EDGE8", "PP_SCORE_FP32",
    "PP_SCORE_MFMA_F32", "PP_SCORE_BF16", "PP_SCORE_FP16",
]


class PPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{N.status_string(status)} ({status}): {msg}")
        self.status = status


@dataclass
class DiffuseConfig:
    iters: int = 20
    lam: float = 0.2
    kappa_mm: float = 30.0
    edge_stop: int = PP_EDGE_EXP
    scheme: int = PP_DIFFUSE_EDGE4

    def c(self) -> N.DiffuseParams:
        return N.DiffuseParams(int(self.iters), float(self.lam), float(self.kappa_mm), int(self.edge_stop),
                               int(self.scheme))


@dataclass
class RansacConfig:
    max_planes: int = 12
    hyps: int = 1024
    min_inliers: int = 615
    thresh_m: float = 0.01
    seed: int = 0
    frame_id: int = 0
    precision: int = PP_SCORE_FP32
    recheck_band_m: float = 0.0

    def c(self) -> N.RansacParams:
        return N.RansacParams(int(self.max_planes), int(self.hyps), int(self.min_inliers), float(self.thresh_m),
                              int(self.seed) & 0xFFFFFFFFFFFFFFFF, int(self.frame_id) & 0xFFFFFFFFFFFFFFFF,
                              int(self.precision), float(self.recheck_band_m))


def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream) -> Optional[int]:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _check_dev(t, name: str, dtypes, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype not in dtypes:
        raise ValueError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Context:
    """A pp_ctx on one device (owns the library's scratch memory)."""

    def __init__(self, device: int = 0):
        L = N.lib()
        h = N.c_vp()
        s = L.pp_ctx_create(int(device), ctypes.byref(h))
        if s != N.PP_OK:
            raise PPError(s, L.pp_last_error(None).decode())
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            N.lib().pp_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, s: int):
        if s != N.PP_OK:
            raise PPError(s, N.lib().pp_last_error(self.h).decode())

    def set_tuning(self, diffuse_tile=0, diffuse_t=0, score_hb=0, score_chunk=0):
        t = N.Tuning(diffuse_tile, diffuse_t, score_hb, score_chunk)
        self.check(N.lib().pp_set_tuning(self.h, ctypes.byref(t)))

    def reset_tuning(self):
        self.check(N.lib().pp_set_tuning(self.h, None))

    def set_stage_timing(self, enable: bool):
        self.check(N.lib().pp_set_stage_timing(self.h, 1 if enable else 0))

    def stage_time(self):
        """(summed ms, launches) of the scoring launches of the last run (stream must be synchronised)."""
        ms, n = N.c_f32(), N.c_i32()
        self.check(N.lib().pp_stage_time(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)

    def stage_breakdown(self) -> dict:
        """ms per stage of the last timed eager batch: diffusion, normals (+ valid list), scoring, rest."""
        out = (N.c_f32 * 4)()
        self.check(N.lib().pp_stage_breakdown(self.h, out))
        return dict(diffusion=out[0], normals=out[1], scoring=out[2], ransac_other=out[3])

    def get_tuning(self) -> dict:
        t = N.Tuning()
        self.check(N.lib().pp_get_tuning(self.h, ctypes.byref(t)))
        return dict(diffuse_tile=t.diffuse_tile, diffuse_t=t.diffuse_t, score_hb=t.score_hb, score_chunk=t.score_chunk)


_default = {}


def default_context(device: Optional[int] = None) -> Context:
    torch = _torch()
    if device is None:
        device = torch.cuda.current_device()
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def _desc(H: int, W: int, pitch: Optional[int] = None) -> N.FrameDesc:
    return N.FrameDesc(int(W), int(H), int(pitch if pitch is not None else W))


def diffuse(depth, iters: int = 20, lam: float = 0.2, kappa_mm: float = 30.0, edge_stop: int = PP_EDGE_EXP,
            out=None, ctx: Optional[Context] = None, stream=None, scheme: int = PP_DIFFUSE_EDGE4):
    """Step 1: Perona-Malik diffusion (Eq. 1, Alg. 1) of a [H][W] uint16/int16
    depth tensor in mm -> float32 [H][W] mm (holes stay 0).  scheme picks the
    discretisation: PP_DIFFUSE_EDGE4 (default), PP_DIFFUSE_PIXEL, PP_DIFFUSE_EDGE8."""
    torch = _torch()
    _check_dev(depth, "depth", (torch.uint16, torch.int16))
    H, W = depth.shape
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=depth.device)
    _check_dev(out, "out", (torch.float32,), (H, W))
    ctx = ctx or default_context(depth.device.index)
    p = DiffuseConfig(iters, lam, kappa_mm, edge_stop, scheme).c()
    ctx.check(N.lib().pp_diffuse(ctx.h, _ptr(depth), _ptr(out), _desc(H, W), ctypes.byref(p), _stream(stream)))
    return out


def normals(depth_mm, K, points=None, nrm=None, valid=None, ctx: Optional[Context] = None, stream=None):
    """Steps 2-3: back-projection and Sobel normals (Alg. 2, Eq. 2, Alg. 1).
    K = (fx, fy, cx, cy).  Returns (points [3][H][W] m, normals [3][H][W], valid u8)."""
    torch = _torch()
    _check_dev(depth_mm, "depth_mm", (torch.float32,))
    H, W = depth_mm.shape
    dev = depth_mm.device
    points = points if points is not None else torch.empty((3, H, W), dtype=torch.float32, device=dev)
    nrm = nrm if nrm is not None else torch.empty((3, H, W), dtype=torch.float32, device=dev)
    valid = valid if valid is not None else torch.empty((H, W), dtype=torch.uint8, device=dev)
    _check_dev(points, "points", (torch.float32,), (3, H, W))
    _check_dev(nrm, "normals", (torch.float32,), (3, H, W))
    _check_dev(valid, "valid", (torch.uint8,), (H, W))
    ctx = ctx or default_context(dev.index)
    Kc = N.Intrinsics(*[float(x) for x in K])
    ctx.check(N.lib().pp_normals(ctx.h, _ptr(depth_mm), _desc(H, W), Kc, _ptr(points), _ptr(nrm), _ptr(valid),
                                 _stream(stream)))
    return points, nrm, valid


PLANE_BYTES = ctypes.sizeof(N.Plane)


def planes_to_numpy(planes_u8, n: int):
    """Decode a byte tensor of pp_plane records into numpy: (n, d, centroid, inliers, hyp_index)."""
    import numpy as np
    raw = planes_u8.detach().cpu().numpy().tobytes()
    recs = (N.Plane * (len(raw) // PLANE_BYTES)).from_buffer_copy(raw)
    out = []
    for i in range(n):
        r = recs[i]
        out.append(dict(n=np.array(r.n[:]), d=r.d, centroid=np.array(r.centroid[:]), inliers=r.inliers,
                        hyp_index=r.hyp_index))
    return out


def _ransac_outputs(H, W, cfg: RansacConfig, dev):
    torch = _torch()
    planes = torch.zeros((cfg.max_planes * PLANE_BYTES,), dtype=torch.uint8, device=dev)
    n = torch.zeros((1,), dtype=torch.int32, device=dev)
    labels = torch.empty((H, W), dtype=torch.int8, device=dev)
    return planes, n, labels


def ransac_planes(points, valid, cfg: RansacConfig, planes=None, n_planes=None, labels=None,
                  ctx: Optional[Context] = None, stream=None):
    """Step 4: sequential RANSAC (Alg. 2, Eq. 3).  Returns (planes as pp_plane
    bytes [max_planes*64] u8, n_planes int32 [1], labels int8 [H][W])."""
    torch = _torch()
    _check_dev(points, "points", (torch.float32,))
    _, H, W = points.shape
    _check_dev(valid, "valid", (torch.uint8,), (H, W))
    dev = points.device
    if planes is None:
        planes, n_planes, labels = _ransac_outputs(H, W, cfg, dev)
    ctx = ctx or default_context(dev.index)
    p = cfg.c()
    ctx.check(N.lib().pp_ransac_planes(ctx.h, _ptr(points), _ptr(valid), None, _desc(H, W), ctypes.byref(p),
                                       _ptr(planes), _ptr(n_planes), _ptr(labels), _stream(stream)))
    return planes, n_planes, labels


def ransac_planes_noalloc(points, valid, cfg: RansacConfig, planes, n_planes, labels, stream=None):
    """Step 4 through pp_ransac_planes_noalloc: the same sequential RANSAC on
    the library's static per-GPU scratch, with no context and no device
    allocation (the caller passes every output).  Runs on the current device
    with the default tuning; calls that overlap on one GPU race."""
    torch = _torch()
    _check_dev(points, "points", (torch.float32,))
    _, H, W = points.shape
    _check_dev(valid, "valid", (torch.uint8,), (H, W))
    _check_dev(labels, "labels", (torch.int8,), (H, W))
    if planes.dtype != torch.uint8 or planes.numel() < cfg.max_planes * PLANE_BYTES or n_planes.numel() < 1:
        raise ValueError("planes must be uint8 [max_planes*64] and n_planes int32 [1]")
    p = cfg.c()
    s = N.lib().pp_ransac_planes_noalloc(_ptr(points), _ptr(valid), _desc(H, W), ctypes.byref(p), _ptr(planes),
                                          _ptr(n_planes), _ptr(labels), _stream(stream))
    if s != N.PP_OK:
        raise PPError(s, N.lib().pp_last_error(None).decode())
    return planes, n_planes, labels


def ransac_planes_debug(points, valid, cfg: RansacConfig, ctx: Optional[Context] = None, stream=None):
    """ransac_planes plus per-round introspection (hypotheses, triples,
    counts, round info, S/F masks, valid list, the tile scorer's decided
    pairs and evaluated residuals)."""
    torch = _torch()
    _, H, W = points.shape
    dev = points.device
    R, Hy = cfg.max_planes, cfg.hyps
    planes, n_planes, labels = _ransac_outputs(H, W, cfg, dev)
    dbg_t = dict(
        counts=torch.zeros((R, Hy), dtype=torch.int32, device=dev),
        hyps=torch.zeros((R, Hy, 4), dtype=torch.float32, device=dev),
        triples=torch.full((R, Hy, 3), -2, dtype=torch.int32, device=dev),
        round_info=torch.zeros((R, 4), dtype=torch.int32, device=dev),
        masks=torch.zeros((R, H * W), dtype=torch.uint8, device=dev),
        valid_list=torch.zeros((H * W,), dtype=torch.int32, device=dev),
        n_valid=torch.zeros((1,), dtype=torch.int32, device=dev),
        scored=torch.zeros((3,), dtype=torch.int64, device=dev),
    )
    dbg = N.RansacDebug(*[_ptr(dbg_t[k]) for k in ("counts", "hyps", "triples", "round_info", "masks",
                                                      "valid_list", "n_valid", "scored")])
    ctx = ctx or default_context(dev.index)
    p = cfg.c()
    ctx.check(N.lib().pp_ransac_planes_dbg(ctx.h, _ptr(points), _ptr(valid), _desc(H, W), ctypes.byref(p),
                                           _ptr(planes), _ptr(n_planes), _ptr(labels), ctypes.byref(dbg),
                                           _stream(stream)))
    return planes, n_planes, labels, dbg_t


def segment(normals, valid, low: float = 0.35, high: float = 0.7, min_area: Optional[int] = None,
            max_regions: int = 127, region=None, n_regions=None, edges: bool = False,
            ctx: Optional[Context] = None, stream=None):
    """Canny edges on the normal image and the regions between them (Sec.
    III-D).  normals float32 [3][H][W], valid uint8 [H][W] (bit1: normal
    valid).  Returns (region int16 [H][W], n_regions int32 [1]) and the edge
    map uint8 [H][W] when edges=True.  min_area defaults to max(50,
    ceil(0.002 W H))."""
    torch = _torch()
    _check_dev(normals, "normals", (torch.float32,))
    _, H, W = normals.shape
    _check_dev(valid, "valid", (torch.uint8,), (H, W))
    dev = normals.device
    if min_area is None:
        min_area = max(50, -(-2 * W * H // 1000))
    if region is None:
        region = torch.empty((H, W), dtype=torch.int16, device=dev)
    if n_regions is None:
        n_regions = torch.zeros((1,), dtype=torch.int32, device=dev)
    e = torch.empty((H, W), dtype=torch.uint8, device=dev) if edges else None
    ctx = ctx or default_context(dev.index)
    prm = N.SegmentParams(float(low), float(high), int(min_area), int(max_regions))
    ctx.check(N.lib().pp_segment(ctx.h, _ptr(normals), _ptr(valid), _desc(H, W), ctypes.byref(prm), _ptr(region),
                                 _ptr(n_regions), _ptr(e), _stream(stream)))
    return (region, n_regions, e) if edges else (region, n_regions)


def region_polygons(region, n_regions: int, eps_px: float = 1.5):
    """Contours of regions 0..n_regions-1 of a label image (host numpy int16
    [H][W] or a device tensor, copied to the host) simplified into polygons:
    a list of int32 [k][2] (x, y) vertex arrays, clockwise from each region's
    first pixel."""
    import numpy as np
    if hasattr(region, "detach"):
        region = region.detach().cpu().numpy()
    reg = np.ascontiguousarray(region, dtype=np.int16)
    H, W = reg.shape
    off = np.zeros(n_regions + 1, np.int32)
    L = N.lib()
    xy = np.zeros((16384, 2), np.int32)
    st = L.pp_region_polygons(reg.ctypes.data, _desc(H, W), int(n_regions), float(eps_px), xy.ctypes.data, len(xy),
                              off.ctypes.data)
    if st == N.PP_E_NOMEM:  # more vertices than the first buffer holds: again with the exact size
        xy = np.zeros((int(off[-1]), 2), np.int32)
        st = L.pp_region_polygons(reg.ctypes.data, _desc(H, W), int(n_regions), float(eps_px), xy.ctypes.data,
                                  len(xy), off.ctypes.data)
    if st != N.PP_OK:
        raise PPError(st, "pp_region_polygons")
    return [xy[off[g]:off[g + 1]].copy() for g in range(n_regions)]


class DriftMap:
    """The polygon map with vertical drift compensation (Sec. III-E, Eqs.
    4-10), host code behind the C ABI.  integrate() takes the intrinsics, the
    odometry pose (R world<-camera, camera centre) and the frame's polygons
    as (n[3], d, centroid[3], support, xy_px int32 [k][2]) in the camera frame."""

    def __init__(self, drift_tolerance_m: float = 0.05, sigma_p: float = 1e-5, sigma_m: float = 1e-4,
                 max_tilt_deg: float = 15.0):
        self._lib = N.lib()
        h = ctypes.c_void_p()
        st = self._lib.pp_map_create(ctypes.byref(N.MapParams(drift_tolerance_m, sigma_p, sigma_m, max_tilt_deg)),
                                     ctypes.byref(h))
        if st != N.PP_OK:
            raise PPError(st, "pp_map_create")
        self.h = h.value

    def integrate(self, K, R, C, polygons):
        import numpy as np
        keep = []
        obs = (N.MapObservation * max(1, len(polygons)))()
        for i, (n, d, cen, sup, xy) in enumerate(polygons):
            xy = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)
            keep.append(xy)
            obs[i].n[:] = [float(v) for v in n]
            obs[i].d = float(d)
            obs[i].centroid[:] = [float(v) for v in cen]
            obs[i].support = int(sup)
            obs[i].n_vertices = len(xy)
            obs[i].xy_px = xy.ctypes.data
        Rm = np.ascontiguousarray(R, dtype=np.float64).reshape(9)
        Cm = np.ascontiguousarray(C, dtype=np.float64).reshape(3)
        match = np.zeros(max(1, len(polygons)), np.int32)
        res = N.MapFrameResult()
        st = self._lib.pp_map_integrate(self.h, N.Intrinsics(*[float(v) for v in K]), Rm.ctypes.data, Cm.ctypes.data,
                                        obs, len(polygons), match.ctypes.data, ctypes.byref(res))
        if st != N.PP_OK:
            raise PPError(st, "pp_map_integrate")
        return dict(matched=res.matched, added=res.added, skipped=res.skipped, measurement=res.measurement,
                    drift=res.drift, variance=res.variance, match_of=match[:len(polygons)].tolist())

    def polygons(self):
        import numpy as np
        n = ctypes.c_int32()
        self._lib.pp_map_size(self.h, ctypes.byref(n))
        out = []
        for i in range(n.value):
            info = N.MapPolygonInfo()
            self._lib.pp_map_polygon(self.h, i, ctypes.byref(info), None, 0)
            xy = np.zeros((max(1, info.n_vertices), 2))
            st = self._lib.pp_map_polygon(self.h, i, ctypes.byref(info), xy.ctypes.data, info.n_vertices)
            if st != N.PP_OK:
                raise PPError(st, "pp_map_polygon")
            out.append(dict(height=info.height, support=info.support, hull=xy[:info.n_vertices].copy()))
        return out

    def close(self):
        if getattr(self, "h", None):
            self._lib.pp_map_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def paper_chain(depth, K, drift_map: Optional["DriftMap"] = None, pose=None, diffuse_cfg: Optional[DiffuseConfig] = None,
                low: float = 0.35, high: float = 0.7, min_area: Optional[int] = None, hyps: int = 10,
                thresh_m: float = 0.01, seed: int = 0, frame_id: int = 0, eps_px: float = 1.5,
                ctx: Optional[Context] = None, stream=None, times: Optional[dict] = None):
    """The paper's per-frame chain through the library: diffusion, normals,
    segmentation and region-mode RANSAC on the GPU, then (on the host) the
    region polygons and, with a map and a pose (R world<-camera, camera
    centre), the drift-compensated map update.  Returns a dict with the
    device outputs, the stored planes and polygons, and the map result.  With
    `times`, per-stage milliseconds are accumulated into it (device stages by
    events on the stream, host stages by the host clock)."""
    import time
    torch = _torch()
    dc = diffuse_cfg or DiffuseConfig()
    H, W = depth.shape
    st = torch.cuda.current_stream() if stream is None else stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)] if times is not None else None
    if ev:
        ev[0].record(st)
    dmm = diffuse(depth, dc.iters, dc.lam, dc.kappa_mm, dc.edge_stop, ctx=ctx, stream=stream, scheme=dc.scheme)
    if ev:
        ev[1].record(st)
    pts, nrm, valid = normals(dmm, K, ctx=ctx, stream=stream)
    if ev:
        ev[2].record(st)
    region, n_reg = segment(nrm, valid, low, high, min_area, 127, ctx=ctx, stream=stream)
    if ev:
        ev[3].record(st)
    cfg = RansacConfig(max_planes=127, hyps=hyps, min_inliers=1, thresh_m=thresh_m, seed=seed, frame_id=frame_id)
    planes, n_planes, labels = ransac_regions(pts, valid, region, cfg, ctx=ctx, stream=stream)
    if ev:
        ev[4].record(st)
    st.synchronize()
    t0 = time.perf_counter()
    nr = int(n_reg.cpu().item())
    recs = planes_to_numpy(planes, 127)
    polys = region_polygons(region, nr, eps_px)
    stored = [g for g in range(nr) if recs[g]["hyp_index"] >= 0]
    t1 = time.perf_counter()
    mres = None
    if drift_map is not None and pose is not None:
        obs = [(recs[g]["n"], recs[g]["d"], recs[g]["centroid"], recs[g]["inliers"], polys[g]) for g in stored]
        mres = drift_map.integrate(K, pose[0], pose[1], obs)
    t2 = time.perf_counter()
    if times is not None:
        for name, a, b in (("diffusion", 0, 1), ("normals", 1, 2), ("segmentation", 2, 3), ("region_ransac", 3, 4)):
            times[name] = times.get(name, 0.0) + ev[a].elapsed_time(ev[b])
        times["polygons_host"] = times.get("polygons_host", 0.0) + (t1 - t0) * 1e3
        times["map_host"] = times.get("map_host", 0.0) + (t2 - t1) * 1e3
    return dict(depth_mm=dmm, points=pts, normals=nrm, valid=valid, region=region, n_regions=nr, labels=labels,
                planes={g: recs[g] for g in stored}, polygons=polys, map=mres)


def ransac_regions(points, valid, region, cfg: RansacConfig, planes=None, n_planes=None, labels=None,
                   ctx: Optional[Context] = None, stream=None, debug: bool = False):
    """Region-mode RANSAC (Alg. 2 as printed) over the regions 0..max_planes-1
    of an int16 [H][W] label image: per region the hypothesis with the
    smallest summed distance, stored iff more than 90 % of the region's points
    are its inliers.  Returns (planes bytes [max_planes*64], n_planes, labels)
    and, with debug=True, a dict of per-hypothesis tensors as well."""
    torch = _torch()
    _check_dev(points, "points", (torch.float32,))
    _, H, W = points.shape
    _check_dev(valid, "valid", (torch.uint8,), (H, W))
    _check_dev(region, "region", (torch.int16,), (H, W))
    dev = points.device
    if planes is None:
        planes, n_planes, labels = _ransac_outputs(H, W, cfg, dev)
    ctx = ctx or default_context(dev.index)
    p = cfg.c()
    if not debug:
        ctx.check(N.lib().pp_ransac_planes(ctx.h, _ptr(points), _ptr(valid), _ptr(region), _desc(H, W),
                                           ctypes.byref(p), _ptr(planes), _ptr(n_planes), _ptr(labels),
                                           _stream(stream)))
        return planes, n_planes, labels
    R, Hy = cfg.max_planes, cfg.hyps
    dbg_t = dict(
        npts=torch.zeros((R,), dtype=torch.int32, device=dev),
        triples=torch.full((R, Hy, 3), -2, dtype=torch.int32, device=dev),
        hyps=torch.zeros((R, Hy, 4), dtype=torch.float32, device=dev),
        errors=torch.zeros((R, Hy), dtype=torch.float64, device=dev),
        counts=torch.zeros((R, Hy), dtype=torch.int32, device=dev),
        jstar=torch.zeros((R,), dtype=torch.int32, device=dev),
    )
    dbg = N.RegionDebug(*[_ptr(dbg_t[k]) for k in ("npts", "triples", "hyps", "errors", "counts", "jstar")])
    ctx.check(N.lib().pp_ransac_regions_dbg(ctx.h, _ptr(points), _ptr(valid), _ptr(region), _desc(H, W),
                                            ctypes.byref(p), _ptr(planes), _ptr(n_planes), _ptr(labels),
                                            ctypes.byref(dbg), _stream(stream)))
    return planes, n_planes, labels, dbg_t


def score_triples(points, valid, triples, thresh_m: float, precision: int = PP_SCORE_FP32,
                  recheck_band_m: float = 0.0, ctx: Optional[Context] = None, stream=None):
    """Inlier counts of caller-given triples of pixel offsets over every
    depth-valid point -> (planes float32 [n][4], counts int32 [n])."""
    torch = _torch()
    _, H, W = points.shape
    _check_dev(triples, "triples", (torch.int32,))
    n = triples.shape[0]
    dev = points.device
    planes = torch.empty((n, 4), dtype=torch.float32, device=dev)
    counts = torch.empty((n,), dtype=torch.int32, device=dev)
    ctx = ctx or default_context(dev.index)
    ctx.check(N.lib().pp_debug_score_triples(ctx.h, _ptr(points), _ptr(valid), _desc(H, W), _ptr(triples), int(n),
                                             float(thresh_m), int(precision), float(recheck_band_m), _ptr(planes),
                                             _ptr(counts), _stream(stream)))
    return planes, counts


@dataclass
class FrameOutputs:
    """Device buffers of one frame's results (allocated once, reused)."""
    depth: object        # uint16/int16 [H][W] input
    depth_mm: object     # float32 [H][W]
    points: object       # float32 [3][H][W]
    normals: object      # float32 [3][H][W]
    valid: object        # uint8 [H][W]
    planes: object       # uint8 [max_planes * 64]
    n_planes: object     # int32 [1]
    labels: object       # int8 [H][W]
    K: Tuple[float, float, float, float]
    diffuse: DiffuseConfig
    ransac: RansacConfig

    def job(self) -> N.FrameJob:
        H, W = self.depth.shape
        return N.FrameJob(_ptr(self.depth), _desc(H, W), N.Intrinsics(*[float(x) for x in self.K]), self.diffuse.c(),
                          self.ransac.c(), _ptr(self.depth_mm), _ptr(self.points), _ptr(self.normals),
                          _ptr(self.valid), _ptr(self.planes), _ptr(self.n_planes), _ptr(self.labels))


def make_outputs(depth, K, diffuse_cfg: DiffuseConfig, ransac_cfg: RansacConfig) -> FrameOutputs:
    torch = _torch()
    _check_dev(depth, "depth", (torch.uint16, torch.int16))
    H, W = depth.shape
    dev = depth.device
    planes, n, labels = _ransac_outputs(H, W, ransac_cfg, dev)
    return FrameOutputs(depth, torch.empty((H, W), dtype=torch.float32, device=dev),
                        torch.empty((3, H, W), dtype=torch.float32, device=dev),
                        torch.empty((3, H, W), dtype=torch.float32, device=dev),
                        torch.empty((H, W), dtype=torch.uint8, device=dev), planes, n, labels, tuple(K),
                        diffuse_cfg, ransac_cfg)


def batch_run(frames: Sequence[FrameOutputs], graph: bool = True, ctx: Optional[Context] = None, stream=None):
    """Run a ragged batch of frames through all four steps in one launch per
    stage (captured once per batch layout into a HIP graph when graph=True)."""
    if not frames:
        return
    jobs = (N.FrameJob * len(frames))(*[f.job() for f in frames])
    ctx = ctx or default_context(frames[0].depth.device.index)
    fn = N.lib().pp_batch_run if graph else N.lib().pp_batch_run_eager
    ctx.check(fn(ctx.h, len(frames), jobs, _stream(stream)))


def run_frame(fo: FrameOutputs, ctx: Optional[Context] = None, stream=None):
    """The plain per-frame path: pp_diffuse, pp_normals, pp_ransac_planes on one stream."""
    H, W = fo.depth.shape
    diffuse(fo.depth, fo.diffuse.iters, fo.diffuse.lam, fo.diffuse.kappa_mm, fo.diffuse.edge_stop, out=fo.depth_mm,
            ctx=ctx, stream=stream, scheme=fo.diffuse.scheme)
    normals(fo.depth_mm, fo.K, fo.points, fo.normals, fo.valid, ctx=ctx, stream=stream)
    ransac_planes(fo.points, fo.valid, fo.ransac, fo.planes, fo.n_planes, fo.labels, ctx=ctx, stream=stream)


class Server:
    """The serving runtime (pp_server_*): camera streams submit host frames,
    results come back through poll().  dry_run_us > 0 exercises admission and
    scheduling without touching a GPU (no planes are computed)."""

    def __init__(self, hbm_budget_bytes: int = 8 << 30, max_batch: int = 32, lanes: int = 4,
                 staging_frames: int = 64, use_graphs: bool = True, device: int = 0, dry_run_us: int = 0,
                 dry_run_fail_batch: int = 0):
        cfg = N.ServerCfg(int(device), int(hbm_budget_bytes), int(max_batch), int(lanes), int(staging_frames),
                          1 if use_graphs else 0, int(dry_run_us), int(dry_run_fail_batch))
        h = N.c_vp()
        s = N.lib().pp_server_create(ctypes.byref(cfg), ctypes.byref(h))
        if s != N.PP_OK:
            raise PPError(s, "pp_server_create")
        self.h = h
        self.streams = {}

    def close(self):
        if self.h:
            N.lib().pp_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, s):
        if s != N.PP_OK:
            raise PPError(s, N.lib().pp_server_last_error(self.h).decode())

    def open_stream(self, stream_id: int, W: int, H: int, K, diffuse_cfg: DiffuseConfig, ransac_cfg: RansacConfig):
        dp, rp = diffuse_cfg.c(), ransac_cfg.c()
        self._check(N.lib().pp_stream_open(self.h, int(stream_id), _desc(H, W), N.Intrinsics(*[float(x) for x in K]),
                                           ctypes.byref(dp), ctypes.byref(rp)))
        self.streams[stream_id] = (W, H, ransac_cfg.max_planes)

    def reset(self):
        """pp_server_reset: fail every frame not yet completed and accept work again."""
        self._check(N.lib().pp_server_reset(self.h))

    def close_stream(self, stream_id: int):
        self._check(N.lib().pp_stream_close(self.h, int(stream_id)))

    def submit(self, stream_id: int, depth_u16, frame_id: int) -> int:
        """Queue a host uint16 [H][W] frame; returns a ticket.  Raises PPError
        (status PP_E_AGAIN) when the stream's staging is full."""
        import numpy as np
        a = np.ascontiguousarray(depth_u16, dtype=np.uint16)
        W, H, _ = self.streams[stream_id]
        if a.shape != (H, W):
            raise ValueError(f"frame shape {a.shape} != {(H, W)}")
        t = N.c_u64()
        self._check(N.lib().pp_submit(self.h, int(stream_id), a.ctypes.data, int(frame_id), ctypes.byref(t)))
        return t.value

    def try_submit(self, stream_id: int, depth_u16, frame_id: int):
        """submit() that returns None instead of raising when staging is full."""
        try:
            return self.submit(stream_id, depth_u16, frame_id)
        except PPError as e:
            if e.status == N.PP_E_AGAIN:
                return None
            raise

    def poll(self, ticket: int, stream_id: int, timeout_us: int = 0, labels: bool = True):
        """None while pending; else dict(n_planes, planes (raw bytes), labels, latency_us, frame_id)."""
        import numpy as np
        W, H, mp = self.streams[stream_id]
        planes = (N.Plane * mp)()
        n = N.c_i32()
        lab = np.empty((H, W), dtype=np.int8) if labels else None
        res = N.Result(ctypes.addressof(planes), ctypes.addressof(n), lab.ctypes.data if labels else None, 0, 0, 0.0)
        s = N.lib().pp_poll(self.h, int(ticket), ctypes.byref(res), int(timeout_us))
        if s == N.PP_PENDING:
            return None
        self._check(s)
        return dict(n_planes=n.value, planes=bytes(planes), labels=lab, latency_us=res.latency_us,
                    frame_id=res.frame_id, stream_id=res.stream_id)

    def stats(self) -> dict:
        st = N.ServerStats()
        self._check(N.lib().pp_server_stats_get(self.h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in N.ServerStats._fields_}

"""CPU FP64 oracle of the plane-extraction path (ctypes binding of ``orc.c``).

TEST INFRASTRUCTURE ONLY.  The slow, plain reference the GPU library is
checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product package never
does, and this module imports nothing from the product package.

Functions take and return numpy arrays; each cites the passage of
arXiv 2411.01919 it follows (see ``orc.c`` for the readings taken).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("ORC_LIB") or os.path.join(_HERE, "liborc.so")
_SRC = os.environ.get("ORC_SRC") or os.path.join(_HERE, "orc.c")


def build(force: bool = True) -> str:
    """Compile ``orc.c`` into ``liborc.so`` with gcc (OpenMP, IEEE float64, no contraction)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", _SRC, "-o", LIB_PATH + ".tmp", "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i, d = ctypes.c_int, ctypes.c_double
        L.orc_philox4x64_10.argtypes = [P, P, P]
        L.orc_diffuse.argtypes = [P, i, i, i, d, d, i, P]
        L.orc_diffuse_variant.argtypes = [P, i, i, i, d, d, i, i, P]
        L.orc_backproject.argtypes = [P, i, i, d, d, d, d, P, P]
        f = ctypes.c_float
        L.orc_seg_grad.argtypes = [P, P, i, i, P, P, P]
        L.orc_seg_edges.argtypes = [P, P, P, i, i, f, f, P, P]
        L.orc_seg_regions.argtypes = [P, i, i, i, i, P]
        L.orc_segment.argtypes = [P, P, i, i, f, f, i, i, P, P]
        L.orc_region_polygons.argtypes = [P, i, i, i, d, P, i, P]
        L.orc_ransac_regions.argtypes = [P, P, P, i, i, i, P, P, P, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_normals.argtypes = [P, P, i, i, P, P, P, P]
        L.orc_valid_list.argtypes = [P, i, P]
        L.orc_valid_list.restype = i
        L.orc_hypotheses.argtypes = [P, i, i, P, i, P, P, i, P, P, P]
        L.orc_score.argtypes = [P, i, i, P, i, P, P, P, i, d, P, P, P, P, P]
        L.orc_refit.argtypes = [P, i, i, P, i, P, P]
        L.orc_refit.restype = i
        L.orc_eig3.argtypes = [P, P, P]
        L.orc_ransac_round.argtypes = [P, i, i, P, i, P, P, i, P, P, P, P, P, P, P, P, P, P]
        L.orc_ransac.argtypes = [P, P, i, i, P, P, P, P, P, P, P]
        L.orc_ransac.restype = i
        L.orc_num_threads.restype = i
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class _Params(ctypes.Structure):
    _fields_ = [("hyps", ctypes.c_int), ("max_planes", ctypes.c_int), ("min_inliers", ctypes.c_int),
                ("thresh", ctypes.c_double), ("seed", ctypes.c_uint64), ("frame", ctypes.c_uint64)]


class _RoundResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("jstar", ctypes.c_int), ("n_remaining", ctypes.c_int),
                ("s_count", ctypes.c_int), ("f_count", ctypes.c_int),
                ("hyp_plane", ctypes.c_double * 4), ("plane", ctypes.c_double * 4),
                ("centroid", ctypes.c_double * 3)]


@dataclass
class RansacParams:
    hyps: int = 256
    max_planes: int = 12
    min_inliers: int = 50
    thresh: float = 0.01
    seed: int = 0
    frame: int = 0

    def _c(self):
        return _Params(self.hyps, self.max_planes, self.min_inliers, self.thresh,
                       self.seed & 0xFFFFFFFFFFFFFFFF, self.frame & 0xFFFFFFFFFFFFFFFF)


def num_threads() -> int:
    return lib().orc_num_threads()


def philox4x64_10(ctr, key) -> np.ndarray:
    """Philox4x64-10 block for counter (4 words) and key (2 words)."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint64))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint64))
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_p(c), _p(k), _p(out))
    return out


def diffuse(depth: np.ndarray, iters: int, lam: float = 0.2, kappa: float = 30.0, edge_stop: int = 0) -> np.ndarray:
    """Eq. 1 / Alg. 1 explicit Perona-Malik diffusion of a depth image in mm
    (uint16 frames or real-valued images; a pixel is a hole iff it is not > 0) -> float64 mm."""
    d = np.ascontiguousarray(depth, dtype=np.float64)
    H, W = d.shape
    out = np.zeros((H, W), dtype=np.float64)
    lib().orc_diffuse(_p(d), W, H, int(iters), float(lam), float(kappa), int(edge_stop), _p(out))
    return out


def diffuse_variant(depth: np.ndarray, iters: int, lam: float, kappa: float, scheme: int, edge_stop: int = 0):
    """Diffusion variants: scheme 1 = Alg. 1 as printed (pixel-centred c_p lap I),
    scheme 2 = 8-neighbour per-edge flux."""
    d = np.ascontiguousarray(depth, dtype=np.float64)
    H, W = d.shape
    out = np.zeros((H, W), dtype=np.float64)
    lib().orc_diffuse_variant(_p(d), W, H, int(iters), float(lam), float(kappa), int(edge_stop), int(scheme), _p(out))
    return out


def backproject(depth_mm: np.ndarray, K) -> tuple:
    """Back-projection with intrinsics K (Alg. 2): -> (P [3][H][W] m, valid [H][W] uint8)."""
    d = np.ascontiguousarray(depth_mm, dtype=np.float64)
    H, W = d.shape
    P = np.zeros((3, H, W))
    valid = np.zeros((H, W), dtype=np.uint8)
    lib().orc_backproject(_p(d), W, H, K.fx, K.fy, K.cx, K.cy, _p(P), _p(valid))
    return P, valid


def normals(P: np.ndarray, valid: np.ndarray, with_grad: bool = False):
    """Eq. 2 / Alg. 1 normal image: -> (N [3][H][W], nvalid [H][W]) (+ Gx, Gy)."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    v = np.ascontiguousarray(valid, dtype=np.uint8)
    _, H, W = P.shape
    N = np.zeros_like(P)
    nv = np.zeros((H, W), dtype=np.uint8)
    gx = np.zeros_like(P) if with_grad else None
    gy = np.zeros_like(P) if with_grad else None
    lib().orc_normals(_p(P), _p(v), W, H, _p(N), _p(nv), _p(gx), _p(gy))
    return (N, nv, gx, gy) if with_grad else (N, nv)


def valid_list(valid: np.ndarray) -> np.ndarray:
    v = np.ascontiguousarray(valid, dtype=np.uint8).reshape(-1)
    L = np.zeros(v.size, dtype=np.int32)
    m = lib().orc_valid_list(_p(v), v.size, _p(L))
    return L[:m].copy()


def hypotheses(P, L, assigned, prm: RansacParams, r: int):
    """Round-r hypotheses (Alg. 2): -> (triples [h][3] L-positions, planes [h][4], hvalid [h])."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    _, H, W = P.shape
    L = np.ascontiguousarray(L, dtype=np.int32)
    a = np.ascontiguousarray(assigned, dtype=np.uint8).reshape(-1)
    tr = np.zeros((prm.hyps, 3), dtype=np.int32)
    pl = np.zeros((prm.hyps, 4))
    hv = np.zeros(prm.hyps, dtype=np.uint8)
    c = prm._c()
    lib().orc_hypotheses(_p(P), W, H, _p(L), len(L), _p(a), ctypes.byref(c), int(r), _p(tr), _p(pl), _p(hv))
    return tr, pl, hv


def score(P, L, assigned, planes, hvalid, thresh: float, eps: Optional[np.ndarray] = None):
    """Inlier counts (Alg. 2, Eq. 3) -> counts (and counts_lo, counts_hi, pmax when eps is given)."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    _, H, W = P.shape
    L = np.ascontiguousarray(L, dtype=np.int32)
    a = np.ascontiguousarray(assigned, dtype=np.uint8).reshape(-1)
    pl = np.ascontiguousarray(planes, dtype=np.float64)
    hv = np.ascontiguousarray(hvalid, dtype=np.uint8)
    nh = len(hv)
    c = np.zeros(nh, dtype=np.int32)
    lo = hi = None
    e = None
    if eps is not None:
        e = np.ascontiguousarray(eps, dtype=np.float64)
        lo = np.zeros(nh, dtype=np.int32)
        hi = np.zeros(nh, dtype=np.int32)
    pmax = np.zeros(1)
    lib().orc_score(_p(P), W, H, _p(L), len(L), _p(a), _p(pl), _p(hv), nh, float(thresh), _p(e),
                    _p(c), _p(lo), _p(hi), _p(pmax))
    if eps is None:
        return c
    return c, lo, hi, float(pmax[0])


def refit(P, idx) -> tuple:
    """Least-squares plane of P[idx] -> (plane (n, d) with d >= 0, centroid)."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    _, H, W = P.shape
    ix = np.ascontiguousarray(idx, dtype=np.int32)
    pl = np.zeros(4)
    ce = np.zeros(3)
    lib().orc_refit(_p(P), W, H, _p(ix), len(ix), _p(pl), _p(ce))
    return pl, ce


def eig3(A) -> tuple:
    A = np.ascontiguousarray(A, dtype=np.float64).reshape(9)
    w = np.zeros(3)
    V = np.zeros(9)
    lib().orc_eig3(_p(A), _p(w), _p(V))
    return w, V.reshape(3, 3)


@dataclass
class RoundResult:
    status: int
    jstar: int
    n_remaining: int
    s_count: int
    f_count: int
    hyp_plane: np.ndarray
    plane: np.ndarray
    centroid: np.ndarray
    triples: np.ndarray
    planes: np.ndarray
    hvalid: np.ndarray
    counts: np.ndarray
    counts_lo: Optional[np.ndarray]
    counts_hi: Optional[np.ndarray]
    smask: np.ndarray
    fmask: np.ndarray


def ransac_round(P, L, assigned, prm: RansacParams, r: int, eps: Optional[np.ndarray] = None) -> RoundResult:
    """One round of sequential RANSAC given the assignment state (follow mode)."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    _, H, W = P.shape
    L = np.ascontiguousarray(L, dtype=np.int32)
    a = np.ascontiguousarray(assigned, dtype=np.uint8).reshape(-1)
    nh = prm.hyps
    tr = np.zeros((nh, 3), dtype=np.int32)
    pl = np.zeros((nh, 4))
    hv = np.zeros(nh, dtype=np.uint8)
    ct = np.zeros(nh, dtype=np.int32)
    lo = hi = e = None
    if eps is not None:
        e = np.ascontiguousarray(eps, dtype=np.float64)
        lo = np.zeros(nh, dtype=np.int32)
        hi = np.zeros(nh, dtype=np.int32)
    sm = np.zeros((H, W), dtype=np.uint8)
    fm = np.zeros((H, W), dtype=np.uint8)
    rr = _RoundResult()
    c = prm._c()
    lib().orc_ransac_round(_p(P), W, H, _p(L), len(L), _p(a), ctypes.byref(c), int(r), _p(e),
                           _p(tr), _p(pl), _p(hv), _p(ct), _p(lo), _p(hi), _p(sm), _p(fm), ctypes.byref(rr))
    return RoundResult(rr.status, rr.jstar, rr.n_remaining, rr.s_count, rr.f_count,
                       np.array(rr.hyp_plane[:]), np.array(rr.plane[:]), np.array(rr.centroid[:]),
                       tr, pl, hv, ct, lo, hi, sm.astype(bool), fm.astype(bool))


@dataclass
class RansacResult:
    n_planes: int
    planes: np.ndarray      # [n][4]
    centroids: np.ndarray   # [n][3]
    inliers: np.ndarray     # [n]
    jstar: np.ndarray       # [n]
    labels: np.ndarray      # int8 [H][W]
    residuals: float        # sum_r |R_r| * hyps


def ransac(P, valid, prm: RansacParams) -> RansacResult:
    """Whole-frame sequential RANSAC (Alg. 2 with the hot-path readings)."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    _, H, W = P.shape
    v = np.ascontiguousarray(valid, dtype=np.uint8)
    labels = np.zeros((H, W), dtype=np.int8)
    mp = prm.max_planes
    pl = np.zeros((mp, 4))
    ce = np.zeros((mp, 3))
    inl = np.zeros(mp, dtype=np.int32)
    js = np.zeros(mp, dtype=np.int32)
    res = np.zeros(1)
    c = prm._c()
    n = lib().orc_ransac(_p(P), _p(v), W, H, ctypes.byref(c), _p(labels), _p(pl), _p(ce), _p(inl), _p(js), _p(res))
    return RansacResult(n, pl[:n].copy(), ce[:n].copy(), inl[:n].copy(), js[:n].copy(), labels, float(res[0]))


@dataclass
class RegionResult:
    n_stored: int
    npts: np.ndarray        # [R]
    triples: np.ndarray     # [R][hyps][3] positions in the region's row-major list
    planes: np.ndarray      # [R][hyps][4]
    hvalid: np.ndarray      # [R][hyps]
    errors: np.ndarray      # [R][hyps] sum |r| (inf without a plane)
    counts: np.ndarray      # [R][hyps]
    counts_lo: np.ndarray
    counts_hi: np.ndarray
    jstar: np.ndarray       # [R] (-1 none)
    stored: np.ndarray      # [R] bool
    centroids: np.ndarray   # [R][3]
    labels: np.ndarray      # [H][W] int8


def ransac_regions(P, valid, region, R: int, prm: RansacParams, eps=None) -> RegionResult:
    """Region-mode RANSAC (Alg. 2 as printed) for region labels 0..R-1."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    _, H, W = P.shape
    v = np.ascontiguousarray(valid, dtype=np.uint8)
    reg = np.ascontiguousarray(region, dtype=np.int16)
    nh = prm.hyps
    npts = np.zeros(R, np.int32)
    tr = np.zeros((R, nh, 3), np.int32)
    pl = np.zeros((R, nh, 4))
    hv = np.zeros((R, nh), np.uint8)
    er = np.zeros((R, nh))
    cn, lo, hi = (np.zeros((R, nh), np.int32) for _ in range(3))
    js = np.zeros(R, np.int32)
    st = np.zeros(R, np.uint8)
    ce = np.zeros((R, 3))
    labels = np.zeros((H, W), np.int8)
    e = None if eps is None else np.ascontiguousarray(np.broadcast_to(eps, (R, nh)), dtype=np.float64)
    c = prm._c()
    ns = lib().orc_ransac_regions(_p(P), _p(v), _p(reg), W, H, int(R), ctypes.byref(c), _p(e) if e is not None else None,
                                  _p(npts), _p(tr), _p(pl), _p(hv), _p(er), _p(cn), _p(lo), _p(hi), _p(js), _p(st),
                                  _p(ce), _p(labels))
    return RegionResult(ns, npts, tr, pl, hv.astype(bool), er, cn, lo, hi, js, st.astype(bool), ce, labels)


def seg_grad(N, nvalid):
    """-> (m2 float32 [H][W], sector u8, barrier u8) of the FP32 normal image N [3][H][W]."""
    N = np.ascontiguousarray(N, dtype=np.float32)
    _, H, W = N.shape
    nv = np.ascontiguousarray(nvalid != 0, dtype=np.uint8)
    m2 = np.zeros((H, W), np.float32)
    sec = np.zeros((H, W), np.uint8)
    bar = np.zeros((H, W), np.uint8)
    lib().orc_seg_grad(_p(N), _p(nv), W, H, _p(m2), _p(sec), _p(bar))
    return m2, sec, bar


def seg_edges(m2, sector, barrier, low: float, high: float):
    """-> (cls u8 0/1/2 after non-maximum suppression, edge u8 after hysteresis)."""
    m2 = np.ascontiguousarray(m2, dtype=np.float32)
    H, W = m2.shape
    sec = np.ascontiguousarray(sector, dtype=np.uint8)
    bar = np.ascontiguousarray(barrier, dtype=np.uint8)
    cls = np.zeros((H, W), np.uint8)
    edge = np.zeros((H, W), np.uint8)
    lib().orc_seg_edges(_p(m2), _p(sec), _p(bar), W, H, float(low), float(high), _p(cls), _p(edge))
    return cls, edge


def seg_regions(mask, min_area: int, max_regions: int):
    """Ranked 4-connected components of mask -> (int16 [H][W] labels, count)."""
    m = np.ascontiguousarray(mask != 0, dtype=np.uint8)
    H, W = m.shape
    reg = np.zeros((H, W), np.int16)
    n = lib().orc_seg_regions(_p(m), W, H, int(min_area), int(max_regions), _p(reg))
    return reg, n


def segment(N, nvalid, low: float, high: float, min_area: int, max_regions: int):
    """Canny on the normal image, then its regions -> (int16 labels, count, edge u8)."""
    N = np.ascontiguousarray(N, dtype=np.float32)
    _, H, W = N.shape
    nv = np.ascontiguousarray(nvalid != 0, dtype=np.uint8)
    reg = np.zeros((H, W), np.int16)
    edge = np.zeros((H, W), np.uint8)
    n = lib().orc_segment(_p(N), _p(nv), W, H, float(low), float(high), int(min_area), int(max_regions), _p(reg),
                          _p(edge))
    return reg, n, edge


def region_polygons(region, n_regions: int, eps: float):
    """Simplified contour polygons of regions 0..n_regions-1 -> list of int32 [k][2] (x, y) arrays."""
    reg = np.ascontiguousarray(region, dtype=np.int16)
    H, W = reg.shape
    off = np.zeros(n_regions + 1, np.int32)
    need = lib().orc_region_polygons(_p(reg), W, H, int(n_regions), float(eps), None, 0, _p(off))
    xy = np.zeros((max(need, 1), 2), np.int32)
    lib().orc_region_polygons(_p(reg), W, H, int(n_regions), float(eps), _p(xy), need, _p(off))
    return [xy[off[g]:off[g + 1]].copy() for g in range(n_regions)]


@dataclass
class PipelineResult:
    depth: np.ndarray
    P: np.ndarray
    valid: np.ndarray
    N: np.ndarray
    nvalid: np.ndarray
    ransac: RansacResult


def pipeline(depth_u16, K, iters: int, lam: float, kappa: float, prm: RansacParams, edge_stop: int = 0) -> PipelineResult:
    """The whole per-frame path: diffusion -> back-projection -> normals -> sequential RANSAC."""
    I = diffuse(depth_u16, iters, lam, kappa, edge_stop)
    P, valid = backproject(I, K)
    N, nvalid = normals(P, valid)
    rr = ransac(P, valid, prm)
    return PipelineResult(I, P, valid, N, nvalid, rr)

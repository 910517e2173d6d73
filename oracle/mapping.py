"""Test infrastructure: a plain float64 reference of the polygon map with
vertical drift compensation (Sec. III-E, Eqs. 4-10).  Only the tests, the
smoke check and the benchmark's CPU baseline use it; the library never does.

Readings (the paper states the rules, not every detail):
  - the map keeps near-horizontal polygons (normal within max_tilt_deg of the
    world up axis, +Z): heights and vertical drift are about steppable
    surfaces; other polygons are skipped;
  - a polygon's height is the world z of its centroid (Eq. 4 compares
    centroid heights); the 2-D footprint is the convex hull of its vertices
    in world x, y;
  - frame k: raw heights z_raw use the given (drifting) pose; corrected
    heights are z_raw - x_{k-1}; a new polygon matches the map polygon whose
    footprint overlaps its own with positive area and whose height is within
    the drift tolerance (Eq. 5), the smallest height difference first (ties:
    the older map polygon);
  - the drift measurement z_k is the mean of z_raw - h_map over the matches;
    with at least one match the filter runs Eqs. 6-10 once, otherwise only
    the prediction (Eqs. 6-7);
  - the new polygons are then corrected by the updated x_k; a matched one is
    merged (footprint: hull of both; height: support-weighted mean; supports
    add), an unmatched one is appended; matches are applied in input order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


def convex_hull(pts: np.ndarray) -> np.ndarray:
    """Counter-clockwise hull of 2-D points (gift wrapping, collinear points dropped)."""
    P = np.unique(np.asarray(pts, dtype=np.float64).reshape(-1, 2), axis=0)
    if len(P) < 3:
        return P
    start = int(np.lexsort((P[:, 1], P[:, 0]))[0])
    hull = [start]
    while True:
        cur = hull[-1]
        cand = (cur + 1) % len(P)
        for j in range(len(P)):
            if j == cur:
                continue
            a, b = P[cand] - P[cur], P[j] - P[cur]
            cr = a[0] * b[1] - a[1] * b[0]
            # j is to the right of cur->cand, or collinear and farther: wrap to j
            if cr < 0 or (cr == 0 and b @ b > a @ a):
                cand = j
        if cand == start:
            break
        hull.append(cand)
        if len(hull) > len(P):
            break
    return P[hull]


def _clip(subject: np.ndarray, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Part of polygon `subject` left of the directed line a->b (Sutherland-Hodgman step)."""
    out = []
    n = len(subject)
    side = lambda p: (b[0] - a[0]) * (p[1] - a[1]) - (b[1] - a[1]) * (p[0] - a[0])
    for i in range(n):
        p, q = subject[i], subject[(i + 1) % n]
        sp, sq = side(p), side(q)
        if sp >= 0:
            out.append(p)
        if (sp >= 0) != (sq >= 0):
            t = sp / (sp - sq)
            out.append(p + t * (q - p))
    return np.array(out).reshape(-1, 2)


def area(poly: np.ndarray) -> float:
    if len(poly) < 3:
        return 0.0
    x, y = poly[:, 0], poly[:, 1]
    return 0.5 * float(np.dot(x, np.roll(y, -1)) - np.dot(y, np.roll(x, -1)))


def overlap_area(h1: np.ndarray, h2: np.ndarray) -> float:
    """Area of the intersection of two counter-clockwise convex polygons."""
    if len(h1) < 3 or len(h2) < 3:
        return 0.0
    poly = h1
    for i in range(len(h2)):
        poly = _clip(poly, h2[i], h2[(i + 1) % len(h2)])
        if len(poly) == 0:
            return 0.0
    return abs(area(poly))


@dataclass
class MapPolygon:
    height: float
    support: int
    hull: np.ndarray  # [k][2] counter-clockwise footprint


@dataclass
class FrameResult:
    matched: int
    added: int
    skipped: int
    measurement: float
    drift: float
    variance: float
    match_of: List[int] = field(default_factory=list)  # map index per input polygon (-1: added, -2: skipped)


class DriftMap:
    def __init__(self, drift_tolerance: float = 0.05, sigma_p: float = 1e-5, sigma_m: float = 1e-4,
                 max_tilt_deg: float = 15.0):
        self.tol = drift_tolerance
        self.sigma_p = sigma_p
        self.sigma_m = sigma_m
        self.cos_tilt = math.cos(math.radians(max_tilt_deg))
        self.x = 0.0   # drift estimate x_{k|k}
        self.P = 0.0   # its variance P_{k|k}
        self.polys: List[MapPolygon] = []

    def integrate(self, R: np.ndarray, C: np.ndarray, polys) -> FrameResult:
        """polys: list of (n[3], d, centroid[3], support, vertices [k][3]) in the camera frame."""
        R = np.asarray(R, dtype=np.float64)
        C = np.asarray(C, dtype=np.float64)
        cands = []
        for (n, d, cen, sup, verts) in polys:
            nw = R @ np.asarray(n, dtype=np.float64)
            if abs(nw[2]) < self.cos_tilt:
                cands.append(None)
                continue
            cw = R @ np.asarray(cen, dtype=np.float64) + C
            vw = (R @ np.asarray(verts, dtype=np.float64).T).T + C
            cands.append((cw[2], int(sup), convex_hull(vw[:, :2])))
        # matching on heights corrected by the previous estimate (Eqs. 4-5)
        match = []
        for c in cands:
            if c is None:
                match.append(-2)
                continue
            zc = c[0] - self.x
            best, bj = None, -1
            for j, mp in enumerate(self.polys):
                dz = abs(zc - mp.height)
                if dz <= self.tol and overlap_area(c[2], mp.hull) > 0.0 and (best is None or dz < best):
                    best, bj = dz, j
            match.append(bj)
        pairs = [(c[0], self.polys[j].height) for c, j in zip(cands, match) if c is not None and j >= 0]
        # Kalman filter of the vertical drift (Eqs. 6-10)
        x_pred, P_pred = self.x, self.P + self.sigma_p
        meas = float("nan")
        if pairs:
            meas = float(np.mean([zr - h for zr, h in pairs]))
            K = P_pred / (P_pred + self.sigma_m)
            self.x = x_pred + K * (meas - x_pred)
            self.P = (1.0 - K) * P_pred
        else:
            self.x, self.P = x_pred, P_pred
        added = 0
        for c, j in zip(cands, match):
            if c is None:
                continue
            z = c[0] - self.x
            if j >= 0:
                mp = self.polys[j]
                mp.height = (mp.height * mp.support + z * c[1]) / (mp.support + c[1])
                mp.support += c[1]
                mp.hull = convex_hull(np.vstack([mp.hull, c[2]]))
            else:
                self.polys.append(MapPolygon(z, c[1], c[2]))
                added += 1
        return FrameResult(len(pairs), added, sum(1 for c in cands if c is None), meas, self.x, self.P, match)


def lift_polygon(xy_px: np.ndarray, plane_n, plane_d: float, K) -> np.ndarray:
    """Pixel vertices of a polygon on the camera-frame plane n.p + d = 0 -> 3-D
    points (the intersections of the pixel rays with the plane)."""
    fx, fy, cx, cy = K
    xy = np.asarray(xy_px, dtype=np.float64).reshape(-1, 2)
    rays = np.stack([(xy[:, 0] - cx) / fx, (xy[:, 1] - cy) / fy, np.ones(len(xy))], axis=1)
    t = -plane_d / (rays @ np.asarray(plane_n, dtype=np.float64))
    return rays * t[:, None]

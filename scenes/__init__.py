"""Seeded synthetic depth frames of staircase scenes.

This module only builds inputs: it ray-casts analytic planar patches (and one
cylinder) in float64, then adds sensor noise and holes.  It holds none of the
plane-extraction arithmetic (no diffusion, no back-projection of a depth
image, no normals, no RANSAC), so that both the CPU oracle and the GPU path
can be fed from it without sharing any of the method's code.

Conventions
-----------
* World frame is Z-up.  The camera frame is x right, y down, z forward; depth
  is the forward z of the hit point, not the range along the ray.
* Pixel (u, v) = (column, row) looks along ((u - cx)/fx, (v - cy)/fy, 1).
* Depth is stored as uint16 millimetres with 0 marking a hole (no return,
  beyond the sensor's range, or a dropped pixel).
* Every frame is a pure function of (config id, frame index): the pose walk,
  noise and holes are drawn from numpy PCG64 streams seeded with
  SeedSequence([config, k]) (frame k) and SeedSequence([config, 65535]) (the
  pose trajectory of a config).

The five workloads are described by ``CONFIGS``; ``make_frame(cfg, k)`` and
``make_batch(cfg, n)`` build frames.  The scene recipe mirrors the workloads
the paper measures on (Sec. IV-A and IV-B: a stair model seen by an L515
depth camera at 320x240 and 640x480) with synthetic geometry.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Intrinsics", "Frame", "SceneConfig", "CONFIGS", "make_frame", "make_batch",
    "straight_stair_patches", "spiral_stair_patches", "two_step_patches",
    "render", "camera_rotation", "frame_rng",
]

MAX_RANGE_M = 8.0  # L515-like maximum range: farther returns become holes


@dataclass(frozen=True)
class Intrinsics:
    fx: float
    fy: float
    cx: float
    cy: float


@dataclass
class Frame:
    depth: np.ndarray            # uint16 [H][W] mm, 0 = hole
    K: Intrinsics
    gt_labels: np.ndarray        # int16 [H][W], index into gt_planes, -1 = miss/hole
    gt_planes: np.ndarray        # float64 [P][4]: camera-frame n.p + d = 0, d > 0 (or d == 0)
    depth_m: np.ndarray          # float64 [H][W] noise-free depth in metres, 0 = miss
    pose: Tuple[np.ndarray, np.ndarray]  # (R world<-camera, camera centre)
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.depth.shape


# --------------------------------------------------------------------------
# Geometry: patches are (world plane n.X + d = 0, inside-test on hit points)
# --------------------------------------------------------------------------
@dataclass
class Patch:
    n: np.ndarray
    d: float
    inside: Callable[[np.ndarray], np.ndarray]
    name: str = ""


@dataclass
class Cylinder:
    """Vertical cylinder x^2 + y^2 = r^2 between z0 and z1 (a non-planar distractor)."""
    r: float
    z0: float
    z1: float
    name: str = "column"


def _rect(axis: int, value: float, lo: Sequence[float], hi: Sequence[float], name: str) -> Patch:
    """Axis-aligned rectangle on the plane X[axis] = value; lo/hi bound the other two axes."""
    n = np.zeros(3)
    n[axis] = 1.0
    others = [a for a in range(3) if a != axis]

    def inside(X, others=others, lo=lo, hi=hi):
        m = np.ones(X.shape[0], dtype=bool)
        for a, l, h in zip(others, lo, hi):
            m &= (X[:, a] >= l) & (X[:, a] <= h)
        return m

    return Patch(n=n, d=-float(value), inside=inside, name=name)


def two_step_patches() -> List[Patch]:
    """Floor plus two steps (rise 0.15 m, tread 0.28 m) with the first riser 1.0 m
    ahead along +X; the stair spans the whole view and the top tread is unbounded."""
    big = 1e3
    rise, tread, x0 = 0.15, 0.28, 1.0
    return [
        _rect(2, 0.0, (-big, -big), (x0, big), "floor"),
        _rect(0, x0, (-big, 0.0), (big, rise), "riser0"),
        _rect(2, rise, (x0, -big), (x0 + tread, big), "tread0"),
        _rect(0, x0 + tread, (-big, rise), (big, 2 * rise), "riser1"),
        _rect(2, 2 * rise, (x0 + tread, -big), (big, big), "tread1"),
    ]


def straight_stair_patches(steps: int = 8, rise: float = 0.15, tread: float = 0.28,
                           width: float = 1.2, x0: float = 1.0, landing: float = 1.0,
                           wall_h: float = 2.5) -> List[Patch]:
    """Straight staircase of ``steps`` steps along +X between side walls at
    y = +-width/2, a floor before it, a top landing ``landing`` m deep and an
    end wall; walls are ``wall_h`` m tall above each local floor level."""
    hw = width / 2.0
    x_end = x0 + steps * tread + landing
    top = steps * rise
    P = [_rect(2, 0.0, (-3.0, -hw), (x0, hw), "floor")]
    for i in range(steps):
        xa = x0 + i * tread
        P.append(_rect(0, xa, (-hw, i * rise), (hw, (i + 1) * rise), f"riser{i}"))
        xb = xa + tread if i < steps - 1 else x_end
        P.append(_rect(2, (i + 1) * rise, (xa, -hw), (xb, hw), f"tread{i}"))
    P.append(_rect(1, -hw, (-3.0, 0.0), (x_end, top + wall_h), "wall_right"))
    P.append(_rect(1, hw, (-3.0, 0.0), (x_end, top + wall_h), "wall_left"))
    P.append(_rect(0, x_end, (-hw, top), (hw, top + wall_h), "end_wall"))
    return P


def spiral_stair_patches(steps: int = 16, step_deg: float = 30.0, rise: float = 0.16,
                         r_in: float = 0.3, r_out: float = 1.3) -> Tuple[List[Patch], List[Cylinder]]:
    """Spiral staircase around the world Z axis: step i is the annular sector
    [i, i+1) * step_deg at tread height (i+1)*rise; its riser is the radial
    rectangle at angle i*step_deg.  A floor and a central column surround it."""
    P = [Patch(n=np.array([0.0, 0.0, 1.0]), d=0.0,
               inside=lambda X: (np.hypot(X[:, 0], X[:, 1]) >= r_in) & (np.abs(X[:, 0]) < 6) & (np.abs(X[:, 1]) < 6),
               name="floor")]
    step = math.radians(step_deg)
    for i in range(steps):
        a0, a1 = i * step, (i + 1) * step
        h = (i + 1) * rise

        def tread_inside(X, a0=a0, a1=a1):
            r = np.hypot(X[:, 0], X[:, 1])
            ang = np.arctan2(X[:, 1], X[:, 0])
            # unwrap the sector test so sectors beyond 2*pi still work
            rel = np.mod(ang - a0, 2 * math.pi)
            return (r >= r_in) & (r <= r_out) & (rel <= (a1 - a0))

        P.append(Patch(n=np.array([0.0, 0.0, 1.0]), d=-h, inside=tread_inside, name=f"tread{i}"))
        # riser: vertical plane through the axis at angle a0, normal pointing to -angle side
        n = np.array([-math.sin(a0), math.cos(a0), 0.0])
        u = np.array([math.cos(a0), math.sin(a0), 0.0])

        def riser_inside(X, u=u, z0=i * rise, z1=h):
            s = X @ u
            return (s >= r_in) & (s <= r_out) & (X[:, 2] >= z0) & (X[:, 2] <= z1)

        P.append(Patch(n=n, d=0.0, inside=riser_inside, name=f"riser{i}"))
    return P, [Cylinder(r=r_in, z0=0.0, z1=steps * rise + 2.0)]


# --------------------------------------------------------------------------
# Camera and ray casting
# --------------------------------------------------------------------------
def camera_rotation(yaw: float, pitch_down: float) -> np.ndarray:
    """World<-camera rotation whose columns are the camera's x (right), y (down)
    and z (forward) axes in the Z-up world; yaw turns about +Z from +X."""
    f = np.array([math.cos(pitch_down) * math.cos(yaw), math.cos(pitch_down) * math.sin(yaw), -math.sin(pitch_down)])
    r = np.array([math.sin(yaw), -math.cos(yaw), 0.0])
    dn = np.cross(f, r)
    return np.stack([r, dn, f], axis=1)


def render(W: int, H: int, K: Intrinsics, R: np.ndarray, C: np.ndarray,
           patches: Sequence[Patch], cylinders: Sequence[Cylinder] = ()) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Ray-cast the scene.  Returns (depth_m [H][W] float64 with 0 for a miss,
    labels int16 [H][W] (patch index, or len(patches)+c for cylinder c, -1 miss),
    camera-frame planes [P][4] of the patches)."""
    u, v = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    rays_c = np.stack([(u - K.cx) / K.fx, (v - K.cy) / K.fy, np.ones_like(u)], axis=-1).reshape(-1, 3)
    dirs = rays_c @ R.T
    best = np.full(dirs.shape[0], np.inf)
    lab = np.full(dirs.shape[0], -1, dtype=np.int16)
    for pi, p in enumerate(patches):
        den = dirs @ p.n
        num = -(p.n @ C + p.d)
        with np.errstate(divide="ignore", invalid="ignore"):
            t = np.where(np.abs(den) > 1e-12, num / den, np.inf)
        ok = (t > 1e-6) & (t < best)
        if not ok.any():
            continue
        idx = np.nonzero(ok)[0]
        X = C[None, :] + t[idx, None] * dirs[idx]
        ins = p.inside(X)
        idx = idx[ins]
        best[idx] = t[idx]
        lab[idx] = pi
    for ci, cyl in enumerate(cylinders):
        # |C_xy + t d_xy|^2 = r^2
        a = dirs[:, 0] ** 2 + dirs[:, 1] ** 2
        b = 2 * (C[0] * dirs[:, 0] + C[1] * dirs[:, 1])
        c = C[0] ** 2 + C[1] ** 2 - cyl.r ** 2
        disc = b * b - 4 * a * c
        with np.errstate(invalid="ignore", divide="ignore"):
            sq = np.sqrt(np.maximum(disc, 0.0))
            t1 = (-b - sq) / (2 * a)
            t2 = (-b + sq) / (2 * a)
        t = np.where(t1 > 1e-6, t1, t2)
        z = C[2] + t * dirs[:, 2]
        ok = (disc > 0) & (a > 1e-12) & (t > 1e-6) & (t < best) & (z >= cyl.z0) & (z <= cyl.z1)
        best[ok] = t[ok]
        lab[ok] = len(patches) + ci
    depth = np.where(np.isfinite(best) & (best <= MAX_RANGE_M), best, 0.0)
    lab = np.where(depth > 0, lab, -1).astype(np.int16)
    planes = np.zeros((len(patches), 4))
    for pi, p in enumerate(patches):
        n_c = R.T @ p.n
        d_c = float(p.n @ C + p.d)
        if d_c < 0:
            n_c, d_c = -n_c, -d_c
        planes[pi, :3] = n_c
        planes[pi, 3] = d_c
    return depth.reshape(H, W), lab.reshape(H, W), planes


def quantize(depth_m: np.ndarray, rng: np.random.Generator, noise: str, sigma: float,
             hole_frac: float) -> np.ndarray:
    """Depth -> uint16 mm with additive Gaussian noise and uniformly dropped pixels.
    noise = 'const': sigma in mm;  'quad': sigma * z^2 metres (z in metres)."""
    valid = depth_m > 0
    if noise == "const":
        s_mm = np.full(depth_m.shape, sigma)
    elif noise == "quad":
        s_mm = 1000.0 * sigma * depth_m ** 2
    elif noise == "none":
        s_mm = np.zeros(depth_m.shape)
    else:
        raise ValueError(noise)
    eps = rng.standard_normal(depth_m.shape) * s_mm
    mm = np.rint(1000.0 * depth_m + eps)
    mm = np.clip(mm, 1, 65535)
    mm = np.where(valid, mm, 0).astype(np.uint16)
    n = mm.size
    nh = int(round(hole_frac * n))
    if nh > 0:
        drop = rng.choice(n, size=nh, replace=False)
        mm.reshape(-1)[drop] = 0
    return mm


# --------------------------------------------------------------------------
# Workload configurations
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class SceneConfig:
    cid: int
    name: str
    sizes: Tuple[Tuple[int, int], ...]     # (W, H) cycle for successive frames
    scene: str                              # 'two_step' | 'straight' | 'spiral' | 'mixed'
    noise: str
    sigma: float
    hole_frac: float
    diffuse_iters: int
    hyps: int
    max_planes: int
    thresh_m: float = 0.01
    lam: float = 0.2
    kappa_mm: float = 30.0
    seed: int = 0

    def intrinsics(self, W: int, H: int) -> Intrinsics:
        if self.cid == 1:
            return Intrinsics(100.0, 100.0, 80.0, 60.0)
        if (W, H) == (1280, 720):
            return Intrinsics(574.5, 574.5, 640.0, 360.0)
        f = 383.0 * H / 480.0
        return Intrinsics(f, f, W / 2.0, H / 2.0)

    def min_inliers(self, W: int, H: int) -> int:
        return max(50, int(math.ceil(0.002 * W * H)))

    @property
    def ransac_seed(self) -> int:
        return 0x5EED0000 + self.cid


CONFIGS = {
    1: SceneConfig(1, "c1_two_step_160x120", ((160, 120),), "two_step", "const", 2.0, 0.01, 10, 256, 12),
    2: SceneConfig(2, "c2_straight_640x480", ((640, 480),), "straight", "quad", 0.002, 0.02, 20, 1024, 12),
    3: SceneConfig(3, "c3_spiral_mixed", ((424, 240), (640, 480), (848, 480)), "spiral", "quad", 0.002, 0.02, 20, 1024, 12),
    4: SceneConfig(4, "c4_straight_720p_480p", ((1280, 720), (848, 480)), "straight", "quad", 0.002, 0.02, 20, 4096, 12),
    5: SceneConfig(5, "c5_serving_mixed", ((424, 240), (640, 480), (1280, 720)), "mixed", "quad", 0.002, 0.02, 20, 1024, 12),
}


def frame_rng(cid: int, k: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([cid, k])))


def _walk(cid: int, n: int, kind: str) -> List[Tuple[float, float, float, float, float]]:
    """Seeded random-walk poses (x, y, h, yaw, pitch) for frames 0..n-1."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([cid, 65535])))
    out = []
    if kind == "spiral":
        phi, h, dpitch, dyaw = 0.0, 1.3, 0.0, 0.0
        for _ in range(n):
            x, y = 2.5 * math.cos(phi), 2.5 * math.sin(phi)
            yaw = phi + math.pi + dyaw
            out.append((x, y, h, yaw, math.radians(30.0) + dpitch))
            phi += rng.normal(0.0, 0.05) / 2.5
            h = float(np.clip(h + rng.normal(0.0, 0.05), 1.0, 1.6))
            dpitch = float(np.clip(dpitch + math.radians(rng.normal(0.0, 2.0)), -math.radians(5), math.radians(5)))
            dyaw = float(np.clip(dyaw + math.radians(rng.normal(0.0, 2.0)), -math.radians(10), math.radians(10)))
    else:
        x, y, h, dpitch, dyaw = 0.0, 0.0, 1.2, 0.0, 0.0
        for _ in range(n):
            out.append((x, y, h, dyaw, math.radians(30.0) + dpitch))
            x = float(np.clip(x + rng.normal(0.0, 0.05), -0.5, 0.3))
            y = float(np.clip(y + rng.normal(0.0, 0.05), -0.3, 0.3))
            h = float(np.clip(h + rng.normal(0.0, 0.05), 1.1, 1.3))
            dpitch = float(np.clip(dpitch + math.radians(rng.normal(0.0, 2.0)), -math.radians(5), math.radians(5)))
            dyaw = float(np.clip(dyaw + math.radians(rng.normal(0.0, 2.0)), -math.radians(5), math.radians(5)))
    return out


def make_frame(cfg, k: int = 0, size: Optional[Tuple[int, int]] = None, noise: Optional[str] = None,
               hole_frac: Optional[float] = None, scene: Optional[str] = None) -> Frame:
    """Frame k of a workload configuration (a SceneConfig or its id).

    ``size``/``noise``/``hole_frac``/``scene`` override the configuration
    (e.g. noise='none', hole_frac=0 for the noise-free variants used to pin
    exact plane recovery)."""
    if isinstance(cfg, int):
        cfg = CONFIGS[cfg]
    W, H = size if size is not None else cfg.sizes[k % len(cfg.sizes)]
    K = cfg.intrinsics(W, H)
    kind = scene or cfg.scene
    if kind == "mixed":
        kind = "straight" if k % 2 == 0 else "spiral"
    cyl: List[Cylinder] = []
    if kind == "two_step":
        patches = two_step_patches()
        R = camera_rotation(0.0, math.radians(30.0))
        C = np.array([0.0, 0.0, 1.0])
    elif kind == "straight":
        patches = straight_stair_patches()
        if k == 0:
            x, y, h, yaw, pitch = 0.0, 0.0, 1.2, 0.0, math.radians(30.0)
        else:
            x, y, h, yaw, pitch = _walk(cfg.cid, k + 1, "straight")[k]
        R = camera_rotation(yaw, pitch)
        C = np.array([x, y, h])
    elif kind == "spiral":
        patches, cyl = spiral_stair_patches()
        x, y, h, yaw, pitch = _walk(cfg.cid, k + 1, "spiral")[k]
        R = camera_rotation(yaw, pitch)
        C = np.array([x, y, h])
    else:
        raise ValueError(kind)
    depth_m, labels, planes = render(W, H, K, R, C, patches, cyl)
    rng = frame_rng(cfg.cid, k)
    nz = noise if noise is not None else cfg.noise
    hf = cfg.hole_frac if hole_frac is None else hole_frac
    mm = quantize(depth_m, rng, nz, cfg.sigma, hf)
    labels = np.where(mm > 0, labels, -1).astype(np.int16)
    return Frame(depth=mm, K=K, gt_labels=labels, gt_planes=planes, depth_m=depth_m, pose=(R, C),
                 meta=dict(config=cfg.cid, k=k, W=W, H=H, scene=kind, noise=nz, hole_frac=hf,
                           patch_names=[p.name for p in patches] + [c.name for c in cyl]))


def make_batch(cfg, n: int, start: int = 0) -> List[Frame]:
    return [make_frame(cfg, start + i) for i in range(n)]

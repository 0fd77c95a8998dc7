"""Seeded synthetic scenes and cameras.

This module only draws inputs: Gaussian attributes (already activated:
linear scales, unit quaternions, opacities in (0, 1)) and pinhole cameras.
It holds none of the visibility-field arithmetic, so the reference checker
and the GPU path can both take their inputs from here.

The shapes and distributions follow the workloads the paper evaluates on
(indoor rooms seen by a robot at 1.5 m, images 512x512 with a 90 degree
field of view in its simulator setup, object scenes seen from a sphere);
the datasets themselves are not available, so these seeded scenes stand in
for them.

Camera convention: x right, y down, z forward; world up is +z.  A camera is
(R, t) with x_cam = R x_world + t, focal lengths in pixels and the principal
point at the image centre; pixel (i, j) is sampled at (i + 0.5, j + 0.5).
All arrays are float32 (the stored precision); checkers promote to float64.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

__all__ = [
    "Scene", "Cameras", "Workload", "look_at", "make_cameras", "tiny_scene",
    "rooms_scene", "sphere_cameras", "ellipse_path_cameras", "room_candidates",
    "workload", "subset_scene", "WORKLOADS", "uniform_draws", "color_sh_variances",
]


@dataclass
class Scene:
    means: np.ndarray      # [N, 3] float32
    scales: np.ndarray     # [N, 3] float32, linear (exp of log-scale)
    quats: np.ndarray      # [N, 4] float32, (w, x, y, z), unit norm
    opacity: np.ndarray    # [N] float32 in (0, 1)
    n_virtual: int = 0     # the last n_virtual rows are virtual particles
    extent: Tuple[Tuple[float, float], ...] = ((-1, 1), (-1, 1), (-1, 1))

    @property
    def n(self) -> int:
        return int(self.means.shape[0])


@dataclass
class Cameras:
    R: np.ndarray          # [V, 3, 3] float32, world -> camera rotation
    t: np.ndarray          # [V, 3] float32
    K: np.ndarray          # [V, 4] float32: fx, fy, cx, cy
    wh: np.ndarray         # [V, 2] int32: width, height

    @property
    def n(self) -> int:
        return int(self.R.shape[0])

    @property
    def centers(self) -> np.ndarray:
        R = self.R.astype(np.float64)
        t = self.t.astype(np.float64)
        return -np.einsum("vji,vj->vi", R, t)

    def pixels(self) -> int:
        return int(np.sum(self.wh[:, 0].astype(np.int64) * self.wh[:, 1]))

    def subset(self, idx: Sequence[int]) -> "Cameras":
        idx = np.asarray(idx, dtype=np.int64)
        return Cameras(self.R[idx].copy(), self.t[idx].copy(), self.K[idx].copy(), self.wh[idx].copy())

    @staticmethod
    def concat(cams: List["Cameras"]) -> "Cameras":
        return Cameras(np.concatenate([c.R for c in cams]), np.concatenate([c.t for c in cams]),
                       np.concatenate([c.K for c in cams]), np.concatenate([c.wh for c in cams]))


def look_at(center, target, up=(0.0, 0.0, 1.0)):
    """World->camera rotation and translation of a camera at `center` looking
    at `target` (x right, y down, z forward)."""
    c = np.asarray(center, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - c
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, dtype=np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    t = -R @ c
    return R, t


def make_cameras(centers, targets, width, height, fov_x_deg) -> Cameras:
    centers = np.asarray(centers, dtype=np.float64).reshape(-1, 3)
    targets = np.asarray(targets, dtype=np.float64).reshape(-1, 3)
    V = centers.shape[0]
    ws = np.broadcast_to(np.asarray(width), (V,)).astype(np.int32)
    hs = np.broadcast_to(np.asarray(height), (V,)).astype(np.int32)
    R = np.zeros((V, 3, 3))
    t = np.zeros((V, 3))
    K = np.zeros((V, 4))
    for i in range(V):
        R[i], t[i] = look_at(centers[i], targets[i])
        fx = ws[i] / (2.0 * np.tan(np.deg2rad(fov_x_deg) / 2.0))
        K[i] = (fx, fx, ws[i] / 2.0, hs[i] / 2.0)
    return Cameras(R.astype(np.float32), t.astype(np.float32), K.astype(np.float32),
                   np.stack([ws, hs], axis=1).astype(np.int32))


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _random_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def tiny_scene(n=2000, seed=1000) -> Scene:
    """Object-like scene: means U[-1,1]^3, per-axis log-scale N(-3, 0.5),
    random unit quaternions, opacity sigmoid(N(0, 1))."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, size=(n, 3))
    scales = np.exp(rng.normal(-3.0, 0.5, size=(n, 3)))
    quats = _random_quats(rng, n)
    opacity = _sigmoid(rng.normal(0.0, 1.0, size=n))
    return Scene(means.astype(np.float32), scales.astype(np.float32), quats.astype(np.float32),
                 opacity.astype(np.float32), 0, ((-1, 1), (-1, 1), (-1, 1)))


def sphere_cameras(n, seed, radius=3.0, width=128, height=128, fov=60.0) -> Cameras:
    """Cameras on a sphere of the given radius, directions uniform on S^2
    (rejecting |z| > 0.95 so that the look-at frame stays defined), looking at
    the origin."""
    rng = np.random.default_rng(seed)
    dirs = []
    while len(dirs) < n:
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        if abs(d[2]) <= 0.95:
            dirs.append(d)
    centers = radius * np.asarray(dirs)
    return make_cameras(centers, np.zeros_like(centers), width, height, fov)


# --- rooms -----------------------------------------------------------------

ROOM = (6.0, 4.0, 3.0)
DOOR_W, DOOR_H = 1.0, 2.1


def _room_surfaces(nx, ny):
    """Axis-aligned rectangles (fixed axis, fixed value, (a0, a1), (b0, b1))
    for the floor, the outer walls and the interior walls (with doors) of an
    nx-by-ny grid of 6x4x3 m rooms."""
    X, Y, Z = ROOM[0] * nx, ROOM[1] * ny, ROOM[2]
    rects = [(2, 0.0, (0.0, X), (0.0, Y))]                     # floor, z = 0
    rects += [(1, 0.0, (0.0, X), (0.0, Z)), (1, Y, (0.0, X), (0.0, Z))]
    rects += [(0, 0.0, (0.0, Y), (0.0, Z)), (0, X, (0.0, Y), (0.0, Z))]
    # interior walls normal to x (x = 6 k), door centred in each room's y span
    for k in range(1, nx):
        x = ROOM[0] * k
        for j in range(ny):
            y0, y1 = ROOM[1] * j, ROOM[1] * (j + 1)
            yc = 0.5 * (y0 + y1)
            d0, d1 = yc - DOOR_W / 2, yc + DOOR_W / 2
            rects += [(0, x, (y0, d0), (0.0, Z)), (0, x, (d1, y1), (0.0, Z)),
                      (0, x, (d0, d1), (DOOR_H, Z))]
    # interior walls normal to y (y = 4 k), door centred in each room's x span
    for k in range(1, ny):
        y = ROOM[1] * k
        for i in range(nx):
            x0, x1 = ROOM[0] * i, ROOM[0] * (i + 1)
            xc = 0.5 * (x0 + x1)
            d0, d1 = xc - DOOR_W / 2, xc + DOOR_W / 2
            rects += [(1, y, (x0, d0), (0.0, Z)), (1, y, (d1, x1), (0.0, Z)),
                      (1, y, (d0, d1), (DOOR_H, Z))]
    return rects


def rooms_scene(n, nx=1, ny=1, seed=2000, clutter_frac=0.2, blobs_per_room=16) -> Scene:
    """Indoor scene: an nx-by-ny grid of 6x4x3 m rooms.  (1 - clutter_frac) of
    the Gaussians lie uniformly by area on the floor and walls, the rest in
    seeded clutter blobs N(c, 0.25^2 I) with c in [0.5, W-0.5] x [0.5, D-0.5] x
    [0, 1.5] per room.  Per-axis log-scale N(-4, 0.5), random unit quaternions,
    opacity sigmoid(N(1, 1))."""
    rng = np.random.default_rng(seed)
    rects = _room_surfaces(nx, ny)
    areas = np.array([(a[1] - a[0]) * (b[1] - b[0]) for _, _, a, b in rects])
    n_surf = int(round(n * (1.0 - clutter_frac)))
    n_clut = n - n_surf
    which = rng.choice(len(rects), size=n_surf, p=areas / areas.sum())
    means = np.zeros((n, 3))
    u = rng.uniform(size=(n_surf, 2))
    for k, (axis, val, a, b) in enumerate(rects):
        sel = which == k
        if not np.any(sel):
            continue
        other = [i for i in range(3) if i != axis]
        means[:n_surf][sel, axis] = val
        means[:n_surf][sel, other[0]] = a[0] + (a[1] - a[0]) * u[sel, 0]
        means[:n_surf][sel, other[1]] = b[0] + (b[1] - b[0]) * u[sel, 1]
    n_blobs = blobs_per_room * nx * ny
    centers = np.zeros((n_blobs, 3))
    b = 0
    for i in range(nx):
        for j in range(ny):
            for _ in range(blobs_per_room):
                centers[b] = (ROOM[0] * i + rng.uniform(0.5, ROOM[0] - 0.5),
                              ROOM[1] * j + rng.uniform(0.5, ROOM[1] - 0.5),
                              rng.uniform(0.0, 1.5))
                b += 1
    blob = rng.integers(0, n_blobs, size=n_clut)
    means[n_surf:] = centers[blob] + 0.25 * rng.standard_normal((n_clut, 3))
    scales = np.exp(rng.normal(-4.0, 0.5, size=(n, 3)))
    quats = _random_quats(rng, n)
    opacity = _sigmoid(rng.normal(1.0, 1.0, size=n))
    ext = ((0.0, ROOM[0] * nx), (0.0, ROOM[1] * ny), (0.0, ROOM[2]))
    return Scene(means.astype(np.float32), scales.astype(np.float32), quats.astype(np.float32),
                 opacity.astype(np.float32), 0, ext)


def ellipse_path_cameras(n, seed, width, height, fov=90.0, center=(1.5, 2.0), radii=(0.8, 1.2),
                         height_m=1.5, yaw_jitter_deg=30.0) -> Cameras:
    """Training path: n poses evenly spaced on an ellipse at camera height
    height_m, each looking radially outward with a yaw jitter U(-j, j) and
    zero pitch (planar robot poses)."""
    rng = np.random.default_rng(seed)
    th = np.linspace(0.0, 2.0 * np.pi, n, endpoint=False)
    c = np.stack([center[0] + radii[0] * np.cos(th), center[1] + radii[1] * np.sin(th),
                  np.full(n, height_m)], axis=1)
    yaw = th + np.deg2rad(rng.uniform(-yaw_jitter_deg, yaw_jitter_deg, size=n))
    tgt = c + np.stack([np.cos(yaw), np.sin(yaw), np.zeros(n)], axis=1)
    return make_cameras(c, tgt, width, height, fov)


def room_candidates(n, seed, extent, width, height, fov=90.0, height_m=1.5, margin=0.3) -> Cameras:
    """Candidate poses: uniform over the floor plan with a wall margin, at
    camera height height_m, yaw U[0, 2 pi), zero pitch."""
    rng = np.random.default_rng(seed)
    (x0, x1), (y0, y1), _ = extent
    c = np.stack([rng.uniform(x0 + margin, x1 - margin, n), rng.uniform(y0 + margin, y1 - margin, n),
                  np.full(n, height_m)], axis=1)
    yaw = rng.uniform(0.0, 2.0 * np.pi, n)
    tgt = c + np.stack([np.cos(yaw), np.sin(yaw), np.zeros(n)], axis=1)
    return make_cameras(c, tgt, width, height, fov)


def morton_order(scene: Scene, bits: int = 10) -> np.ndarray:
    """Permutation that sorts the Gaussians along a 3D Morton (Z-order) curve,
    so that consecutive blocks are spatially compact (block-anchored half
    storage of the means relies on it)."""
    lo = scene.means.min(0)
    span = np.maximum(scene.means.max(0) - lo, 1e-9)
    q = np.clip(((scene.means - lo) / span * ((1 << bits) - 1)).astype(np.int64), 0, (1 << bits) - 1)
    code = np.zeros(scene.n, dtype=np.int64)
    for b in range(bits):
        for a in range(3):
            code |= ((q[:, a] >> b) & 1) << (3 * b + a)
    return np.argsort(code, kind="stable")


def uniform_draws(n: int, seed: int) -> np.ndarray:
    """n seeded samples of U[0, 1)^3 (the random positions density control
    draws are passed in from here)."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=(n, 3))


def color_sh_variances(n: int, Lc: int, seed: int) -> np.ndarray:
    """Seeded stand-in for the diagonal variances of the colour SH
    coefficients a Laplace approximation would give: float32 [3][Kc][n],
    Kc = (Lc + 1)^2.  Per Gaussian a log-uniform scale in [1e-4, 1e-1] (well
    and poorly observed particles), times 2^-l for degree l and a log-normal
    factor (sigma 0.5) per coefficient and channel."""
    rng = np.random.default_rng(seed)
    Kc = (Lc + 1) ** 2
    base = 10.0 ** rng.uniform(-4.0, -1.0, size=n)
    deg = np.array([l for l in range(Lc + 1) for _ in range(2 * l + 1)], dtype=np.float64)
    f = np.exp(rng.normal(0.0, 0.5, size=(3, Kc, n)))
    return (base[None, None, :] * (2.0 ** -deg)[None, :, None] * f).astype(np.float32)


def subset_scene(scene: Scene, idx) -> Scene:
    idx = np.asarray(idx)
    return Scene(scene.means[idx].copy(), scene.scales[idx].copy(), scene.quats[idx].copy(),
                 scene.opacity[idx].copy(), 0, scene.extent)


@dataclass
class Workload:
    name: str
    scene: Scene
    train: Cameras
    cand: Cameras
    sh_degree: int
    kappa: float = 1.0
    notes: dict = field(default_factory=dict)


RES_CLASSES = ((160, 120), (320, 240), (640, 480))


def mixed_candidates(n, seed, extent):
    rng = np.random.default_rng(seed + 7)
    cls = rng.integers(0, len(RES_CLASSES), size=n)
    cams = []
    for i in range(n):
        w, h = RES_CLASSES[cls[i]]
        cams.append(room_candidates(1, seed * 1009 + i, extent, w, h))
    return Cameras.concat(cams)


WORKLOADS = ("tiny", "room", "batched", "precision", "ctx512")


def workload(name: str, scale: float = 1.0) -> Workload:
    """The synthetic workloads.  `scale` shrinks Gaussian and view counts for
    quick checks (1.0 = full size)."""
    def s(x):
        return max(1, int(round(x * scale)))
    if name == "tiny":
        sc = tiny_scene(s(2000), seed=1000)
        return Workload(name, sc, sphere_cameras(s(8), 1001), sphere_cameras(s(4), 1002), 2)
    if name in ("room", "ctx512"):
        sc = rooms_scene(s(200_000), 1, 1, seed=2000)
        train = ellipse_path_cameras(s(100), 2001, 800, 800)
        if name == "room":
            cand = room_candidates(s(64), 2002, sc.extent, 400, 400)
        else:
            cand = room_candidates(s(64), 2002, sc.extent, 512, 512)
        return Workload(name, sc, train, cand, 3)
    if name == "batched":
        sc = rooms_scene(s(1_000_000), 2, 1, seed=3000)
        train = ellipse_path_cameras(s(300), 3001, 1280, 720)
        cand = mixed_candidates(s(256), 3002, sc.extent)
        return Workload(name, sc, train, cand, 3)
    if name == "precision":
        sc = rooms_scene(s(3_000_000), 2, 2, seed=4000)
        sc = subset_scene(sc, morton_order(sc))
        train = ellipse_path_cameras(s(300), 4001, 640, 480)
        cand = room_candidates(s(512), 4002, sc.extent, 320, 240)
        return Workload(name, sc, train, cand, 3)
    raise ValueError(f"unknown workload {name!r}")

"""Seeded synthetic depth-camera scenes (input generator only).

This module renders z-depth images of axis-aligned solids with an analytic
FP64 ray/box caster, adds the depth-dependent sensor noise of the workload
descriptions, and packs everything the ray-MRF method consumes: depth frames,
camera-to-world poses, pinhole intrinsics, the voxel grid, the 64-bin
Gaussian-sigma table and the truncation parameters.  It holds none of the
method's arithmetic (no voxel traversal, no potentials, no messages) and is
shared by the FP64 oracle tests, the GPU parity tests and the benchmark.

Conventions
-----------
* World frame in metres, voxel (i, j, k) covers
  [o + i h, o + (i + 1) h) x ... ; linear id = i + nx (j + ny k).
* Cameras use OpenCV axes (x right, y down, z forward); ``T_wc`` maps camera
  to world, row-major 4x4.  The ray through pixel (u, v) is
  c + t R ((u - cx)/fx, (v - cy)/fy, 1), so t is z-depth.
* Depth is float32 z-depth in metres; 0 marks an invalid pixel.
* All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64).

Workloads (names used throughout the repository)
------------------------------------------------
``c1``   one 64x48 frame, 64^3 grid at 0.05 m, floor + 4 boxes, 5 sweeps.
``c2``   one 640x480 frame in a 5x5x3 m room with 20 boxes and bumpy walls,
         100x100x60 grid at 0.05 m, 10 sweeps.
``c3``   30 keyframes of 640x480 along a smooth loop in the same room,
         250x250x150 grid at 0.02 m, 10 sweeps.
``c4``   ``c3`` with 8 sweeps plus ground-truth occupancy for a BCE loss.
``fd``   32^3 grid at 0.05 m, 2 boxes, 3 frames of 64x48, 8 sweeps (small
         enough for finite differences over every parameter).
``c5``   8 independent rooms of different grids and frame counts.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

N_BINS = 64


@dataclass
class Intrinsics:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float


@dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    voxel: float
    origin: tuple = (0.0, 0.0, 0.0)

    @property
    def n_voxels(self) -> int:
        return self.nx * self.ny * self.nz


@dataclass
class BuildParams:
    """Ray validity window and truncation (frozen at build time)."""
    z_min: float = 0.1
    z_max: float = 8.0
    trunc_nsigma: float = 3.0
    trunc_c0: float = 0.001
    trunc_c2: float = 0.003
    trunc_min: float = 0.0
    table_dmax: float = 8.0
    min_ray_voxels: int = 2
    sparse_bricks: int = 0      # 1: only 8^3 bricks around the measured points carry voxels
    brick_radius: int = 1       # bricks allocated around each measured point's brick
    skip_empty_bricks: int = 0  # 1: the traversal steps over unallocated bricks a brick at a time
    group_slots_log2: int = 0   # 0: scenes grouped under 2^32 edge slots; 12..31 force smaller groups (tests)


@dataclass
class Scene:
    name: str
    depth: np.ndarray            # (F, H, W) float32, 0 = invalid
    T_wc: np.ndarray             # (F, 4, 4) float64
    intr: Intrinsics
    grid: Grid
    solids: np.ndarray           # (S, 2, 3) float64 AABBs [lo, hi)
    params: BuildParams
    sigma_table: np.ndarray      # (64,) float64, sigma at bin centres
    prior: float = 0.1
    sweeps: int = 10
    extra: dict = field(default_factory=dict)

    @property
    def n_frames(self) -> int:
        return int(self.depth.shape[0])

    @property
    def n_rays(self) -> int:
        return int(self.depth.size)

    def occupancy(self) -> np.ndarray:
        """Ground truth y_v (float32, V): 1 iff the voxel centre is inside a solid."""
        return voxel_centres_inside(self.grid, self.solids)

    def prior_logit(self) -> np.ndarray:
        return np.full(self.grid.n_voxels, math.log(self.prior / (1.0 - self.prior)),
                       dtype=np.float32)


# --------------------------------------------------------------------------
# geometry helpers (rendering only)
# --------------------------------------------------------------------------

def look_at(c, target, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """Camera-to-world pose with OpenCV axes looking from ``c`` at ``target``."""
    c = np.asarray(c, np.float64)
    f = np.asarray(target, np.float64) - c
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    T = np.eye(4)
    T[:3, 0], T[:3, 1], T[:3, 2], T[:3, 3] = r, d, f, c
    return T


def pixel_rays(intr: Intrinsics, T: np.ndarray):
    """Origin (3,) and z-depth-parameterised directions (H, W, 3)."""
    u = np.arange(intr.width, dtype=np.float64)
    v = np.arange(intr.height, dtype=np.float64)
    dx = (u - intr.cx) / intr.fx
    dy = (v - intr.cy) / intr.fy
    cam = np.stack(np.broadcast_arrays(dx[None, :], dy[:, None], np.ones((1, 1))), -1)
    w = cam @ T[:3, :3].T
    return T[:3, 3].copy(), w


def ray_box_hits(c, w, solids):
    """First-hit z-depth of rays c + t w against AABBs; +inf on a miss.

    Returns (t_hit, solid_index) with solid_index = -1 on a miss.
    """
    shape = w.shape[:-1]
    w2 = w.reshape(-1, 3)
    best = np.full(w2.shape[0], np.inf)
    idx = np.full(w2.shape[0], -1, dtype=np.int64)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / w2
    for s, (lo, hi) in enumerate(solids):
        tn = np.full(w2.shape[0], -np.inf)
        tf = np.full(w2.shape[0], np.inf)
        ok = np.ones(w2.shape[0], dtype=bool)
        for a in range(3):
            zero = w2[:, a] == 0.0
            with np.errstate(invalid="ignore", over="ignore"):
                t0 = (lo[a] - c[a]) * inv[:, a]
                t1 = (hi[a] - c[a]) * inv[:, a]
            tmin = np.where(zero, -np.inf, np.minimum(t0, t1))
            tmax = np.where(zero, np.inf, np.maximum(t0, t1))
            inside = (c[a] >= lo[a]) & (c[a] < hi[a])
            ok &= ~zero | inside
            tn = np.maximum(tn, tmin)
            tf = np.minimum(tf, tmax)
        hit = ok & (tn <= tf) & (tf > 0.0)
        th = np.where(tn > 0.0, tn, 0.0)
        better = hit & (th < best)
        best = np.where(better, th, best)
        idx = np.where(better, s, idx)
    return best.reshape(shape), idx.reshape(shape)


def voxel_centres_inside(grid: Grid, solids) -> np.ndarray:
    o = np.asarray(grid.origin, np.float64)
    xs = o[0] + (np.arange(grid.nx) + 0.5) * grid.voxel
    ys = o[1] + (np.arange(grid.ny) + 0.5) * grid.voxel
    zs = o[2] + (np.arange(grid.nz) + 0.5) * grid.voxel
    occ = np.zeros((grid.nz, grid.ny, grid.nx), dtype=bool)
    for lo, hi in solids:
        ix = (xs >= lo[0]) & (xs < hi[0])
        iy = (ys >= lo[1]) & (ys < hi[1])
        iz = (zs >= lo[2]) & (zs < hi[2])
        occ |= iz[:, None, None] & iy[None, :, None] & ix[None, None, :]
    return occ.reshape(-1).astype(np.float32)


def sigma_table(kind: str, dmax: float) -> np.ndarray:
    """64-bin Gaussian-sigma table at bin centres."""
    d = (np.arange(N_BINS) + 0.5) * (dmax / N_BINS)
    if kind == "quad_c1":
        return np.maximum(0.0025 * d * d, 1e-3)
    if kind == "room":
        return 0.001 + 0.003 * d * d
    raise ValueError(kind)


def bias_table(sigma: np.ndarray, seed: int) -> np.ndarray:
    """64-bin depth bias table (metres) for a learnt sensor model: a smooth
    trend of a quarter sigma that changes sign over the range, plus a seeded
    tenth-of-sigma wobble per bin, so every bin carries its own value."""
    rng = np.random.default_rng(seed)
    sigma = np.asarray(sigma, np.float64)
    trend = np.cos(np.linspace(0.0, np.pi, N_BINS))
    return sigma * (0.25 * trend + 0.1 * rng.standard_normal(N_BINS))


# --------------------------------------------------------------------------
# noise
# --------------------------------------------------------------------------

def _clean(t_true, z_min, z_max):
    """Noise-free z-depth of the rendered surfaces (0 where nothing is hit or
    outside the sensor's window): the reference the paper scores maps against."""
    hit = np.isfinite(t_true) & (t_true > 0)
    z = np.where(hit, t_true, 0.0)
    return np.where(hit & (z >= z_min) & (z <= z_max), z, 0.0).astype(np.float32)


def _noisy(rng, t_true, sigma_fn, z_min, z_max, outlier_frac):
    z = np.where(np.isfinite(t_true), t_true, 0.0)
    hit = np.isfinite(t_true) & (t_true > 0)
    n = rng.standard_normal(z.shape)
    z = np.where(hit, z + n * sigma_fn(z), 0.0)
    if outlier_frac > 0:
        pick = rng.random(z.shape) < outlier_frac
        uni = rng.uniform(z_min, z_max, z.shape)
        z = np.where(hit & pick, uni, z)
    valid = hit & (z >= z_min) & (z <= z_max)
    return np.where(valid, z, 0.0).astype(np.float32)


# --------------------------------------------------------------------------
# rooms with bumpy walls
# --------------------------------------------------------------------------

def _bump_field(rng):
    """Smooth seeded field b(p) on a wall face, |b| <= 1 cm."""
    k = rng.uniform(2.0, 9.0, size=(3, 2))
    ph = rng.uniform(0, 2 * math.pi, size=(3, 2))
    amp = rng.uniform(0.3, 1.0, size=3)
    amp = 0.01 * amp / amp.sum()

    def f(p, q):
        out = np.zeros_like(p)
        for i in range(3):
            out += amp[i] * np.sin(k[i, 0] * p + ph[i, 0]) * np.sin(k[i, 1] * q + ph[i, 1])
        return out
    return f


def _room_solids(L, rng, n_boxes, path=None, clearance=0.4, thick=0.1,
                 box_xy=(0.1, 0.8), box_h=(0.1, 1.5)):
    Lx, Ly, Lz = L
    walls = [
        ((0, 0, 0), (Lx, Ly, thick)),                  # floor
        ((0, 0, Lz - thick), (Lx, Ly, Lz)),            # ceiling
        ((0, 0, 0), (thick, Ly, Lz)),                  # x- wall
        ((Lx - thick, 0, 0), (Lx, Ly, Lz)),            # x+ wall
        ((0, 0, 0), (Lx, thick, Lz)),                  # y- wall
        ((0, Ly - thick, 0), (Lx, Ly, Lz)),            # y+ wall
    ]
    # inward normal axis/sign of the inner face of each wall (floor/ceiling flat)
    faces = [None, None, (0, +1), (0, -1), (1, +1), (1, -1)]
    boxes = []
    margin = 0.3
    tries = 0
    while len(boxes) < n_boxes and tries < 10000:
        tries += 1
        sx, sy = rng.uniform(*box_xy, size=2)
        sz = rng.uniform(*box_h)
        cx = rng.uniform(margin + sx / 2, Lx - margin - sx / 2)
        cy = rng.uniform(margin + sy / 2, Ly - margin - sy / 2)
        lo = np.array([cx - sx / 2, cy - sy / 2, thick])
        hi = np.array([cx + sx / 2, cy + sy / 2, min(thick + sz, Lz - thick - 0.05)])
        if path is not None:
            # reject boxes within `clearance` of any camera centre
            q = np.clip(path, lo, hi)
            if np.min(np.linalg.norm(q - path, axis=1)) < clearance:
                continue
        boxes.append((tuple(lo), tuple(hi)))
    solids = np.array(walls + boxes, dtype=np.float64)
    return solids, faces + [None] * len(boxes)


def _render_room(rng, intr, poses, solids, faces, sigma_fn, z_min, z_max, outlier_frac):
    bumps = [(_bump_field(rng) if fc is not None else None) for fc in faces]
    depth = np.zeros((len(poses), intr.height, intr.width), np.float32)
    clean = np.zeros_like(depth)
    for f, T in enumerate(poses):
        c, w = pixel_rays(intr, T)
        t, idx = ray_box_hits(c, w, solids)
        # bumpy inner wall faces: shift the face along its inward normal by b(p)
        for s, fc in enumerate(faces):
            if fc is None:
                continue
            a, sgn = fc
            m = idx == s
            if not np.any(m):
                continue
            p = c[None, :] + t[m][:, None] * w[m]
            oth = [x for x in range(3) if x != a]
            b = bumps[s](p[:, oth[0]], p[:, oth[1]])
            nw = sgn * w[m][:, a]
            with np.errstate(divide="ignore", invalid="ignore"):
                dt = np.where(nw < -1e-3, b / nw, 0.0)
            t[m] = t[m] + np.clip(dt, -0.05, 0.05)
        clean[f] = _clean(t, z_min, z_max)
        depth[f] = _noisy(rng, t, sigma_fn, z_min, z_max, outlier_frac)
    return depth, clean


def _room_sigma(d):
    return 0.001 + 0.003 * d * d


ROOM_INTR = Intrinsics(640, 480, 525.0, 525.0, 319.5, 239.5)
SMALL_INTR = Intrinsics(64, 48, 60.0, 60.0, 32.0, 24.0)


def _room_params():
    return BuildParams(z_min=0.1, z_max=8.0, trunc_nsigma=3.0, trunc_c0=0.001,
                       trunc_c2=0.003, trunc_min=0.0, table_dmax=8.0, min_ray_voxels=2)


def loop_trajectory(rng, n_frames, L, radius=1.5, height=1.3, target_z=1.0):
    """Smooth closed-ish loop of look-at poses around the room centre."""
    Lx, Ly, _ = L
    phi0, phi1 = rng.uniform(0, 2 * math.pi, size=2)
    poses, centres = [], []
    for k in range(n_frames):
        s = k / max(n_frames - 1, 1)
        a = phi0 + 1.6 * math.pi * s
        c = np.array([Lx / 2 + radius * math.cos(a), Ly / 2 + radius * math.sin(a),
                      height + 0.15 * math.sin(2 * math.pi * s + phi1)])
        tgt = np.array([Lx / 2, Ly / 2, target_z]) + rng.uniform(-0.2, 0.2, size=3) / math.sqrt(3)
        poses.append(look_at(c, tgt))
        centres.append(c)
    return poses, np.array(centres)


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------

def make_c1(seed: int = 1000) -> Scene:
    """64x48 frame, camera at (1.6, 1.6, 0.2) looking +z, floor slab + 4 boxes."""
    rng = np.random.default_rng(seed)
    grid = Grid(64, 64, 64, 0.05)
    ext = 64 * 0.05
    floor = ((0.0, 2.4, 0.0), (ext, 2.5, ext))
    solids = [floor]
    for _ in range(4):
        s = rng.uniform(0.2, 0.6, size=3)
        cx = rng.uniform(0.5, 2.7)
        cz = rng.uniform(1.0, 2.8)
        solids.append(((cx - s[0] / 2, 2.4 - s[1], cz - s[2] / 2),
                       (cx + s[0] / 2, 2.4, cz + s[2] / 2)))
    solids = np.array(solids, np.float64)
    T = np.eye(4)
    T[:3, 3] = (1.6, 1.6, 0.2)
    intr = SMALL_INTR
    c, w = pixel_rays(intr, T)
    t, _ = ray_box_hits(c, w, solids)
    p = BuildParams(z_min=0.1, z_max=3.0, trunc_nsigma=3.0, trunc_c0=0.0, trunc_c2=0.0025,
                    trunc_min=1e-3, table_dmax=3.2, min_ray_voxels=2)
    depth = _noisy(rng, t, lambda d: 0.0025 * d * d, p.z_min, p.z_max, 0.0)[None]
    return Scene("c1", depth, T[None].copy(), intr, grid, solids, p,
                 sigma_table("quad_c1", p.table_dmax), 0.1, 5, {"clean_depth": _clean(t, p.z_min, p.z_max)[None]})


def make_c2(seed: int = 2000) -> Scene:
    """640x480 frame in a 5x5x3 m room, 20 boxes, bumpy walls, 1% outliers."""
    rng = np.random.default_rng(seed)
    L = (5.0, 5.0, 3.0)
    grid = Grid(100, 100, 60, 0.05)
    cam = np.array([2.5, 0.6, 1.4])
    solids, faces = _room_solids(L, rng, 20, path=cam[None], clearance=0.4)
    pitch = math.radians(10.0)
    T = look_at(cam, cam + np.array([0.0, math.cos(pitch), -math.sin(pitch)]))
    p = _room_params()
    depth, clean = _render_room(rng, ROOM_INTR, [T], solids, faces, _room_sigma, p.z_min, p.z_max, 0.01)
    return Scene("c2", depth, T[None].copy(), ROOM_INTR, grid, solids, p,
                 sigma_table("room", p.table_dmax), 0.1, 10, {"clean_depth": clean})


def make_room_batch(name, seed, grid: Grid, n_frames, sweeps, n_boxes=20,
                    intr: Intrinsics = ROOM_INTR) -> Scene:
    rng = np.random.default_rng(seed)
    L = (grid.nx * grid.voxel, grid.ny * grid.voxel, grid.nz * grid.voxel)
    radius = 0.3 * min(L[0], L[1])
    height = min(1.3, 0.45 * L[2])
    poses, centres = loop_trajectory(rng, n_frames, L, radius=radius, height=height,
                                     target_z=min(1.0, 0.35 * L[2]))
    solids, faces = _room_solids(L, rng, n_boxes, path=centres, clearance=0.4,
                                 box_h=(0.1, min(1.5, 0.5 * L[2])))
    p = _room_params()
    depth, clean = _render_room(rng, intr, poses, solids, faces, _room_sigma, p.z_min, p.z_max, 0.01)
    return Scene(name, depth, np.array(poses), intr, grid, solids, p,
                 sigma_table("room", p.table_dmax), 0.1, sweeps, {"clean_depth": clean})


def make_c3(seed: int = 3000, n_frames: int = 30) -> Scene:
    """30 keyframes of 640x480 along a loop, 250x250x150 grid at 0.02 m."""
    return make_room_batch("c3", seed, Grid(250, 250, 150, 0.02), n_frames, 10)


def make_c4(seed: int = 3000, n_frames: int = 30) -> Scene:
    """The c3 batch with 8 unrolled sweeps (differentiable workload)."""
    s = make_room_batch("c4", seed, Grid(250, 250, 150, 0.02), n_frames, 8)
    return s


def make_fd(seed: int = 4000) -> Scene:
    """32^3 grid at 0.05 m, floor + 2 boxes, 3 frames of 64x48, 8 sweeps."""
    rng = np.random.default_rng(seed)
    grid = Grid(32, 32, 32, 0.05)
    ext = 32 * 0.05
    solids = [((0.0, 0.0, 0.0), (ext, ext, 0.1))]
    for _ in range(2):
        s = rng.uniform(0.15, 0.35, size=3)
        cx, cy = rng.uniform(0.5, 1.1, size=2)
        solids.append(((cx - s[0] / 2, cy - s[1] / 2, 0.1), (cx + s[0] / 2, cy + s[1] / 2, 0.1 + s[2])))
    solids = np.array(solids, np.float64)
    poses = []
    phi = rng.uniform(0, 2 * math.pi)
    for k in range(3):
        a = phi + 2 * math.pi * k / 3
        c = (0.8 + 0.6 * math.cos(a), 0.8 + 0.6 * math.sin(a), 1.2)
        poses.append(look_at(c, (0.8, 0.8, 0.25)))
    intr = SMALL_INTR
    p = BuildParams(z_min=0.1, z_max=3.0, trunc_nsigma=3.0, trunc_c0=0.0, trunc_c2=0.0025,
                    trunc_min=1e-3, table_dmax=3.2, min_ray_voxels=2)
    depth = np.zeros((3, intr.height, intr.width), np.float32)
    clean = np.zeros_like(depth)
    for f, T in enumerate(poses):
        c, w = pixel_rays(intr, T)
        t, _ = ray_box_hits(c, w, solids)
        clean[f] = _clean(t, p.z_min, p.z_max)
        depth[f] = _noisy(rng, t, lambda d: np.maximum(0.0025 * d * d, 2e-3), p.z_min, p.z_max, 0.0)
    return Scene("fd", depth, np.array(poses), intr, grid, solids, p,
                 sigma_table("quad_c1", p.table_dmax), 0.1, 8, {"clean_depth": clean})


C5_LAYOUT = [  # (grid, voxel size, frames)
    ((64, 64, 64), 0.05, 120),
    ((100, 100, 60), 0.05, 20),
    ((128, 128, 64), 0.04, 10),
    ((160, 160, 96), 0.03125, 10),
    ((200, 200, 120), 0.025, 10),
    ((250, 250, 150), 0.02, 10),
    ((320, 320, 150), 0.015625, 10),
    ((400, 400, 150), 0.0125, 10),
]


def make_c5(frame_scale: float = 1.0, scenes=None) -> list:
    """Eight independent rooms; ``frame_scale`` shrinks frame counts to fit memory."""
    out = []
    for i, (g, h, nf) in enumerate(C5_LAYOUT):
        if scenes is not None and i not in scenes:
            continue
        nf = max(1, int(round(nf * frame_scale)))
        out.append(make_room_batch(f"c5s{i}", 5000 + i, Grid(*g, h), nf, 10))
    return out


def make(name: str, **kw):
    return {"c1": make_c1, "c2": make_c2, "c3": make_c3, "c4": make_c4, "fd": make_fd,
            "c5": make_c5}[name](**kw)


def random_scene(seed: int, grid=(16, 16, 16), voxel=0.1, n_frames=2, intr=None,
                 n_boxes=3, sweeps=5) -> Scene:
    """Small randomised scene for property tests (random poses inside the grid)."""
    rng = np.random.default_rng(seed)
    g = Grid(*grid, voxel)
    L = np.array(grid, np.float64) * voxel
    solids = [((0.0, 0.0, 0.0), (L[0], L[1], 0.5 * voxel + 0.3 * voxel))]
    for _ in range(n_boxes):
        s = rng.uniform(0.1, 0.3, size=3) * L
        cxy = rng.uniform(0.2, 0.8, size=2) * L[:2]
        solids.append(((cxy[0] - s[0] / 2, cxy[1] - s[1] / 2, 0.0),
                       (cxy[0] + s[0] / 2, cxy[1] + s[1] / 2, s[2])))
    solids = np.array(solids, np.float64)
    intr = intr or Intrinsics(24, 18, 20.0, 20.0, 11.5, 8.5)
    poses = []
    for _ in range(n_frames):
        c = rng.uniform(0.15, 0.85, size=3) * L
        c[2] = rng.uniform(0.5, 0.9) * L[2]
        tgt = rng.uniform(0.3, 0.7, size=3) * L
        tgt[2] = 0.2 * L[2]
        poses.append(look_at(c, tgt))
    p = BuildParams(z_min=0.05, z_max=float(np.linalg.norm(L)), trunc_nsigma=3.0, trunc_c0=0.005,
                    trunc_c2=0.01, trunc_min=0.0, table_dmax=float(np.linalg.norm(L)),
                    min_ray_voxels=2)
    depth = np.zeros((n_frames, intr.height, intr.width), np.float32)
    for f, T in enumerate(poses):
        c, w = pixel_rays(intr, T)
        t, _ = ray_box_hits(c, w, solids)
        depth[f] = _noisy(rng, t, lambda d: 0.005 + 0.01 * d * d, p.z_min, p.z_max, 0.02)
    tab = 0.005 + 0.01 * ((np.arange(N_BINS) + 0.5) * (p.table_dmax / N_BINS)) ** 2
    return Scene(f"rand{seed}", depth, np.array(poses), intr, g, solids, p, tab, 0.1, sweeps)

"""Seeded synthetic inputs: Gaussian sets, block scenes and pinhole cameras.

This module only draws random numbers and builds cameras; it holds none of the
rendering or level-of-detail arithmetic.  Both the GPU path and the CPU oracle
are fed from here, so every test and benchmark input is reproducible from a seed.

Gaussian sets are structure-of-arrays float32 (the layout the rasterizer reads):
    means  [3, N]      world position (x, y, z), metres
    scales [3, N]      per-axis standard deviation (> 0)
    quats  [4, N]      rotation quaternion (w, x, y, z), unit norm
    opac   [N]         opacity in (0, 1)
    sh     [16, 3, N]  degree-3 real SH coefficients, coefficient-major, then RGB

Workload shapes follow the paper's evaluation (Sec. 4.1: aerial city views,
1600 px wide images, camera heights 150-500 m; Sec. 3.3: a block grid with three
detail levels).  The paper's MatrixCity scenes are not available, so these
synthetic city-shaped scenes stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------
@dataclass
class Camera:
    """Pinhole camera, world->camera rotation R (row-major) and translation t.

    Camera axes: x right, y down, z forward.  A world point p maps to
    p_cam = R p + t; the pixel centre of pixel (i, j) is (i + 0.5, j + 0.5).
    """
    R: np.ndarray
    t: np.ndarray
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    znear: float = 0.2

    @property
    def center(self) -> np.ndarray:
        return -self.R.T @ self.t


def look_camera(center, yaw, pitch, width, height, fov_x_deg=60.0, znear=0.2) -> Camera:
    """Camera at `center` with heading `yaw` (radians, from +x toward +y in the
    world xy plane) and `pitch` (radians, negative looks down); z is world up.
    The field of view is horizontal; fy = fx; principal point at the image centre.
    """
    c = np.asarray(center, dtype=np.float64)
    hd = np.array([math.cos(yaw), math.sin(yaw), 0.0])
    fwd = math.cos(pitch) * hd + np.array([0.0, 0.0, math.sin(pitch)])
    fwd /= np.linalg.norm(fwd)
    right = np.array([math.sin(yaw), -math.cos(yaw), 0.0])
    down = np.cross(fwd, right)
    down /= np.linalg.norm(down)
    R = np.stack([right, down, fwd])
    t = -R @ c
    fx = (0.5 * width) / math.tan(math.radians(0.5 * fov_x_deg))
    return Camera(R=R, t=t, fx=fx, fy=fx, cx=0.5 * width, cy=0.5 * height,
                  width=int(width), height=int(height), znear=znear)


def axis_camera(width=256, height=256, dist=3.0, fov_x_deg=60.0) -> Camera:
    """Identity-rotation camera at (0, 0, -dist) looking along +z."""
    fx = (0.5 * width) / math.tan(math.radians(0.5 * fov_x_deg))
    return Camera(R=np.eye(3), t=np.array([0.0, 0.0, dist]), fx=fx, fy=fx,
                  cx=0.5 * width, cy=0.5 * height, width=width, height=height)


# --------------------------------------------------------------------------
# Gaussian sets
# --------------------------------------------------------------------------
@dataclass
class GaussianSet:
    means: np.ndarray
    scales: np.ndarray
    quats: np.ndarray
    opac: np.ndarray
    sh: np.ndarray

    @property
    def n(self) -> int:
        return int(self.opac.shape[0])

    def subset(self, idx) -> "GaussianSet":
        return GaussianSet(self.means[:, idx], self.scales[:, idx], self.quats[:, idx],
                           self.opac[idx], self.sh[:, :, idx])

    def astuple(self):
        return (self.means, self.scales, self.quats, self.opac, self.sh)


def draw_attributes(rng: np.random.Generator, n: int, log_scale_mu=-3.0, log_scale_sd=0.5,
                    sh_sd=0.3):
    """Scales, rotations, opacities and SH drawn in that order."""
    log_s = rng.normal(log_scale_mu, log_scale_sd, size=(3, n))
    scales = np.exp(log_s).astype(np.float32)
    q = rng.standard_normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    quats = q.astype(np.float32)
    logit = rng.standard_normal(size=n)
    opac = (1.0 / (1.0 + np.exp(-logit))).astype(np.float32)
    sh = rng.standard_normal(size=(16, 3, n), dtype=np.float32)
    sh *= np.float32(sh_sd)
    return scales, quats, opac, sh


def cube_gaussians(n=4096, seed=0) -> GaussianSet:
    """Means uniform in [-1, 1]^3 plus the standard attribute draws."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, size=(3, n)).astype(np.float32)
    scales, quats, opac, sh = draw_attributes(rng, n)
    return GaussianSet(means, scales, quats, opac, sh)


def small_render_case(n=4096, seed=0, width=256, height=256):
    """Plain forward render: n Gaussians in [-1,1]^3, camera at z=-3, fov 60 deg."""
    return cube_gaussians(n, seed), axis_camera(width, height)


def box_gaussians(n, seed, extent=((-100.0, 100.0), (-100.0, 100.0), (0.0, 40.0))) -> GaussianSet:
    rng = np.random.default_rng(seed)
    lo = np.array([e[0] for e in extent])[:, None]
    hi = np.array([e[1] for e in extent])[:, None]
    means = (lo + (hi - lo) * rng.uniform(size=(3, n))).astype(np.float32)
    scales, quats, opac, sh = draw_attributes(rng, n)
    return GaussianSet(means, scales, quats, opac, sh)


def single_view_training_case(n=1_000_000, seed=1, width=1920, height=1080):
    """Means over a 200 x 200 x 40 m box; camera 60 m up looking 45 deg down."""
    g = box_gaussians(n, seed)
    cam = look_camera((0.0, -100.0, 60.0), yaw=math.pi / 2, pitch=-math.pi / 4,
                      width=width, height=height)
    rng = np.random.default_rng(seed + 1000)
    target = rng.uniform(size=(3, height, width)).astype(np.float32)
    return g, cam, target


# --------------------------------------------------------------------------
# city-shaped scenes split into an xy block grid with nested detail levels
# --------------------------------------------------------------------------
def city_points(rng: np.random.Generator, n: int, x0: float, y0: float, side_x: float,
                side_y: float, lot=40.0, footprint=25.0, floater_top=300.0):
    """Means of a synthetic city: 40 % ground, 0.5 % floaters, the rest on the
    walls and roofs of one box building per lot (area weighted)."""
    n_ground = int(round(0.40 * n))
    n_float = int(round(0.005 * n))
    n_bld = n - n_ground - n_float
    nlx = max(1, int(side_x // lot))
    nly = max(1, int(side_y // lot))
    h = np.clip(rng.lognormal(math.log(20.0), 0.6, size=nlx * nly), 5.0, 150.0)
    lx = np.repeat(np.arange(nlx), nly)
    ly = np.tile(np.arange(nly), nlx)
    bx0 = x0 + lot * lx + 0.5 * (lot - footprint)
    by0 = y0 + lot * ly + 0.5 * (lot - footprint)
    wall = footprint * h
    roof = footprint * footprint
    area = 4.0 * wall + roof
    cdf = np.cumsum(area)
    b = np.searchsorted(cdf, rng.uniform(0.0, cdf[-1], size=n_bld), side="right")
    b = np.minimum(b, len(area) - 1)
    face_u = rng.uniform(size=n_bld) * area[b]
    s = rng.uniform(size=n_bld)
    t = rng.uniform(size=n_bld)
    px = np.empty(n_bld)
    py = np.empty(n_bld)
    pz = np.empty(n_bld)
    on_roof = face_u < roof
    px[on_roof] = bx0[b[on_roof]] + footprint * s[on_roof]
    py[on_roof] = by0[b[on_roof]] + footprint * t[on_roof]
    pz[on_roof] = h[b[on_roof]]
    w = ~on_roof
    face = np.minimum(((face_u[w] - roof) // wall[b[w]]).astype(np.int64), 3)
    along = footprint * s[w]
    up = h[b[w]] * t[w]
    fx = np.where(face == 0, along, np.where(face == 1, footprint, np.where(face == 2, footprint - along, 0.0)))
    fy = np.where(face == 0, 0.0, np.where(face == 1, along, np.where(face == 2, footprint, footprint - along)))
    px[w] = bx0[b[w]] + fx
    py[w] = by0[b[w]] + fy
    pz[w] = up
    gx = x0 + side_x * rng.uniform(size=n_ground)
    gy = y0 + side_y * rng.uniform(size=n_ground)
    gz = rng.uniform(0.0, 0.5, size=n_ground)
    fxl = x0 + side_x * rng.uniform(size=n_float)
    fyl = y0 + side_y * rng.uniform(size=n_float)
    fzl = rng.uniform(0.0, floater_top, size=n_float)
    means = np.stack([np.concatenate([gx, px, fxl]),
                      np.concatenate([gy, py, fyl]),
                      np.concatenate([gz, pz, fzl])])
    perm = rng.permutation(n)
    return means[:, perm]


@dataclass
class BlockScene:
    """Gaussians split into an xy grid of blocks, each stored at several detail levels.

    levels[l] is a GaussianSet; level 0 is the coarsest, level L-1 the finest.
    Within each level, block b occupies [lvl_off[b, l], lvl_off[b, l] + lvl_cnt[b, l]).
    cells[b] = (x0, x1, y0, y1) is the half-open xy cell of block b.
    """
    levels: list
    lvl_off: np.ndarray
    lvl_cnt: np.ndarray
    cells: np.ndarray
    finest_block_means: list = field(default_factory=list)

    @property
    def n_blocks(self) -> int:
        return int(self.cells.shape[0])

    @property
    def n_levels(self) -> int:
        return len(self.levels)


def block_scene_from_finest(fine: GaussianSet, block_id: np.ndarray, cells: np.ndarray, u: np.ndarray,
                            fractions=(0.30, 0.50, 1.00), coarse_scale=1.3) -> BlockScene:
    """Sort Gaussians by block (stable), then derive nested level subsets:
    a Gaussian belongs to level l if its uniform draw u < fractions[l]; levels
    below the finest have their scales multiplied by `coarse_scale`."""
    order = np.argsort(block_id, kind="stable")
    fine = fine.subset(order)
    block_id = block_id[order]
    u = u[order]
    B = cells.shape[0]
    L = len(fractions)
    lvl_off = np.zeros((B, L), np.int64)
    lvl_cnt = np.zeros((B, L), np.int64)
    levels = []
    for l, frac in enumerate(fractions):
        if frac >= 1.0:
            idx = np.arange(fine.n)
            lev = fine
        else:
            idx = np.nonzero(u < frac)[0]
            lev = fine.subset(idx)
            lev.scales = (lev.scales * np.float32(coarse_scale)).astype(np.float32)
        cnt = np.bincount(block_id[idx], minlength=B)
        lvl_cnt[:, l] = cnt
        lvl_off[:, l] = np.concatenate([[0], np.cumsum(cnt)[:-1]])
        levels.append(lev)
    return BlockScene(levels=levels, lvl_off=lvl_off, lvl_cnt=lvl_cnt, cells=cells)


def grid_cells(x0, y0, cell, nx, ny):
    cells = np.zeros((nx * ny, 4))
    for by in range(ny):
        for bx in range(nx):
            b = by * nx + bx
            cells[b] = (x0 + cell * bx, x0 + cell * (bx + 1), y0 + cell * by, y0 + cell * (by + 1))
    return cells


def city_finest(n=20_000_000, seed=2, area_m2=1.5e6, grid=(8, 8)):
    """Finest level of the synthetic city, sorted by block (row-major xy cells).

    Returns (GaussianSet, block_id [n], u [n], cells [B, 4]); u is the uniform
    draw that decides membership of the coarser nested levels.  Centres are
    drawn and sorted first, attributes are drawn afterwards in block order, so
    no large array is permuted."""
    rng = np.random.default_rng(seed)
    side = math.sqrt(area_m2)
    x0 = y0 = -0.5 * side
    nx, ny = grid
    cell = side / nx
    means = city_points(rng, n, x0, y0, side, side)
    bx = np.clip(np.floor((means[0] - x0) / cell), 0, nx - 1).astype(np.int64)
    by = np.clip(np.floor((means[1] - y0) / cell), 0, ny - 1).astype(np.int64)
    block_id = by * nx + bx
    order = block_morton_order(means, block_id, x0, y0, cell, bx, by)
    means = np.ascontiguousarray(means[:, order], dtype=np.float32)
    block_id = block_id[order]
    scales, quats, opac, sh = draw_attributes(rng, n)
    u = rng.uniform(size=n)
    cells = grid_cells(x0, y0, cell, nx, ny)
    return GaussianSet(means, scales, quats, opac, sh), block_id, u, cells


def _spread_bits10(v):
    """Interleave the low 10 bits of v with two zero bits between each."""
    v = v.astype(np.int64) & 0x3FF
    v = (v | (v << 16)) & 0x030000FF
    v = (v | (v << 8)) & 0x0300F00F
    v = (v | (v << 4)) & 0x030C30C3
    v = (v | (v << 2)) & 0x09249249
    return v


def block_morton_order(means, block_id, x0, y0, cell, bx, by, z_top=160.0):
    """Storage order: by block, then by the 30-bit Morton code of the centre
    inside its block (10 bits per axis), so Gaussians that are culled together
    share cache lines.  This is a layout choice only; it changes no result
    except which of two Gaussians at exactly equal depth is drawn first."""
    q = lambda a: np.clip(a * 1024.0, 0, 1023).astype(np.int64)
    ux = q((means[0] - (x0 + bx * cell)) / cell)
    uy = q((means[1] - (y0 + by * cell)) / cell)
    uz = q(means[2] / z_top)
    code = _spread_bits10(ux) | (_spread_bits10(uy) << 1) | (_spread_bits10(uz) << 2)
    return np.argsort((block_id.astype(np.int64) << 30) | code, kind="stable")


def city_block_scene(n=20_000_000, seed=2, area_m2=1.5e6, grid=(8, 8),
                     fractions=(0.30, 0.50, 1.00)) -> BlockScene:
    """Square city of `area_m2`, split into grid[0] x grid[1] blocks, n finest Gaussians."""
    fine, block_id, u, cells = city_finest(n, seed, area_m2, grid)
    return block_scene_from_finest(fine, block_id, cells, u, fractions)


def level_membership(block_id, u, n_blocks, fractions=(0.30, 0.50, 1.00)):
    """For each level: the (sorted) finest-level indices it keeps, and per-block counts."""
    out = []
    for frac in fractions:
        idx = np.arange(block_id.shape[0]) if frac >= 1.0 else np.nonzero(u < frac)[0]
        out.append((idx, np.bincount(block_id[idx], minlength=n_blocks)))
    return out


def city_views(seed=2, area_m2=1.5e6, heights=(50.0, 150.0, 400.0), n_xy=8,
               pitches_deg=(-90.0, -45.0), width=1600, height=900):
    """Cameras over the central 80 % of the city at each height and pitch."""
    rng = np.random.default_rng(seed + 7)
    half = 0.5 * math.sqrt(area_m2) * 0.8
    cams = []
    for h in heights:
        xy = rng.uniform(-half, half, size=(n_xy, 2))
        yaw = rng.uniform(0.0, 2 * math.pi, size=n_xy)
        for p in pitches_deg:
            for k in range(n_xy):
                cams.append(look_camera((xy[k, 0], xy[k, 1], h), yaw[k], math.radians(p), width, height))
    return cams


def orbit_views(center, n_views=16, radius=60.0, height=60.0, width=1600, h_px=900):
    """Cameras on a circle of `radius` at `height`, all looking at `center` (z = 0)."""
    cams = []
    for k in range(n_views):
        a = 2 * math.pi * k / n_views
        pos = (center[0] + radius * math.cos(a), center[1] + radius * math.sin(a), height)
        yaw = math.atan2(center[1] - pos[1], center[0] - pos[0])
        pitch = -math.atan2(height, radius)
        cams.append(look_camera(pos, yaw, pitch, width, h_px))
    return cams


def uneven_finest(seed=4, grid=(8, 4), cell=153.1, n_min=200_000, n_max=3_000_000):
    """Finest level of the uneven scene (blocks with log-uniform Gaussian counts),
    in block order, and 4 views per block: (fine, block_id, u, cells, cams)."""
    rng = np.random.default_rng(seed)
    nx, ny = grid
    counts = np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=nx * ny)).astype(np.int64)
    x0 = -0.5 * nx * cell
    y0 = -0.5 * ny * cell
    cells = grid_cells(x0, y0, cell, nx, ny)
    parts = []
    for b in range(nx * ny):
        parts.append(city_points(rng, int(counts[b]), cells[b, 0], cells[b, 2], cell, cell))
    means = np.concatenate(parts, axis=1).astype(np.float32)
    del parts
    n = means.shape[1]
    block_id = np.repeat(np.arange(nx * ny), counts)
    scales, quats, opac, sh = draw_attributes(rng, n)
    u = rng.uniform(size=n)
    cams = []
    for b in range(nx * ny):
        for _ in range(4):
            x = rng.uniform(cells[b, 0], cells[b, 1])
            y = rng.uniform(cells[b, 2], cells[b, 3])
            h = rng.uniform(30.0, 300.0)
            pitch = math.radians(rng.uniform(-90.0, -30.0))
            yaw = rng.uniform(0.0, 2 * math.pi)
            cams.append(look_camera((x, y, h), yaw, pitch, 1280, 720))
    return GaussianSet(means, scales, quats, opac, sh), block_id, u, cells, cams


def uneven_block_scene(seed=4, grid=(8, 4), cell=153.1, n_min=200_000, n_max=3_000_000,
                       fractions=(0.30, 0.50, 1.00)):
    """Blocks with log-uniform Gaussian counts; returns the scene and 4 views per block."""
    fine, block_id, u, cells, cams = uneven_finest(seed, grid, cell, n_min, n_max)
    return block_scene_from_finest(fine, block_id, cells, u, fractions), cams

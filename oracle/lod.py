"""Block-wise level-of-detail selection, plain FP64 NumPy: TEST INFRASTRUCTURE ONLY.

Follows Sec. 3.3.2 of the paper step by step:
  1. per block, a floater-robust bounding box from the Median Absolute Deviation
     of the finest-level Gaussian centres (Eq. 6, n_MAD = 4);
  2. per (view, block), the minimum distance from the box's eight corners to the
     camera centre picks the detail level against the distance intervals;
  3. the corners in front of the camera are projected; the block is visible when
     the bounding box of those projections overlaps the screen with positive
     area (IoU > 0), or when the camera stands inside the block's xy cell;
  4. the chosen levels of the visible blocks are concatenated in block order.

Readings of points the paper leaves open (also listed in the design notes):
  * median of an even count = the lower middle element (rank floor((n-1)/2));
  * distance intervals are half-open [t_k, t_{k+1});
  * a corner counts as in front of the camera when its camera-space z > znear;
  * the block that contains the camera is the one whose half-open xy cell holds
    the camera centre;
  * levels are indexed 0 (coarsest) .. L-1 (finest); a near block gets L-1.
"""
from __future__ import annotations

import numpy as np

N_MAD = 4.0


def lower_median(x: np.ndarray) -> float:
    """Element of rank floor((n-1)/2) in ascending order."""
    s = np.sort(np.asarray(x, np.float64))
    return float(s[(s.shape[0] - 1) // 2])


def mad_bounds(means_block: np.ndarray, n_mad: float = N_MAD):
    """Eq. 6 per axis: lo = max(min p, med - n*MAD), hi = min(max p, med + n*MAD)."""
    p = np.asarray(means_block, np.float64)
    lo = np.zeros(3)
    hi = np.zeros(3)
    for ax in range(3):
        x = p[ax]
        med = lower_median(x)
        mad = lower_median(np.abs(x - med))
        lo[ax] = max(float(x.min()), med - n_mad * mad)
        hi[ax] = min(float(x.max()), med + n_mad * mad)
    return lo, hi


def scene_bounds(scene, n_mad: float = N_MAD):
    """MAD boxes of every block from its finest-level centres: lo, hi [B, 3]."""
    fine = scene.levels[-1]
    L = scene.n_levels
    B = scene.n_blocks
    lo = np.zeros((B, 3))
    hi = np.zeros((B, 3))
    for b in range(B):
        o, c = scene.lvl_off[b, L - 1], scene.lvl_cnt[b, L - 1]
        if c == 0:
            lo[b] = np.inf
            hi[b] = -np.inf
            continue
        lo[b], hi[b] = mad_bounds(fine.means[:, o:o + c], n_mad)
    return lo, hi


def camera_center(cam):
    R = np.asarray(cam.R, np.float64)
    t = np.asarray(cam.t, np.float64)
    return np.array([-((R[0, k] * t[0] + R[1, k] * t[1]) + R[2, k] * t[2]) for k in range(3)])


def corners(lo, hi):
    return np.array([[(hi if (c >> 0) & 1 else lo)[0], (hi if (c >> 1) & 1 else lo)[1],
                      (hi if (c >> 2) & 1 else lo)[2]] for c in range(8)])


def select_block(lo, hi, cell, thresholds, cam, n_levels, contraction=None):
    """Level for one (view, block): -1 if culled, else 0 (coarsest) .. n_levels-1.

    contraction: None (cell is a world xy rectangle) or (p_min, p_max) of a
    contracted partition (Sec. 3.2.2): the camera centre is then normalised and
    contracted by Eq. 2, as a Gaussian centre would be, before the cell test."""
    if not (lo[0] <= hi[0]):
        return -1  # empty block
    C = camera_center(cam)
    R = np.asarray(cam.R, np.float64).reshape(9)
    t = np.asarray(cam.t, np.float64)
    dmin2 = np.inf
    front = []
    for p in corners(lo, hi):
        d2 = ((p[0] - C[0]) * (p[0] - C[0]) + (p[1] - C[1]) * (p[1] - C[1])) + (p[2] - C[2]) * (p[2] - C[2])
        dmin2 = min(dmin2, d2)
        zc = ((R[6] * p[0] + R[7] * p[1]) + R[8] * p[2]) + t[2]
        if zc > cam.znear:
            xc = ((R[0] * p[0] + R[1] * p[1]) + R[2] * p[2]) + t[0]
            yc = ((R[3] * p[0] + R[4] * p[1]) + R[5] * p[2]) + t[1]
            rz = 1.0 / zc
            front.append((cam.fx * (xc * rz) + cam.cx, cam.fy * (yc * rz) + cam.cy))
    visible = False
    if front:
        f = np.array(front)
        umin, vmin = f.min(axis=0)
        umax, vmax = f.max(axis=0)
        # intersection of [umin, umax] x [vmin, vmax] with the screen has positive area
        visible = (min(umax, float(cam.width)) > max(umin, 0.0)) and (min(vmax, float(cam.height)) > max(vmin, 0.0))
    X, Y = C[0], C[1]
    if contraction is not None:
        from oracle import partition
        c = partition.contract(partition.normalise(C[:, None], contraction[0], contraction[1]))[:, 0]
        X, Y = c[0], c[1]
    in_cell = (cell[0] <= X < cell[1]) and (cell[2] <= Y < cell[3])
    if not (visible or in_cell):
        return -1
    level = n_levels - 1
    for tk in thresholds:
        if dmin2 >= tk * tk:
            level -= 1
    return level


def lod_select(lo, hi, cells, thresholds, cams, lvl_cnt, contraction=None):
    """level [V, B] int8 and offsets [V, B+1] int64 (exclusive prefix of chosen counts)."""
    B = cells.shape[0]
    L = lvl_cnt.shape[1]
    V = len(cams)
    level = np.full((V, B), -1, np.int8)
    offsets = np.zeros((V, B + 1), np.int64)
    for v, cam in enumerate(cams):
        for b in range(B):
            level[v, b] = select_block(lo[b], hi[b], cells[b], thresholds, cam, L, contraction)
        counts = np.array([lvl_cnt[b, level[v, b]] if level[v, b] >= 0 else 0 for b in range(B)], np.int64)
        offsets[v, 1:] = np.cumsum(counts)
    return level, offsets


def aggregate(scene, level_row):
    """Concatenate the chosen level of every selected block, in block order."""
    from types import SimpleNamespace
    parts = {k: [] for k in ("means", "scales", "quats", "opac", "sh")}
    for b, l in enumerate(level_row):
        if l < 0:
            continue
        o, c = scene.lvl_off[b, l], scene.lvl_cnt[b, l]
        lev = scene.levels[l]
        parts["means"].append(lev.means[:, o:o + c])
        parts["scales"].append(lev.scales[:, o:o + c])
        parts["quats"].append(lev.quats[:, o:o + c])
        parts["opac"].append(lev.opac[o:o + c])
        parts["sh"].append(lev.sh[:, :, o:o + c])
    if not parts["opac"]:
        return SimpleNamespace(means=np.zeros((3, 0), np.float32), scales=np.zeros((3, 0), np.float32),
                               quats=np.zeros((4, 0), np.float32), opac=np.zeros(0, np.float32),
                               sh=np.zeros((16, 3, 0), np.float32))
    return SimpleNamespace(means=np.concatenate(parts["means"], 1), scales=np.concatenate(parts["scales"], 1),
                           quats=np.concatenate(parts["quats"], 1), opac=np.concatenate(parts["opac"]),
                           sh=np.concatenate(parts["sh"], 2))


# ---------------------------------------------------------------------------
# Point-wise baseline (Sec. 3.3.2 opening, ablated in Table 5): every Gaussian
# of every level is tested on its own.  Level l keeps the Gaussians of level l
# whose centre distance to the camera centre falls in level l's interval and
# whose centre lies in the view frustum.
#
# Readings (also listed in the design notes):
#   * distance = Euclidean distance from the Gaussian centre to the camera
#     centre, same intervals and the same level numbering as the block-wise
#     selection;
#   * in the frustum: camera-space z > znear and the projected centre inside
#     the screen widened by POINT_GUARD of its size on every side (the 1.3x
#     guard band of the rasterizer's projection for a centred principal point),
#     so Gaussians centred just off screen still reach the rasterizer;
#   * the selection of view v is laid out as L segments (level 0 .. L-1), each
#     listing its Gaussians by ascending index within the level.
# ---------------------------------------------------------------------------
POINT_GUARD = 0.15


def point_levels(means, cam, thresholds, n_levels):
    """Per centre (means [3, n]): level from the distance intervals, and the
    frustum test; returns (level int array, in_frustum bool array)."""
    p = np.asarray(means, np.float64)
    C = camera_center(cam)
    R = np.asarray(cam.R, np.float64).reshape(9)
    t = np.asarray(cam.t, np.float64)
    dx, dy, dz = p[0] - C[0], p[1] - C[1], p[2] - C[2]
    d2 = (dx * dx + dy * dy) + dz * dz
    level = np.full(p.shape[1], n_levels - 1, np.int64)
    for tk in thresholds:
        level -= (d2 >= tk * tk).astype(np.int64)
    zc = ((R[6] * p[0] + R[7] * p[1]) + R[8] * p[2]) + t[2]
    xc = ((R[0] * p[0] + R[1] * p[1]) + R[2] * p[2]) + t[0]
    yc = ((R[3] * p[0] + R[4] * p[1]) + R[5] * p[2]) + t[1]
    front = zc > cam.znear
    with np.errstate(divide="ignore", invalid="ignore"):
        rz = 1.0 / zc
        u = cam.fx * (xc * rz) + cam.cx
        v = cam.fy * (yc * rz) + cam.cy
    W, H = float(cam.width), float(cam.height)
    inside = ((u > -POINT_GUARD * W) & (u < (1.0 + POINT_GUARD) * W) &
              (v > -POINT_GUARD * H) & (v < (1.0 + POINT_GUARD) * H))
    return level, front & inside


def pointwise_select(level_means, thresholds, cams):
    """level_means: list of [3, n_l] centre arrays, level 0 (coarsest) first.
    Returns offsets [V*L + 1] (int64) and gather (uint32): segment v*L + l of
    the selection holds gather[offsets[s]:offsets[s+1]], indices into level l."""
    L = len(level_means)
    parts = []
    for cam in cams:
        for l, m in enumerate(level_means):
            level, ok = point_levels(m, cam, thresholds, L)
            parts.append(np.nonzero(ok & (level == l))[0].astype(np.uint32))
    sizes = np.array([p.shape[0] for p in parts], np.int64)
    offsets = np.zeros(len(parts) + 1, np.int64)
    offsets[1:] = np.cumsum(sizes)
    gather = np.concatenate(parts) if parts else np.zeros(0, np.uint32)
    return offsets, gather


def gather_selection(level_sets, offsets, gather, view, n_levels):
    """Concatenate view `view`'s point-wise selection (level 0 first) into one
    Gaussian set with the attributes of the chosen Gaussians."""
    from types import SimpleNamespace
    parts = {k: [] for k in ("means", "scales", "quats", "opac", "sh")}
    for l in range(n_levels):
        s = view * n_levels + l
        idx = gather[offsets[s]:offsets[s + 1]].astype(np.int64)
        lev = level_sets[l]
        parts["means"].append(lev.means[:, idx])
        parts["scales"].append(lev.scales[:, idx])
        parts["quats"].append(lev.quats[:, idx])
        parts["opac"].append(lev.opac[idx])
        parts["sh"].append(lev.sh[:, :, idx])
    return SimpleNamespace(means=np.concatenate(parts["means"], 1), scales=np.concatenate(parts["scales"], 1),
                           quats=np.concatenate(parts["quats"], 1), opac=np.concatenate(parts["opac"]),
                           sh=np.concatenate(parts["sh"], 2))

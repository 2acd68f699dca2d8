"""Frame pipeline over the C ABI: device-resident scenes, frame buffers, and the
differentiable render (torch.autograd.Function).

A frame is five library calls on one stream (Sec. 3.3.2 then Sec. 3.1):
    lod_select -> preprocess -> bin_sort -> rasterize_fwd  [-> rasterize_bwd]
(lod_select_points in place of lod_select for the point-wise baseline; with
refine=True, lod_refine between lod_select and preprocess drops the chunks the
projection would cull whole, with identical images.)
Buffers are allocated once per capacity and reused; data-dependent sizes stay
on the device (the counts array), so a frame issues no host synchronisation
unless a capacity check is requested.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import gs

# selection mode of render_frame besides gs.GS_LOD_BLOCKWISE / gs.GS_LOD_ALL_FINEST:
# the point-wise baseline (gs_lod_select_points)
LOD_POINTWISE = "pointwise"

# ---------------------------------------------------------------------------
# scenes
# ---------------------------------------------------------------------------
@dataclass
class DeviceLevel:
    means: torch.Tensor
    scales: torch.Tensor
    quats: torch.Tensor
    opac: torch.Tensor
    sh: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.opac.shape[0])

    def struct(self) -> gs.gs_gaussians:
        return gs.gaussians_struct(self.means, self.scales, self.quats, self.opac, self.sh)

    def zeros_like(self) -> "DeviceLevel":
        """FP32 gradient buffers shaped like this level (whatever its storage precision)."""
        return DeviceLevel(*(torch.zeros(t.shape, dtype=torch.float32, device=t.device)
                             for t in (self.means, self.scales, self.quats, self.opac, self.sh)))

    def reduced(self, sh_degree: int, half: bool) -> "DeviceLevel":
        """Copy with `sh_degree` SH bands stored and, if `half`, every attribute but
        the centre stored as binary16 (the storage of a coarse detail level)."""
        k = (sh_degree + 1) ** 2
        cast = (lambda t: t.to(torch.float16).contiguous()) if half else (lambda t: t.contiguous())
        return DeviceLevel(self.means, cast(self.scales), cast(self.quats), cast(self.opac), cast(self.sh[:k]))


class DeviceScene:
    """Gaussians of every detail level plus the block table, in device memory."""

    def __init__(self, levels, lvl_off, lvl_cnt, cells=None, lo=None, hi=None, device="cuda"):
        self.levels = levels
        self.device = device
        self.lvl_off = torch.as_tensor(np.asarray(lvl_off, np.int64)).to(device)
        self.lvl_cnt = torch.as_tensor(np.asarray(lvl_cnt, np.int64)).to(device)
        self.lvl_cnt_host = np.asarray(lvl_cnt, np.int64)
        self.cells = None if cells is None else torch.as_tensor(np.asarray(cells, np.float64)).to(device)
        self.lo = None if lo is None else torch.as_tensor(np.asarray(lo, np.float64)).to(device)
        self.hi = None if hi is None else torch.as_tensor(np.asarray(hi, np.float64)).to(device)
        self.contraction = None  # device [6] p_min, p_max of a contracted partition
        self.chunk_off = None    # chunk tables of the refinement, made on first use
        self.chunk_bounds = None
        self.max_chunks = 0

    @property
    def n_blocks(self) -> int:
        return int(self.lvl_off.shape[0])

    @property
    def n_levels(self) -> int:
        return len(self.levels)

    @property
    def n_finest(self) -> int:
        return self.levels[-1].n

    def max_records_per_view(self) -> int:
        """Upper bound of the records one view can select."""
        return int(self.lvl_cnt_host.max(axis=1).sum())

    @staticmethod
    def from_sets(levels_np, lvl_off, lvl_cnt, cells=None, lo=None, hi=None, device="cuda"):
        levels = [DeviceLevel(*(torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
                                for a in (g.means, g.scales, g.quats, g.opac, g.sh))) for g in levels_np]
        return DeviceScene(levels, lvl_off, lvl_cnt, cells, lo, hi, device)

    @staticmethod
    def single(g, device="cuda") -> "DeviceScene":
        """One block, one level: the plain rasterizer input."""
        n = int(np.asarray(g.opac).shape[0])
        return DeviceScene.from_sets([g], [[0]], [[n]], device=device)

    @staticmethod
    def from_tensors(means, scales, quats, opac, sh) -> "DeviceScene":
        lev = DeviceLevel(means, scales, quats, opac, sh)
        n = lev.n
        return DeviceScene([lev], [[0]], [[n]], device=means.device)

    @staticmethod
    def from_finest(fine, block_id, u, cells, fractions=(0.30, 0.50, 1.00), coarse_scale=1.3,
                    device="cuda") -> "DeviceScene":
        """Upload the finest level and derive the nested coarser levels on the
        device (level l keeps the Gaussians with u < fractions[l]; coarser
        levels have scales x coarse_scale), so a 20M-Gaussian scene is built
        without host copies of the coarse levels."""
        fine_dev = DeviceLevel(*(torch.from_numpy(np.ascontiguousarray(a)).to(device) for a in fine.astuple()))
        return DeviceScene._nested(fine_dev, block_id, u, cells, fractions, coarse_scale, device)

    @staticmethod
    def _nested(fine_dev, block_id, u, cells, fractions, coarse_scale, device, contraction=None):
        B = cells.shape[0]
        L = len(fractions)
        lvl_cnt = np.zeros((B, L), np.int64)
        levels = []
        for l, frac in enumerate(fractions):
            if frac >= 1.0:
                lvl_cnt[:, l] = np.bincount(block_id, minlength=B)
                levels.append(fine_dev)
                continue
            idx_np = np.nonzero(u < frac)[0]
            lvl_cnt[:, l] = np.bincount(block_id[idx_np], minlength=B)
            idx = torch.from_numpy(idx_np).to(device)
            k = torch.tensor(np.float32(coarse_scale), device=device)
            levels.append(DeviceLevel(fine_dev.means.index_select(1, idx).contiguous(),
                                      (fine_dev.scales.index_select(1, idx) * k).contiguous(),
                                      fine_dev.quats.index_select(1, idx).contiguous(),
                                      fine_dev.opac.index_select(0, idx).contiguous(),
                                      fine_dev.sh.index_select(2, idx).contiguous()))
            del idx
        lvl_off = np.zeros_like(lvl_cnt)
        lvl_off[1:] = np.cumsum(lvl_cnt, axis=0)[:-1]
        scene = DeviceScene(levels, lvl_off, lvl_cnt, cells=cells, device=device)
        if contraction is not None:
            scene.contraction = torch.as_tensor(np.asarray(contraction, np.float64)).to(device)
        return scene

    @staticmethod
    def from_partition(fine, u, xy_box, nx, ny, fractions=(0.30, 0.50, 1.00), coarse_scale=1.3,
                       device="cuda") -> "DeviceScene":
        """Partition a finest-level Gaussian cloud (any order) into an nx x ny grid
        over the contracted space of Sec. 3.2.2 on the GPU (gs_partition), store
        it block by block (gs_gather_gaussians) and derive the nested coarser
        levels as from_finest does.  Cells are the contracted grid cells and the
        block table carries the contraction, so the camera's block is found in
        the same space.  Returns (scene, perm) with perm the new order."""
        n = fine.n
        src = DeviceLevel(*(torch.from_numpy(np.ascontiguousarray(a)).to(device) for a in fine.astuple()))
        perm = torch.empty(max(1, n), dtype=torch.int32, device=device)
        block_off = torch.empty(nx * ny + 1, dtype=torch.int64, device=device)
        cells = torch.empty((nx * ny, 4), dtype=torch.float64, device=device)
        ws = torch.empty(max(1, gs.partition_workspace_bytes(n)), dtype=torch.uint8, device=device)
        gs.partition(src.means, n, xy_box, nx, ny, perm, block_off, ws, cells=cells)
        dst = DeviceLevel(*(torch.empty_like(t) for t in (src.means, src.scales, src.quats, src.opac, src.sh)))
        gs.gather_gaussians(src.struct(), perm, n, gs.grads_struct(dst.means, dst.scales, dst.quats, dst.opac,
                                                                    dst.sh))
        del src, ws
        perm_host = perm[:n].cpu().numpy().view(np.uint32).astype(np.int64)
        counts = np.diff(block_off.cpu().numpy())
        block_id = np.repeat(np.arange(nx * ny), counts)
        z = np.asarray(fine.means[2])
        x0, x1 = sorted((float(xy_box[0]), float(xy_box[2])))
        y0, y1 = sorted((float(xy_box[1]), float(xy_box[3])))
        contraction = [x0, y0, float(z.min()), x1, y1, float(z.max())]
        scene = DeviceScene._nested(dst, block_id, np.asarray(u)[perm_host], cells.cpu().numpy(), fractions,
                                    coarse_scale, device, contraction)
        return scene, perm_host

    @staticmethod
    def from_block_scene(bs, device="cuda") -> "DeviceScene":
        return DeviceScene.from_sets(bs.levels, bs.lvl_off, bs.lvl_cnt, cells=bs.cells, device=device)

    def compute_bounds(self, n_mad: float = 4.0, stream=None):
        """Eq. 6 block boxes from the finest level, on the GPU."""
        B = self.n_blocks
        self.lo = torch.empty((B, 3), dtype=torch.float64, device=self.device)
        self.hi = torch.empty((B, 3), dtype=torch.float64, device=self.device)
        max_cnt = int(self.lvl_cnt_host[:, -1].max()) if B else 0
        ws = torch.empty(gs.mad_workspace_bytes(max_cnt), dtype=torch.uint8, device=self.device)
        gs.mad_bounds(self.levels[-1].struct(), self.lvl_off, self.lvl_cnt, n_mad, self.lo, self.hi, max_cnt, ws,
                      stream)
        return self.lo, self.hi

    def reduced_precision(self, sh_degrees=(1, 2, 3), half_levels=(0, 1)) -> "DeviceScene":
        """Same blocks and centres; level l stores sh_degrees[l] SH bands and, for
        l in half_levels, binary16 attributes."""
        levels = [lv.reduced(sh_degrees[l], l in half_levels) for l, lv in enumerate(self.levels)]
        out = DeviceScene(levels, self.lvl_off.cpu().numpy(), self.lvl_cnt_host, device=self.device)
        out.cells, out.lo, out.hi, out.contraction = self.cells, self.lo, self.hi, self.contraction
        return out

    def blocks_struct(self) -> gs.gs_blocks:
        return gs.blocks_struct(self.lo, self.hi, self.cells, self.lvl_off, self.lvl_cnt, self.contraction)

    def ensure_chunks(self, stream=None):
        """Chunk boxes of every (block, level) run (gs_chunk_bounds), once per scene;
        call invalidate_chunks() after moving or rescaling Gaussians."""
        if self.chunk_off is not None:
            return
        levels = [lv.struct() for lv in self.levels]
        blocks = self.blocks_struct()
        self.max_chunks = gs.chunk_capacity(levels, blocks)
        self.chunk_off = torch.empty(self.n_blocks * self.n_levels + 1, dtype=torch.int64, device=self.device)
        self.chunk_bounds = torch.empty((self.max_chunks, 8), dtype=torch.float32, device=self.device)
        gs.chunk_bounds(levels, blocks, self.chunk_off, self.chunk_bounds, self.max_chunks, stream)

    def invalidate_chunks(self):
        self.chunk_off = self.chunk_bounds = None
        self.max_chunks = 0


# ---------------------------------------------------------------------------
# frame buffers
# ---------------------------------------------------------------------------
class Frame:
    """All buffers of one batched frame (V views at one resolution)."""

    def __init__(self, n_blocks, n_views, width, height, record_capacity, pair_capacity, tuning=None,
                 device="cuda"):
        self.B, self.V, self.W, self.H = n_blocks, n_views, width, height
        self.tuning = tuning or gs.tuning_struct()
        self.device = device
        tw, th = self.tuning.tile_w, self.tuning.tile_h
        self.tiles_x = (width + tw - 1) // tw
        self.tiles_y = (height + th - 1) // th
        self.n_tiles = self.tiles_x * self.tiles_y * n_views
        d = device
        self.level = torch.empty((n_views, n_blocks), dtype=torch.int8, device=d)
        self.offsets = torch.empty(n_views * n_blocks + 1, dtype=torch.int64, device=d)
        self.counts = torch.zeros(gs.GS_COUNT_SLOTS, dtype=torch.int64, device=d)
        self.rgb = torch.empty((n_views, 3, height, width), dtype=torch.float32, device=d)
        self.T = torch.empty((n_views, height, width), dtype=torch.float32, device=d)
        self.n_last = torch.empty((n_views, height, width), dtype=torch.int32, device=d)
        self.tile_ranges = torch.empty((self.n_tiles, 2), dtype=torch.int32, device=d)
        # device work queue of the persistent tile kernels (used with GS_TUNE_WORK_QUEUE)
        self.tile_queue = torch.zeros(2 + self.n_tiles, dtype=torch.int32, device=d)
        self.record_capacity = 0
        self.pair_capacity = 0
        self.gather = None        # point-wise selection buffers, made on first use
        self.pts_offsets = None
        self.pts_ws = None
        self.pointwise = False    # selection kind of the last render_frame
        self.refined = None       # refined selection (gather, view offsets, workspace), made on first use
        self.refined_last = False  # whether the last render_frame used it
        self.reserve(record_capacity, pair_capacity)

    def reserve(self, record_capacity, pair_capacity):
        d = self.device
        if record_capacity > self.record_capacity:
            self.record_capacity = int(record_capacity)
            rb = gs.record_bytes()
            self.records = torch.empty(self.record_capacity * rb, dtype=torch.uint8, device=d)
            self.depth_keys = torch.empty(self.record_capacity, dtype=torch.int32, device=d)
            self.tiles_touched = torch.empty(self.record_capacity, dtype=torch.int32, device=d)
            self.bwd_ws = None
            if self.gather is not None:
                self.gather = torch.empty(self.record_capacity, dtype=torch.int32, device=d)
            if self.refined is not None:
                self.refined["gather"] = torch.empty(self.record_capacity, dtype=torch.int32, device=d)
        if pair_capacity > self.pair_capacity:
            self.pair_capacity = int(pair_capacity)
            self.pair_tiles = torch.empty(self.pair_capacity, dtype=torch.int32, device=d)
            self.pair_records = torch.empty(self.pair_capacity, dtype=torch.int32, device=d)
        nbytes = gs.workspace_bytes(gs.GS_WS_BIN_SORT, self.record_capacity, self.pair_capacity, self.V, self.W,
                                    self.H, self.tuning)
        if getattr(self, "sort_ws", None) is None or self.sort_ws.numel() < nbytes:
            self.sort_ws = torch.empty(nbytes, dtype=torch.uint8, device=d)

    def ensure_pointwise(self, scene):
        d = self.device
        L = scene.n_levels
        if self.gather is None or self.gather.numel() < self.record_capacity:
            self.gather = torch.empty(max(1, self.record_capacity), dtype=torch.int32, device=d)
        if self.pts_offsets is None or self.pts_offsets.numel() != self.V * L + 1:
            self.pts_offsets = torch.empty(self.V * L + 1, dtype=torch.int64, device=d)
        nbytes = gs.points_workspace_bytes([lv.n for lv in scene.levels], self.V)
        if self.pts_ws is None or self.pts_ws.numel() < nbytes:
            self.pts_ws = torch.empty(nbytes, dtype=torch.uint8, device=d)

    def ensure_refined(self, scene, stream=None):
        scene.ensure_chunks(stream)
        d = self.device
        nbytes = gs.refine_workspace_bytes(self.V, scene.max_chunks)
        r = self.refined
        if r is None or r["ws"].numel() < nbytes:
            self.refined = r = dict(gather=torch.empty(max(1, self.record_capacity), dtype=torch.int32, device=d),
                                    view_off=torch.empty(self.V + 1, dtype=torch.int64, device=d),
                                    ws=torch.empty(nbytes, dtype=torch.uint8, device=d))
        return r

    def pre_tuning(self):
        """Tuning gs_preprocess takes for the last selection."""
        if not self.refined_last:
            return self.tuning
        t = gs.tuning_struct(self.tuning.tile_w, self.tuning.tile_h, self.tuning.batch, self.tuning.flags)
        t.flags |= gs.GS_TUNE_PACKED_SELECTION
        return t

    def selection(self):
        """(level, offsets, gather) of the last selection, as gs_preprocess takes them."""
        if self.refined_last:
            return None, self.refined["view_off"], self.refined["gather"]
        if self.pointwise:
            return None, self.pts_offsets, self.gather
        return self.level, self.offsets, None

    def host_counts(self):
        c = self.counts.cpu().numpy()
        return dict(records=int(c[0]), visible=int(c[1]), pairs=int(c[2]), flags=int(c[3]))


def render_frame(scene: DeviceScene, frame: Frame, cams_dev, mode=gs.GS_LOD_BLOCKWISE, thresholds=(200.0, 500.0),
                 sh_degree=3, bg=(0.0, 0.0, 0.0), stream=None, check=True, refine=False):
    """LoD select + preprocess + bin/sort + composite for every view of `frame`.

    With check=True the counts are read back once (a host sync); if a capacity
    was too small the buffers grow and the frame is rendered again.  refine=True
    (block-wise selections only) adds the chunk refinement (gs_lod_refine); the
    images are the same, and backward_frame takes the refined selection (not with
    GS_TUNE_SHARED_SELECTION, nor GS_TUNE_DETERMINISTIC over several views).  The
    chunk boxes are made once per scene: after moving or rescaling Gaussians (an
    optimiser step) call scene.invalidate_chunks(), or the refinement may drop
    Gaussians that have become visible."""
    if refine and mode == LOD_POINTWISE:
        raise ValueError("the chunk refinement applies to block-wise selections")
    for _ in range(4):
        blocks = scene.blocks_struct()
        levels = [lv.struct() for lv in scene.levels]
        frame.pointwise = mode == LOD_POINTWISE
        frame.refined_last = False
        if frame.pointwise:
            frame.ensure_pointwise(scene)
            gs.lod_select_points(levels, thresholds, cams_dev, frame.V, frame.record_capacity, frame.gather,
                                 frame.pts_offsets, frame.counts, frame.pts_ws, stream)
        else:
            gs.lod_select(blocks, thresholds, mode, cams_dev, frame.V, frame.level, frame.offsets, frame.counts,
                          stream)
            if refine:
                r = frame.ensure_refined(scene, stream)
                gs.lod_refine(blocks, frame.level, cams_dev, frame.V, frame.W, frame.H, scene.chunk_off,
                              scene.chunk_bounds, scene.max_chunks, frame.record_capacity, r["gather"],
                              r["view_off"], frame.counts, r["ws"], stream)
                frame.refined_last = True
        level, offsets, gather = frame.selection()
        gs.preprocess(levels, blocks, level, offsets, cams_dev, frame.V, frame.W, frame.H, sh_degree,
                      frame.pre_tuning(), frame.record_capacity, frame.records, frame.depth_keys, frame.tiles_touched,
                      frame.counts, stream, gather=gather)
        gs.bin_sort(frame.records, frame.depth_keys, frame.tiles_touched, frame.V, frame.W, frame.H, frame.tuning,
                    frame.record_capacity, frame.pair_capacity, frame.pair_tiles, frame.pair_records,
                    frame.tile_ranges, frame.counts, frame.sort_ws, stream, frame.tile_queue)
        gs.rasterize_fwd(frame.records, frame.pair_records, frame.tile_ranges, frame.V, frame.W, frame.H, bg,
                         frame.tuning, frame.rgb, frame.T, frame.n_last, stream, frame.tile_queue)
        if not check:
            return frame.rgb
        c = frame.host_counts()
        if c["flags"] & gs.GS_FLAG_WAIT:
            raise RuntimeError("a device-side wait gave up during the frame (counts=%s)" % c)
        if c["flags"] & gs.GS_FLAG_SELECTION:
            raise RuntimeError("GS_TUNE_SHARED_SELECTION was set but the views selected different records "
                               "(counts=%s)" % c)
        if c["flags"] == 0:
            return frame.rgb
        frame.reserve(max(frame.record_capacity, int(c["records"] * 1.1) + 1024),
                      max(frame.pair_capacity, int(c["pairs"] * 1.25) + 4096))
    raise RuntimeError("frame did not fit after growing the buffers: %s" % frame.host_counts())


def backward_frame(scene: DeviceScene, frame: Frame, cams_dev, d_rgb, grads, sh_degree=3, bg=(0.0, 0.0, 0.0),
                   stream=None):
    """Accumulate dL/d(parameters) of every level into `grads` (list of DeviceLevel)."""
    tuning = frame.pre_tuning()  # with the packed-selection flag after a refined render
    nbytes = gs.workspace_bytes(gs.GS_WS_RASTERIZE_BWD, frame.record_capacity, frame.pair_capacity, frame.V, frame.W,
                                frame.H, tuning)
    if getattr(frame, "bwd_ws", None) is None or frame.bwd_ws.numel() < nbytes:
        frame.bwd_ws = torch.empty(nbytes, dtype=torch.uint8, device=frame.device)
    level, offsets, gather = frame.selection()
    gs.rasterize_bwd(frame.records, frame.pair_records, frame.tile_ranges, frame.V, frame.W, frame.H, bg,
                     tuning, frame.rgb, frame.T, frame.n_last, d_rgb.contiguous(),
                     [lv.struct() for lv in scene.levels], scene.blocks_struct(), level, offsets,
                     cams_dev, sh_degree, frame.record_capacity, frame.counts,
                     [gs.grads_struct(g.means, g.scales, g.quats, g.opac, g.sh) for g in grads], frame.bwd_ws, stream,
                     frame.tile_queue, gather=gather)


# ---------------------------------------------------------------------------
# differentiable render of one Gaussian set
# ---------------------------------------------------------------------------
class GaussianRasterize(torch.autograd.Function):
    """image[V,3,H,W] = render(means[3,N], scales[3,N], quats[4,N], opac[N], sh[16,3,N]; cameras).

    Forward runs the library's preprocess, bin_sort and rasterize_fwd; backward
    runs rasterize_bwd, which recomputes the per-pixel blend state."""

    @staticmethod
    def forward(ctx, means, scales, quats, opac, sh, cams_dev, n_views, width, height, sh_degree, bg, frame):
        scene = DeviceScene.from_tensors(means.detach().contiguous(), scales.detach().contiguous(),
                                         quats.detach().contiguous(), opac.detach().contiguous(),
                                         sh.detach().contiguous())
        if frame is None:
            frame = Frame(1, n_views, width, height, n_views * scene.n_finest, max(4096, 4 * n_views * scene.n_finest))
        else:
            frame.reserve(n_views * scene.n_finest, 0)
        render_frame(scene, frame, cams_dev, mode=gs.GS_LOD_ALL_FINEST, thresholds=(), sh_degree=sh_degree, bg=bg)
        ctx.scene, ctx.frame, ctx.cams = scene, frame, cams_dev
        ctx.sh_degree, ctx.bg = sh_degree, bg
        return frame.rgb.clone()

    @staticmethod
    def backward(ctx, d_rgb):
        scene, frame = ctx.scene, ctx.frame
        grads = [scene.levels[0].zeros_like()]
        backward_frame(scene, frame, ctx.cams, d_rgb, grads, ctx.sh_degree, ctx.bg)
        g = grads[0]
        return g.means, g.scales, g.quats, g.opac, g.sh, None, None, None, None, None, None, None


def rasterize(means, scales, quats, opac, sh, cams, sh_degree=3, bg=(0.0, 0.0, 0.0), frame=None):
    """Differentiable render of one Gaussian set for a list of cameras (same size)."""
    cams_dev = gs.cameras_to_device(cams, means.device)
    W, H = cams[0].width, cams[0].height
    return GaussianRasterize.apply(means, scales, quats, opac, sh, cams_dev, len(cams), W, H, sh_degree, bg, frame)

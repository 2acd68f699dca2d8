"""Training-data assignment of Sec. 3.2.2 (Eqs. 3-5) over the C ABI.

For each pose and block j: B1 = the SSIM loss between the render of every block
and the render without block j exceeds eps; B2 = the contracted camera centre
lies in block j; B = B1 or B2.  Per batch of poses:

  1. one batched render of every pose with all blocks (gs_lod_select_exclude, -1)
  2. per (pose, block) count of records that survived the cull (gs_segment_visible):
     a block with none cannot change the pose's image, its SSIM is 1 exactly and
     its leave-one-out render is skipped
  3. batched leave-one-out renders of the remaining (pose, block) pairs
  4. SSIM of each (full, leave-one-out) image pair (gs_ssim)
  5. Eqs. 3-5 on the device (gs_assign)

The scene is the coarse global prior, a single level partitioned into blocks
(render.DeviceScene.from_partition with fractions=(1.0,)).
"""
from __future__ import annotations

import numpy as np
import torch

from . import gs, render


def _render_views(scene, frame, cams_dev, exclude, sh_degree, stream):
    """Render the views of `frame` with per-view excluded blocks (grow-and-retry on overflow)."""
    for _ in range(4):
        blocks = scene.blocks_struct()
        gs.lod_select_exclude(blocks, cams_dev, frame.V, exclude, frame.level, frame.offsets, frame.counts, stream)
        gs.preprocess([lv.struct() for lv in scene.levels], blocks, frame.level, frame.offsets, cams_dev, frame.V,
                      frame.W, frame.H, sh_degree, frame.tuning, frame.record_capacity, frame.records,
                      frame.depth_keys, frame.tiles_touched, frame.counts, stream)
        gs.bin_sort(frame.records, frame.depth_keys, frame.tiles_touched, frame.V, frame.W, frame.H, frame.tuning,
                    frame.record_capacity, frame.pair_capacity, frame.pair_tiles, frame.pair_records,
                    frame.tile_ranges, frame.counts, frame.sort_ws, stream, frame.tile_queue)
        gs.rasterize_fwd(frame.records, frame.pair_records, frame.tile_ranges, frame.V, frame.W, frame.H,
                         (0.0, 0.0, 0.0), frame.tuning, frame.rgb, frame.T, frame.n_last, stream, frame.tile_queue)
        c = frame.host_counts()
        if c["flags"] & gs.GS_FLAG_WAIT:
            raise RuntimeError("a device-side wait gave up (counts=%s)" % c)
        if c["flags"] == 0:
            return
        frame.reserve(max(frame.record_capacity, int(c["records"] * 1.1) + 1024),
                      max(frame.pair_capacity, int(c["pairs"] * 1.25) + 4096))
    raise RuntimeError("views did not fit after growing the buffers: %s" % frame.host_counts())


def assign_poses(scene, cams, width, height, eps=0.05, poses_per_call=4, views_per_call=16, sh_degree=3,
                 skip_invisible=True, tuning=None, stream=None):
    """Returns dict(b1, b2, b: bool [P, B], ssim: float [P, B], renders: leave-one-out renders done)."""
    dev = scene.device
    P, B = len(cams), scene.n_blocks
    tuning = tuning or gs.tuning_struct(16, 16, 256, gs.GS_TUNE_WORK_QUEUE)
    n_per_view = int(scene.lvl_cnt_host[:, -1].sum())
    ssim_all = torch.ones((P, B), dtype=torch.float32, device=dev)
    full = render.Frame(B, poses_per_call, width, height, poses_per_call * n_per_view, 1 << 22, tuning, dev)
    loo = render.Frame(B, views_per_call, width, height, views_per_call * n_per_view, 1 << 22, tuning, dev)
    vis = torch.empty(poses_per_call * B, dtype=torch.int32, device=dev)
    n_loo = 0
    for p0 in range(0, P, poses_per_call):
        batch = list(range(p0, min(P, p0 + poses_per_call)))
        nb = len(batch)
        cams_dev = gs.cameras_to_device([cams[p] for p in batch], dev)
        if nb != full.V:
            full = render.Frame(B, nb, width, height, nb * n_per_view, full.pair_capacity, tuning, dev)
        exclude = torch.full((nb,), -1, dtype=torch.int32, device=dev)
        _render_views(scene, full, cams_dev, exclude, sh_degree, stream)
        full_img = full.rgb.clone()
        if skip_invisible:
            gs.segment_visible(full.tiles_touched, full.offsets, nb * B, full.record_capacity, vis, stream)
            v = vis[: nb * B].view(nb, B).cpu().numpy()
            todo = [(i, j) for i in range(nb) for j in range(B) if v[i, j] > 0]
        else:
            todo = [(i, j) for i in range(nb) for j in range(B)]
        for k0 in range(0, len(todo), views_per_call):
            chunk = todo[k0:k0 + views_per_call]
            nv = len(chunk)
            if nv != loo.V:
                loo = render.Frame(B, nv, width, height, nv * n_per_view, loo.pair_capacity, tuning, dev)
            ccams = gs.cameras_to_device([cams[batch[i]] for i, _ in chunk], dev)
            excl = torch.tensor([j for _, j in chunk], dtype=torch.int32, device=dev)
            _render_views(scene, loo, ccams, excl, sh_degree, stream)
            n_loo += nv
            # SSIM of (full image of the pose, leave-one-out image): both stacked into one batch
            images = torch.cat([full_img, loo.rgb], dim=0).contiguous()
            pairs = torch.tensor([[i, nb + k] for k, (i, _) in enumerate(chunk)], dtype=torch.int32, device=dev)
            out = torch.empty(nv, dtype=torch.float32, device=dev)
            ws = torch.empty(gs.ssim_workspace_bytes(nv, width, height), dtype=torch.uint8, device=dev)
            gs.ssim(images, images.shape[0], width, height, pairs, nv, out, ws, stream)
            rows = torch.tensor([batch[i] for i, _ in chunk], device=dev)
            cols = torch.tensor([j for _, j in chunk], device=dev)
            ssim_all[rows, cols] = out
    b = torch.empty((P, B), dtype=torch.uint8, device=dev)
    b1 = torch.empty_like(b)
    b2 = torch.empty_like(b)
    gs.assign(scene.blocks_struct(), gs.cameras_to_device(cams, dev), P, ssim_all, eps, b, b1, b2, stream)
    torch.cuda.synchronize()
    return dict(b1=b1.cpu().numpy().astype(bool), b2=b2.cpu().numpy().astype(bool), b=b.cpu().numpy().astype(bool),
                ssim=ssim_all.cpu().numpy(), renders=n_loo)

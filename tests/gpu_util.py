"""Helpers shared by the GPU tests: run the library on seeded inputs and pull
results back as NumPy arrays."""
import numpy as np
import torch

from paper_2404_01133_amd import gs, render, synth


def run_single(g, cam, tuning=None, sh_degree=3, bg=(0.0, 0.0, 0.0), pair_capacity=None):
    """Plain render of one Gaussian set through the five entry points."""
    scene = render.DeviceScene.single(g)
    cams_dev = gs.cameras_to_device([cam])
    n = scene.n_finest
    frame = render.Frame(1, 1, cam.width, cam.height, max(1, n), pair_capacity or max(4096, 8 * n),
                         tuning or gs.tuning_struct())
    render.render_frame(scene, frame, cams_dev, mode=gs.GS_LOD_ALL_FINEST, thresholds=(), sh_degree=sh_degree, bg=bg)
    torch.cuda.synchronize()
    return scene, frame, cams_dev


def records_np(frame, n):
    raw = frame.records[: n * gs.record_bytes()].view(torch.int32).reshape(n, 12).cpu().numpy()
    f = raw.view(np.float32)
    px = raw[:, 2].view(np.uint32)
    py = raw[:, 3].view(np.uint32)
    i0 = (px & 0xFFFF).astype(np.int64)
    j0 = (py & 0xFFFF).astype(np.int64)
    rect = np.stack([i0, i0 + (px >> 16), j0, j0 + (py >> 16)], axis=1)
    return dict(u=f[:, 0] + i0 + 0.5, v=f[:, 11] + j0 + 0.5, rect=rect, conic_factor=f[:, 4:7], opac=f[:, 7],
                rgb=f[:, 8:11], view=raw[:, 1])


def frame_pairs(frame):
    c = frame.host_counts()
    m = c["pairs"]
    tiles = frame.pair_tiles[:m].cpu().numpy().view(np.uint32)
    recs = frame.pair_records[:m].cpu().numpy().view(np.uint32)
    return tiles, recs


def image_np(frame):
    return frame.rgb.cpu().numpy(), frame.T.cpu().numpy(), frame.n_last.cpu().numpy()


def scaled_city(n=200_000, seed=21, grid=(8, 8)):
    return synth.city_block_scene(n=n, seed=seed, area_m2=1.5e6, grid=grid)

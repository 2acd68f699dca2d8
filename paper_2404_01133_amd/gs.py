"""Thin ctypes binding of libgs (include/gs.h): same names as the C entry points,
argument marshalling only.  torch supplies device memory and the stream; every
step of the rendering path runs in the HIP kernels of libgs.

Importing this module loads torch first so that libgs binds to the HIP runtime
torch already uses; if libgs.so is missing it raises immediately (there is no
fallback path).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgs.so")

GS_OK = 0
GS_ERR_INVALID_ARG = -1
GS_ERR_UNSUPPORTED = -2
GS_ERR_WORKSPACE = -3
GS_ERR_CAPACITY = -4
GS_ERR_HIP = -5
GS_ERR_SCRATCH = -6
GS_STATIC_SCRATCH_BYTES = 64 << 20

GS_COUNT_RECORDS, GS_COUNT_VISIBLE, GS_COUNT_PAIRS, GS_COUNT_FLAGS = 0, 1, 2, 3
GS_COUNT_SLOTS = 8
GS_FLAG_RECORDS, GS_FLAG_PAIRS, GS_FLAG_WAIT, GS_FLAG_SELECTION = 1, 2, 4, 8
GS_WS_BIN_SORT, GS_WS_RASTERIZE_BWD = 1, 2
GS_LOD_BLOCKWISE, GS_LOD_ALL_FINEST = 0, 1
GS_TUNE_SHARED_SELECTION, GS_TUNE_WORK_QUEUE, GS_TUNE_DETERMINISTIC, GS_TUNE_PACKED_SELECTION = 1, 2, 4, 8
GS_CHUNK, GS_PACKED_INDEX_BITS = 2048, 29

c_double, c_int32, c_int64, c_void_p, c_size_t = (ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p,
                                                  ctypes.c_size_t)


class gs_camera(ctypes.Structure):
    _fields_ = [("R", c_double * 9), ("t", c_double * 3), ("fx", c_double), ("fy", c_double), ("cx", c_double),
                ("cy", c_double), ("znear", c_double), ("width", c_int32), ("height", c_int32),
                ("pad", c_int32 * 2)]


class gs_gaussians(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("scales", c_void_p), ("quats", c_void_p), ("opac", c_void_p),
                ("sh", c_void_p), ("n", c_int64), ("sh_degree", c_int32), ("attr_half", c_int32)]


class gs_gaussian_grads(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("scales", c_void_p), ("quats", c_void_p), ("opac", c_void_p),
                ("sh", c_void_p)]


class gs_blocks(ctypes.Structure):
    _fields_ = [("lo", c_void_p), ("hi", c_void_p), ("cell", c_void_p), ("lvl_off", c_void_p),
                ("lvl_cnt", c_void_p), ("n_blocks", c_int32), ("n_levels", c_int32), ("contraction", c_void_p)]


class gs_tuning(ctypes.Structure):
    _fields_ = [("tile_w", c_int32), ("tile_h", c_int32), ("batch", c_int32), ("flags", c_int32)]


assert ctypes.sizeof(gs_camera) == 152

_lib = None

_SIGNATURES = {
    "gs_record_bytes": (c_size_t, []),
    "gs_workspace_bytes": (c_size_t, [c_int32, c_int64, c_int64, c_int32, c_int32, c_int32, c_void_p]),
    "gs_lod_select": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_int32, c_void_p, c_void_p, c_void_p,
                                c_void_p]),
    "gs_points_workspace_bytes": (c_size_t, [c_void_p, c_int32, c_int32]),
    "gs_lod_select_points": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_int64, c_void_p, c_void_p,
                                       c_void_p, c_void_p, c_size_t, c_void_p]),
    "gs_preprocess": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int32,
                                c_int32, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "gs_bin_sort": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p, c_int64, c_int64,
                              c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "gs_bin_sort_static": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p, c_int64,
                                     c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "gs_rasterize_fwd": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p,
                                   c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "gs_rasterize_bwd": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p,
                                   c_void_p,
                                   c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_void_p, c_int32, c_int64, c_void_p, c_void_p, c_void_p, c_size_t,
                                   c_void_p]),
    "gs_partition_workspace_bytes": (c_size_t, [c_int64]),
    "gs_partition": (c_int32, [c_void_p, c_int64, c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                               c_void_p, c_size_t, c_void_p]),
    "gs_gather_gaussians": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p]),
    "gs_lod_select_exclude": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_void_p]),
    "gs_segment_visible": (c_int32, [c_void_p, c_void_p, c_int32, c_int64, c_void_p, c_void_p]),
    "gs_ssim_workspace_bytes": (c_size_t, [c_int32, c_int32, c_int32]),
    "gs_ssim": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_int32, c_void_p, c_void_p, c_size_t,
                          c_void_p]),
    "gs_assign": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_double, c_void_p, c_void_p, c_void_p,
                            c_void_p]),
    "gs_mad_workspace_bytes": (c_size_t, [c_int64]),
    "gs_mad_bounds": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int64, c_double, c_void_p,
                                c_void_p, c_void_p, c_size_t, c_void_p]),
    "gs_chunk_capacity": (c_int64, [c_void_p, c_void_p]),
    "gs_chunk_bounds": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_void_p]),
    "gs_refine_workspace_bytes": (c_size_t, [c_int32, c_int64]),
    "gs_lod_refine": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_int64,
                                c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "gs_status_string": (ctypes.c_char_p, [c_int32]),
}


def lib():
    """Load libgs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libgs.so not found at %s: build it with __graft_entry__.build() "
                               "(the HIP path has no fallback)" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class GsError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__("%s failed: %s" % (where, status_string(status)))
        self.status = status


def status_string(status: int) -> str:
    return lib().gs_status_string(status).decode()


def _check(status: int, where: str):
    if status != GS_OK:
        raise GsError(status, where)


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def record_bytes() -> int:
    return int(lib().gs_record_bytes())


def workspace_bytes(which: int, record_capacity: int, pair_capacity: int, n_views: int, width: int, height: int,
                    tuning: gs_tuning) -> int:
    return int(lib().gs_workspace_bytes(which, record_capacity, pair_capacity, n_views, width, height,
                                        ctypes.byref(tuning)))


def mad_workspace_bytes(max_block_count: int) -> int:
    return int(lib().gs_mad_workspace_bytes(max_block_count))


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------
def camera_struct(cam) -> gs_camera:
    c = gs_camera()
    R = np.asarray(cam.R, np.float64).reshape(9)
    t = np.asarray(cam.t, np.float64).reshape(3)
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
    c.fx, c.fy, c.cx, c.cy, c.znear = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy), float(cam.znear)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def cameras_to_device(cams, device="cuda") -> torch.Tensor:
    """Pack cameras into a device byte tensor holding gs_camera[V]."""
    arr = (gs_camera * len(cams))(*[camera_struct(c) for c in cams])
    host = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8)
    return host.to(device)


SH_PLANES = {1: 0, 4: 1, 9: 2, 16: 3}


def gaussians_struct(means, scales, quats, opac, sh) -> gs_gaussians:
    """Centres FP32 [3, n]; the other attributes all float32 or all float16;
    sh [K, 3, n] with K in (1, 4, 9, 16) coefficient planes (SH degree 0..3)."""
    n = int(opac.shape[0])
    half = scales.dtype == torch.float16
    adt = torch.float16 if half else torch.float32
    K = int(sh.shape[0])
    if K not in SH_PLANES:
        raise ValueError("sh must hold 1, 4, 9 or 16 coefficient planes, got %d" % K)
    for t, shape, dt in ((means, (3, n), torch.float32), (scales, (3, n), adt), (quats, (4, n), adt),
                         (opac, (n,), adt), (sh, (K, 3, n), adt)):
        if tuple(t.shape) != shape or t.dtype != dt or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("Gaussian arrays must be contiguous device tensors in SoA layout (centres float32, "
                             "other attributes all float32 or all float16); got %s %s" % (tuple(t.shape), t.dtype))
    return gs_gaussians(means.data_ptr(), scales.data_ptr(), quats.data_ptr(), opac.data_ptr(), sh.data_ptr(), n,
                        SH_PLANES[K], 1 if half else 0)


def grads_struct(gm, gs_, gq, go, gsh) -> gs_gaussian_grads:
    for t in (gm, gs_, gq, go, gsh):
        if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("gradient buffers must be contiguous float32 device tensors, got %s" % (t.dtype,))
    return gs_gaussian_grads(gm.data_ptr(), gs_.data_ptr(), gq.data_ptr(), go.data_ptr(), gsh.data_ptr())


def blocks_struct(lo, hi, cell, lvl_off, lvl_cnt, contraction=None) -> gs_blocks:
    B, L = lvl_off.shape
    ptr = lambda t: None if t is None else t.data_ptr()
    return gs_blocks(ptr(lo), ptr(hi), ptr(cell), lvl_off.data_ptr(), lvl_cnt.data_ptr(), B, L, ptr(contraction))


def tuning_struct(tile_w=16, tile_h=16, batch=256, flags=0) -> gs_tuning:
    return gs_tuning(tile_w, tile_h, batch, flags)


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI, without the gs_ prefix)
# ---------------------------------------------------------------------------
def lod_select(blocks: gs_blocks, thresholds, mode, cams_dev, n_views, level, offsets, counts, stream=None):
    thr = (c_double * max(1, len(thresholds)))(*[float(x) for x in thresholds])
    _check(lib().gs_lod_select(ctypes.byref(blocks), thr, mode, _p(cams_dev), n_views, _p(level), _p(offsets),
                               _p(counts), _stream(stream)), "gs_lod_select")


def chunk_capacity(levels, blocks: gs_blocks) -> int:
    arr = (gs_gaussians * len(levels))(*levels)
    c = int(lib().gs_chunk_capacity(arr, ctypes.byref(blocks)))
    if c < 0:
        raise GsError(GS_ERR_INVALID_ARG, "gs_chunk_capacity")
    return c


def chunk_bounds(levels, blocks: gs_blocks, chunk_off, bounds, max_chunks, stream=None):
    arr = (gs_gaussians * len(levels))(*levels)
    _check(lib().gs_chunk_bounds(arr, ctypes.byref(blocks), _p(chunk_off), _p(bounds), max_chunks, _stream(stream)),
           "gs_chunk_bounds")


def refine_workspace_bytes(n_views, max_chunks) -> int:
    return int(lib().gs_refine_workspace_bytes(n_views, max_chunks))


def lod_refine(blocks: gs_blocks, level, cams_dev, n_views, width, height, chunk_off, bounds, max_chunks,
               record_capacity, gather, view_offsets, counts, ws, stream=None):
    _check(lib().gs_lod_refine(ctypes.byref(blocks), _p(level), _p(cams_dev), n_views, width, height, _p(chunk_off),
                               _p(bounds), max_chunks, record_capacity, _p(gather), _p(view_offsets), _p(counts),
                               _p(ws), ws.numel() * ws.element_size(), _stream(stream)), "gs_lod_refine")


def points_workspace_bytes(level_sizes, n_views) -> int:
    sizes = (c_int64 * len(level_sizes))(*[int(x) for x in level_sizes])
    return int(lib().gs_points_workspace_bytes(sizes, len(level_sizes), n_views))


def lod_select_points(levels, thresholds, cams_dev, n_views, record_capacity, gather, offsets, counts, ws,
                      stream=None):
    arr = (gs_gaussians * len(levels))(*levels)
    thr = (c_double * max(1, len(thresholds)))(*[float(x) for x in thresholds])
    _check(lib().gs_lod_select_points(arr, len(levels), thr, _p(cams_dev), n_views, record_capacity, _p(gather),
                                      _p(offsets), _p(counts), _p(ws), ws.numel() * ws.element_size(),
                                      _stream(stream)), "gs_lod_select_points")


def preprocess(levels, blocks: gs_blocks, level, offsets, cams_dev, n_views, width, height, sh_degree,
               tuning: gs_tuning, record_capacity, records, depth_keys, tiles_touched, counts, stream=None,
               gather=None):
    arr = (gs_gaussians * len(levels))(*levels)
    _check(lib().gs_preprocess(arr, ctypes.byref(blocks), _p(level), _p(offsets), _p(gather), _p(cams_dev), n_views,
                               width, height, sh_degree, ctypes.byref(tuning), record_capacity, _p(records),
                               _p(depth_keys), _p(tiles_touched), _p(counts), _stream(stream)), "gs_preprocess")


def bin_sort(records, depth_keys, tiles_touched, n_views, width, height, tuning: gs_tuning, record_capacity,
             pair_capacity, pair_tiles, pair_records, tile_ranges, counts, ws, stream=None, tile_queue=None):
    _check(lib().gs_bin_sort(_p(records), _p(depth_keys), _p(tiles_touched), n_views, width, height,
                             ctypes.byref(tuning), record_capacity, pair_capacity, _p(pair_tiles), _p(pair_records),
                             _p(tile_ranges), _p(tile_queue), _p(counts), _p(ws), ws.numel() * ws.element_size(),
                             _stream(stream)), "gs_bin_sort")


def bin_sort_static(records, depth_keys, tiles_touched, n_views, width, height, tuning: gs_tuning, record_capacity,
                    pair_capacity, pair_tiles, pair_records, tile_ranges, counts, stream=None, tile_queue=None):
    """gs_bin_sort with the library's static scratch array as workspace (no allocation)."""
    _check(lib().gs_bin_sort_static(_p(records), _p(depth_keys), _p(tiles_touched), n_views, width, height,
                                    ctypes.byref(tuning), record_capacity, pair_capacity, _p(pair_tiles),
                                    _p(pair_records), _p(tile_ranges), _p(tile_queue), _p(counts), _stream(stream)),
           "gs_bin_sort_static")


def rasterize_fwd(records, pair_records, tile_ranges, n_views, width, height, bg, tuning: gs_tuning, rgb, T_final,
                  n_last, stream=None, tile_queue=None):
    bgv = (ctypes.c_float * 3)(*[float(x) for x in bg])
    _check(lib().gs_rasterize_fwd(_p(records), _p(pair_records), _p(tile_ranges), _p(tile_queue), n_views, width,
                                  height, bgv, ctypes.byref(tuning), _p(rgb), _p(T_final), _p(n_last),
                                  _stream(stream)), "gs_rasterize_fwd")


def rasterize_bwd(records, pair_records, tile_ranges, n_views, width, height, bg, tuning: gs_tuning, rgb, T_final,
                  n_last, d_rgb, levels, blocks: gs_blocks, level, offsets, cams_dev, sh_degree, record_capacity,
                  counts, grads, ws, stream=None, tile_queue=None, gather=None):
    bgv = (ctypes.c_float * 3)(*[float(x) for x in bg])
    lv = (gs_gaussians * len(levels))(*levels)
    gr = (gs_gaussian_grads * len(grads))(*grads)
    _check(lib().gs_rasterize_bwd(_p(records), _p(pair_records), _p(tile_ranges), _p(tile_queue), n_views, width,
                                  height, bgv,
                                  ctypes.byref(tuning), _p(rgb), _p(T_final), _p(n_last), _p(d_rgb), lv,
                                  ctypes.byref(blocks), _p(level), _p(offsets), _p(gather), _p(cams_dev), sh_degree,
                                  record_capacity, _p(counts), gr, _p(ws), ws.numel() * ws.element_size(),
                                  _stream(stream)), "gs_rasterize_bwd")


def partition_workspace_bytes(n) -> int:
    return int(lib().gs_partition_workspace_bytes(int(n)))


def partition(means, n, xy_box, nx, ny, perm, block_off, ws, block_id=None, cells=None, stream=None):
    box = (c_double * 4)(*[float(x) for x in xy_box])
    _check(lib().gs_partition(_p(means), int(n), box, nx, ny, _p(block_id), _p(perm), _p(block_off), _p(cells),
                              _p(ws), 0 if ws is None else ws.numel() * ws.element_size(), _stream(stream)),
           "gs_partition")


def gather_gaussians(src: gs_gaussians, perm, n, dst: gs_gaussian_grads, stream=None):
    _check(lib().gs_gather_gaussians(ctypes.byref(src), _p(perm), int(n), ctypes.byref(dst), _stream(stream)),
           "gs_gather_gaussians")


def lod_select_exclude(blocks: gs_blocks, cams_dev, n_views, exclude, level, offsets, counts, stream=None):
    _check(lib().gs_lod_select_exclude(ctypes.byref(blocks), _p(cams_dev), n_views, _p(exclude), _p(level),
                                       _p(offsets), _p(counts), _stream(stream)), "gs_lod_select_exclude")


def segment_visible(tiles_touched, offsets, n_segments, record_capacity, visible, stream=None):
    _check(lib().gs_segment_visible(_p(tiles_touched), _p(offsets), n_segments, record_capacity, _p(visible),
                                    _stream(stream)), "gs_segment_visible")


def ssim_workspace_bytes(n_pairs, width, height) -> int:
    return int(lib().gs_ssim_workspace_bytes(n_pairs, width, height))


def ssim(images, n_images, width, height, pairs, n_pairs, out, ws, stream=None):
    _check(lib().gs_ssim(_p(images), n_images, width, height, _p(pairs), n_pairs, _p(out), _p(ws),
                         ws.numel() * ws.element_size(), _stream(stream)), "gs_ssim")


def assign(blocks: gs_blocks, cams_dev, n_poses, ssim_vals, eps, b, b1=None, b2=None, stream=None):
    _check(lib().gs_assign(ctypes.byref(blocks), _p(cams_dev), n_poses, _p(ssim_vals), float(eps), _p(b1), _p(b2),
                           _p(b), _stream(stream)), "gs_assign")


def mad_bounds(finest: gs_gaussians, lvl_off, lvl_cnt, n_mad, lo, hi, max_block_count, ws, stream=None):
    B, L = lvl_off.shape
    _check(lib().gs_mad_bounds(ctypes.byref(finest), _p(lvl_off), _p(lvl_cnt), B, L, max_block_count, float(n_mad),
                               _p(lo), _p(hi), _p(ws), ws.numel() * ws.element_size(), _stream(stream)),
           "gs_mad_bounds")

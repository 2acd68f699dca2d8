"""CPU oracle: TEST INFRASTRUCTURE ONLY.

A plain, slow FP64 implementation of the rendering path, written from the paper
(Sec. 3.1, Eq. 1 for projection + compositing; Sec. 3.3.2, Eq. 6 for the
block-wise level-of-detail selection).  Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import it; the GPU path never does, and the
two share no code.

    raster.cpp   projection, untiled per-pixel compositing, tile-pair listing,
                 exact FP64 gradients (built into _build/liboracle.so)
    lod.py       MAD block bounds (Eq. 6), per-view level selection, frustum test,
                 concatenation of the chosen levels
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "raster.cpp")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle library with g++ (FP64, no FMA contraction, OpenMP)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        i32 = ctypes.c_int
        L.orc_project.argtypes = [i64, P, P, P, P, P, i32, P, P, i32, i32, P, P, P, P, P, P, P, P, P, P]
        L.orc_project.restype = i32
        L.orc_render.argtypes = [i64, P, P, P, P, P, i32, P, P, P, P, i64, P, P, P, P, P, P, P]
        L.orc_render.restype = i32
        L.orc_render_tiled.argtypes = [i64, P, P, P, P, P, i32, P, P, P, i32, i32, P, P, P]
        L.orc_render_tiled.restype = i32
        L.orc_pairs.argtypes = [i64, P, P, P, P, P, i32, P, P, i32, i32, i64, P, P]
        L.orc_pairs.restype = i64
        L.orc_render_bwd.argtypes = [i64, P, P, P, P, P, i32, P, P, P, P, P, P, P, P, P, P, ctypes.c_double, P, P,
                                     ctypes.c_double]
        L.orc_render_bwd.restype = i32
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _cam_arrays(cam):
    d = np.ascontiguousarray(np.concatenate([np.asarray(cam.R, np.float64).reshape(9),
                                             np.asarray(cam.t, np.float64).reshape(3),
                                             [cam.fx, cam.fy, cam.cx, cam.cy, cam.znear]]), np.float64)
    i = np.array([cam.width, cam.height], np.int32)
    return d, i


def _params(g):
    # FP32 inputs are promoted to FP64 exactly; FP64 inputs (finite-difference
    # tests) pass through unchanged.
    arrs = [np.ascontiguousarray(a, np.float64) for a in (g.means, g.scales, g.quats, g.opac, g.sh)]
    n = arrs[3].shape[0]
    assert arrs[0].shape == (3, n) and arrs[1].shape == (3, n) and arrs[2].shape == (4, n)
    assert arrs[4].shape == (16, 3, n)
    return n, arrs


def project(g, cam, sh_degree=3, tile=(16, 16)):
    """Per-Gaussian projection results (dict of arrays)."""
    n, arrs = _params(g)
    cd, ci = _cam_arrays(cam)
    out = dict(visible=np.zeros(n, np.int32), depth_bits=np.zeros(n, np.uint32), rect=np.zeros((n, 4), np.int32),
               tiles_touched=np.zeros(n, np.int32), uv=np.zeros((n, 2)), cov2d=np.zeros((n, 3)),
               conic=np.zeros((n, 3)), rgb=np.zeros((n, 3)), rgb_clamped=np.zeros((n, 3), np.int32),
               radius=np.zeros(n))
    lib().orc_project(n, *[_ptr(a) for a in arrs], sh_degree, _ptr(cd), _ptr(ci), tile[0], tile[1],
                      *[_ptr(out[k]) for k in ("visible", "depth_bits", "rect", "tiles_touched", "uv", "cov2d",
                                               "conic", "rgb", "rgb_clamped", "radius")])
    return out


def render(g, cam, sh_degree=3, bg=(0.0, 0.0, 0.0), pixels=None):
    """Untiled FP64 render.  Returns (img [3,H,W] or [3,npix], T_final, n_contrib, ambiguous)."""
    r = render_branches(g, cam, sh_degree, bg, pixels, branches=False)
    return r["img"], r["T"], r["n_contrib"], r["ambiguous"]


def render_branches(g, cam, sh_degree=3, bg=(0.0, 0.0, 0.0), pixels=None, branches=True):
    """Untiled FP64 render with the bookkeeping of threshold decisions.

    Returns a dict (shapes [3,H,W] / [H,W], or [3,npix] / [npix] for a pixel list):
      img, T, n_contrib  the render;
      ambiguous          image decisions that fall inside a threshold band (the
                         skip of alpha < 1/255, the stop before T < 1e-4);
      img_alt, T_alt     (branches=True) the result with the other branch taken at
                         a pixel's only ambiguous decision (equal to img, T elsewhere):
                         both are correct results, a pixel with two or more such
                         decisions has more than two;
      grad_ambiguous     contributing entries whose raw alpha lies in the band of the
                         0.99 clamp (image continuous, gradient not)."""
    n, arrs = _params(g)
    cd, ci = _cam_arrays(cam)
    bgv = np.asarray(bg, np.float64)
    if pixels is None:
        P = cam.width * cam.height
        pix = None
    else:
        pix = np.ascontiguousarray(pixels, np.int64)
        P = pix.shape[0]
    img = np.zeros((3, P))
    T = np.zeros(P)
    nc = np.zeros(P, np.int32)
    amb = np.zeros(P, np.int32)
    gamb = np.zeros(P, np.int32)
    img_alt = np.zeros((3, P)) if branches else None
    T_alt = np.zeros(P) if branches else None
    lib().orc_render(n, *[_ptr(a) for a in arrs], sh_degree, _ptr(cd), _ptr(ci), _ptr(bgv), _ptr(pix),
                     0 if pix is None else P, _ptr(img), _ptr(T), _ptr(nc), _ptr(amb), _ptr(img_alt), _ptr(T_alt),
                     _ptr(gamb))
    out = dict(img=img, T=T, n_contrib=nc, ambiguous=amb, grad_ambiguous=gamb, img_alt=img_alt, T_alt=T_alt)
    if pixels is None:
        H, W = cam.height, cam.width
        out = {k: (None if v is None else v.reshape((3, H, W) if v.ndim == 2 else (H, W))) for k, v in out.items()}
    return out


def render_tiled(g, cam, sh_degree=3, bg=(0.0, 0.0, 0.0), tile=(16, 16)):
    n, arrs = _params(g)
    cd, ci = _cam_arrays(cam)
    bgv = np.asarray(bg, np.float64)
    H, W = cam.height, cam.width
    img = np.zeros((3, H, W))
    T = np.zeros((H, W))
    nc = np.zeros((H, W), np.int32)
    lib().orc_render_tiled(n, *[_ptr(a) for a in arrs], sh_degree, _ptr(cd), _ptr(ci), _ptr(bgv), tile[0],
                           tile[1], _ptr(img), _ptr(T), _ptr(nc))
    return img, T, nc


def pairs(g, cam, sh_degree=3, tile=(16, 16)):
    """(tile id, Gaussian index) pairs sorted by (tile, depth bits, index)."""
    n, arrs = _params(g)
    cd, ci = _cam_arrays(cam)
    m = lib().orc_pairs(n, *[_ptr(a) for a in arrs], sh_degree, _ptr(cd), _ptr(ci), tile[0], tile[1], 0,
                        None, None)
    t = np.zeros(m, np.uint32)
    idx = np.zeros(m, np.uint32)
    lib().orc_pairs(n, *[_ptr(a) for a in arrs], sh_degree, _ptr(cd), _ptr(ci), tile[0], tile[1], m,
                    _ptr(t), _ptr(idx))
    return t, idx


def tile_ranges(tile_ids, n_tiles):
    """[start, end) of each tile in a tile-sorted pair list."""
    starts = np.searchsorted(tile_ids, np.arange(n_tiles), side="left")
    ends = np.searchsorted(tile_ids, np.arange(n_tiles), side="right")
    return np.stack([starts, ends], axis=1).astype(np.uint32)


def render_bwd(g, cam, dimg, sh_degree=3, bg=(0.0, 0.0, 0.0), near_band=None, magnitudes=False, mag_offset=1.0):
    """Exact FP64 gradient of sum(dimg * render(g)) w.r.t. every parameter.

    Returns dict(means [3,n], scales [3,n], quats [4,n], opac [n], sh [16,3,n],
    g2d [n,9] = d/d(u, v, conicA, conicB, conicC, opacity, r, g, b)).  With
    near_band, also near [n] (bool): the Gaussians that contribute to a pixel
    with a decision within that relative distance of its threshold (alpha vs
    1/255, T vs 1e-4, raw alpha vs 0.99), and those at the band: the gradient
    jumps there.  With magnitudes=True, also
    abs:<name> (same shapes): the chain rule applied to the sums of the
    magnitudes of the per-pixel terms, each weighted by (k + mag_offset) for an
    entry with k contributors in front of it at that pixel (the size of what
    each entry's summands add up to before they cancel, scaled by how the
    rounding of a front-to-back evaluation grows along the list)."""
    n, arrs = _params(g)
    cd, ci = _cam_arrays(cam)
    bgv = np.asarray(bg, np.float64)
    d = np.ascontiguousarray(dimg, np.float64)
    assert d.shape == (3, cam.height, cam.width)
    out = dict(g2d=np.zeros((n, 9)), means=np.zeros((3, n)), scales=np.zeros((3, n)), quats=np.zeros((4, n)),
               opac=np.zeros(n), sh=np.zeros((16, 3, n)))
    near = np.zeros(n, np.int32) if near_band is not None else None
    mag = np.zeros(59 * n) if magnitudes else None
    lib().orc_render_bwd(n, *[_ptr(a) for a in arrs], sh_degree, _ptr(cd), _ptr(ci), _ptr(bgv), _ptr(d),
                         *[_ptr(out[k]) for k in ("g2d", "means", "scales", "quats", "opac", "sh")],
                         0.0 if near_band is None else float(near_band), _ptr(near), _ptr(mag), float(mag_offset))
    if near is not None:
        out["near"] = near > 0
    if mag is not None:
        out["abs:means"] = mag[:3 * n].reshape(3, n)
        out["abs:scales"] = mag[3 * n:6 * n].reshape(3, n)
        out["abs:quats"] = mag[6 * n:10 * n].reshape(4, n)
        out["abs:opac"] = mag[10 * n:11 * n]
        out["abs:sh"] = mag[11 * n:].reshape(16, 3, n)
    return out

"""Host-only checks of the C ABI (no GPU needed): the library loads, exports
every function include/gs.h declares, and rejects bad arguments before any
launch."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gs.h")
LIB = os.path.join(ROOT, "paper_2404_01133_amd", "libgs.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libgs():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_five_path_entry_points():
    names = declared_functions()
    for fn in ("gs_lod_select", "gs_preprocess", "gs_bin_sort", "gs_rasterize_fwd", "gs_rasterize_bwd"):
        assert fn in names


def test_every_declared_function_is_exported(libgs):
    missing = [fn for fn in declared_functions() if not hasattr(libgs, fn)]
    assert not missing, missing


def test_status_strings_and_sizes(libgs):
    libgs.gs_status_string.restype = ctypes.c_char_p
    for code in (0, -1, -2, -3, -4):
        assert libgs.gs_status_string(code).decode().startswith("GS_")
    libgs.gs_record_bytes.restype = ctypes.c_size_t
    assert libgs.gs_record_bytes() == 48
    libgs.gs_workspace_bytes.restype = ctypes.c_size_t
    libgs.gs_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
    a = libgs.gs_workspace_bytes(1, 1000, 4000, 1, 256, 256, None)
    b = libgs.gs_workspace_bytes(1, 100000, 400000, 1, 256, 256, None)
    assert 0 < a < b
    assert libgs.gs_workspace_bytes(2, 1000, 0, 1, 256, 256, None) >= 1000 * 9 * 4


def test_invalid_arguments_rejected_before_launch(libgs):
    # NULL structures and pointers: every entry point returns GS_ERR_INVALID_ARG
    assert libgs.gs_lod_select(None, None, 0, None, 1, None, None, None, None) == -1
    assert libgs.gs_bin_sort(*([None] * 3), 1, 64, 64, *([None] * 1), ctypes.c_int64(10), ctypes.c_int64(10),
                             *([None] * 6), ctypes.c_size_t(0), None) == -1
    assert libgs.gs_rasterize_fwd(*([None] * 4), 1, 64, 64, *([None] * 6)) == -1
    assert libgs.gs_lod_select_points(None, 3, None, None, 1, ctypes.c_int64(0), None, None, None, None,
                                      ctypes.c_size_t(0), None) == -1


def test_pointwise_workspace_and_threshold_checks(libgs):
    libgs.gs_points_workspace_bytes.restype = ctypes.c_size_t
    sizes = (ctypes.c_int64 * 3)(5000, 0, 2048)
    a = libgs.gs_points_workspace_bytes(sizes, 3, 1)
    b = libgs.gs_points_workspace_bytes(sizes, 3, 4)
    assert 0 < a < b and b - a == 3 * (a - 256)
    assert libgs.gs_points_workspace_bytes(None, 3, 1) == 0

    class Gaussians(ctypes.Structure):
        _fields_ = [("means", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                    ("opac", ctypes.c_void_p), ("sh", ctypes.c_void_p), ("n", ctypes.c_int64),
                    ("sh_degree", ctypes.c_int32), ("attr_half", ctypes.c_int32)]
    dummy = 0x1000
    lv = (Gaussians * 3)(*[Gaussians(dummy, dummy, dummy, dummy, dummy, 10, 3, 0) for _ in range(3)])
    thr = (ctypes.c_double * 2)(500.0, 200.0)   # descending: rejected
    r = libgs.gs_lod_select_points(lv, 3, thr, ctypes.c_void_p(dummy), 1, ctypes.c_int64(16), ctypes.c_void_p(dummy),
                                   ctypes.c_void_p(dummy), ctypes.c_void_p(dummy), ctypes.c_void_p(dummy),
                                   ctypes.c_size_t(1 << 20), None)
    assert r == -1
    thr2 = (ctypes.c_double * 2)(200.0, 500.0)
    r = libgs.gs_lod_select_points(lv, 3, thr2, ctypes.c_void_p(dummy), 1, ctypes.c_int64(16), ctypes.c_void_p(dummy),
                                   ctypes.c_void_p(dummy), ctypes.c_void_p(dummy), ctypes.c_void_p(dummy),
                                   ctypes.c_size_t(8), None)
    assert r == -3   # workspace too small
    # gathering a binary16 set is not supported
    half = Gaussians(dummy, dummy, dummy, dummy, dummy, 10, 3, 1)
    r = libgs.gs_gather_gaussians(ctypes.byref(half), ctypes.c_void_p(dummy), ctypes.c_int64(10),
                                  ctypes.byref(Gaussians(dummy, dummy, dummy, dummy, dummy, 0, 0, 0)), None)
    assert r == -2


def test_unsupported_tile_shape_rejected(libgs):
    class Tuning(ctypes.Structure):
        _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("batch", ctypes.c_int32),
                    ("flags", ctypes.c_int32)]
    t = Tuning(12, 12, 256, 0)
    dummy = ctypes.c_void_p(0x1000)
    bg = (ctypes.c_float * 3)(0, 0, 0)
    r = libgs.gs_rasterize_fwd(dummy, dummy, dummy, None, 1, 64, 64, bg, ctypes.byref(t), dummy, dummy, dummy, None)
    assert r == -2


def test_static_scratch_variant_checks_before_any_device_call(libgs):
    # gs_bin_sort_static rejects NULL buffers and capacities whose workspace exceeds
    # the static array (GS_ERR_SCRATCH) before it looks the array up on a device
    P = ctypes.c_void_p
    f = libgs.gs_bin_sort_static
    f.restype = ctypes.c_int32
    f.argtypes = [P, P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int64, ctypes.c_int64,
                  P, P, P, P, P, P]

    class Tuning(ctypes.Structure):
        _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("batch", ctypes.c_int32),
                    ("flags", ctypes.c_int32)]

    t = Tuning(16, 16, 256, 0)
    one = P(1)  # never dereferenced: the call returns before any launch
    assert f(None, None, None, 1, 64, 64, None, 10, 10, None, None, None, None, None, None) == -1
    assert f(one, one, one, 1, 64, 64, ctypes.byref(t), 0, 10, one, one, one, None, one, None) == -1
    assert f(one, one, one, 1, 64, 64, ctypes.byref(t), 1 << 22, 1 << 24, one, one, one, None, one, None) == -6
    libgs.gs_status_string.restype = ctypes.c_char_p
    assert libgs.gs_status_string(-6).decode().startswith("GS_ERR_SCRATCH")


def test_chunk_refinement_sizes_and_checks(libgs):
    # chunk table sizes and the argument checks of gs_chunk_bounds / gs_lod_refine,
    # all decided on the host before any launch
    class Gaussians(ctypes.Structure):
        _fields_ = [("means", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                    ("opac", ctypes.c_void_p), ("sh", ctypes.c_void_p), ("n", ctypes.c_int64),
                    ("sh_degree", ctypes.c_int32), ("attr_half", ctypes.c_int32)]

    class Blocks(ctypes.Structure):
        _fields_ = [("lo", ctypes.c_void_p), ("hi", ctypes.c_void_p), ("cell", ctypes.c_void_p),
                    ("lvl_off", ctypes.c_void_p), ("lvl_cnt", ctypes.c_void_p), ("n_blocks", ctypes.c_int32),
                    ("n_levels", ctypes.c_int32), ("contraction", ctypes.c_void_p)]

    P = ctypes.c_void_p
    dummy = 0x1000
    sizes = (5000, 4096, 4097 * 3)
    lv = (Gaussians * 3)(*[Gaussians(dummy, dummy, dummy, dummy, dummy, n, 3, 0) for n in sizes])
    blk = Blocks(dummy, dummy, dummy, dummy, dummy, 4, 3, None)
    cap = libgs.gs_chunk_capacity
    cap.restype = ctypes.c_int64
    cap.argtypes = [P, P]
    # per level ceil(n / GS_CHUNK) chunks, plus one partial chunk per (block, level) run
    ch = 2048
    assert cap(lv, ctypes.byref(blk)) == 4 * 3 + sum((n + ch - 1) // ch for n in sizes)
    assert cap(None, ctypes.byref(blk)) == -1
    assert cap(lv, ctypes.byref(Blocks(dummy, dummy, dummy, dummy, dummy, 4, 0, None))) == -1

    wsb = libgs.gs_refine_workspace_bytes
    wsb.restype = ctypes.c_size_t
    wsb.argtypes = [ctypes.c_int32, ctypes.c_int64]
    a, b = wsb(1, 1000), wsb(8, 1000)
    assert 0 < a < b and b >= 8 * 1000 * 8   # a size and an offset per (view, chunk)
    assert wsb(0, 1000) == 0 and wsb(1, 0) == 0

    cb = libgs.gs_chunk_bounds
    cb.restype = ctypes.c_int32
    cb.argtypes = [P, P, P, P, ctypes.c_int64, P]
    assert cb(None, None, None, None, 10, None) == -1
    assert cb(lv, ctypes.byref(blk), P(dummy), P(dummy), 5, None) == -4   # fewer entries than chunks
    # a level too large for the packed gather entries (index bits) is refused before any launch
    big = (Gaussians * 3)(*[Gaussians(dummy, dummy, dummy, dummy, dummy, n, 3, 0) for n in (10, 10, 1 << 29)])
    need = cap(big, ctypes.byref(blk))
    assert cb(big, ctypes.byref(blk), P(dummy), P(dummy), need, None) == -2

    rf = libgs.gs_lod_refine
    rf.restype = ctypes.c_int32
    rf.argtypes = [P, P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_int64, ctypes.c_int64,
                   P, P, P, P, ctypes.c_size_t, P]
    one = P(dummy)
    assert rf(None, *([None] * 2), 1, 64, 64, *([None] * 2), 10, 10, *([None] * 4), 0, None) == -1
    ok_args = (ctypes.byref(blk), one, one, 2, 64, 64, one, one, 19, 1000, one, one, one, one)
    assert rf(*ok_args, ctypes.c_size_t(16), None) == -3                       # workspace too small
    bad_cap = ok_args[:9] + (1 << 32,) + ok_args[10:]
    assert rf(*bad_cap, ctypes.c_size_t(wsb(2, 19)), None) == -1               # record ids are u32
    bad_size = ok_args[:3] + (2, 0, 64) + ok_args[6:]
    assert rf(*bad_size, ctypes.c_size_t(wsb(2, 19)), None) == -1


def test_refinement_constants_match_the_header():
    import paper_2404_01133_amd.gs as gsmod
    text = open(HEADER).read()
    for name, value in (("GS_TUNE_PACKED_SELECTION", 8), ("GS_CHUNK", 2048), ("GS_PACKED_INDEX_BITS", 29)):
        assert re.search(r"#define %s %d\b" % (name, value), text)
        assert getattr(gsmod, name) == value

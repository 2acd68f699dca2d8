"""Host-only sanitizer runs (no GPU): the oracle's every entry point under
AddressSanitizer and UndefinedBehaviorSanitizer (built with g++ together with
tests/sanitize_oracle.cpp), and the library's host-side argument checks,
workspace sizing and status strings with the host half of every HIP translation
unit built with ASan/UBSan (hipcc -Xarch_host), driven through ctypes in a
child process with the sanitizer runtime preloaded."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def _asan_runtime():
    out = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


def test_oracle_under_address_and_undefined_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "oracle_san")
        subprocess.check_call(["g++", "-std=c++17", "-O1", "-ffp-contract=off"] + SAN +
                              [os.path.join(ROOT, "tests", "sanitize_oracle.cpp"),
                               os.path.join(ROOT, "oracle", "raster.cpp"), "-o", exe])
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                           env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1"))
        assert r.returncode == 0, r.stderr[-4000:]
        assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
        assert r.stdout.count("pairs") == 3


HOST_DRIVER = r'''
import ctypes, sys
L = ctypes.CDLL(sys.argv[1])
P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
L.gs_status_string.restype = ctypes.c_char_p
for c in range(-7, 1):
    assert L.gs_status_string(c)
L.gs_workspace_bytes.restype = sz
L.gs_workspace_bytes.argtypes = [i32, i64, i64, i32, i32, i32, P]
class Tuning(ctypes.Structure):
    _fields_ = [("tile_w", i32), ("tile_h", i32), ("batch", i32), ("flags", i32)]
for flags in (0, 4):
    t = Tuning(16, 16, 256, flags)
    for rc, pc in ((0, 0), (1, 1), (1000, 4000), (1 << 20, 1 << 22)):
        for which in (1, 2, 3):
            L.gs_workspace_bytes(which, rc, pc, 1, 64, 48, ctypes.byref(t))
    assert L.gs_workspace_bytes(1, -1, 10, 1, 64, 48, None) == 0
one = P(1)
t = Tuning(16, 16, 256, 0)
bad = Tuning(15, 16, 256, 0)
L.gs_bin_sort.restype = i32
L.gs_bin_sort.argtypes = [P, P, P, i32, i32, i32, P, i64, i64, P, P, P, P, P, P, sz, P]
assert L.gs_bin_sort(None, None, None, 1, 64, 48, None, 10, 10, None, None, None, None, None, None, 0, None) == -1
assert L.gs_bin_sort(one, one, one, 1, 64, 48, ctypes.byref(bad), 10, 10, one, one, one, None, one, one, 1 << 20, None) == -2
assert L.gs_bin_sort(one, one, one, 1, 64, 48, ctypes.byref(t), 10, 10, one, one, one, None, one, one, 16, None) == -3
assert L.gs_bin_sort(one, one, one, 0, 64, 48, ctypes.byref(t), 10, 10, one, one, one, None, one, one, 1 << 20, None) == -1
L.gs_bin_sort_static.restype = i32
L.gs_bin_sort_static.argtypes = [P, P, P, i32, i32, i32, P, i64, i64, P, P, P, P, P, P]
assert L.gs_bin_sort_static(one, one, one, 1, 64, 48, ctypes.byref(t), 1 << 22, 1 << 24, one, one, one, None, one, None) == -6
L.gs_rasterize_fwd.restype = i32
assert L.gs_rasterize_fwd(*([None] * 4), 1, 64, 48, *([None] * 6)) == -1
L.gs_lod_select.restype = i32
assert L.gs_lod_select(None, None, 0, None, 1, None, None, None, None) == -1
print("host checks ok")
'''


def test_library_host_side_under_address_and_undefined_sanitizers():
    asan = _asan_runtime()
    if asan is None:
        pytest.skip("no host AddressSanitizer runtime")
    sys.path.insert(0, ROOT)
    from paper_2404_01133_amd import build as b
    with tempfile.TemporaryDirectory() as d:
        objs = []
        procs = []
        for src in b.SOURCES:
            obj = os.path.join(d, os.path.splitext(src)[0] + ".o")
            cmd = [b.hipcc()] + b.flags() + [x for s in SAN[:2] for x in ("-Xarch_host", s)] + \
                ["-c", os.path.join(b.CSRC, src), "-o", obj]
            procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE))
            objs.append(obj)
        for p in procs:
            _, err = p.communicate(timeout=600)
            assert p.returncode == 0, err.decode()[-4000:]
        lib = os.path.join(d, "libgs_san.so")
        subprocess.check_call([b.hipcc(), "--offload-arch=" + b.ARCH, "-shared", "-fPIC", "-Xarch_host",
                               "-fsanitize=address,undefined", "-o", lib] + objs)
        ubsan = subprocess.run(["g++", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
        pre = asan + ((":" + ubsan) if os.path.isabs(ubsan) else "")
        r = subprocess.run([sys.executable, "-c", HOST_DRIVER, lib], capture_output=True, text=True, timeout=300,
                           env=dict(os.environ, LD_PRELOAD=pre, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0"))
        assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
        assert "host checks ok" in r.stdout
        assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr

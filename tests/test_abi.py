"""CPU checks of the C ABI: the library loads, exports every function that
include/canny.h declares, and rejects bad arguments on the host before any
device work (no GPU is touched by these calls)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "canny.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(?:int|size_t|int64_t|void|const char\*)\s+\**\s*(canny_\w+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_1710_07745_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libcanny.so not built")
    return _lib.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("canny_u8", "canny_f32", "canny_f32_sector", "canny_batch", "canny_mag_backward",
                     "canny_mag_forward", "canny_hysteresis", "canny_batch_plan_create"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_the_header():
    from paper_1710_07745_amd import _lib
    assert set(declared_functions()) <= set(_lib.SIGNATURES)


def test_status_strings_and_pitch(lib):
    assert lib.canny_status_string(0) == b"ok"
    assert lib.canny_status_string(2).startswith(b"workspace")
    assert lib.canny_status_string(99) == b"unknown status"
    assert lib.canny_abi_version() == 5
    for W, p in [(0, 0), (1, 4), (4, 4), (5, 4), (16, 4), (17, 8), (4096, 1024), (4097, 1028)]:
        assert lib.canny_class_pitch(W) == p, W


def test_workspace_sizes(lib):
    assert lib.canny_u8_workspace_bytes(4096, 4096) > 4096 * 1024
    assert lib.canny_f32_workspace_bytes(1, 1) > 0
    assert lib.canny_hysteresis_workspace_bytes(0, 5) == 0
    assert lib.canny_mag_backward_workspace_bytes(2, 64, 64, 9) >= 2 * 64 * 64 * 4
    assert lib.canny_mag_backward_workspace_bytes(2, 64, 64, 13) == 0


FAKE = C.c_void_p(0x1000)  # never dereferenced: validation fails first


def test_host_validation_u8(lib):
    ws, n = FAKE, 1 << 40
    assert lib.canny_u8(None, 8, 8, 8, 10, 20, None, 8, None, ws, n, None) == 1
    assert lib.canny_u8(FAKE, 7, 8, 8, 10, 20, None, 8, None, ws, n, None) == 1  # pitch < W
    assert lib.canny_u8(FAKE, 8, 0, 8, 10, 20, None, 8, None, ws, n, None) == 1
    assert lib.canny_u8(FAKE, 8, 8, 8, 30, 20, None, 8, None, ws, n, None) == 1  # low > high
    assert lib.canny_u8(FAKE, 8, 8, 8, -1, 20, None, 8, None, ws, n, None) == 1
    assert lib.canny_u8(FAKE, 8, 8, 8, 10, 20, C.c_void_p(0x1002), 8, None, ws, n, None) == 1  # alias
    assert lib.canny_u8(FAKE, 8, 8, 8, 10, 20, None, 8, C.c_void_p(0x2002), ws, n, None) == 1  # align
    assert lib.canny_u8(FAKE, 8, 8, 8, 10, 20, None, 8, None, None, n, None) == 2
    assert lib.canny_u8(FAKE, 8, 8, 8, 10, 20, None, 8, None, ws, 16, None) == 2


def test_host_validation_u8_noalloc(lib):
    """The allocation-free entry point validates like canny_u8 and rejects
    images whose workspace exceeds its static scratch before any device work."""
    from paper_1710_07745_amd import _lib
    f = lib.canny_u8_noalloc
    assert f(None, 8, 8, 8, 10, 20, None, 8, None, None) == 1
    assert f(FAKE, 7, 8, 8, 10, 20, None, 8, None, None) == 1  # pitch < W
    assert f(FAKE, 8, 8, 8, 30, 20, None, 8, None, None) == 1  # low > high
    assert f(FAKE, 8, 8, 8, 10, 20, C.c_void_p(0x1002), 8, None, None) == 1  # alias
    assert f(FAKE, 8, 8, 8, 10, 20, None, 8, C.c_void_p(0x2002), None) == 1  # align
    H = W = 8192
    assert lib.canny_u8_workspace_bytes(H, W) > _lib.CANNY_NOALLOC_SCRATCH_BYTES
    assert f(FAKE, W, H, W, 10, 20, None, W, None, None) == _lib.CANNY_ERR_TOO_LARGE
    assert lib.canny_status_string(_lib.CANNY_ERR_TOO_LARGE).startswith(b"image too large")


def test_host_validation_log(lib):
    f = lib.canny_log_u8
    E = C.c_void_p(0x900000)
    assert f(None, 8, 8, 8, 10, E, 8, None, 0, None) == 1
    assert f(FAKE, 8, 8, 8, 10, None, 8, None, 0, None) == 1
    assert f(FAKE, 7, 8, 8, 10, E, 8, None, 0, None) == 1      # pitch < W
    assert f(FAKE, 8, 8, 8, 10, E, 7, None, 0, None) == 1      # edges pitch < W
    assert f(FAKE, 8, 8, 8, -1, E, 8, None, 0, None) == 1      # t < 0
    assert f(FAKE, 8, 0, 8, 10, E, 8, None, 0, None) == 1
    assert f(FAKE, 8, 8, 8, 10, C.c_void_p(0x1004), 8, None, 0, None) == 1  # aliases the input
    assert f(FAKE, 8, 8, 8, 10, E, 8, C.c_void_p(0x800001), 8, None) == 1  # lap misaligned
    assert f(FAKE, 8, 8, 8, 10, E, 8, C.c_void_p(0x800000), 7, None) == 1  # lap pitch < W
    assert f(FAKE, 8, 8, 8, 10, E, 8, C.c_void_p(0x900004), 8, None) == 1  # lap aliases edges


def test_host_validation_f32(lib):
    n = 1 << 40
    f = lib.canny_f32
    assert f(FAKE, 8, 8, 8, 0.0, 3, 0.1, 0.2, 1, None, 8, None, None, None, FAKE, n, None) == 1
    assert f(FAKE, 8, 8, 8, 1.4, 9, 0.1, 0.2, 1, None, 8, None, None, None, FAKE, n, None) == 1
    assert f(FAKE, 8, 8, 8, 1.4, 3, 0.3, 0.2, 1, None, 8, None, None, None, FAKE, n, None) == 1
    assert f(FAKE, 8, 8, 8, float("nan"), 3, 0.1, 0.2, 1, None, 8, None, None, None, FAKE, n, None) == 1
    assert f(FAKE, 8, 8, 8, 1.4, 3, 0.1, 0.2, 1, None, 8, None, None, None, None, n, None) == 2


def test_host_validation_f32_sector(lib):
    n = 1 << 40
    f = lib.canny_f32_sector
    assert f(FAKE, 8, 8, 8, 0.0, 3, 10.0, 20.0, None, 8, None, None, FAKE, n, None) == 1
    assert f(FAKE, 8, 8, 8, 1.4, 0, 10.0, 20.0, None, 8, None, None, FAKE, n, None) == 1
    assert f(FAKE, 8, 8, 8, 1.4, 3, 30.0, 20.0, None, 8, None, None, FAKE, n, None) == 1
    assert f(FAKE, 4, 8, 8, 1.4, 3, 10.0, 20.0, None, 8, None, None, FAKE, n, None) == 1
    assert f(FAKE, 8, 8, 8, 1.4, 3, 10.0, 20.0, None, 8, None, None, None, n, None) == 2


def test_host_validation_video(lib):
    out = C.c_void_p()
    assert lib.canny_video_create(0, 8, 1, 2, 3, C.byref(out)) == 1
    assert lib.canny_video_create(8, 8, 3, 2, 3, C.byref(out)) == 1
    assert lib.canny_video_create(8, 8, 1, 2, 0, C.byref(out)) == 1
    assert lib.canny_video_create(8, 8, 1, 2, 17, C.byref(out)) == 1
    assert lib.canny_video_create(8, 8, 1, 2, 3, None) == 1
    # sizes canny_u8 rejects are rejected at creation: a side above 2^20
    assert lib.canny_video_create(1, (1 << 20) + 1, 1, 2, 3, C.byref(out)) == 1
    assert lib.canny_video_create((1 << 20) + 1, 1, 1, 2, 3, C.byref(out)) == 1
    assert lib.canny_video_push(None, FAKE, FAKE) == 1
    assert lib.canny_video_sync(None) == 1
    lib.canny_video_destroy(None)


def test_host_validation_mag_and_batch(lib):
    assert lib.canny_mag_forward(None, FAKE, 1, 8, 8, 9, FAKE, None) == 1
    assert lib.canny_mag_forward(FAKE, FAKE, 1, 8, 8, 13, C.c_void_p(0x900000), None) == 1
    assert lib.canny_mag_backward(FAKE, FAKE, FAKE, 0, 8, 8, 9, FAKE, FAKE, FAKE, 1 << 30, None) == 1
    out = C.c_void_p()
    H = (C.c_int32 * 1)(10)
    W = (C.c_int32 * 1)(10)
    assert lib.canny_batch_plan_create(0, H, W, 1, 2, 0, C.byref(out)) == 1
    assert lib.canny_batch_plan_create(1, H, W, 3, 2, 0, C.byref(out)) == 1
    assert lib.canny_batch_plan_create(1, H, W, 1, 2, 0, None) == 1
    assert lib.canny_batch(None, None, None, None, None, None, 0, None) == 1
    assert lib.canny_batch_workspace_bytes(None) == 0
    lib.canny_batch_plan_destroy(None)


def test_timing_validation(lib):
    """Argument checks of the stage-timing calls (no events are created)."""
    ms = C.c_double(-1.0)
    n = C.c_int64(-1)
    assert lib.canny_timing_begin(0) == 1
    assert lib.canny_timing_begin(65537) == 1
    assert lib.canny_timing_read(7, C.byref(ms), C.byref(n)) == 1
    assert lib.canny_timing_read(-1, C.byref(ms), C.byref(n)) == 1
    assert lib.canny_timing_read(2, None, C.byref(n)) == 1
    assert lib.canny_timing_read(2, C.byref(ms), C.byref(n)) == 0  # nothing recorded
    assert ms.value == 0.0 and n.value == 0
    assert lib.canny_timing_end() == 0

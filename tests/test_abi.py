"""C-ABI checks that need no GPU: the library loads, exports every symbol that
include/pdiv.h declares, and rejects bad arguments synchronously (before any
device work) with PDIV_ERR_INVALID and a message."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_2510_01190_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdiv.h")
INVALID = 1

pytestmark = pytest.mark.skipif(not os.path.exists(P.LIB_PATH), reason="libpdiv.so not built")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdiv_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_core_calls():
    names = _declared()
    for core in ("pdiv_moments", "pdiv_divergence_gaussian", "pdiv_lcp", "pdiv_mc_lcp"):
        assert core in names


def test_every_declared_symbol_is_exported():
    L = P.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(_declared()) == set(P.EXPORTS)


def test_version_and_status_strings():
    L = P.lib()
    assert L.pdiv_version().decode().count(".") == 2
    assert L.pdiv_status_string(0) == b"ok"
    assert L.pdiv_status_string(1) == b"invalid argument"


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
NUL = ctypes.c_void_p(0)


def _iso(vals):
    a = np.asarray(vals, np.float32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _expect_invalid(status, fragment):
    assert status == INVALID
    assert fragment in P.lib().pdiv_last_error().decode()


def test_lcp_rejects_bad_arguments():
    L = P.lib()
    keep, ip = _iso([0.1, 0.2])
    _expect_invalid(L.pdiv_lcp(FAKE, FAKE, 1, 8, ip, 2, FAKE, 0, 0, NUL), "at least 2x2")
    _expect_invalid(L.pdiv_lcp(FAKE, FAKE, 8, 1, ip, 2, FAKE, 0, 0, NUL), "at least 2x2")
    _expect_invalid(L.pdiv_lcp(NUL, FAKE, 8, 8, ip, 2, FAKE, 0, 0, NUL), "div_mean is NULL")
    _expect_invalid(L.pdiv_lcp(FAKE, FAKE, 8, 8, ip, 2, NUL, 0, 0, NUL), "lcp is NULL")
    _expect_invalid(L.pdiv_lcp(FAKE, FAKE, 8, 8, ip, 2, ctypes.c_void_p(0x1002), 0, 0, NUL),
                    "4-byte aligned")
    _expect_invalid(L.pdiv_lcp_from_moments(FAKE, FAKE, FAKE, FAKE, 0, 8, 8, 1.0, 1.0, ip, 2,
                                            ctypes.c_void_p(0x1001), 0, 0, NUL), "4-byte aligned")
    _expect_invalid(L.pdiv_lcp(FAKE, FAKE, 8, 8, ip, 0, FAKE, 0, 0, NUL), "n_iso")
    _expect_invalid(L.pdiv_lcp(FAKE, FAKE, 8, 8, ip, 257, FAKE, 0, 0, NUL), "n_iso")
    _expect_invalid(L.pdiv_lcp(FAKE, FAKE, 8, 8, None, 2, FAKE, 0, 0, NUL), "isovalues_host")
    _expect_invalid(L.pdiv_lcp(FAKE, FAKE, 1 << 22, 8, ip, 2, FAKE, 0, 0, NUL), "too large")
    _expect_invalid(L.pdiv_lcp(FAKE, FAKE, 8, 8, ip, 2, FAKE, 6, 0, NUL), "lcp_row_pitch")
    _expect_invalid(L.pdiv_lcp(FAKE, FAKE, 8, 8, ip, 2, FAKE, -1, 0, NUL), "lcp_row_pitch")
    _expect_invalid(L.pdiv_lcp(FAKE, FAKE, 8, 8, ip, 2, FAKE, 1 << 62, 0, NUL), "lcp_row_pitch")
    # the largest pitch on the most rows: rows x pitch exceeds 2^52 floats and
    # is rejected before any int64 product of the two is formed
    _expect_invalid(L.pdiv_lcp(FAKE, FAKE, 1 << 21, 8, ip, 2, FAKE, 1 << 52, 0, NUL),
                    "too large")
    _expect_invalid(L.pdiv_lcp(FAKE, FAKE, 1 << 21, 8, ip, 2, FAKE, 1 << 40, 1 << 20, NUL),
                    "too large")
    # maps that overlap: plane stride between a row and a map, or rows too short
    _expect_invalid(L.pdiv_lcp(FAKE, FAKE, 8, 8, ip, 2, FAKE, 7, 20, NUL), "overlap")
    _expect_invalid(L.pdiv_lcp(FAKE, FAKE, 8, 8, ip, 2, FAKE, 10, 7, NUL), "overlap")
    _expect_invalid(L.pdiv_lcp(FAKE, FAKE, 8, 8, ip, 2, FAKE, 0, -5, NUL), "lcp_plane_stride")


def test_fused_and_divergence_reject_bad_spacing_and_dtype():
    L = P.lib()
    keep, ip = _iso([0.0])
    for dx, dy in ((0.0, 1.0), (1.0, -2.0), (float("nan"), 1.0), (1.0, float("inf"))):
        _expect_invalid(L.pdiv_lcp_from_moments(FAKE, FAKE, FAKE, FAKE, 0, 8, 8, dx, dy, ip, 1,
                                                FAKE, 0, 0, NUL), "dx and dy")
        _expect_invalid(L.pdiv_divergence_gaussian(FAKE, FAKE, FAKE, FAKE, 0, 8, 8, dx, dy,
                                                   FAKE, FAKE, NUL), "dx and dy")
    _expect_invalid(L.pdiv_lcp_from_moments(FAKE, FAKE, FAKE, FAKE, 7, 8, 8, 1.0, 1.0, ip, 1,
                                            FAKE, 0, 0, NUL), "dtype")
    _expect_invalid(L.pdiv_divergence_gaussian(FAKE, NUL, FAKE, FAKE, 0, 8, 8, 1.0, 1.0, FAKE,
                                               FAKE, NUL), "var_u is NULL")


def test_moments_rejects_bad_arguments():
    L = P.lib()
    _expect_invalid(L.pdiv_moments(FAKE, FAKE, 0, 1, 4, 4, 0, 1, FAKE, FAKE, FAKE, FAKE, 0, NUL),
                    "n_members")
    _expect_invalid(L.pdiv_moments(FAKE, FAKE, 0, 5, 4, 4, 0, 2, FAKE, FAKE, FAKE, FAKE, 0, NUL),
                    "ddof")
    _expect_invalid(L.pdiv_moments(FAKE, FAKE, 0, 5, 4, 4, 15, 1, FAKE, FAKE, FAKE, FAKE, 0, NUL),
                    "member_stride")
    _expect_invalid(L.pdiv_moments(FAKE, FAKE, 0, 5, 4, 4, 0, 1, FAKE, FAKE, NUL, FAKE, 0, NUL),
                    "mean_v is NULL")
    _expect_invalid(L.pdiv_moments(FAKE, FAKE, 0, 5, 4, 4, 0, 1, FAKE, FAKE, FAKE, FAKE, 9, NUL),
                    "out_dtype")


def test_mc_rejects_bad_arguments():
    L = P.lib()
    keep, ip = _iso([0.0])
    _expect_invalid(L.pdiv_mc_lcp(FAKE, FAKE, FAKE, FAKE, 0, 8, 8, 1.0, 1.0, ip, 1, 0, 1, 0,
                                  FAKE, NUL), "n_samples")
    _expect_invalid(L.pdiv_mc_lcp(FAKE, FAKE, FAKE, FAKE, 0, 8, 8, 1.0, 1.0, ip, 1, 1 << 31, 1,
                                  0, FAKE, NUL), "n_samples")
    _expect_invalid(L.pdiv_mc_lcp(FAKE, FAKE, FAKE, FAKE, 0, 1 << 21, 1 << 11, 1.0, 1.0, ip, 1,
                                  10, 1, 0, FAKE, NUL), "2^32")
    for mode in (2, 7, 0xFFFFFFFF):
        _expect_invalid(L.pdiv_mc_lcp(FAKE, FAKE, FAKE, FAKE, 0, 8, 8, 1.0, 1.0, ip, 1, 10, 1,
                                      mode, FAKE, NUL), "mode")
    # nx = 2^29 with ny = 7 keeps ny*nx below 2^32, but the launch would need
    # 2^24 blocks of 256 threads, one work-item more than a dispatch holds
    for mode in (0, 1):
        _expect_invalid(L.pdiv_mc_lcp(FAKE, FAKE, FAKE, FAKE, 0, 7, 1 << 29, 1.0, 1.0, ip, 1,
                                      10, 1, mode, FAKE, NUL), "too large")
    _expect_invalid(L.pdiv_mc_sample_field(FAKE, FAKE, FAKE, FAKE, 0, 8, 8, -1, 1, FAKE, FAKE,
                                           NUL), "sample")


def test_error_message_is_per_thread():
    import threading
    L = P.lib()
    keep, ip = _iso([0.0])
    assert L.pdiv_lcp(FAKE, FAKE, 1, 8, ip, 1, FAKE, 0, 0, NUL) == INVALID
    seen = {}

    def other():
        seen["msg"] = L.pdiv_last_error().decode()

    t = threading.Thread(target=other)
    t.start()
    t.join()
    assert seen["msg"] == ""
    assert "2x2" in L.pdiv_last_error().decode()


def test_batch_rejects_bad_fields():
    L = P.lib()
    iso_dev = FAKE
    good = P._Field(FAKE, FAKE, FAKE, FAKE, 8, 8, 1.0, 1.0, iso_dev, 4, FAKE)
    out = ctypes.c_void_p()
    for bad, frag in (
        (P._Field(FAKE, FAKE, FAKE, FAKE, 8, 8, 1.0, 1.0, iso_dev, 17, FAKE), "n_iso"),
        (P._Field(FAKE, FAKE, FAKE, FAKE, 1, 8, 1.0, 1.0, iso_dev, 4, FAKE), "bad grid"),
        (P._Field(NUL, FAKE, FAKE, FAKE, 8, 8, 1.0, 1.0, iso_dev, 4, FAKE), "NULL"),
        (P._Field(FAKE, FAKE, FAKE, FAKE, 8, 8, 0.0, 1.0, iso_dev, 4, FAKE), "dx and dy"),
        (P._Field(FAKE, FAKE, FAKE, FAKE, 8, 8, 1.0, 1.0, iso_dev, 4, FAKE, 6), "lcp_row_pitch"),
    ):
        arr = (P._Field * 2)(good, bad)
        _expect_invalid(L.pdiv_batch_create(arr, 2, 0, 0, NUL, ctypes.byref(out)), frag)
        assert out.value is None
    arr = (P._Field * 1)(good)
    _expect_invalid(L.pdiv_batch_create(arr, 0, 0, 0, NUL, ctypes.byref(out)), "n_fields")
    _expect_invalid(L.pdiv_batch_create(arr, 1, 5, 0, NUL, ctypes.byref(out)), "dtype")
    _expect_invalid(L.pdiv_batch_create(arr, 1, 0, 8, NUL, ctypes.byref(out)), "flags")
    _expect_invalid(L.pdiv_batch_launch(NUL, NUL), "batch is NULL")


def test_server_calls_reject_null_handles():
    L = P.lib()
    _expect_invalid(L.pdiv_server_reserve_staging(NUL, 1024, 0, 1), "server is NULL")
    _expect_invalid(L.pdiv_server_destroy(NUL), "server is NULL")



def test_3d_calls_reject_bad_arguments():
    L = P.lib()
    iso, ip = _iso([0.1])
    six = [FAKE] * 6
    _expect_invalid(L.pdiv_divergence_gaussian_3d(*six, 0, 1, 8, 8, 1.0, 1.0, 1.0, FAKE, FAKE,
                                                  NUL), "at least 2x2x2")
    _expect_invalid(L.pdiv_divergence_gaussian_3d(*six, 0, 4, 8, 8, 1.0, 1.0, 0.0, FAKE, FAKE,
                                                  NUL), "dz")
    _expect_invalid(L.pdiv_divergence_gaussian_3d(*six, 0, 4, 8, 8, 1.0, -1.0, 1.0, FAKE, FAKE,
                                                  NUL), "dx and dy")
    _expect_invalid(L.pdiv_divergence_gaussian_3d(*six[:5], NUL, 0, 4, 8, 8, 1.0, 1.0, 1.0,
                                                  FAKE, FAKE, NUL), "var_w")
    _expect_invalid(L.pdiv_divergence_gaussian_3d(*six, 5, 4, 8, 8, 1.0, 1.0, 1.0, FAKE, FAKE,
                                                  NUL), "dtype")
    _expect_invalid(L.pdiv_divergence_gaussian_3d(*six, 0, 1 << 14, 1 << 14, 1 << 14, 1.0, 1.0,
                                                  1.0, FAKE, FAKE, NUL), "too large")
    _expect_invalid(L.pdiv_lcp_3d(FAKE, FAKE, 4, 8, 1, ip, 1, FAKE, 0, 0, NUL), "at least 2x2x2")
    _expect_invalid(L.pdiv_lcp_3d(FAKE, FAKE, 4, 8, 8, ip, 0, FAKE, 0, 0, NUL), "n_iso")
    _expect_invalid(L.pdiv_lcp_3d(FAKE, FAKE, 4, 8, 8, ip, 257, FAKE, 0, 0, NUL), "n_iso")
    _expect_invalid(L.pdiv_lcp_3d(FAKE, FAKE, 4, 8, 8, ip, 1, NUL, 0, 0, NUL), "lcp")
    _expect_invalid(L.pdiv_lcp_3d(FAKE, FAKE, 4, 1 << 22, 8, ip, 1, FAKE, 0, 0, NUL), "too large")
    _expect_invalid(L.pdiv_lcp_3d(FAKE, FAKE, 4, 9000, 9000, ip, 1, FAKE, 0, 0, NUL), "limited")
    _expect_invalid(L.pdiv_lcp_3d_from_moments(*six, 1, 4, 13000, 13000, 1.0, 1.0, 1.0, ip, 1,
                                               FAKE, 0, 0, NUL), "limited")
    _expect_invalid(L.pdiv_lcp_3d(FAKE, FAKE, 4, 8, 8, ip, 1, FAKE, 6, 0, NUL), "lcp_row_pitch")
    _expect_invalid(L.pdiv_lcp_3d(FAKE, FAKE, 4, 8, 8, ip, 2, FAKE, 32, 32 * 7 * 3 - 1, NUL),
                    "lcp_plane_stride")
    _expect_invalid(L.pdiv_lcp_3d(FAKE, FAKE, 4, 8, 8, ip, 2, FAKE, 1 << 50, 0, NUL),
                    "too large")
    _expect_invalid(L.pdiv_lcp_3d_from_moments(*six, 0, 4, 8, 8, 1.0, 1.0, -2.0, ip, 1, FAKE,
                                               0, 0, NUL), "dz")
    _expect_invalid(L.pdiv_lcp_3d_from_moments(*six, 0, 4, 8, 8, 1.0, 1.0, 1.0, ip, 0, FAKE,
                                               0, 0, NUL), "n_iso")
    _expect_invalid(L.pdiv_lcp_3d_from_moments(*six, 3, 4, 8, 8, 1.0, 1.0, 1.0, ip, 1, FAKE,
                                               0, 0, NUL), "dtype")
    _expect_invalid(L.pdiv_lcp_3d_from_moments(*six, 0, 2, 1, 8, 1.0, 1.0, 1.0, ip, 1, FAKE,
                                               0, 0, NUL), "at least 2x2x2")
    _expect_invalid(L.pdiv_lcp_3d_from_moments(*six, 0, 4, 8, 8, 1.0, 1.0, 1.0, ip, 1, NUL,
                                               0, 0, NUL), "lcp")


def test_speed_gradient_rejects_bad_arguments():
    L = P.lib()
    outs = [FAKE] * 4
    _expect_invalid(L.pdiv_speed_gradient_moments(FAKE, FAKE, 0, 5, 1, 8, 0, 1.0, 1.0, 1, *outs, 0,
                                                  NUL), "at least 2x2")
    _expect_invalid(L.pdiv_speed_gradient_moments(FAKE, FAKE, 0, 1, 8, 8, 0, 1.0, 1.0, 1, *outs, 0,
                                                  NUL), "n_members")
    _expect_invalid(L.pdiv_speed_gradient_moments(FAKE, FAKE, 0, 5, 8, 8, 0, 1.0, 1.0, 2, *outs, 0,
                                                  NUL), "ddof")
    _expect_invalid(L.pdiv_speed_gradient_moments(FAKE, FAKE, 0, 5, 8, 8, 10, 1.0, 1.0, 1, *outs,
                                                  0, NUL), "member_stride")
    _expect_invalid(L.pdiv_speed_gradient_moments(FAKE, FAKE, 0, 5, 8, 8, 0, 0.0, 1.0, 1, *outs, 0,
                                                  NUL), "dx and dy")
    _expect_invalid(L.pdiv_speed_gradient_moments(FAKE, FAKE, 0, 5, 8, 8, 0, 1.0, 1.0, 1, *outs, 9,
                                                  NUL), "out_dtype")
    _expect_invalid(L.pdiv_speed_gradient_moments(NUL, FAKE, 0, 5, 8, 8, 0, 1.0, 1.0, 1, *outs, 0,
                                                  NUL), "u_members")


def test_isocontour_rejects_bad_arguments():
    L = P.lib()
    _expect_invalid(L.pdiv_isocontour(FAKE, 1, 8, ctypes.c_float(0.0), FAKE, FAKE, 4, NUL),
                    "at least 2x2")
    _expect_invalid(L.pdiv_isocontour(FAKE, 8, 8, ctypes.c_float(0.0), NUL, FAKE, 4, NUL),
                    "row_offsets")
    _expect_invalid(L.pdiv_isocontour(FAKE, 8, 8, ctypes.c_float(0.0), FAKE, NUL, 4, NUL),
                    "segments is NULL")
    _expect_invalid(L.pdiv_isocontour(FAKE, 8, 8, ctypes.c_float(0.0), FAKE, FAKE, -1, NUL),
                    "max_segments")
    _expect_invalid(L.pdiv_isocontour(FAKE, 8, 8, ctypes.c_float(0.0), FAKE,
                                      ctypes.c_void_p(0x1004), 4, NUL), "aligned")


def test_spaghetti_rejects_bad_arguments():
    L = P.lib()
    c = ctypes.c_float(0.0)
    _expect_invalid(L.pdiv_spaghetti(FAKE, FAKE, 0, 0, 8, 8, 0, 1.0, 1.0, c, FAKE, FAKE, FAKE, 4,
                                     NUL), "n_members")
    _expect_invalid(L.pdiv_spaghetti(FAKE, FAKE, 0, 3, 8, 8, 10, 1.0, 1.0, c, FAKE, FAKE, FAKE, 4,
                                     NUL), "member_stride")
    _expect_invalid(L.pdiv_spaghetti(FAKE, FAKE, 0, 3, 8, 8, 0, 1.0, 1.0, c, NUL, FAKE, FAKE, 4,
                                     NUL), "div_workspace")
    _expect_invalid(L.pdiv_spaghetti(FAKE, FAKE, 0, 3, 8, 8, 0, 1.0, 1.0, c, FAKE, FAKE, NUL, 4,
                                     NUL), "segments is NULL")
    _expect_invalid(L.pdiv_spaghetti(FAKE, FAKE, 0, 3, 1, 8, 0, 1.0, 1.0, c, FAKE, FAKE, FAKE, 4,
                                     NUL), "at least 2x2")
    # 4096 members of 1024 x 1024: 2^32 threads in one launch
    _expect_invalid(L.pdiv_spaghetti(FAKE, FAKE, 0, 4096, 1024, 1024, 0, 1.0, 1.0, c, FAKE, FAKE,
                                     FAKE, 4, NUL), "n_members")


def test_debug_flags_reject_unknown_bits():
    L = P.lib()
    _expect_invalid(L.pdiv_set_debug(8), "unknown debug flags")
    assert L.pdiv_set_debug(0) == 0
    assert L.pdiv_set_debug(1 | 2 | 4) == 0
    assert L.pdiv_set_debug(0) == 0


def test_log_mode_writes_one_line_per_call():
    """PDIV_LOG=1 at load: each core call (even one that is rejected) writes
    its name and sizes to stderr; without it nothing is written."""
    import subprocess
    import sys
    code = ("import ctypes, sys; sys.path.insert(0, %r); import paper_2510_01190_amd as P; "
            "L = P.lib(); iso = (ctypes.c_float * 1)(0.0); "
            "print(L.pdiv_lcp(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000), 1, 8, iso, 1, "
            "ctypes.c_void_p(0x1000), 0, 0, None))" % ROOT)
    for env_val, expect in (("1", True), ("0", False)):
        env = dict(os.environ, PDIV_LOG=env_val)
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                           timeout=120)
        assert r.stdout.strip() == str(INVALID)
        assert ("[pdiv] pdiv_lcp ny=1 nx=8 n_iso=1" in r.stderr) == expect, r.stderr

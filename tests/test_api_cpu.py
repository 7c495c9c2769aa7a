"""The C ABI library loads, exports every declared entry point, and rejects bad arguments
before touching the GPU (these calls make no HIP call, so they run without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_1609_01839_amd as gfd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gfdeconv.h")

pytestmark = pytest.mark.skipif(not os.path.exists(gfd.library_path()), reason="library not built")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:gfd_status|void|const char \*)\s*\*?\s*(\w+)\s*\(", src, flags=re.M)))


def test_every_declared_symbol_is_exported_and_bound():
    lib = gfd.load_library()
    names = declared_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
        assert n in gfd.EXPORTS, n
    assert set(gfd.EXPORTS) == set(names)


def test_invalid_arguments_are_rejected_without_gpu():
    lib = gfd.load_library()
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)
    cases = [
        # (M, N, kh, kw, sigma2, w, eps, rho, expected)
        (7 * 16, 64, 3, 3, 1.0, 3, 1.0, 1.0, -2),     # 7 is not 2^a 3^b 5^c
        (8192, 64, 3, 3, 1.0, 3, 1.0, 1.0, -2),       # too large
        (64, 64, 4, 3, 1.0, 3, 1.0, 1.0, -2),         # even PSF side
        (64, 64, 65, 3, 1.0, 3, 1.0, 1.0, -2),        # PSF larger than the image
        (64, 64, 3, 3, -1.0, 3, 1.0, 1.0, -1),        # negative noise variance
        (64, 64, 3, 3, 1.0, 4, 1.0, 1.0, -1),         # even window
        (64, 64, 3, 3, 1.0, 65, 1.0, 1.0, -1),        # window larger than the image
        (64, 64, 3, 3, 1.0, 3, 0.0, 1.0, -1),         # eps must be > 0
        (64, 64, 3, 3, 1.0, 3, float("nan"), 1.0, -1),
        (64, 64, 3, 3, 1.0, 3, 1.0, 1.5, -1),         # rho > 1
        (64, 32, 3, 3, 1.0, 33, 1.0, 1.0, -1),        # window wider than the image (N = 32)
    ]
    for M, N, kh, kw, s2, w, eps, rho, want in cases:
        rc = lib.deconv_init(ctypes.byref(ctx), fake, M, N, fake, kh, kw, s2, w, eps, rho, None)
        assert rc == want, (M, N, kh, kw, s2, w, eps, rho, rc, lib.gfd_last_error())
        assert ctx.value is None
        assert lib.gfd_last_error()
    assert lib.deconv_init(ctypes.byref(ctx), None, 64, 64, fake, 3, 3, 1.0, 3, 1.0, 1.0, None) == -1
    assert lib.deconv_init(None, fake, 64, 64, fake, 3, 3, 1.0, 3, 1.0, 1.0, None) == -1


def test_guided_filter_argument_checks():
    lib = gfd.load_library()
    a, b, c = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000), ctypes.c_void_p(0x30000)
    assert lib.guided_filter(None, b, c, 16, 16, 3, 1.0, None) == -1
    assert lib.guided_filter(a, b, c, 16, 16, 2, 1.0, None) == -1
    assert lib.guided_filter(a, b, c, 16, 16, 17, 1.0, None) == -1
    assert lib.guided_filter(a, b, c, 0, 16, 1, 1.0, None) == -2
    assert lib.guided_filter(a, b, c, 16, 16, 3, -1.0, None) == -1
    assert lib.guided_filter(a, b, ctypes.c_void_p(0x10000 + 64), 16, 16, 3, 1.0, None) == -1  # u overlaps uI


def test_guided_filter_clipped_argument_checks():
    lib = gfd.load_library()
    a, b, c = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000), ctypes.c_void_p(0x30000)
    assert lib.guided_filter_clipped(None, b, c, 16, 16, 3, 1.0, None) == -1
    assert lib.guided_filter_clipped(a, b, c, 16, 16, 2, 1.0, None) == -1
    assert lib.guided_filter_clipped(a, b, c, 16, 16, 3, 0.0, None) == -1
    assert lib.guided_filter_clipped(a, b, c, 64, 32, 33, 1.0, None) == -1  # w > N
    assert lib.guided_filter_clipped(a, ctypes.c_void_p(0x30000 - 8), c, 16, 16, 3, 1.0, None) == -1


def test_guided_filter_color_argument_checks():
    lib = gfd.load_library()
    a, b, c = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x200000), ctypes.c_void_p(0x300000)
    assert lib.guided_filter_color(None, b, c, 16, 16, 3, 1.0, None) == -1
    assert lib.guided_filter_color(a, b, c, 16, 16, 4, 1.0, None) == -1
    assert lib.guided_filter_color(a, b, c, 16, 16, 17, 1.0, None) == -1
    assert lib.guided_filter_color(a, b, c, 16, 0, 1, 1.0, None) == -2
    assert lib.guided_filter_color(a, b, c, 16, 16, 3, 0.0, None) == -1
    assert lib.guided_filter_color(a, b, c, 16, 64, 19, 1.0, None) == -1   # w > M
    # u inside the third channel plane of I3 (planes of 16 * 16 floats)
    assert lib.guided_filter_color(a, b, ctypes.c_void_p(0x100000 + 2 * 1024 + 8), 16, 16, 3, 1.0, None) == -1
    assert lib.guided_filter_color(a, b, ctypes.c_void_p(0x200000 - 4), 16, 16, 3, 1.0, None) == -1  # overlaps up
    assert lib.gfd_last_error()


def test_foreign_and_null_contexts():
    lib = gfd.load_library()
    bogus = ctypes.c_void_p(0xDEAD0)
    assert lib.deconv_iterate(bogus, 1, None, None, None) == -5
    assert lib.deconv_iterate(None, 1, None, None, None) == -5
    assert lib.deconv_reset(bogus, None) == -5
    assert lib.deconv_set_graph(bogus, 1) == -5
    flags = ctypes.c_uint()
    assert lib.deconv_get_status(bogus, ctypes.byref(flags)) == -5
    lib.deconv_destroy(None)
    lib.deconv_destroy(bogus)   # unknown pointers are ignored, never dereferenced
    assert "invalid" in lib.gfd_last_error().decode() or lib.gfd_last_error() is not None


def test_batch_descriptors_are_checked_without_gpu():
    lib = gfd.load_library()
    ctx = ctypes.c_void_p()
    fake = 0x1000
    good = gfd.GfdImage(fake, 64, 64, fake, 3, 3, 1.0, 3, 1.0, -1.0)
    bad = gfd.GfdImage(fake, 64, 64, fake, 3, 3, 1.0, 4, 1.0, -1.0)      # even window
    arr = (gfd.GfdImage * 3)(good, good, bad)
    rc = lib.deconv_init_batch(ctypes.byref(ctx), ctypes.cast(arr, ctypes.c_void_p), 3, None)
    assert rc == -1 and ctx.value is None
    assert "image 2" in lib.gfd_last_error().decode()
    assert lib.deconv_init_batch(ctypes.byref(ctx), ctypes.cast(arr, ctypes.c_void_p), 0, None) == -1
    assert lib.deconv_init_batch(ctypes.byref(ctx), None, 1, None) == -1
    assert lib.deconv_init_batch(ctypes.byref(ctx), ctypes.cast(arr, ctypes.c_void_p), 5000, None) == -1
    assert lib.deconv_image_info(None, 0, None, None, None, None) == -5
    assert lib.deconv_image_domain(None, 0, None, None, None) == -5
    assert ctypes.sizeof(gfd.GfdImage) == 64


def test_boundary_flags_are_checked_without_gpu():
    lib = gfd.load_library()
    ctx = ctypes.c_void_p()
    fake = 0x1000

    def init(M, N, kh, boundary):
        img = gfd.GfdImage(fake, M, N, fake, kh, kh, 1.0, 3, 1.0, -1.0, boundary)
        return lib.deconv_init_batch(ctypes.byref(ctx), ctypes.byref(img), 1, None)

    assert init(64, 64, 3, 4) == -1                      # unknown flag
    assert init(64, 64, 3, -1) == -1
    assert init(4096, 64, 3, gfd.BOUNDARY_PAD) == -2     # padded domain 4098 -> 4320 > 4096
    assert init(7 * 16, 64, 3, gfd.BOUNDARY_CLIP) == -2  # unpadded sizes must be 2^a 3^b 5^c
    assert init(1, 64, 1, gfd.BOUNDARY_PAD) == -2        # observed sides of at least 2
    assert init(64, 64, 65, gfd.BOUNDARY_PAD) == -2      # PSF larger than the observation
    assert ctx.value is None


def test_static_entry_point_rejects_before_touching_the_device():
    """deconvolve_static validates its arguments and the size of its problem against the fixed
    array before any HIP call (1024 x 1024 needs about 80 MB of the 32 MiB)."""
    lib = gfd.load_library()
    fake = ctypes.c_void_p(0x1000)
    rc = lib.deconvolve_static(fake, 1024, 1024, fake, 9, 9, 1.0, 5, 1.0, -1.0, 3, fake, None, None)
    assert rc == -2 and "static scratch" in lib.gfd_last_error().decode()
    assert lib.deconvolve_static(fake, 64, 64, fake, 9, 9, 1.0, 4, 1.0, -1.0, 3, fake, None, None) == -1
    assert lib.deconvolve_static(fake, 64, 64, fake, 9, 9, 1.0, 5, 1.0, -1.0, -1, fake, None, None) == -1
    assert lib.deconvolve_static(fake, 64, 64, fake, 9, 9, 1.0, 5, 1.0, -1.0, 3, None, None, None) == -1
    assert lib.deconvolve_static(fake, 64, 64, fake, 9, 9, 1.0, 65, 1.0, -1.0, 3, fake, None, None) == -1

"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/dsnlm.h, and rejects bad arguments with
DSNLM_EINVAL before touching the device."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dsnlm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z_0-9\s\*]*?\b([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("dsnlm_", "ladmm_"))))


@pytest.fixture(scope="module")
def lib():
    from paper_1901_06110_amd import _lib
    return _lib.get()


def test_header_lists_the_entry_points():
    names = _declared_functions()
    for must in ["dsnlm_build_weights", "dsnlm_apply", "dsnlm_apply_backward", "dsnlm_forward",
                 "dsnlm_forward_batched", "ladmm_step", "ladmm_solve", "ladmm_operator_norm2"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    from paper_1901_06110_amd import _lib
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (\w+)$", out, flags=re.M))
    missing = [n for n in _declared_functions() if n not in exported]
    assert not missing, missing
    assert set(_lib.EXPORTED) <= exported


def test_invalid_arguments_rejected_on_host(lib):
    hp = C.c_void_p()
    fake = C.c_void_p(0x1000)
    cases = [
        lib.dsnlm_build_weights(None, 8, 8, 1, 1, 0.1, None, C.byref(hp)),
        lib.dsnlm_build_weights(fake, 0, 8, 1, 1, 0.1, None, C.byref(hp)),
        lib.dsnlm_build_weights(fake, 8, 8, -1, 1, 0.1, None, C.byref(hp)),
        lib.dsnlm_build_weights(fake, 8, 8, 1, -1, 0.1, None, C.byref(hp)),
        lib.dsnlm_build_weights(fake, 8, 8, 1, 8, 0.1, None, C.byref(hp)),
        lib.dsnlm_build_weights(fake, 8, 8, 1, 1, 0.0, None, C.byref(hp)),
        lib.dsnlm_build_weights(fake, 8, 8, 1, 1, float("nan"), None, C.byref(hp)),
        lib.dsnlm_build_weights(fake, 8, 8, 1, 1, float("inf"), None, C.byref(hp)),
        lib.dsnlm_forward(fake, fake, fake, 8, 8, 1, 1, 0.1, None, None),  # y aliases x
        lib.dsnlm_apply(None, fake, fake, None),
    ]
    assert all(c == -1 for c in cases), cases
    assert not hp.value
    assert b"overlap" in lib.dsnlm_last_error() or len(lib.dsnlm_last_error()) > 0


def test_unsupported_sizes_reported(lib):
    hp = C.c_void_p()
    fake = C.c_void_p(0x1000)
    assert lib.dsnlm_build_weights(fake, 64, 64, 25, 1, 0.1, None, C.byref(hp)) == -5
    assert lib.dsnlm_build_weights(fake, 64, 64, 3, 16, 0.1, None, C.byref(hp)) == -5


def test_images_past_the_32bit_offsets_refused(lib):
    """An image of more than 2^28 pixels (or one whose guide padded by S + P
    exceeds that) is refused on the host, single-image and batched, before
    any device work: the kernels form element offsets in 32-bit ints."""
    from paper_1901_06110_amd import _lib
    hp = C.c_void_p()
    fake = C.c_void_p(0x1000)
    assert lib.dsnlm_build_weights(fake, 16385, 16384, 1, 1, 0.1, None, C.byref(hp)) == -5
    assert lib.dsnlm_forward(fake, C.c_void_p(0x2000), C.c_void_p(1 << 40), 16384, 16384, 10, 3, 0.1,
                             None, None) == -5
    assert b"2^28" in lib.dsnlm_last_error()
    arr = (_lib.DsnlmImage * 1)()
    arr[0] = _lib.DsnlmImage(0x1000, 0x1000, 1 << 40, 1 << 15, 1 << 14, 0.1)
    assert lib.dsnlm_forward_batched(arr, 1, 10, 3, None) == -5
    assert not hp.value


def test_noalloc_forward_refuses_past_its_scratch(lib):
    """The allocation-free forward serves images whose intermediates fit its
    fixed scratch and refuses larger ones on the host, before any device call."""
    limit = lib.dsnlm_forward_noalloc_limit()
    assert limit == 48 << 20
    assert 0 < lib.dsnlm_forward_noalloc_bytes(1024, 1024, 10, 3) <= limit
    assert lib.dsnlm_forward_noalloc_bytes(2048, 2048, 10, 3) > limit
    assert lib.dsnlm_forward_noalloc_bytes(64, 64, 10, 6) == 0
    fake = C.c_void_p(0x1000)
    assert lib.dsnlm_forward_noalloc(fake, fake, C.c_void_p(1 << 40), 2048, 2048, 10, 3, 0.1, None) == -5
    assert b"scratch" in lib.dsnlm_last_error()
    assert lib.dsnlm_forward_noalloc(fake, fake, C.c_void_p(1 << 40), 64, 64, 10, 6, 0.1, None) == -5
    assert lib.dsnlm_forward_noalloc(fake, fake, fake, 64, 64, 10, 3, 0.1, None) == -1  # y aliases x
    assert lib.dsnlm_forward_noalloc(None, fake, C.c_void_p(1 << 40), 64, 64, 10, 3, 0.1, None) == -1

"""CPU checks of the C ABI: the built library exports every function declared in
include/he.h, the binding covers them, and argument validation rejects bad
parameter sets before touching a device (error paths forced from the host)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "he.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(he_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2409_05205_amd import he
    if not os.path.exists(he.LIB_PATH):
        pytest.fail("libhe.so is not built (run __graft_entry__.build())")
    return he.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("he_setup", "he_pack_filters", "he_conv_layer", "he_fc_layer"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_lists_every_symbol():
    from paper_2409_05205_amd import he
    assert sorted(he.EXPORTED) == declared_functions()


def test_setup_rejects_bad_parameters(lib):
    from paper_2409_05205_amd import he
    h = ctypes.c_void_p()
    U = ctypes.c_uint32
    assert lib.he_setup(1000, 3, None, 786433, ctypes.byref(h)) == he.HE_EINVAL        # not a power of two
    assert lib.he_setup(128, 3, None, 786433, ctypes.byref(h)) == he.HE_EINVAL         # too small
    assert lib.he_setup(32768, 3, None, 786433, ctypes.byref(h)) == he.HE_EINVAL       # too large
    assert lib.he_setup(4096, 0, None, 786433, ctypes.byref(h)) == he.HE_EINVAL        # no limbs
    assert lib.he_setup(4096, 9, None, 786433, ctypes.byref(h)) == he.HE_EINVAL        # too many limbs
    assert lib.he_setup(4096, 3, None, 1, ctypes.byref(h)) == he.HE_EINVAL             # t < 2
    assert lib.he_setup(4096, 1, None, 1 << 30, ctypes.byref(h)) == he.HE_EINVAL       # t >= q
    bad = (U * 1)(1073692673 + 2 * 4096 * 0 + 2)                                      # not prime / not 1 mod 2N
    assert lib.he_setup(4096, 1, bad, 786433, ctypes.byref(h)) == he.HE_EINVAL
    not_friendly = (U * 1)(1073741789)                                                # prime, != 1 mod 2N
    assert lib.he_setup(4096, 1, not_friendly, 786433, ctypes.byref(h)) == he.HE_EINVAL
    dup = (U * 2)(1073692673, 1073692673)
    assert lib.he_setup(4096, 2, dup, 786433, ctypes.byref(h)) == he.HE_EINVAL
    assert lib.he_setup(4096, 3, None, 786433, None) == he.HE_EINVAL
    assert not h.value


def test_null_handles_rejected(lib):
    from paper_2409_05205_amd import he
    assert lib.he_conv_layer(None, None, 1, None, None, None, None, None) == he.HE_EINVAL
    assert lib.he_fc_layer(None, None, 1, None, None, None, None, None) == he.HE_EINVAL
    assert lib.he_pack_filters(None, None, None, None, None, 0, None) == he.HE_EINVAL
    assert lib.he_layer_workspace_bytes(None, 4) == 0
    assert lib.he_strerror(he.HE_EINVAL) == b"invalid argument"


def test_new_calls_reject_null_handles(lib):
    from paper_2409_05205_amd import he
    info = he.LayerInfo()
    d = he.LayerDesc(he.HE_LAYER_CONV, 3, 16, 32, 32, 3, 1, 1, 0, 0)
    assert lib.he_layer_geometry(None, ctypes.byref(d), 0, ctypes.byref(info)) == he.HE_EINVAL
    assert lib.he_workspace_reserve(None, None, 1 << 20) == he.HE_EINVAL
    assert lib.he_ctx_workspace_bytes(None, 4) == 0

"""C ABI checks that need no GPU: the library loads, exports every function
include/xdrop.h declares, and rejects bad arguments before touching a
device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "xdrop.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(xdrop_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2304_08662_amd import xdrop
    if not os.path.exists(xdrop.LIB_PATH):
        from paper_2304_08662_amd import build
        build.build()
    return xdrop.load_library()


def test_header_lists_the_entry_points():
    names = declared_functions()
    for f in ("xdrop_extend_batch", "xdrop_ctx_create", "xdrop_server_submit",
              "xdrop_autotune", "xdrop_extend_batch_graph"):
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2304_08662_amd import xdrop
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(xdrop.EXPORTS) == declared_functions()


def test_strerror(lib):
    assert lib.xdrop_strerror(0) == b"ok"
    assert b"invalid" in lib.xdrop_strerror(-1)


def test_null_handles_are_rejected(lib):
    from paper_2304_08662_amd import xdrop
    assert lib.xdrop_extend_batch(None, None, None, 0, None, 0, None, None,
                                  None, None) == xdrop.E_INVALID
    assert lib.xdrop_ctx_destroy(None) == xdrop.E_INVALID
    assert lib.xdrop_server_destroy(None) == xdrop.E_INVALID
    assert lib.xdrop_server_poll(None, 1, None) == xdrop.E_INVALID
    assert lib.xdrop_last_stats(None, None, 0) == xdrop.E_INVALID


def test_ctx_create_rejects_missing_device(lib):
    from paper_2304_08662_amd import xdrop
    h = ctypes.c_void_p()
    rc = lib.xdrop_ctx_create(4096, None, ctypes.byref(h))
    assert rc == xdrop.E_INVALID and not h.value


def test_product_package_does_not_import_the_oracle():
    # the oracle is test infrastructure: no product module may reach it
    pkg = os.path.join(ROOT, "paper_2304_08662_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text, f
                assert "xdrop_oracle" not in text, f
                assert "liboracle" not in text, f
                # nor the CPU emulation of the kernels (tests/emu)
                assert "xdrop_emu" not in text, f
                assert "tests/emu" not in text, f

"""C-ABI contract checks that need no GPU: the library loads, exports every
entry point that include/dpvr.h declares, and rejects bad arguments on the
host with the documented status and a message (nothing is launched)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpvr.h")

dp = pytest.importorskip("paper_2501_01628_amd")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vr_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 18
    lib = C.CDLL(dp.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(dp.EXPORTED)


def test_abi_version_and_status_strings():
    assert dp.vr_abi_version() == 2
    assert dp.vr_status_string(dp.VR_ERR_WORKSPACE) == "VR_ERR_WORKSPACE"
    assert dp.vr_status_string(12345) == "VR_ERR_UNKNOWN"


@pytest.mark.parametrize("dims,ghost,storage,status", [
    ((0, 4, 4), 1, dp.VR_F32, dp.VR_ERR_INVALID_ARG),
    ((4, -1, 4), 1, dp.VR_F32, dp.VR_ERR_INVALID_ARG),
    ((4, 4, 4), 0, dp.VR_F32, dp.VR_ERR_INVALID_ARG),
    ((4, 4, 4), 2, dp.VR_F32, dp.VR_ERR_INVALID_ARG),
    ((4, 4, 4), 1, 7, dp.VR_ERR_INVALID_ARG),
])
def test_workspace_size_rejects(dims, ghost, storage, status):
    with pytest.raises(dp.VRError) as e:
        dp.vr_brick_workspace_size(dims, ghost, storage)
    assert e.value.status == status
    assert dp.vr_last_error(None)


def test_workspace_size_values():
    # rows of nx + 2 voxels padded to a multiple of 8 elements
    assert dp.vr_brick_workspace_size((32, 64, 64), 1, dp.VR_F32) == ((40 * 66 * 66 * 4 + 255) // 256) * 256
    assert dp.vr_brick_workspace_size((32, 64, 64), 1, dp.VR_F16) == ((40 * 66 * 66 * 2 + 255) // 256) * 256
    assert dp.vr_brick_workspace_size((6, 1, 1), 1, dp.VR_F32) == 512   # 8 x 3 x 3 x 4 B


def test_workspace_size_rejects_bricks_beyond_32bit_offsets():
    # 1026 x 1026 x 2050 stored voxels (pitch 1032) >= 2^31: unsupported
    with pytest.raises(dp.VRError) as e:
        dp.vr_brick_workspace_size((1024, 1024, 2048), 1, dp.VR_F16)
    assert e.value.status == dp.VR_ERR_UNSUPPORTED
    # just below the limit: 1032 x 1026 x 2028 < 2^31
    assert dp.vr_brick_workspace_size((1024, 1024, 2026), 1, dp.VR_F16) > 0


def test_null_handles_are_rejected():
    for call in (lambda: dp.vr_context_release(None), lambda: dp.vr_synchronize(None),
                 lambda: dp.vr_brick_release(None),
                 lambda: dp.vr_set_render_params(None, 0.5, 0.0),
                 lambda: dp.vr_render_partial(None, None, dp.make_partial((0, 0, 1, 1), 16, 16)),
                 lambda: dp.vr_partial_roi(None, None)):
        with pytest.raises(dp.VRError) as e:
            call()
        assert e.value.status == dp.VR_ERR_INVALID_HANDLE


def test_bogus_handle_is_rejected_without_dereference():
    with pytest.raises(dp.VRError) as e:
        dp.vr_set_render_params(0xDEAD0000, 0.5, 0.0)
    assert e.value.status == dp.VR_ERR_INVALID_HANDLE


def test_context_create_needs_out_pointer():
    st = dp._lib.vr_context_create(0, None, None)
    assert st == dp.VR_ERR_INVALID_ARG


def test_no_cpu_fallback_in_product_path():
    """The package imports nothing from the oracle and has no host
    rendering path: its Python sources never mention the oracle."""
    pkg = os.path.dirname(dp.__file__)
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "oracle" not in src, fn

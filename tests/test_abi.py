"""The C-ABI library loads and exports what include/lnm.h declares (CPU only;
no compute calls)."""
import ctypes as C
import os
import re

import pytest

from synth.weights import n_params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^LNM_API\s+[^(]*?\b(lnm_\w+)\s*\(", text, flags=re.M))
    return names


@pytest.fixture(scope="module")
def L():
    from paper_2604_03748_amd import lnm

    return lnm


def test_header_declares_entry_points():
    d = _declared()
    for name in ("lnm_march", "lnm_infer", "lnm_frame", "lnm_ctx_create", "lnm_net_create"):
        assert name in d


def test_library_exports_every_declared_symbol(L):
    lib = L.lib()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(L.EXPORTS) == _declared()


def test_struct_sizes_match_binding(L):
    lib = L.lib()
    for i, s in enumerate([L.Volume, L.Camera, L.MarchParams, L.Light, L.ShadowFrame]):
        assert lib.lnm_abi_struct_size(i) == C.sizeof(s)
    assert lib.lnm_abi_struct_size(99) == 0


def test_param_count_and_device_bytes(L):
    lib = L.lib()
    for lv, b in ((2, 16), (3, 16), (4, 32), (4, 48)):
        assert L.param_count(lv, b) == n_params(lv, b)
        assert lib.lnm_net_device_bytes(lv, b, L.FP32) >= 4 * n_params(lv, b)
    assert L.param_count(1, 16) == 0  # unsupported depth
    assert L.param_count(3, 8) == 0  # width not a multiple of 16
    assert lib.lnm_version().startswith(b"liblnm")


def test_work_order_choice_by_grid_size(L):
    """lnm_march_workspace_bytes is host arithmetic, and the z orders add a
    bucket byte and a list entry per record: the automatic order for a 128^3
    grid is the cell order with the top/bottom lights (a cell's two 130 x 130
    planes fit in LDS) and the band order with the left/right lights (whose
    marches leave their z cell); 192^3 and 256^3 grids (60 and 141 MB of
    bricks, above the 32 MiB of the eight L2 caches) take the z order; the
    cell order is refused where the planes do not fit."""
    from synth.scene import headline

    cam = L.make_camera(headline().camera)
    lib = L.lib()

    def ws(n, **kw):
        vol = L.Volume()
        vol.density, vol.nx, vol.ny, vol.nz, vol.sigma_scale, vol.bricks = 0x1000, n, n, n, 8.0, None
        return lib.lnm_march_workspace_bytes(C.byref(vol), C.byref(cam), C.byref(L.make_params(4.0, **kw)))

    for n in (128, 192, 256):
        assert ws(n, work_order=L.ORDER_Z) > ws(n, work_order=L.ORDER_BANDS) > 0, n
    # cell order: the z orders' bucket plane and sorted list, no band lists
    assert ws(128, work_order=L.ORDER_Z) > ws(128, work_order=L.ORDER_CELLS) > ws(128, work_order=L.ORDER_BANDS)
    assert ws(128) == ws(128, work_order=L.ORDER_CELLS)
    assert ws(128, light_set=L.LIGHTS_LEFT_RIGHT) == ws(128, work_order=L.ORDER_BANDS)
    assert ws(192) == ws(192, work_order=L.ORDER_Z)  # 60 MB of bricks: z layers
    assert ws(192, work_order=L.ORDER_CELLS) == 0 and ws(256, work_order=L.ORDER_CELLS) == 0
    assert ws(256) == ws(256, work_order=L.ORDER_Z)
    assert ws(128, work_order=4) == 0

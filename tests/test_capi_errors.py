"""Argument checks of the C ABI that return before any device call (no GPU
needed): sizes, precision and scheme codes, workspace pointer, alignment,
size and the 2^29-site limit. lbm_create reads the workspace pointer only
after these checks pass, so a host address stands in for device memory."""
import ctypes

import pytest

from paper_2208_13769_amd import lbm

FAKE_WS = ctypes.c_void_p(1 << 20)  # 256-byte aligned, never dereferenced by a rejected call
BIG = 1 << 40


def _create(nx=32, ny=32, dx=1.0, prec=lbm.LBM_FP32, scheme=lbm.LBM_SCHEME_PC, ws=FAKE_WS, nbytes=BIG):
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(nx, ny, dx, prec, scheme, ws, nbytes, None)
    return e.value.status


def test_workspace_bytes_rejects_small_sizes_and_unknown_precision():
    assert lbm.lbm_workspace_bytes(4, 64, lbm.LBM_FP32) == 0
    assert lbm.lbm_workspace_bytes(64, 4, lbm.LBM_FP32) == 0
    assert lbm.lbm_workspace_bytes(64, 64, 99) == 0
    assert lbm.lbm_workspace_bytes_walled(4, 64, lbm.LBM_FP32) == 0
    assert lbm.lbm_workspace_bytes(5, 5, lbm.LBM_FP64) > 0
    # the walled workspace holds the regular one plus the passes' scratch
    assert lbm.lbm_workspace_bytes_walled(64, 48, lbm.LBM_FP64) > lbm.lbm_workspace_bytes(64, 48, lbm.LBM_FP64)


@pytest.mark.parametrize("kw,status", [
    (dict(nx=4), lbm.LBM_ERR_ARG),
    (dict(ny=3), lbm.LBM_ERR_ARG),
    (dict(dx=0.0), lbm.LBM_ERR_ARG),
    (dict(dx=float("nan")), lbm.LBM_ERR_ARG),
    (dict(prec=17), lbm.LBM_ERR_ARG),
    (dict(scheme=5), lbm.LBM_ERR_ARG),
    (dict(ws=None), lbm.LBM_ERR_ARG),
    (dict(ws=ctypes.c_void_p((1 << 20) + 8)), lbm.LBM_ERR_ARG),       # not 256-byte aligned
    (dict(nx=1 << 15, ny=(1 << 14) + 1), lbm.LBM_ERR_UNSUPPORTED),  # more than 2^29 sites
    (dict(nbytes=1024), lbm.LBM_ERR_NOMEM),
])
def test_create_rejects(kw, status):
    assert _create(**kw) == status


def test_extrapolation_scheme_needs_the_walled_workspace():
    nb = lbm.lbm_workspace_bytes(32, 32, lbm.LBM_FP64)
    assert _create(prec=lbm.LBM_FP64, scheme=lbm.LBM_SCHEME_EXTRAP, nbytes=nb) == lbm.LBM_ERR_NOMEM


def test_error_message_is_set():
    lib = lbm.load_library()
    _create(nx=4)
    msg = lib.lbm_last_error(None)
    assert msg and b"nx" in msg

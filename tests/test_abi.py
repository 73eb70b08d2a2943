"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the GPU."""

import ctypes
import os
import re

import pytest

from paper_2106_04649_amd import mk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mk.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:mk_status|const char\*|int32_t)\s+(mk_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    return mk.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ["mk_plan", "mk_load_R", "mk_set_focal", "mk_iterate", "mk_get", "mk_destroy",
                 "mk_strerror", "mk_last_error", "mk_net_forward", "mk_net_backward", "mk_net_adam",
                 "mk_net_param_count"]:
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_device_checks_need_the_checked_build(lib):
    v = ctypes.c_uint32(7)
    assert lib.mk_device_checks(None) == mk.MK_ERR_ARG
    assert lib.mk_device_checks(ctypes.byref(v)) == mk.MK_ERR_UNSUPPORTED and v.value == 0


def test_checked_build_exports_every_declared_symbol():
    if not os.path.exists(mk.CHECKED_LIB_PATH):
        pytest.skip("libmk_checked.so is not built (python -m paper_2106_04649_amd.build --device-checks)")
    checked = ctypes.CDLL(mk.CHECKED_LIB_PATH)
    for name in declared_functions():
        assert hasattr(checked, name), name


def test_strerror(lib):
    for s in range(7):
        assert lib.mk_strerror(s).decode()
    assert lib.mk_strerror(99).decode() == "unknown status"


def _desc(**kw):
    base = dict(nr=8, ns=8, nt=64, iw_lo=0, iw_hi=32, nf_max=1, dt=0.004, dx=10.0, div_factor=0.0,
                rprec=0, flags=0, stream=None, r_dev_bytes=0)
    base.update(kw)
    return mk.mk_plan_desc(*[base[f] for f, _ in mk.mk_plan_desc._fields_])


@pytest.mark.parametrize("kw,status", [
    (dict(ns=9), mk.MK_ERR_ARG),                 # nr != ns
    (dict(nr=0, ns=0), mk.MK_ERR_ARG),
    (dict(nt=48), mk.MK_ERR_ARG),                # not a power of two
    (dict(nt=8), mk.MK_ERR_ARG),                 # below 16
    (dict(nt=8192, iw_hi=100), mk.MK_ERR_ARG),   # above 4096
    (dict(iw_lo=5, iw_hi=4), mk.MK_ERR_ARG),
    (dict(iw_hi=33), mk.MK_ERR_ARG),             # above nt/2
    (dict(iw_lo=-1), mk.MK_ERR_ARG),
    (dict(nf_max=0), mk.MK_ERR_ARG),
    (dict(dt=0.0), mk.MK_ERR_ARG),
    (dict(dx=-1.0), mk.MK_ERR_ARG),
    (dict(dt=float("inf")), mk.MK_ERR_ARG),
    (dict(div_factor=float("nan")), mk.MK_ERR_ARG),
    (dict(rprec=7), mk.MK_ERR_ARG),
    (dict(flags=0x100), mk.MK_ERR_ARG),
    # streamed R: a cap below two bins of R (one bin is 8 x 32 complex64 = 2 KiB)
    (dict(r_dev_bytes=4095), mk.MK_ERR_ARG),
    (dict(r_dev_bytes=8192, flags=0x1), mk.MK_ERR_UNSUPPORTED),      # with graph replay
    (dict(r_dev_bytes=8192, flags=0x4), mk.MK_ERR_UNSUPPORTED),      # with the autotuner
    (dict(r_dev_bytes=8192, flags=0x20), mk.MK_ERR_UNSUPPORTED),     # with the tile walk
    (dict(flags=0x24), mk.MK_ERR_UNSUPPORTED),                       # tile walk with the autotuner
    (dict(flags=0x60), mk.MK_ERR_ARG),                               # tile walk and grid form
    (dict(flags=0x80), mk.MK_ERR_ARG),                               # unknown bit
])
def test_plan_rejects_bad_descriptions(lib, kw, status):
    d = _desc(**kw)
    h = ctypes.c_void_p()
    st = lib.mk_plan(ctypes.byref(d), ctypes.byref(h))
    assert st == status
    assert h.value is None
    assert lib.mk_last_error(None).decode().startswith("mk_plan")


def test_null_arguments(lib):
    h = ctypes.c_void_p()
    assert lib.mk_plan(None, ctypes.byref(h)) == mk.MK_ERR_ARG
    d = _desc()
    assert lib.mk_plan(ctypes.byref(d), None) == mk.MK_ERR_ARG
    assert lib.mk_load_R(None, None, 0) == mk.MK_ERR_ARG
    assert lib.mk_set_focal(None, 1, None, None, 0, None, 0) == mk.MK_ERR_ARG
    assert lib.mk_iterate(None, 1, None) == mk.MK_ERR_ARG
    assert lib.mk_get(None, 0, None, 0) == mk.MK_ERR_ARG
    assert lib.mk_passes(None, None) == mk.MK_ERR_ARG
    assert lib.mk_image(None, None) == mk.MK_ERR_ARG
    assert lib.mk_profile(None, 0, None, None, 0) == mk.MK_ERR_ARG
    assert lib.mk_destroy(None) == mk.MK_OK


def test_net_param_count(lib):
    for H in (64, 16, 1):
        assert lib.mk_net_param_count(4, H) == H * 4 * 5 + H + H * H * 5 + H + 2 * H * 5 + 2
    assert lib.mk_net_param_count(0, 64) == -1
    assert lib.mk_net_param_count(4, 0) == -1
    assert lib.mk_net_param_count(4, 129) == -1


def _fake_plan(nf_max=2, nr=8, nt=64, lo=0, hi=32):
    """A binding-side plan with no library handle: the shape checks below run
    before any library call, so they need no GPU."""
    d = _desc(nr=nr, ns=nr, nt=nt, iw_lo=lo, iw_hi=hi, nf_max=nf_max)
    plan = mk.Plan(0, d)
    plan.handle = None
    return plan


def test_binding_checks_shapes_before_the_library_reads():
    import numpy as np

    plan = _fake_plan()
    ok_R = np.zeros((8, 33, 8), np.complex64)
    for bad in (np.zeros((8, 32, 8), np.complex64), np.zeros((8, 33, 9), np.complex64),
                np.zeros((8, 33, 8), np.float32), np.zeros((8, 33, 8, 2), np.float32)[:, :, :7]):
        with pytest.raises(ValueError):
            mk.mk_load_R(plan, bad)
    assert ok_R.shape == (8, 33, 8)
    Gd, itd = np.zeros((2, 8, 64), np.float32), np.zeros((2, 8), np.int32)
    for g, i, b in ((np.zeros((3, 8, 64), np.float32), np.zeros((3, 8), np.int32), None),   # nf > nf_max
                    (np.zeros((2, 8, 32), np.float32), itd, None),                          # wrong nt
                    (Gd, np.zeros((2, 7), np.int32), None),                                  # wrong itd
                    (Gd, itd, np.zeros((1, 2), np.int32)),                                   # wrong band
                    (np.zeros((8, 64), np.float32), itd, None)):                             # no focal axis
        with pytest.raises(ValueError):
            mk.mk_set_focal(plan, g, i, 1, b)
    plan.nf, plan.tail_kT = 2, (4, 16)
    for out in (np.zeros((2, 8, 4, 8), np.float32), np.zeros((1, 8, 4, 16), np.float32)):
        with pytest.raises(ValueError):
            mk.mk_tail_history(plan, out)
    with pytest.raises(TypeError):
        mk.mk_tail_history(plan, np.zeros((2, 8, 4, 16), np.float64))
    with pytest.raises(TypeError):
        mk.mk_tail_history(plan, np.zeros((2, 8, 16, 4), np.float32).transpose(0, 1, 3, 2))


def test_state_calls_reject_null_arguments(lib):
    n = ctypes.c_size_t()
    assert lib.mk_state_bytes(None, ctypes.byref(n)) == mk.MK_ERR_ARG
    buf = ctypes.create_string_buffer(64)
    assert lib.mk_get_state(None, buf, 64) == mk.MK_ERR_ARG
    assert lib.mk_set_state(None, buf, 64) == mk.MK_ERR_ARG

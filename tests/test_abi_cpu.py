"""CPU-only checks of the C ABI: the library loads, exports every entry point
that include/ebsd.h declares, and its host-side logic (defaults, error codes,
argument validation, ROI layout) behaves as documented.  No kernel runs."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ebsd.h")


@pytest.fixture(scope="module")
def E():
    from paper_1907_05993_amd import build, ebsd
    if not os.path.exists(ebsd.LIB_PATH):
        build.build()
    ebsd.lib()
    return ebsd


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w]+\s*\**\s*(ebsd_\w+)\s*\(", text, flags=re.M)))


def test_every_declared_symbol_is_exported(E):
    names = declared_functions()
    assert len(names) >= 16
    lib = C.CDLL(E.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(E.EXPORTED)


def test_version_defaults_strerror(E):
    L = E.lib()
    assert L.ebsd_version() == 5
    p = E.CParams()
    assert L.ebsd_params_default(C.byref(p)) == 0
    assert p.struct_size == C.sizeof(E.CParams)
    assert p.levels == 3 and list(p.max_iters)[:3] == [150, 150, 150]
    assert abs(p.sigma_px - 1.0) < 1e-7 and p.n_roi == 20 and p.roi_size == 64
    assert p.window == 1 and p.second_pass == 1
    assert p.warm_start == 0 and abs(p.fallback_residual_px - 0.5) < 1e-7
    assert p.remap_interp == 3 and p.xcf_passes == 1 and p.first_pass == 0
    # the defaults are exactly the Python mirror's (pattern centre and ring radius as doubles)
    q = E.Params().to_c()
    for f, _ in E.CParams._fields_:
        a, b = getattr(p, f), getattr(q, f)
        assert (list(a)[:3] == list(b)[:3]) if f == "max_iters" else a == b, f
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -99):
        assert len(L.ebsd_strerror(code)) > 0


def test_create_validates_before_touching_the_device(E):
    L = E.lib()
    h = C.c_void_p()
    p = E.Params().to_c()
    p.struct_size = 4
    assert L.ebsd_create(C.byref(p), 0, C.byref(h)) == -8
    for field, val, code in [("sigma_px", -1.0, -1), ("sigma_px", 2.0, -1), ("levels", 0, -1),
                             ("levels", 9, -1), ("n_roi", 3, -1), ("roi_size", 48, -3),
                             ("window", 2, -1), ("pc_z", 0.0, -1), ("tol_px", float("nan"), -1),
                             ("warm_start", 3, -1), ("fallback_residual_px", -1.0, -1),
                             ("remap_interp", 2, -1), ("remap_interp", 0, -1), ("xcf_passes", 0, -1),
                             ("xcf_passes", 17, -1), ("first_pass", 2, -1), ("first_pass", -1, -1),
                             ("bandpass_lo_px", -1.0, -1), ("bandpass_hi_px", 33.0, -1),
                             ("bandpass_hi_px", float("nan"), -1)]:
        p = E.Params().to_c()
        setattr(p, field, val)
        assert L.ebsd_create(C.byref(p), 0, C.byref(h)) == code, field
    assert L.ebsd_create(C.byref(E.Params().to_c()), 0, None) == -1
    # the conventional first pass takes no warm start
    p = E.Params(first_pass=1, warm_start=1).to_c()
    assert L.ebsd_create(C.byref(p), 0, C.byref(h)) == -1


def test_create_without_gpu_reports_device_error(E):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert E.lib().ebsd_create(C.byref(E.Params().to_c()), 0, C.byref(h)) == -5


@pytest.mark.parametrize("HW,roi", [((256, 256), 64), ((128, 128), 32), ((400, 400), 128),
                                    ((512, 512), 128), ((160, 96), 32)])
def test_roi_layout_equals_oracle(E, orc, HW, roi):
    H, W = HW
    gp = E.Params(roi_size=roi)
    cx, cy, x0, y0 = E.roi_layout(gp, H, W)
    ocx, ocy, ox0, oy0, bad = orc.roi_layout(H, W, orc.make_params(roi_size=roi))
    assert not bad
    assert np.array_equal(x0, ox0) and np.array_equal(y0, oy0)
    assert np.array_equal(cx, ocx) and np.array_equal(cy, ocy)


def test_roi_layout_out_of_bounds(E):
    with pytest.raises(E.EbsdError) as ei:
        E.roi_layout(E.Params(roi_size=128), 128, 128)
    assert ei.value.code == -3


def test_null_arguments_rejected(E):
    L = E.lib()
    assert L.ebsd_register_batch(None, None, 0, None, None) == -1
    assert L.ebsd_stage_xcf(None, None, 1, 64, 1, None, None, None) == -1
    assert L.ebsd_stage_xcf(None, None, 0, 48, 1, None, None, None) == -3
    assert L.ebsd_stage_restrict(None, 0, 1, 8, None, None) == -2  # odd sizes are accepted, 1 row is not
    fake = C.c_void_p(16)  # never dereferenced: validation fails first
    assert L.ebsd_stage_remap(None, 1, 64, 64, None, 31.5, 31.5, 44.8, 3, None, None, None) == -1
    assert L.ebsd_stage_remap(fake, 1, 64, 64, fake, 31.5, 31.5, 44.8, 3, None, fake, None) == -1  # no coef
    assert L.ebsd_stage_remap(fake, 1, 64, 64, fake, 31.5, 31.5, 44.8, 2, fake, fake, None) == -1
    assert L.ebsd_stage_remap(fake, 1, 64, 64, fake, 31.5, 31.5, 0.0, 1, None, fake, None) == -1
    assert L.ebsd_stage_remap(fake, 1, 2, 64, fake, 31.5, 31.5, 44.8, 1, None, fake, None) == -2
    assert L.ebsd_stage_remap(None, 0, 64, 64, None, 31.5, 31.5, 44.8, 3, None, None, None) == 0
    assert L.ebsd_stage_bandpass(None, 1, 64, 64, C.c_float(1.0), C.c_float(8.0), fake, None) == -1
    assert L.ebsd_stage_bandpass(fake, 1, 64, 64, C.c_float(40.0), C.c_float(8.0), fake, None) == -1
    assert L.ebsd_stage_bandpass(fake, 1, 64, 20000, C.c_float(1.0), C.c_float(8.0), fake, None) == -2
    assert L.ebsd_stage_bandpass(None, 0, 64, 64, C.c_float(1.0), C.c_float(8.0), None, None) == 0
    assert L.ebsd_stage_prolong(fake, 1, 64, 8193, fake, None) == -2  # output over 16384 px a side
    assert L.ebsd_stage_prolong(None, 1, 64, 64, fake, None) == -1
    assert L.ebsd_destroy(None) == 0
    assert L.ebsd_set_gating(None, 8) == -1
    assert L.ebsd_tilt_rotation(0.1, None) == -1
    # the allocation-free pre-filter validates before touching a device
    assert L.ebsd_stage_bandpass_static(None, 1, 64, 64, C.c_float(1.0), C.c_float(8.0), fake, None) == -1
    assert L.ebsd_stage_bandpass_static(fake, 17, 512, 512, C.c_float(1.0), C.c_float(8.0), fake, None) == -10
    assert L.ebsd_stage_bandpass_static(None, 0, 64, 64, C.c_float(1.0), C.c_float(8.0), None, None) == 0
    assert L.ebsd_get_launch_counts(None, None, None) == -1
    # traction-free solve: validation before any launch
    eye = (C.c_double * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1)
    bad = (C.c_double * 9)(1, 0, 0, 0, 1, 0, 0, 0, -1)  # a reflection
    ni = (2.76e11, 1.59e11, 1.32e11)
    tf = L.ebsd_traction_free
    assert tf(None, 1, 20, fake, fake, 127.5, 127.5, 179.2, None, fake, eye, *ni, fake, None, None, None, None) == -1
    assert tf(fake, 1, 20, fake, fake, 127.5, 127.5, 179.2, None, fake, None, *ni, fake, None, None, None, None) == -1
    assert tf(fake, 1, 20, fake, fake, 127.5, 127.5, 179.2, None, fake, bad, *ni, fake, None, None, None, None) == -1
    assert tf(fake, 1, 4, fake, fake, 127.5, 127.5, 179.2, None, fake, eye, *ni, fake, None, None, None, None) == -1
    assert tf(fake, 1, 20, fake, fake, 127.5, 127.5, 0.0, None, fake, eye, *ni, fake, None, None, None, None) == -1
    for c in [(1.0, 2.0, 1.0), (1.0, 0.5, 0.0), (1.0, -0.6, 1.0), (float("nan"), 0.5, 1.0)]:
        assert tf(fake, 1, 20, fake, fake, 127.5, 127.5, 179.2, None, fake, eye, *c, fake, None, None, None,
                  None) == -1
    assert tf(None, 0, 20, None, None, 127.5, 127.5, 179.2, None, None, eye, *ni, None, None, None, None, None) == 0


def test_network_entry_points_validate_without_a_gpu(E):
    import torch
    from oracle import cnn
    L = E.lib()
    assert L.ebsd_cnn_num_params() == E.CNN_PARAMS == cnn.flatten(cnn.init_params(0)).size
    h = C.c_void_p()
    assert L.ebsd_cnn_create(0, 0, C.byref(h)) == -1
    assert L.ebsd_cnn_create(0, 5000, C.byref(h)) == -1
    assert L.ebsd_cnn_create(0, 4, None) == -1
    if not torch.cuda.is_available():
        assert L.ebsd_cnn_create(0, 4, C.byref(h)) == -5
    assert L.ebsd_cnn_destroy(None) == 0
    assert L.ebsd_cnn_set_params(None, None, E.CNN_PARAMS) == -1
    assert L.ebsd_cnn_forward(None, None, None, 1, 256, 256, None, None) == -1
    assert L.ebsd_cnn_train_step(None, None, None, None, 1, 256, 256, 1e-3, 1, None, None) == -1
    assert L.ebsd_cnn_load(None, b"x") == -1
    assert L.ebsd_load_model(None, b"x") == -1
    assert L.ebsd_set_model(None, None) == -1
    assert L.ebsd_cnn_set_fusion(None, 1) == -1


def test_pipeline_entry_points_validate_without_a_gpu(E):
    import torch
    L = E.lib()
    h = C.c_void_p()
    p = E.Params().to_c()
    assert L.ebsd_pipeline_create(C.byref(p), 0, 0, C.byref(h)) == -1
    assert L.ebsd_pipeline_create(C.byref(p), 0, 9, C.byref(h)) == -1
    assert L.ebsd_pipeline_create(C.byref(p), 0, 2, None) == -1
    bad = E.Params(sigma_px=-1.0).to_c()
    assert L.ebsd_pipeline_create(C.byref(bad), 0, 2, C.byref(h)) == -1
    if not torch.cuda.is_available():
        assert L.ebsd_pipeline_create(C.byref(p), 0, 2, C.byref(h)) == -5
    assert L.ebsd_pipeline_handle(None, 0, C.byref(h)) == -1
    assert L.ebsd_pipeline_submit(None, None, 0, None, None) == -1
    assert L.ebsd_pipeline_wait(None, None) == -1
    assert L.ebsd_pipeline_destroy(None) == 0


def test_tilt_rotation_is_eq13_as_printed(E, orc):
    """ebsd_tilt_rotation (host) against the tests' own transcription of Eq. (13)."""
    import math
    import test_oracle_pins as pins
    for th in (0.0, math.radians(70.0), -1.3):
        np.testing.assert_allclose(np.array(E.r_tilt(th)), np.array(pins._r_tilt(th)), atol=1e-15)
    S = np.array(E.r_tilt(0.7))
    np.testing.assert_allclose(S @ S.T, np.eye(3), atol=1e-15)
    assert abs(np.linalg.det(S) - 1.0) < 1e-15

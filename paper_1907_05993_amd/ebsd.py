"""Python binding of the gfx950 HIP library (``lib/libebsd.so``, C ABI in ``include/ebsd.h``).

Argument marshalling only: every step of the registration runs in the library's
HIP kernels.  PyTorch provides device memory and the current stream.  If the
library has not been built this module raises instead of falling back to
anything else.

Method: Zhu, Kaufmann & Vecchio, arXiv:1907.05993 -- multi-resolution demons
(section 1, Eq. (1)), shifts at ROI centres and the Eq. (2)-(3) solve for F
(section 2), R = P Q^T (Eq. (4)-(5)), remap + second-pass cross-correlation,
F = F_inf R_finite (Eq. (12)).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libebsd.so")

EBSD_OK = 0
ERRORS = {-1: "EINVAL", -2: "ESHAPE", -3: "EROI", -4: "ENOMEM", -5: "EDEVICE", -6: "ENOTSUP",
          -7: "ENOMODEL", -8: "EVERSION", -9: "EIO"}
CONVERGED, HIT_CAP, SOLVE_ILLCOND, NONFINITE_INPUT, DEGENERATE_INPUT = 1, 2, 16, 32, 64
WARM_USED, WARM_FALLBACK = 4, 8
CNN_PARAMS = 1762306
MAX_LEVELS = 8


class EbsdError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {ERRORS.get(code, code)} ({_strerror(code)})")


class CParams(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("levels", C.c_int32),
        ("max_iters", C.c_int32 * MAX_LEVELS),
        ("sigma_px", C.c_float),
        ("tol_px", C.c_float),
        ("pc_x", C.c_double),
        ("pc_y", C.c_double),
        ("pc_z", C.c_double),
        ("n_roi", C.c_int32),
        ("roi_size", C.c_int32),
        ("roi_radius_frac", C.c_double),
        ("window", C.c_int32),
        ("second_pass", C.c_int32),
        ("warm_start", C.c_int32),
        ("fallback_residual_px", C.c_float),
        ("remap_interp", C.c_int32),
        ("xcf_passes", C.c_int32),
        ("first_pass", C.c_int32),
        ("bandpass_lo_px", C.c_float),
        ("bandpass_hi_px", C.c_float),
        ("background_static", C.c_int32),
        ("background_dynamic_px", C.c_float),
    ]


class CGenSpec(C.Structure):
    _fields_ = [("G", C.c_double * 9), ("F", C.c_double * 9), ("gx", C.c_double), ("gy", C.c_double),
                ("counts", C.c_double), ("key", C.c_uint32 * 2), ("noise", C.c_int32), ("bands", C.c_int32)]


class CPair(C.Structure):
    _fields_ = [("ref", C.c_void_p), ("test", C.c_void_p), ("H", C.c_int32), ("W", C.c_int32),
                ("ref_id", C.c_int32)]


class COutputs(C.Structure):
    _fields_ = [
        ("field", C.c_void_p),
        ("field_offset", C.c_void_p),
        ("F", C.c_void_p),
        ("R", C.c_void_p),
        ("rotvec", C.c_void_p),
        ("R_finite", C.c_void_p),
        ("F_first", C.c_void_p),
        ("q1", C.c_void_p),
        ("q2", C.c_void_p),
        ("peak_height", C.c_void_p),
        ("iters", C.c_void_p),
        ("status", C.c_void_p),
        ("warm_field", C.c_void_p),
        ("warm_misfit", C.c_void_p),
        ("mae_first", C.c_void_p),
        ("mae", C.c_void_p),
        ("ssim", C.c_void_p),
        ("omega", C.c_void_p),
    ]


_lib = None

EXPORTED = ["ebsd_version", "ebsd_params_default", "ebsd_strerror", "ebsd_create", "ebsd_destroy",
            "ebsd_get_params", "ebsd_roi_layout", "ebsd_register_batch",
            "ebsd_register_batch_init", "ebsd_second_pass_batch", "ebsd_stage_normalize",
            "ebsd_stage_restrict", "ebsd_stage_demons_iter", "ebsd_stage_prolong",
            "ebsd_stage_xcf", "ebsd_stage_solve", "ebsd_stage_remap", "ebsd_traction_free",
            "ebsd_stage_bandpass", "ebsd_set_timing", "ebsd_get_timing",
            "ebsd_autotune", "ebsd_get_strip_height", "ebsd_set_strip_height", "ebsd_set_graphs",
            "ebsd_set_resident",
            "ebsd_cnn_num_params", "ebsd_cnn_create", "ebsd_cnn_destroy", "ebsd_cnn_set_params",
            "ebsd_cnn_get_params", "ebsd_cnn_get_grads", "ebsd_cnn_load", "ebsd_cnn_save",
            "ebsd_cnn_forward", "ebsd_cnn_train_step", "ebsd_cnn_reset_optimizer",
            "ebsd_load_model", "ebsd_set_model", "ebsd_stage_conv3x3", "ebsd_stage_conv3x3_dgrad",
            "ebsd_stage_conv3x3_wgrad", "ebsd_gen_pairs", "ebsd_get_fused_height", "ebsd_set_fused_height",
            "ebsd_set_gating", "ebsd_get_launch_counts", "ebsd_tilt_rotation", "ebsd_cnn_get_optimizer",
            "ebsd_cnn_set_optimizer", "ebsd_stage_bandpass_static", "ebsd_cnn_set_fusion",
            "ebsd_pipeline_create", "ebsd_pipeline_handle", "ebsd_pipeline_submit", "ebsd_pipeline_wait",
            "ebsd_pipeline_destroy"]


def lib():
    """Load libebsd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run paper_1907_05993_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.ebsd_version.restype = C.c_int
        L.ebsd_params_default.argtypes = [C.POINTER(CParams)]
        L.ebsd_strerror.restype = C.c_char_p
        L.ebsd_strerror.argtypes = [C.c_int]
        L.ebsd_create.argtypes = [C.POINTER(CParams), C.c_int, C.POINTER(vp)]
        L.ebsd_destroy.argtypes = [vp]
        L.ebsd_get_params.argtypes = [vp, C.POINTER(CParams)]
        L.ebsd_roi_layout.argtypes = [C.POINTER(CParams), i32, i32, vp, vp, vp, vp]
        L.ebsd_register_batch.argtypes = [vp, C.POINTER(CPair), i32, C.POINTER(COutputs), vp]
        L.ebsd_pipeline_create.argtypes = [C.POINTER(CParams), C.c_int, i32, C.POINTER(vp)]
        L.ebsd_pipeline_handle.argtypes = [vp, i32, C.POINTER(vp)]
        L.ebsd_pipeline_submit.argtypes = [vp, C.POINTER(CPair), i32, C.POINTER(COutputs), vp]
        L.ebsd_pipeline_wait.argtypes = [vp, vp]
        L.ebsd_pipeline_destroy.argtypes = [vp]
        L.ebsd_register_batch_init.argtypes = [vp, C.POINTER(CPair), i32, vp, C.POINTER(COutputs), vp]
        L.ebsd_second_pass_batch.argtypes = [vp, C.POINTER(CPair), i32, vp, C.POINTER(COutputs), vp]
        L.ebsd_autotune.argtypes = [vp, C.POINTER(CPair), i32, vp]
        L.ebsd_set_graphs.argtypes = [vp, C.c_int]
        L.ebsd_set_resident.argtypes = [vp, C.c_int]
        L.ebsd_get_strip_height.argtypes = [vp, i32, i32]
        L.ebsd_set_strip_height.argtypes = [vp, i32, i32, i32]
        L.ebsd_get_fused_height.argtypes = [vp, i32, i32]
        L.ebsd_set_fused_height.argtypes = [vp, i32, i32, i32]
        L.ebsd_set_gating.argtypes = [vp, i32]
        L.ebsd_tilt_rotation.argtypes = [C.c_double, C.POINTER(C.c_double)]
        L.ebsd_get_launch_counts.argtypes = [vp, vp, vp]
        L.ebsd_set_timing.argtypes = [vp, C.c_int]
        L.ebsd_get_timing.argtypes = [vp, vp, vp]
        L.ebsd_stage_normalize.argtypes = [vp, i32, i64, vp, vp, vp]
        L.ebsd_stage_restrict.argtypes = [vp, i32, i32, i32, vp, vp]
        L.ebsd_stage_demons_iter.argtypes = [vp, vp, i32, i32, i32, vp, C.c_float, vp, vp, vp]
        L.ebsd_stage_prolong.argtypes = [vp, i32, i32, i32, vp, vp]
        L.ebsd_stage_xcf.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp]
        L.ebsd_stage_solve.argtypes = [vp, i32, i32, vp, vp, C.c_double, C.c_double, C.c_double,
                                       vp, vp, vp, vp]
        L.ebsd_stage_remap.argtypes = [vp, i32, i32, i32, vp, C.c_double, C.c_double, C.c_double, i32,
                                       vp, vp, vp]
        L.ebsd_stage_bandpass.argtypes = [vp, i32, i32, i32, C.c_float, C.c_float, vp, vp]
        L.ebsd_stage_bandpass_static.argtypes = [vp, i32, i32, i32, C.c_float, C.c_float, vp, vp]
        L.ebsd_traction_free.argtypes = [vp, i32, i32, vp, vp, C.c_double, C.c_double, C.c_double, vp, vp,
                                         C.POINTER(C.c_double), C.c_double, C.c_double, C.c_double, vp, vp, vp,
                                         vp, vp]
        L.ebsd_cnn_num_params.restype = i64
        L.ebsd_cnn_create.argtypes = [C.c_int, i32, C.POINTER(vp)]
        L.ebsd_cnn_destroy.argtypes = [vp]
        L.ebsd_cnn_set_params.argtypes = [vp, vp, i64]
        L.ebsd_cnn_get_params.argtypes = [vp, vp, i64]
        L.ebsd_cnn_get_grads.argtypes = [vp, vp, i64]
        L.ebsd_cnn_load.argtypes = [vp, C.c_char_p]
        L.ebsd_cnn_save.argtypes = [vp, C.c_char_p]
        L.ebsd_cnn_forward.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp]
        L.ebsd_cnn_train_step.argtypes = [vp, vp, vp, vp, i32, i32, i32, C.c_float, i32,
                                          C.POINTER(C.c_float), vp]
        L.ebsd_cnn_reset_optimizer.argtypes = [vp]
        L.ebsd_cnn_set_fusion.argtypes = [vp, i32]
        L.ebsd_cnn_get_optimizer.argtypes = [vp, vp, vp, i64, vp]
        L.ebsd_cnn_set_optimizer.argtypes = [vp, vp, vp, i64, i64]
        L.ebsd_load_model.argtypes = [vp, C.c_char_p]
        L.ebsd_set_model.argtypes = [vp, vp]
        L.ebsd_gen_pairs.argtypes = [C.POINTER(CGenSpec), i32, i32, i32, C.c_double, C.c_double, C.c_double,
                                     vp, vp, vp, vp]
        L.ebsd_stage_conv3x3.argtypes = [vp, i32, i32, i32, i32, vp, vp, i32, i32, vp, vp]
        L.ebsd_stage_conv3x3_dgrad.argtypes = [vp, i32, i32, i32, i32, vp, i32, vp, vp]
        L.ebsd_stage_conv3x3_wgrad.argtypes = [vp, vp, i32, i32, i32, i32, i32, vp, vp]
        for name in EXPORTED:
            if name not in ("ebsd_strerror", "ebsd_version", "ebsd_cnn_num_params"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _strerror(code):
    try:
        return lib().ebsd_strerror(int(code)).decode()
    except Exception:  # library missing: no text available
        return "?"


def _check(code, what):
    if code != EBSD_OK:
        raise EbsdError(code, what)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class Params:
    """Mirror of ebsd_params with the library defaults."""
    levels: int = 3
    iters: tuple = (150, 150, 150)
    sigma_px: float = 1.0
    tol_px: float = 0.0
    pc: tuple = (0.5, 0.5, 0.7)
    n_roi: int = 20
    roi_size: int = 64
    roi_radius_frac: float = 0.3
    window: int = 1
    second_pass: int = 1
    warm_start: int = 0
    fallback_residual_px: float = 0.5
    remap_interp: int = 3
    xcf_passes: int = 1
    first_pass: int = 0
    bandpass: tuple = (0.0, 0.0)   # pre-filter sigmas (low-pass, background), px; 0 = off
    background: tuple = (0, 0.0)   # background correction: (static 0/1, dynamic sigma px)

    def to_c(self):
        p = CParams()
        p.struct_size = C.sizeof(CParams)
        p.levels = self.levels
        its = list(self.iters) if not isinstance(self.iters, int) else [self.iters] * self.levels
        its = its + [0] * (MAX_LEVELS - len(its))
        for i in range(MAX_LEVELS):
            p.max_iters[i] = int(its[i])
        p.sigma_px = self.sigma_px
        p.tol_px = self.tol_px
        p.pc_x, p.pc_y, p.pc_z = self.pc
        p.n_roi = self.n_roi
        p.roi_size = self.roi_size
        p.roi_radius_frac = self.roi_radius_frac
        p.window = self.window
        p.second_pass = self.second_pass
        p.warm_start = self.warm_start
        p.fallback_residual_px = self.fallback_residual_px
        p.remap_interp = self.remap_interp
        p.xcf_passes = self.xcf_passes
        p.first_pass = self.first_pass
        p.bandpass_lo_px, p.bandpass_hi_px = (float(v) for v in self.bandpass)
        p.background_static, p.background_dynamic_px = int(self.background[0]), float(self.background[1])
        return p


def level_size(H, W, level):
    """(h, w) of pyramid level `level`: H and W halved that many times, rounding up."""
    for _ in range(level):
        H, W = (H + 1) // 2, (W + 1) // 2
    return H, W


def roi_layout(params: Params, H, W):
    """ROI centres (cx, cy) and corners (x0, y0) as computed by the library."""
    import numpy as np
    n = params.n_roi
    cx = np.empty(n, np.float64)
    cy = np.empty(n, np.float64)
    x0 = np.empty(n, np.int32)
    y0 = np.empty(n, np.int32)
    p = params.to_c()
    _check(lib().ebsd_roi_layout(C.byref(p), H, W, cx.ctypes.data, cy.ctypes.data,
                                 x0.ctypes.data, y0.ctypes.data), "ebsd_roi_layout")
    return cx, cy, x0, y0


class Registrar:
    """A library handle bound to one device with fixed parameters."""

    def __init__(self, params: Params | None = None, device: int = 0, _handle=None):
        self.params = params or Params()
        self._p = self.params.to_c()
        self.device = device
        self._owned = _handle is None
        if _handle is None:
            h = C.c_void_p()
            _check(lib().ebsd_create(C.byref(self._p), device, C.byref(h)), "ebsd_create")
            self._h = h
        else:
            self._h = _handle

    def close(self):
        if getattr(self, "_h", None):
            if self._owned:
                lib().ebsd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _pairs(self, refs, tests, ref_ids):
        if (isinstance(refs, torch.Tensor) and isinstance(tests, torch.Tensor) and refs.dim() == 3
                and tests.dim() == 3 and refs.shape == tests.shape):
            return self._pairs_batched(refs, tests, ref_ids)
        if isinstance(refs, torch.Tensor):
            refs = list(refs.unbind(0)) if refs.dim() == 3 else [refs]
            tests = list(tests.unbind(0)) if tests.dim() == 3 else [tests]
        n = len(tests)
        arr = (CPair * max(n, 1))()
        keep = []
        for i in range(n):
            r, t = refs[i], tests[i]
            for x in (r, t):
                if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()):
                    raise ValueError("patterns must be contiguous float32 device tensors")
            arr[i].ref = r.data_ptr()
            arr[i].test = t.data_ptr()
            arr[i].H, arr[i].W = t.shape[-2], t.shape[-1]
            arr[i].ref_id = -1 if ref_ids is None else int(ref_ids[i])
            keep += [r, t]
        return arr, n, [(t.shape[-2], t.shape[-1]) for t in tests], keep

    @staticmethod
    def _pairs_batched(refs, tests, ref_ids):
        """The pair table of two [n, H, W] tensors, filled without a Python
        object per pair (pair i: base pointer + i H W floats)."""
        import numpy as np
        for x in (refs, tests):
            if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()):
                raise ValueError("patterns must be contiguous float32 device tensors")
        n, H, W = tests.shape
        arr = (CPair * max(n, 1))()
        if n:
            view = np.frombuffer(arr, dtype=np.dtype({"names": ["ref", "test", "H", "W", "ref_id"],
                                                       "formats": [np.uint64, np.uint64, np.int32, np.int32,
                                                                   np.int32],
                                                       "offsets": [CPair.ref.offset, CPair.test.offset,
                                                                   CPair.H.offset, CPair.W.offset,
                                                                   CPair.ref_id.offset],
                                                       "itemsize": C.sizeof(CPair)}), count=max(n, 1))
            step = np.arange(n, dtype=np.uint64) * np.uint64(4 * H * W)
            view["ref"][:n] = np.uint64(refs.data_ptr()) + step
            view["test"][:n] = np.uint64(tests.data_ptr()) + step
            view["H"][:n] = H
            view["W"][:n] = W
            view["ref_id"][:n] = -1 if ref_ids is None else np.asarray(ref_ids, np.int32)
        return arr, n, [(H, W)] * n, [refs, tests]

    def _outputs(self, shapes, want_field, dev, want_ssim=False):
        n = len(shapes)
        nr = self.params.n_roi
        f64 = dict(dtype=torch.float64, device=dev)
        f32 = dict(dtype=torch.float32, device=dev)
        out = {
            "F": torch.empty(n, 3, 3, **f64),
            "R": torch.empty(n, 3, 3, **f64),
            "rotvec": torch.empty(n, 3, **f64),
            "R_finite": torch.empty(n, 3, 3, **f64),
            "F_first": torch.empty(n, 3, 3, **f64),
            "q1": torch.empty(n, nr, 2, **f32),
            "q2": torch.empty(n, nr, 2, **f32),
            "peak_height": torch.empty(n, nr, **f32),
            "iters": torch.empty(n, self.params.levels, dtype=torch.int32, device=dev),
            "status": torch.empty(n, dtype=torch.int32, device=dev),
            "mae_first": torch.empty(n, **f64),
            "mae": torch.empty(n, **f64),
            "omega": torch.empty(n, 3, 3, **f64),
        }
        if want_ssim:
            out["ssim"] = torch.empty(n, **f64)
        if self.params.warm_start and shapes:
            out["warm_field"] = torch.empty(n, 64, 64, 2, **f32)
            out["warm_misfit"] = torch.empty(n, **f32)
        offs = None
        if want_field:
            sizes = [2 * h * w for h, w in shapes]
            import numpy as np
            offs = np.zeros(n, np.int64)
            if n:
                offs[1:] = np.cumsum(sizes)[:-1]
            flat = torch.empty(int(sum(sizes)), **f32)
            out["_field_flat"] = flat
            out["_field_offsets"] = offs
        co = COutputs()
        co.field = out["_field_flat"].data_ptr() if want_field else None
        co.field_offset = offs.ctypes.data if want_field else None
        for k in ("F", "R", "rotvec", "R_finite", "F_first", "q1", "q2", "peak_height", "iters",
                  "status", "warm_field", "warm_misfit", "mae_first", "mae", "ssim", "omega"):
            if k in out:
                setattr(co, k, out[k].data_ptr())
        return out, co

    @staticmethod
    def _unflatten_field(out, shapes):
        if "_field_flat" not in out:
            return out
        flat, offs = out.pop("_field_flat"), out.pop("_field_offsets")
        if shapes and len(set(shapes)) == 1:
            out["field"] = flat.view(len(shapes), 2, shapes[0][0], shapes[0][1])
        else:
            out["field"] = [flat[int(o):int(o) + 2 * h * w].view(2, h, w) for o, (h, w) in zip(offs, shapes)]
        return out

    def register(self, refs, tests, ref_ids=None, want_field=True, u_init=None, want_ssim=False):
        """Register test patterns against references (the whole path).

        refs, tests: float32 device tensors [n, H, W] (or lists of [H, W]
        tensors, sizes may differ).  ref_ids: optional ints; equal ids share
        one reference pyramid.  u_init: optional [n, 2, h, w] coarsest-level
        initial field (full-res px).  Returns a dict of device tensors:
        field, F, R, rotvec, R_finite, F_first, q1, q2, peak_height, iters,
        status, mae_first, mae (mean angular errors of the first and the last
        fit, rad) and, with want_ssim, ssim (structural similarity of the
        reference and the test warped by the final field).  With first_pass =
        1 (the conventional XCF first pass) no field is returned.  Runs on
        torch's current stream.
        """
        arr, n, shapes, keep = self._pairs(refs, tests, ref_ids)
        dev = keep[0].device if keep else torch.device("cuda", self.device)
        want_field = want_field and self.params.first_pass == 0
        out, co = self._outputs(shapes, want_field, dev, want_ssim)
        if u_init is not None:
            if not (u_init.is_cuda and u_init.dtype == torch.float32 and u_init.is_contiguous()):
                raise ValueError("u_init must be a contiguous float32 device tensor")
            rc = lib().ebsd_register_batch_init(self._h, arr, n, _ptr(u_init), C.byref(co), _stream())
        else:
            rc = lib().ebsd_register_batch(self._h, arr, n, C.byref(co), _stream())
        _check(rc, "ebsd_register_batch")
        out["_keep"] = (keep, co, arr, u_init)
        return self._unflatten_field(out, shapes)

    def load_model(self, path):
        """Network parameters for the warm start, from a parameter file."""
        _check(lib().ebsd_load_model(self._h, os.fsencode(path)), "ebsd_load_model")

    def set_model(self, net: "Cnn"):
        """Network parameters for the warm start, copied from a Cnn object."""
        _check(lib().ebsd_set_model(self._h, net._h), "ebsd_set_model")

    def autotune(self, refs, tests, ref_ids=None):
        """Time the demons strip heights on this batch and keep the fastest per
        level; returns {(h, w): rows}."""
        arr, n, shapes, keep = self._pairs(refs, tests, ref_ids)
        _check(lib().ebsd_autotune(self._h, arr, n, _stream()), "ebsd_autotune")
        out = {}
        if shapes:
            H, W = shapes[0]
            for l in range(self.params.levels):
                h, w = level_size(H, W, l)
                out[(h, w)] = lib().ebsd_get_strip_height(self._h, h, w)
        return out

    def set_graphs(self, on=True):
        """Replay captured HIP graphs (default) or launch every kernel directly."""
        _check(lib().ebsd_set_graphs(self._h, int(bool(on))), "ebsd_set_graphs")

    def set_resident(self, on=True):
        """Run levels of at most 64 x 64 px in one launch each (default) or like
        the finer levels."""
        _check(lib().ebsd_set_resident(self._h, int(bool(on))), "ebsd_set_resident")

    def set_gating(self, chunk_launches=8):
        """With a tolerance, issue each level's launches in chunks of this many
        and stop once no pair is left iterating (0 = issue every launch)."""
        _check(lib().ebsd_set_gating(self._h, int(chunk_launches)), "ebsd_set_gating")

    def launch_counts(self):
        """(issued, planned) demons launches per level of the last call."""
        import numpy as np
        issued = np.zeros(MAX_LEVELS, np.int32)
        planned = np.zeros(MAX_LEVELS, np.int32)
        _check(lib().ebsd_get_launch_counts(self._h, issued.ctypes.data, planned.ctypes.data),
               "ebsd_get_launch_counts")
        return issued[:self.params.levels], planned[:self.params.levels]

    def set_strip_height(self, level_h, level_w, rows):
        _check(lib().ebsd_set_strip_height(self._h, level_h, level_w, rows), "ebsd_set_strip_height")

    def set_fused_height(self, level_h, level_w, rows):
        """Two iterations per launch at this strip height (0 = one per launch)."""
        _check(lib().ebsd_set_fused_height(self._h, level_h, level_w, rows), "ebsd_set_fused_height")

    def fused_heights(self, H, W):
        """{(h, w): fused strip height or 0} for the levels of an H x W pattern."""
        sizes = [level_size(H, W, l) for l in range(self.params.levels)]
        return {(h, w): lib().ebsd_get_fused_height(self._h, h, w) for h, w in sizes}

    def set_timing(self, on=True):
        _check(lib().ebsd_set_timing(self._h, int(bool(on))), "ebsd_set_timing")

    def timing(self):
        """(level_ms [levels], total_ms) of the last timed call (waits for it)."""
        import numpy as np
        lv = np.zeros(MAX_LEVELS, np.float64)
        tot = np.zeros(1, np.float64)
        _check(lib().ebsd_get_timing(self._h, lv.ctypes.data, tot.ctypes.data), "ebsd_get_timing")
        return lv[:self.params.levels], float(tot[0])

    def second_pass(self, refs, tests, R_finite, ref_ids=None):
        """Second pass only, with a given R_finite [n, 3, 3] (float64 device)."""
        arr, n, shapes, keep = self._pairs(refs, tests, ref_ids)
        dev = keep[0].device if keep else torch.device("cuda", self.device)
        out, co = self._outputs(shapes, False, dev)
        rf = R_finite.to(device=dev, dtype=torch.float64).contiguous()
        _check(lib().ebsd_second_pass_batch(self._h, arr, n, _ptr(rf), C.byref(co), _stream()),
               "ebsd_second_pass_batch")
        out["_keep"] = (keep, co, arr, rf)
        for k in ("F_first", "q1", "iters", "mae_first"):
            out.pop(k)
        return out


class Pipeline:
    """Pipelined registration (ebsd_pipeline_*): batches submitted in turn run on
    `depth` library handles with their own streams and host threads, back to back
    on each, so that `depth` batches are in flight and one batch's network
    forward and coarse levels overlap another's finest demons level.  Outputs
    equal Registrar.register's bit for bit.  `slots` are Registrar views of the handles
    for configuration (load_model, autotune, set_graphs, ...) while nothing is
    pending."""

    def __init__(self, params: Params | None = None, depth: int = 2, device: int = 0):
        self.params = params or Params()
        self.device = device
        self.depth = depth
        h = C.c_void_p()
        _check(lib().ebsd_pipeline_create(C.byref(self.params.to_c()), device, depth, C.byref(h)),
               "ebsd_pipeline_create")
        self._pl = h
        self.slots = []
        for k in range(depth):
            hk = C.c_void_p()
            _check(lib().ebsd_pipeline_handle(self._pl, k, C.byref(hk)), "ebsd_pipeline_handle")
            self.slots.append(Registrar(self.params, device, _handle=hk))
        self._pending = []

    def load_model(self, path):
        for r in self.slots:
            r.load_model(path)

    def set_graphs(self, on=True):
        for r in self.slots:
            r.set_graphs(on)

    def set_resident(self, on=True):
        for r in self.slots:
            r.set_resident(on)

    def autotune(self, refs, tests, ref_ids=None):
        return [r.autotune(refs, tests, ref_ids) for r in self.slots]

    def submit(self, refs, tests, ref_ids=None, want_field=True):
        """Queue one batch (as Registrar.register, on torch's current stream);
        returns its output dict, valid after wait()."""
        r0 = self.slots[0]
        arr, n, shapes, keep = r0._pairs(refs, tests, ref_ids)
        dev = keep[0].device if keep else torch.device("cuda", self.device)
        want_field = want_field and self.params.first_pass == 0
        out, co = r0._outputs(shapes, want_field, dev)
        _check(lib().ebsd_pipeline_submit(self._pl, arr, n, C.byref(co), _stream()), "ebsd_pipeline_submit")
        out["_keep"] = (keep, co, arr)
        self._pending.append(out)
        return r0._unflatten_field(out, shapes)

    def wait(self):
        """Make torch's current stream wait for every submitted batch."""
        rc = lib().ebsd_pipeline_wait(self._pl, _stream())
        self._pending.clear()
        _check(rc, "ebsd_pipeline_wait")

    def close(self):
        if getattr(self, "_pl", None):
            for r in self.slots:
                r._h = None
            lib().ebsd_pipeline_destroy(self._pl)
            self._pl = None
            self._pending.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Cnn:
    """The warm-start network (ebsd_cnn_* entry points) on one device."""

    def __init__(self, device: int = 0, max_batch: int = 64):
        self.device = device
        self.max_batch = max_batch
        h = C.c_void_p()
        _check(lib().ebsd_cnn_create(device, max_batch, C.byref(h)), "ebsd_cnn_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().ebsd_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, vec):
        """Flat float32 parameter vector (host numpy array)."""
        import numpy as np
        v = np.ascontiguousarray(vec, np.float32)
        _check(lib().ebsd_cnn_set_params(self._h, v.ctypes.data, v.size), "ebsd_cnn_set_params")

    def get_params(self):
        import numpy as np
        v = np.empty(CNN_PARAMS, np.float32)
        _check(lib().ebsd_cnn_get_params(self._h, v.ctypes.data, v.size), "ebsd_cnn_get_params")
        return v

    def get_grads(self):
        import numpy as np
        v = np.empty(CNN_PARAMS, np.float32)
        _check(lib().ebsd_cnn_get_grads(self._h, v.ctypes.data, v.size), "ebsd_cnn_get_grads")
        return v

    def load(self, path):
        _check(lib().ebsd_cnn_load(self._h, os.fsencode(path)), "ebsd_cnn_load")

    def save(self, path):
        _check(lib().ebsd_cnn_save(self._h, os.fsencode(path)), "ebsd_cnn_save")

    def forward(self, refs, tests, out=None):
        """refs, tests: [n, 256, 256] float32 device (raw patterns).  Returns
        [n, 64, 64, 2] (x, y) full-res px."""
        refs, tests = _dev_f32(refs), _dev_f32(tests)
        n, H, W = tests.shape
        if out is None:
            out = torch.empty(n, H // 4, W // 4, 2, dtype=torch.float32, device=tests.device)
        _check(lib().ebsd_cnn_forward(self._h, _ptr(refs), _ptr(tests), n, H, W, _ptr(out), _stream()),
               "ebsd_cnn_forward")
        return out

    def train_step(self, refs, tests, labels, lr=1e-3, update=True):
        """One step (forward, loss, backward, Adam if update); returns the loss."""
        refs, tests, labels = _dev_f32(refs), _dev_f32(tests), _dev_f32(labels)
        n, H, W = tests.shape
        loss = C.c_float()
        _check(lib().ebsd_cnn_train_step(self._h, _ptr(refs), _ptr(tests), _ptr(labels), n, H, W,
                                         float(lr), int(bool(update)), C.byref(loss), _stream()),
               "ebsd_cnn_train_step")
        return float(loss.value)

    def get_optimizer(self):
        """Adam's state: (m, v, step) with m, v float32 host arrays."""
        import numpy as np
        m = np.zeros(CNN_PARAMS, np.float32)
        v = np.zeros(CNN_PARAMS, np.float32)
        st = C.c_int64(0)
        _check(lib().ebsd_cnn_get_optimizer(self._h, m.ctypes.data, v.ctypes.data, CNN_PARAMS, C.byref(st)),
               "ebsd_cnn_get_optimizer")
        return m, v, int(st.value)

    def set_optimizer(self, m, v, step):
        """Restore Adam's state (moments and step count)."""
        import numpy as np
        m = np.ascontiguousarray(m, np.float32)
        v = np.ascontiguousarray(v, np.float32)
        _check(lib().ebsd_cnn_set_optimizer(self._h, m.ctypes.data, v.ctypes.data, CNN_PARAMS, int(step)),
               "ebsd_cnn_set_optimizer")

    def reset_optimizer(self):
        _check(lib().ebsd_cnn_reset_optimizer(self._h), "ebsd_cnn_reset_optimizer")

    def set_fusion(self, on):
        """Inference forward with the fused kernels (True, the default) or one
        kernel per layer (False); equal outputs."""
        _check(lib().ebsd_cnn_set_fusion(self._h, 1 if on else 0), "ebsd_cnn_set_fusion")


# -- single-stage entry points -------------------------------------------------------

def _dev_f32(x):
    if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()):
        raise ValueError("expected a contiguous float32 device tensor")
    return x


def stage_normalize(p):
    """z-score each pattern of p [n, ...]; returns (out, flags)."""
    p = _dev_f32(p)
    n = p.shape[0]
    out = torch.empty_like(p)
    flags = torch.empty(n, dtype=torch.int32, device=p.device)
    _check(lib().ebsd_stage_normalize(_ptr(p), n, p[0].numel() if n else 1, _ptr(out), _ptr(flags),
                                      _stream()), "ebsd_stage_normalize")
    return out, flags


def stage_bandpass(img, lo, hi):
    """Pre-filter (Gaussian low-pass sigma lo minus Gaussian background sigma
    hi, 0 = off) of raw images [n, H, W] float32 device."""
    img = _dev_f32(img)
    n, H, W = img.shape
    out = torch.empty_like(img)
    _check(lib().ebsd_stage_bandpass(_ptr(img), n, H, W, float(lo), float(hi), _ptr(out), _stream()),
           "ebsd_stage_bandpass")
    return out


def stage_restrict(img):
    img = _dev_f32(img)
    n, H, W = img.shape
    out = torch.empty(n, (H + 1) // 2, (W + 1) // 2, dtype=torch.float32, device=img.device)
    _check(lib().ebsd_stage_restrict(_ptr(img), n, H, W, _ptr(out), _stream()), "ebsd_stage_restrict")
    return out


def stage_demons_iter(R, T, u, sigma):
    R, T, u = _dev_f32(R), _dev_f32(T), _dev_f32(u)
    n, H, W = R.shape
    out = torch.empty_like(u)
    rms = torch.empty(n, dtype=torch.float64, device=R.device)
    _check(lib().ebsd_stage_demons_iter(_ptr(R), _ptr(T), n, H, W, _ptr(u), float(sigma), _ptr(out),
                                        _ptr(rms), _stream()), "ebsd_stage_demons_iter")
    return out, rms


def stage_prolong(u):
    u = _dev_f32(u)
    n, _, h, w = u.shape
    out = torch.empty(n, 2, 2 * h, 2 * w, dtype=torch.float32, device=u.device)
    _check(lib().ebsd_stage_prolong(_ptr(u), n, h, w, _ptr(out), _stream()), "ebsd_stage_prolong")
    return out


def stage_xcf(A, B, window=1):
    A, B = _dev_f32(A), _dev_f32(B)
    n, N, _ = A.shape
    q = torch.empty(n, 2, dtype=torch.float32, device=A.device)
    ph = torch.empty(n, dtype=torch.float32, device=A.device)
    _check(lib().ebsd_stage_xcf(_ptr(A), _ptr(B), n, N, window, _ptr(q), _ptr(ph), _stream()),
           "ebsd_stage_xcf")
    return q, ph


def stage_remap(img, R, pcs, interp=3):
    """Remap of n images [n, H, W] by rotations R [n, 3, 3]: returns (out,
    coef); coef holds the cubic B-spline coefficients (None for bilinear)."""
    img = _dev_f32(img)
    n, H, W = img.shape
    R = torch.as_tensor(R, dtype=torch.float64).to(img.device).reshape(n, 9).contiguous()
    out = torch.empty_like(img)
    coef = torch.empty_like(img) if interp == 3 else None
    _check(lib().ebsd_stage_remap(_ptr(img), n, H, W, _ptr(R), float(pcs[0]), float(pcs[1]), float(pcs[2]),
                                  interp, _ptr(coef) if coef is not None else None, _ptr(out), _stream()),
           "ebsd_stage_remap")
    return out, coef


def stage_solve(q, cx, cy, pcs):
    """Eq. (3) solve: q [n, n_roi, 2] float32 device; cx, cy [n_roi] float64."""
    q = _dev_f32(q)
    n, nr, _ = q.shape
    cx = torch.as_tensor(cx, dtype=torch.float64).to(q.device).contiguous()
    cy = torch.as_tensor(cy, dtype=torch.float64).to(q.device).contiguous()
    F = torch.empty(n, 3, 3, dtype=torch.float64, device=q.device)
    R = torch.empty(n, 3, 3, dtype=torch.float64, device=q.device)
    st = torch.empty(n, dtype=torch.int32, device=q.device)
    _check(lib().ebsd_stage_solve(_ptr(q), n, nr, _ptr(cx), _ptr(cy), float(pcs[0]), float(pcs[1]),
                                  float(pcs[2]), _ptr(F), _ptr(R), _ptr(st), _stream()),
           "ebsd_stage_solve")
    return F, R, st


# the paper's nickel constants (C11, C12, C44), Pa
NICKEL_STIFFNESS = (2.76e11, 1.59e11, 1.32e11)


def r_tilt(theta):
    """Eq. (13)'s detector-to-sample rotation for a tilt theta (rad), from
    ebsd_tilt_rotation; a 3 x 3 tuple of rows."""
    S = (C.c_double * 9)()
    _check(lib().ebsd_tilt_rotation(float(theta), S), "ebsd_tilt_rotation")
    return tuple(tuple(S[3 * i + j] for j in range(3)) for i in range(3))


def traction_free(q, cx, cy, pcs, g, S, stiffness=NICKEL_STIFFNESS, M=None):
    """Eq. (3) under the traction-free constraint with strain and stress
    (ebsd_traction_free).  q [n, n_roi, 2] float32 device shifts; cx, cy
    [n_roi] ROI centres; pcs = (x*, y*, Z*) px; g [n, 3, 3] passive
    sample-to-crystal orientations; S 3 x 3 detector-to-sample rotation
    (host); stiffness = (C11, C12, C44); M [n, 3, 3] what the fit composes with
    (R_finite for second-pass shifts) or None.  Returns a dict of device
    tensors F, eps_S, sigma_S [n, 3, 3] and status [n]."""
    q = _dev_f32(q)
    n, nr, _ = q.shape
    dev = q.device
    cx = torch.as_tensor(cx, dtype=torch.float64).to(dev).contiguous()
    cy = torch.as_tensor(cy, dtype=torch.float64).to(dev).contiguous()
    g = torch.as_tensor(g, dtype=torch.float64).to(dev).reshape(n, 3, 3).contiguous()
    Mt = None if M is None else torch.as_tensor(M, dtype=torch.float64).to(dev).reshape(n, 3, 3).contiguous()
    Sh = (C.c_double * 9)(*[float(v) for row in S for v in row])
    out = {k: torch.empty(n, 3, 3, dtype=torch.float64, device=dev) for k in ("F", "eps_S", "sigma_S")}
    out["status"] = torch.empty(n, dtype=torch.int32, device=dev)
    _check(lib().ebsd_traction_free(_ptr(q), n, nr, _ptr(cx), _ptr(cy), float(pcs[0]), float(pcs[1]),
                                    float(pcs[2]), _ptr(Mt) if Mt is not None else None, _ptr(g), Sh,
                                    float(stiffness[0]), float(stiffness[1]), float(stiffness[2]),
                                    _ptr(out["F"]), _ptr(out["eps_S"]),
                                    _ptr(out["sigma_S"]), _ptr(out["status"]), _stream()),
           "ebsd_traction_free")
    return out


def _dev_bf16(x):
    if not (x.is_cuda and x.dtype == torch.bfloat16 and x.is_contiguous()):
        raise ValueError("expected a contiguous bfloat16 device tensor")
    return x


def stage_conv3x3(x, w, bias=None, relu_bf16=True):
    """3x3 convolution kernel alone.  x [n, H, W, Cin] bfloat16, w [3, 3, Cin,
    Cout] float32, bias [Cout] float32.  relu_bf16: bfloat16 max(conv + bias,
    0); otherwise the float32 convolution."""
    x = _dev_bf16(x)
    w = _dev_f32(w)
    n, H, W, Cin = x.shape
    Cout = w.shape[3]
    if relu_bf16:
        bias = _dev_f32(bias)
        out = torch.empty(n, H, W, Cout, dtype=torch.bfloat16, device=x.device)
    else:
        out = torch.empty(n, H, W, Cout, dtype=torch.float32, device=x.device)
    _check(lib().ebsd_stage_conv3x3(_ptr(x), n, H, W, Cin, _ptr(w), _ptr(bias), Cout, 0 if relu_bf16 else 1,
                                    _ptr(out), _stream()), "ebsd_stage_conv3x3")
    return out


def stage_conv3x3_dgrad(dz, w):
    """Input gradient kernel alone: dz [n, H, W, Cout] bfloat16, w [3, 3, Cin, Cout] float32."""
    dz = _dev_bf16(dz)
    w = _dev_f32(w)
    n, H, W, Cout = dz.shape
    Cin = w.shape[2]
    dx = torch.empty(n, H, W, Cin, dtype=torch.float32, device=dz.device)
    _check(lib().ebsd_stage_conv3x3_dgrad(_ptr(dz), n, H, W, Cout, _ptr(w), Cin, _ptr(dx), _stream()),
           "ebsd_stage_conv3x3_dgrad")
    return dx


def stage_conv3x3_wgrad(x, dz):
    """Weight gradient kernel alone: x [n, H, W, Cin], dz [n, H, W, Cout] bfloat16 -> [3, 3, Cin, Cout]."""
    x, dz = _dev_bf16(x), _dev_bf16(dz)
    n, H, W, Cin = x.shape
    Cout = dz.shape[3]
    dw = torch.empty(3, 3, Cin, Cout, dtype=torch.float32, device=x.device)
    _check(lib().ebsd_stage_conv3x3_wgrad(_ptr(x), _ptr(dz), n, H, W, Cin, Cout, _ptr(dw), _stream()),
           "ebsd_stage_conv3x3_wgrad")
    return dw


def gen_pairs(specs, labels=True, device=0):
    """Render pattern pairs on the GPU from synth.PairSpec descriptions (same
    size, pattern centre and band set "basic" for all).  The noise key of a
    spec is its (config_id, pair_index) seeds.  Returns (ref, test, label)
    device tensors [n, H, W], [n, H, W], [n, H/4, W/4, 2] (label None if not
    wanted)."""
    n = len(specs)
    if n == 0:
        raise ValueError("no specs")
    H, W, pc = specs[0].H, specs[0].W, tuple(specs[0].pc)
    arr = (CGenSpec * n)()
    for i, s in enumerate(specs):
        if (s.H, s.W, tuple(s.pc)) != (H, W, pc) or s.bands != "basic":
            raise ValueError("all specs need the same size, pattern centre and the basic band set")
        G = [float(v) for v in list(s.G.ravel())]
        F = [float(v) for v in list(s.F.ravel())]
        for j in range(9):
            arr[i].G[j] = G[j]
            arr[i].F[j] = F[j]
        arr[i].gx, arr[i].gy = float(s.gxy[0]), float(s.gxy[1])
        arr[i].counts = float(s.counts)
        arr[i].key[0], arr[i].key[1] = int(s.seeds[0]) & 0xFFFFFFFF, int(s.seeds[1]) & 0xFFFFFFFF
        arr[i].noise = int(bool(s.noise))
        arr[i].bands = 1
    dev = torch.device("cuda", device)
    ref = torch.empty(n, H, W, dtype=torch.float32, device=dev)
    test = torch.empty(n, H, W, dtype=torch.float32, device=dev)
    label = torch.empty(n, H // 4, W // 4, 2, dtype=torch.float32, device=dev) if labels else None
    _check(lib().ebsd_gen_pairs(arr, n, H, W, pc[0], pc[1], pc[2], _ptr(ref), _ptr(test), _ptr(label),
                                _stream()), "ebsd_gen_pairs")
    return ref, test, label

"""FP64 CPU oracle for demons-based HR-EBSD remapping (arXiv:1907.05993).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg import this package.  The product (the HIP library in
``paper_1907_05993_amd`` and its binding) never imports, loads or calls it,
and the two share no code.

This module is a thin ctypes wrapper over ``ebsd_oracle.c`` (plain loops, FP64,
OpenMP over pairs).  Every function restates which part of the paper it follows;
the arithmetic itself lives in the C file.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB may name another build of the same source (the sanitizer build of build.py)
_LIBPATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

CONVERGED = 1
HIT_CAP = 2
SOLVE_ILLCOND = 16
NONFINITE_INPUT = 32
DEGENERATE_INPUT = 64
MAX_LEVELS = 8


class Params(C.Structure):
    _fields_ = [
        ("levels", C.c_int32),
        ("max_iters", C.c_int32 * MAX_LEVELS),
        ("sigma", C.c_double),
        ("tol", C.c_double),
        ("pc_x", C.c_double),
        ("pc_y", C.c_double),
        ("pc_z", C.c_double),
        ("n_roi", C.c_int32),
        ("roi_size", C.c_int32),
        ("roi_radius_frac", C.c_double),
        ("window", C.c_int32),
        ("second_pass", C.c_int32),
        ("remap_interp", C.c_int32),
        ("xcf_passes", C.c_int32),
        ("first_pass", C.c_int32),
        ("bandpass_lo", C.c_double),
        ("bandpass_hi", C.c_double),
        ("background_static", C.c_int32),
        ("background_dynamic", C.c_double),
        ("background", C.c_void_p),
        ("peak_fit", C.c_int32),
    ]


class _Outputs(C.Structure):
    _fields_ = [
        ("field", C.c_void_p),
        ("q1", C.c_void_p),
        ("F1", C.c_void_p),
        ("Rfin", C.c_void_p),
        ("q2", C.c_void_p),
        ("ph", C.c_void_p),
        ("F", C.c_void_p),
        ("R", C.c_void_p),
        ("rotvec", C.c_void_p),
        ("iters", C.c_void_p),
        ("status", C.c_void_p),
        ("mae1", C.c_void_p),
        ("mae", C.c_void_p),
        ("ssim", C.c_void_p),
        ("omega", C.c_void_p),
    ]


def make_params(levels=3, iters=100, sigma=1.0, tol=0.0, pc=(0.5, 0.5, 0.7), n_roi=20,
                roi_size=32, roi_radius_frac=0.3, window=1, second_pass=1, remap_interp=3,
                xcf_passes=1, first_pass=0, bandpass=(0.0, 0.0), background=(0, 0.0), peak_fit=0):
    p = Params()
    p.levels = levels
    its = [iters] * MAX_LEVELS if np.isscalar(iters) else list(iters) + [0] * (MAX_LEVELS - len(iters))
    for i in range(MAX_LEVELS):
        p.max_iters[i] = int(its[i])
    p.sigma = sigma
    p.tol = tol
    p.pc_x, p.pc_y, p.pc_z = pc
    p.n_roi = n_roi
    p.roi_size = roi_size
    p.roi_radius_frac = roi_radius_frac
    p.window = window
    p.second_pass = second_pass
    p.remap_interp = remap_interp
    p.xcf_passes = xcf_passes
    p.first_pass = first_pass
    p.bandpass_lo, p.bandpass_hi = bandpass
    p.background_static, p.background_dynamic = int(background[0]), float(background[1])
    p.background = None
    p.peak_fit = peak_fit
    return p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIBPATH)
        d = C.POINTER(C.c_double)
        f = C.POINTER(C.c_float)
        L.orc_normalize.restype = C.c_uint32
        L.orc_normalize.argtypes = [f, C.c_int64, d]
        L.orc_restrict.argtypes = [d, C.c_int, C.c_int, d]
        L.orc_gradient.argtypes = [d, C.c_int, C.c_int, d, d]
        L.orc_bilinear.restype = C.c_double
        L.orc_bilinear.argtypes = [d, C.c_int, C.c_int, C.c_double, C.c_double]
        L.orc_bilinear_points.argtypes = [d, C.c_int, C.c_int, d, d, C.c_int64, d]
        L.orc_warp.argtypes = [d, C.c_int, C.c_int, d, d]
        L.orc_smooth.argtypes = [d, C.c_int, C.c_int, C.c_double, d]
        L.orc_demons_iter.restype = C.c_double
        L.orc_demons_iter.argtypes = [d, d, d, d, C.c_int, C.c_int, d, C.c_double, d]
        L.orc_prolong.argtypes = [d, C.c_int, C.c_int, C.c_int, C.c_int, d]
        L.orc_demons.restype = C.c_uint32
        L.orc_demons.argtypes = [d, d, C.c_int, C.c_int, C.POINTER(Params), d, d,
                                 C.POINTER(C.c_int32)]
        L.orc_roi_layout.restype = C.c_int
        L.orc_roi_layout.argtypes = [C.c_int, C.c_int, C.POINTER(Params), d, d,
                                     C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.orc_jacobi_eig.argtypes = [d, C.c_int, d, d]
        L.orc_det_normalize.argtypes = [d]
        L.orc_solve_F.restype = C.c_uint32
        L.orc_solve_F.argtypes = [d, d, d, C.c_int, C.c_double, C.c_double, C.c_double, d]
        L.orc_stress.argtypes = [d, d, C.c_double, C.c_double, C.c_double, d]
        L.orc_strain_stress.argtypes = [d, d, d, C.c_double, C.c_double, C.c_double, d, d, d]
        L.orc_solve_F_traction_free.restype = C.c_uint32
        L.orc_solve_F_traction_free.argtypes = [d, d, d, C.c_int, C.c_double, C.c_double, C.c_double, d, d,
                                                d, C.c_double, C.c_double, C.c_double, d, d, d]
        L.orc_bandpass.argtypes = [f, C.c_int, C.c_int, C.c_double, C.c_double, d]
        L.orc_background.argtypes = [f, C.c_int, C.c_int, d, C.c_double, d]
        L.orc_mean_pattern.argtypes = [f, C.c_int, C.c_int, C.c_int, d]
        L.orc_ssim.restype = C.c_double
        L.orc_ssim.argtypes = [d, d, C.c_int, C.c_int]
        L.orc_mae.restype = C.c_double
        L.orc_mae.argtypes = [d, d, d, C.c_int, C.c_double, C.c_double, C.c_double, d]
        L.orc_polar.argtypes = [d, d]
        L.orc_rotvec.argtypes = [d, d]
        L.orc_omega.argtypes = [d, d]
        L.orc_remap.argtypes = [d, C.c_int, C.c_int, d, C.c_double, C.c_double, C.c_double, C.c_int, d]
        L.orc_bspline_coeffs.argtypes = [d, C.c_int, C.c_int, d]
        L.orc_bspline_at.restype = C.c_double
        L.orc_bspline_at.argtypes = [d, C.c_int, C.c_int, C.c_double, C.c_double]
        L.orc_bspline_points.argtypes = [d, C.c_int, C.c_int, d, d, C.c_int64, d]
        L.orc_fft1.argtypes = [d, d, C.c_int, C.c_int]
        L.orc_fft2.argtypes = [d, d, C.c_int, C.c_int]
        L.orc_xcf.argtypes = [d, d, C.c_int, C.c_int, d, d, d]
        L.orc_xcf_fit.argtypes = [d, d, C.c_int, C.c_int, C.c_int, d, d, d]
        L.orc_peak_fourier.restype = C.c_int
        L.orc_peak_fourier.argtypes = [d, d, C.c_int, C.c_int, C.c_int, d, d]
        L.orc_peak_subpixel.restype = C.c_int
        L.orc_peak_subpixel.argtypes = [d, d]
        L.orc_register_pair.restype = C.c_int
        L.orc_register_pair.argtypes = [f, f, C.c_int, C.c_int, C.POINTER(Params), d, d,
                                        C.POINTER(_Outputs)]
        L.orc_register_batch.restype = C.c_int
        L.orc_register_batch.argtypes = [f, f, C.c_int, C.c_int, C.c_int, C.POINTER(Params), d,
                                         C.POINTER(_Outputs)]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# -- stage functions ------------------------------------------------------------

def normalize(p):
    """Per-pattern z-score (zero mean as in section 2).  Returns (out, status)."""
    a = np.ascontiguousarray(p, dtype=np.float32)
    out = np.empty(a.shape, np.float64)
    st = lib().orc_normalize(_f(a), a.size, _d(out))
    return out, int(st)


def restrict(img):
    """Factor-2 pyramid restriction with the [1,3,3,1]/8 filter (section 1);
    ceil(H/2) x ceil(W/2) outputs."""
    a = _f64(img)
    H, W = a.shape
    out = np.empty(((H + 1) // 2, (W + 1) // 2), np.float64)
    lib().orc_restrict(_d(a), H, W, _d(out))
    return out


def gradient(img):
    """Image gradient of Eq. (1): central inside, one-sided on the border."""
    a = _f64(img)
    H, W = a.shape
    gx = np.empty_like(a)
    gy = np.empty_like(a)
    lib().orc_gradient(_d(a), H, W, _d(gx), _d(gy))
    return gx, gy


def bilinear_points(img, xs, ys):
    a = _f64(img)
    H, W = a.shape
    xs = _f64(xs).ravel()
    ys = _f64(ys).ravel()
    out = np.empty(xs.shape, np.float64)
    lib().orc_bilinear_points(_d(a), H, W, _d(xs), _d(ys), xs.size, _d(out))
    return out


def warp(img, u):
    """out(x) = img(x + u(x)), bilinear, clamped."""
    a = _f64(img)
    u = _f64(u)
    H, W = a.shape
    out = np.empty_like(a)
    lib().orc_warp(_d(a), H, W, _d(u), _d(out))
    return out


def smooth(v, sigma):
    a = _f64(v)
    H, W = a.shape
    out = np.empty_like(a)
    lib().orc_smooth(_d(a), H, W, float(sigma), _d(out))
    return out


def demons_iter(R, T, u, sigma):
    """One demons iteration (Eq. 1 force, then field smoothing).  Returns (u_new, rms)."""
    R = _f64(R)
    T = _f64(T)
    u = _f64(u)
    H, W = R.shape
    gx, gy = gradient(R)
    out = np.empty_like(u)
    rms = lib().orc_demons_iter(_d(R), _d(T), _d(gx), _d(gy), H, W, _d(u), float(sigma), _d(out))
    return out, rms


def prolong(u, shape=None):
    """Field [2, h, w] to the finer level, shape (H, W) (default (2h, 2w))."""
    u = _f64(u)
    _, h, w = u.shape
    H, W = shape if shape is not None else (2 * h, 2 * w)
    out = np.empty((2, H, W), np.float64)
    lib().orc_prolong(_d(u), h, w, H, W, _d(out))
    return out


def demons(Rn, Tn, params, u_init=None):
    """Multi-resolution demons on normalised images.  Returns (field, iters, status)."""
    Rn = _f64(Rn)
    Tn = _f64(Tn)
    H, W = Rn.shape
    field = np.empty((2, H, W), np.float64)
    its = (C.c_int32 * MAX_LEVELS)()
    ui = None
    if u_init is not None:
        ui = _f64(u_init)
    st = lib().orc_demons(_d(Rn), _d(Tn), H, W, C.byref(params), _d(ui) if ui is not None else None,
                          _d(field), its)
    return field, np.array(its[:params.levels]), int(st)


def roi_layout(H, W, params):
    """ROI centres and corners: one at the pattern centre, the rest on a ring."""
    n = params.n_roi
    cx = np.empty(n)
    cy = np.empty(n)
    x0 = np.empty(n, np.int32)
    y0 = np.empty(n, np.int32)
    bad = lib().orc_roi_layout(H, W, C.byref(params), _d(cx), _d(cy),
                               x0.ctypes.data_as(C.POINTER(C.c_int32)),
                               y0.ctypes.data_as(C.POINTER(C.c_int32)))
    return cx, cy, x0, y0, bool(bad)


def jacobi_eig(A):
    A = _f64(A).copy()
    n = A.shape[0]
    ev = np.empty(n)
    V = np.empty((n, n))
    lib().orc_jacobi_eig(_d(A), n, _d(ev), _d(V))
    return ev, V


def solve_F(q, cx, cy, pcs):
    """Eq. (3) minimiser for the Eq. (2) model, det F = 1.  pcs = (x*, y*, Z*) in px."""
    q = _f64(q).reshape(-1, 2)
    cx = _f64(cx)
    cy = _f64(cy)
    F = np.empty(9)
    st = lib().orc_solve_F(_d(q), _d(cx), _d(cy), len(cx), float(pcs[0]), float(pcs[1]),
                           float(pcs[2]), _d(F))
    return F.reshape(3, 3), int(st)


def mae(q, F, cx, cy, pcs):
    """Mean angular error (rad) of the Eq. (3) fit F to the shifts q at the ROI
    centres (cx, cy): the mean over ROIs of the angle between F r_i and
    r_i + q_i (the reading of the figure section 3 compares methods by)."""
    q = _f64(q).reshape(-1, 2)
    cx = _f64(cx)
    cy = _f64(cy)
    F = _f64(F).reshape(9)
    return float(lib().orc_mae(_d(q), _d(cx), _d(cy), len(cx), float(pcs[0]), float(pcs[1]),
                               float(pcs[2]), _d(F)))


def stress(eps_S, g, C):
    """Sample-frame stress of a sample-frame strain (Eq. (16), supplementary
    Eq. (2.4)-(2.8)): g is the passive sample-to-crystal orientation, C =
    (C11, C12, C44) the cubic stiffness of the crystal frame."""
    e = _f64(eps_S).reshape(9)
    out = np.empty(9)
    lib().orc_stress(_d(e), _d(_f64(g).reshape(9)), float(C[0]), float(C[1]), float(C[2]), _d(out))
    return out.reshape(3, 3)


def strain_stress(F, S, g, C):
    """(F_S, eps_S, sigma_S) of a detector-frame F (Eq. (14)-(16)); S is the
    detector-to-sample rotation."""
    FS, e, sg = np.empty(9), np.empty(9), np.empty(9)
    lib().orc_strain_stress(_d(_f64(F).reshape(9)), _d(_f64(S).reshape(9)), _d(_f64(g).reshape(9)),
                            float(C[0]), float(C[1]), float(C[2]), _d(FS), _d(e), _d(sg))
    return FS.reshape(3, 3), e.reshape(3, 3), sg.reshape(3, 3)


def solve_F_traction_free(q, cx, cy, pcs, S, g, C, M=None):
    """Eq. (3) under the traction-free constraint sigma_S33 = sigma_S23 =
    sigma_S13 = 0 of the total F = F_inf M.  Returns (F, eps_S, sigma_S,
    status)."""
    q = _f64(q).reshape(-1, 2)
    cx = _f64(cx)
    cy = _f64(cy)
    F, e, sg = np.empty(9), np.empty(9), np.empty(9)
    Mm = _f64(M).reshape(9) if M is not None else None
    st = lib().orc_solve_F_traction_free(_d(q), _d(cx), _d(cy), len(cx), float(pcs[0]), float(pcs[1]),
                                         float(pcs[2]), _d(Mm) if Mm is not None else None,
                                         _d(_f64(S).reshape(9)), _d(_f64(g).reshape(9)), float(C[0]),
                                         float(C[1]), float(C[2]), _d(F), _d(e), _d(sg))
    return F.reshape(3, 3), e.reshape(3, 3), sg.reshape(3, 3), int(st)


def bandpass(img, lo, hi):
    """Pre-filter of a raw pattern: Gaussian low-pass (sigma lo) minus the
    Gaussian background (sigma hi); 0 turns a filter off."""
    a = np.ascontiguousarray(img, dtype=np.float32)
    H, W = a.shape
    out = np.empty((H, W), np.float64)
    lib().orc_bandpass(_f(a), H, W, float(lo), float(hi), _d(out))
    return out


def background(img, bg=None, dyn=0.0):
    """Background correction of a raw pattern: divided by the static
    background bg (None = off), then by its own Gaussian blur of sigma dyn."""
    a = np.ascontiguousarray(img, dtype=np.float32)
    H, W = a.shape
    out = np.empty((H, W), np.float64)
    b = _f64(bg) if bg is not None else None
    lib().orc_background(_f(a), H, W, _d(b) if b is not None else None, float(dyn), _d(out))
    return out


def mean_pattern(p):
    """Pixelwise mean of patterns [n, H, W] (the static background)."""
    a = np.ascontiguousarray(p, dtype=np.float32)
    n, H, W = a.shape
    out = np.empty((H, W), np.float64)
    lib().orc_mean_pattern(_f(a), n, H, W, _d(out))
    return out


def ssim(R, Tw):
    """Mean structural similarity of R and Tw (11 x 11 Gaussian window of
    sigma 1.5, L = 6 for z-scored patterns, pixels whose window fits)."""
    a = _f64(R)
    b = _f64(Tw)
    H, W = a.shape
    return float(lib().orc_ssim(_d(a), _d(b), H, W))


def polar(F):
    """Rotation factor of F via SVD, Eq. (4)-(5)."""
    F = _f64(F).reshape(9)
    R = np.empty(9)
    lib().orc_polar(_d(F), _d(R))
    return R.reshape(3, 3)


def rotvec(R):
    R = _f64(R).reshape(9)
    out = np.empty(3)
    lib().orc_rotvec(_d(R), _d(out))
    return out


def omega(rotvec):
    """Eq. (6): omega_ij = -eps_ijk theta_k of a rotation vector theta (3 x 3)."""
    th = _f64(rotvec).reshape(3)
    om = np.empty(9)
    lib().orc_omega(_d(th), _d(om))
    return om.reshape(3, 3)


def det_normalize(F):
    F = _f64(F).reshape(9).copy()
    lib().orc_det_normalize(_d(F))
    return F.reshape(3, 3)


def remap(ref, Rfin, pcs, interp=3):
    """Reference remapped by R_finite: Rm(x') = ref(pi(R^T r(x'))) (section 2,
    before Eq. (12)); interp 3 = cubic B-spline, 1 = bilinear."""
    a = _f64(ref)
    H, W = a.shape
    Rf = _f64(Rfin).reshape(9)
    out = np.empty_like(a)
    lib().orc_remap(_d(a), H, W, _d(Rf), float(pcs[0]), float(pcs[1]), float(pcs[2]), int(interp),
                    _d(out))
    return out


def bspline_coeffs(img):
    """Cubic B-spline coefficients of img under whole-sample mirroring."""
    a = _f64(img)
    H, W = a.shape
    out = np.empty_like(a)
    lib().orc_bspline_coeffs(_d(a), H, W, _d(out))
    return out


def bspline_points(coef, xs, ys):
    """Cubic B-spline interpolant with coefficients coef at (xs, ys), clamped."""
    c = _f64(coef)
    H, W = c.shape
    xs = _f64(xs).ravel()
    ys = _f64(ys).ravel()
    out = np.empty(xs.size)
    lib().orc_bspline_points(_d(c), H, W, _d(xs), _d(ys), xs.size, _d(out))
    return out


def fft1(x, inverse=False):
    x = np.asarray(x, np.complex128)
    re = np.ascontiguousarray(x.real)
    im = np.ascontiguousarray(x.imag)
    lib().orc_fft1(_d(re), _d(im), x.size, int(inverse))
    return re + 1j * im


def fft2(x, inverse=False):
    x = np.asarray(x, np.complex128)
    re = np.ascontiguousarray(x.real)
    im = np.ascontiguousarray(x.imag)
    lib().orc_fft2(_d(re), _d(im), x.shape[0], int(inverse))
    return re + 1j * im


def xcf(A, B, window=1, peak_fit=0):
    """ROI cross-correlation (section 2).  peak_fit 0: the 2-D quadratic fit
    of the peak's 3 x 3 neighbourhood; 1: the maximum of the correlation's
    band-limited interpolant.  Returns (q, ph, C)."""
    A = _f64(A)
    B = _f64(B)
    N = A.shape[0]
    Cm = np.empty((N, N))
    q = np.empty(2)
    ph = np.empty(1)
    lib().orc_xcf_fit(_d(A), _d(B), N, int(window), int(peak_fit), _d(Cm), _d(q), _d(ph))
    return q, float(ph[0]), Cm


def peak_fourier(P, start, integer_peak):
    """Maximum of the band-limited interpolant of C = IFFT2(P) near `start`
    (x, y), starting integer peak (sx, sy) in signed coordinates.  Returns
    ((x, y), ok)."""
    P = np.asarray(P, np.complex128)
    N = P.shape[0]
    re = np.ascontiguousarray(P.real)
    im = np.ascontiguousarray(P.imag)
    x = C.c_double(start[0])
    y = C.c_double(start[1])
    ok = lib().orc_peak_fourier(_d(re), _d(im), N, int(integer_peak[0]), int(integer_peak[1]), C.byref(x),
                                C.byref(y))
    return (x.value, y.value), bool(ok)


def peak_subpixel(nb):
    """Sub-pixel offset (dx, dy) of a correlation peak from its 3 x 3
    neighbourhood nb[dy + 1, dx + 1] (section 2's interpolated peak: the
    quadratic surface through the neighbourhood, its stationary point when
    negative definite, each component clamped to +-1).  Returns (d, ok)."""
    nb = np.ascontiguousarray(np.asarray(nb, np.float64).reshape(9))
    d = np.zeros(2)
    ok = lib().orc_peak_subpixel(_d(nb), _d(d))
    return d, bool(ok)


def pc_pixels(H, W, params):
    """(x*, y*, Z*) in px from the fractional pattern centre."""
    return (params.pc_x * W - 0.5, params.pc_y * H - 0.5, params.pc_z * W)


_OUT_KEYS = ("field", "q1", "F1", "Rfin", "q2", "ph", "F", "R", "rotvec", "iters", "status", "mae1", "mae",
             "ssim", "omega")


def register_batch(refs, tests, params, rfin=None, want_field=True, u_init=None):
    """Whole pipeline for a batch of pairs (OpenMP over pairs).

    refs, tests: [n, H, W] float32.  rfin: optional [n, 3, 3] R_finite that
    replaces the first pass's (second pass checked in isolation).  u_init:
    optional [n, 2, h, w] coarsest-level initial field (runs pair by pair).
    Returns a dict of numpy arrays and the number of threads used.
    """
    refs = np.ascontiguousarray(refs, np.float32)
    tests = np.ascontiguousarray(tests, np.float32)
    if refs.ndim == 2:
        refs = refs[None]
        tests = tests[None]
    n, H, W = refs.shape
    nr = params.n_roi
    out = {
        "field": np.empty((n, 2, H, W)) if want_field else None,
        "q1": np.empty((n, nr, 2)),
        "F1": np.empty((n, 3, 3)),
        "Rfin": np.empty((n, 3, 3)),
        "q2": np.empty((n, nr, 2)),
        "ph": np.empty((n, nr)),
        "F": np.empty((n, 3, 3)),
        "R": np.empty((n, 3, 3)),
        "rotvec": np.empty((n, 3)),
        "iters": np.empty((n, params.levels), np.int32),
        "status": np.empty(n, np.uint32),
        "mae1": np.empty(n),
        "mae": np.empty(n),
        "ssim": np.empty(n),
        "omega": np.empty((n, 3, 3)),
    }
    o = _Outputs()
    for k in _OUT_KEYS:
        setattr(o, k, out[k].ctypes.data if out[k] is not None else None)
    rf = None
    if rfin is not None:
        rf = _f64(rfin).reshape(n, 9)
    if u_init is None:
        used = lib().orc_register_batch(_f(refs), _f(tests), n, H, W, C.byref(params),
                                        _d(rf) if rf is not None else None, C.byref(o))
    else:
        ui = _f64(u_init)
        used = 1
        bgm = None
        if params.background_static and not params.background:
            # the static background of the whole call, as orc_register_batch forms it
            bgm = mean_pattern(tests)
            params.background = bgm.ctypes.data
        for i in range(n):
            oi = _Outputs()
            for k in _OUT_KEYS:
                a = out[k]
                setattr(oi, k, a[i:i + 1].ctypes.data if a is not None else None)
            r_i = np.ascontiguousarray(refs[i])
            t_i = np.ascontiguousarray(tests[i])
            u_i = np.ascontiguousarray(ui[i])
            lib().orc_register_pair(_f(r_i), _f(t_i), H, W, C.byref(params), _d(u_i),
                                    _d(np.ascontiguousarray(rf[i])) if rf is not None else None,
                                    C.byref(oi))
        if bgm is not None:
            params.background = None
    out["threads"] = used
    return out

"""The remap before the second-pass XCF (section 2, before Eq. (12)) and the
repeated remap/XCF passes, on the GPU through the C ABI, against the FP64
oracle.  Needs an MI355X; run with -m gpu.

Bars:
  * B-spline coefficients and remapped images: the GPU runs the two
    first-order recursions in FP32 on 32-sample blocks started from zero 16
    samples outside the block (rows, then columns), the oracle runs them in
    FP64 with the exact start.  Each recursion step rounds once and damps
    earlier errors by |z| = 0.268, so a recursion adds at most
    2^-24 x max|input| / (1 - |z|); the row pass sees inputs up to max|img|,
    its output is bounded by 3 max|img| (the gain of the inverse filter), so
    the four recursions stay below 4 x 6 x 3 x 2^-24 / 0.73 max|img| =
    5.9e-6 max|img|, and the 16-sample starts add 2 x 6 x 1.4 x 7.1e-10
    max|img|.  Bar: 4e-5 max|img| (the 16 products of a cubic sample
    included).  Bilinear samples: 4 products, bar 1e-5 max|img|;
  * deformation gradient after P passes from the same R_finite: |dF| <= 1e-6
    (the single-pass bar: each pass starts from the previous pass's F, which
    agrees to ~1e-7 between the two sides);
  * known rotations and affine warps (noise-free rich band set, 256 px):
    rotation recovered to within 1e-5 rad and the isochoric F to 2e-5 after
    8 passes, as the oracle does.
"""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    from paper_1907_05993_amd import ebsd
    ebsd.lib()
    return ebsd


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def smooth_images(n, H, W, seed):
    import scipy.ndimage as ndi
    r = np.random.default_rng(seed)
    imgs = np.stack([ndi.gaussian_filter(r.normal(size=(H, W)), 1.2) for _ in range(n)])
    imgs /= imgs.std(axis=(1, 2), keepdims=True)
    return imgs.astype(np.float32)


def rotations(n, deg, seed):
    r = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        ax = r.normal(size=3)
        ax /= np.linalg.norm(ax)
        out.append(Rotation.from_rotvec(ax * math.radians(deg) * r.uniform(0.3, 1.0)).as_matrix())
    return np.stack(out)


@pytest.mark.parametrize("HW", [(64, 64), (100, 72), (37, 200), (256, 256)])
@pytest.mark.parametrize("interp", [3, 1])
def test_stage_remap_matches_oracle(E, orc, HW, interp):
    H, W = HW
    n = 3
    imgs = smooth_images(n, H, W, seed=H + W)
    Rs = rotations(n, 4.0, seed=H * W)
    pcs = (0.5 * W - 0.5, 0.5 * H - 0.5, 0.7 * W)
    print(f"stage remap {H}x{W} interp {interp}", flush=True)
    out, coef = E.stage_remap(cuda(imgs), torch.from_numpy(Rs), pcs, interp=interp)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    for i in range(n):
        mx = float(np.abs(imgs[i]).max())
        ref = orc.remap(imgs[i].astype(np.float64), Rs[i], pcs, interp=interp)
        bar = 4e-5 * mx if interp == 3 else 1e-5 * mx
        d = np.abs(out[i] - ref).max()
        print(f"  image {i}: max |d remap| {d:.2e} (bar {bar:.2e})")
        assert d <= bar
        if interp == 3:
            dc = np.abs(coef[i].cpu().numpy() - orc.bspline_coeffs(imgs[i].astype(np.float64))).max()
            print(f"  image {i}: max |d coef| {dc:.2e}")
            assert dc <= bar
    # the identity remap returns the samples (cubic: the interpolant passes through them)
    eye = torch.from_numpy(np.stack([np.eye(3)] * n))
    same, _ = E.stage_remap(cuda(imgs), eye, pcs, interp=interp)
    torch.cuda.synchronize()
    assert np.abs(same.cpu().numpy() - imgs).max() <= 4e-5 * float(np.abs(imgs).max())


def _gen(name, n):
    from paper_1907_05993_amd import synth as S
    specs = S.workload_specs(name, n=n)
    return S.render_batch(specs)


def _second_pass_parity(E, orc, gp, op, refs, tests):
    reg = E.Registrar(gp)
    g = reg.register(cuda(refs), cuda(tests), want_field=False)
    torch.cuda.synchronize()
    rf = g["R_finite"].cpu().numpy()
    o2 = orc.register_batch(refs, tests, op, rfin=rf, want_field=False)
    dF = np.abs(g["F"].cpu().numpy() - o2["F"]).max()
    dq2 = np.abs(g["q2"].cpu().numpy() - o2["q2"]).max()
    print("from the GPU's R_finite: max |dF| %.2e, max |dq2| %.2e px" % (dF, dq2))
    assert dF <= 1e-6
    assert np.array_equal(g["status"].cpu().numpy().astype(np.uint32), o2["status"])
    return g


def test_bilinear_remap_option_parity(E, orc):
    refs, tests = _gen("batch_256", 4)
    gp = E.Params(levels=3, iters=(15, 15, 15), roi_size=64, remap_interp=1)
    op = orc.make_params(levels=3, iters=15, roi_size=64, n_roi=20, remap_interp=1)
    print("bilinear remap, 4 pairs of 256", flush=True)
    _second_pass_parity(E, orc, gp, op, refs, tests)


@pytest.mark.parametrize("passes", [2, 4])
def test_repeated_passes_parity(E, orc, passes):
    refs, tests = _gen("batch_256", 4)
    gp = E.Params(levels=3, iters=(15, 15, 15), roi_size=64, xcf_passes=passes)
    op = orc.make_params(levels=3, iters=15, roi_size=64, n_roi=20, xcf_passes=passes)
    print(f"{passes} passes, 4 pairs of 256", flush=True)
    _second_pass_parity(E, orc, gp, op, refs, tests)


def test_known_small_rotation_recovered(E, orc):
    """The oracle's pinned noise-free cases (rotations about random axes and
    about z, and affine warps (I + eps) R): the GPU path with 8 passes
    recovers the rotation vector to within 1e-5 rad and the isochoric F to
    2e-5, and agrees with the oracle's 8 passes from the same R_finite."""
    import importlib.util, os
    spec = importlib.util.spec_from_file_location(
        "pins", os.path.join(os.path.dirname(__file__), "test_oracle_pins.py"))
    pins = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(pins)
    import scipy.linalg
    refs, tests, Fs = [], [], []
    for kind, angle, seed in pins.KNOWN_ROTATION_CASES:
        a, b, F = pins.known_rotation_pair(kind, angle, seed)
        refs.append(a)
        tests.append(b)
        Fs.append(F)
    refs, tests = np.stack(refs), np.stack(tests)
    truth = np.stack([Rotation.from_matrix(scipy.linalg.polar(F)[0]).as_rotvec() for F in Fs])
    Fiso = np.stack([F / np.cbrt(np.linalg.det(F)) for F in Fs])
    print(f"known rotations, {len(Fs)} noise-free pairs of 256, 8 passes", flush=True)
    reg = E.Registrar(E.Params(levels=3, iters=(50, 50, 50), roi_size=64, xcf_passes=8))
    g = reg.register(cuda(refs), cuda(tests), want_field=False)
    torch.cuda.synchronize()
    err = np.linalg.norm(g["rotvec"].cpu().numpy() - truth, axis=1)
    dF = np.abs(g["F"].cpu().numpy() - Fiso).max(axis=(1, 2))
    print("rotation error per pair (rad):", ["%.1e" % e for e in err])
    print("isochoric F error per pair:", ["%.1e" % e for e in dF])
    assert (err < 1e-5).all()
    assert (dF < 2e-5).all()
    op = orc.make_params(levels=3, iters=50, sigma=1.0, roi_size=64, n_roi=20, xcf_passes=8)
    o2 = orc.register_batch(refs, tests, op, rfin=g["R_finite"].cpu().numpy(), want_field=False)
    d = np.abs(g["F"].cpu().numpy() - o2["F"]).max()
    print("8 passes from the GPU's R_finite: max |dF| vs oracle %.2e" % d)
    assert d <= 1e-6

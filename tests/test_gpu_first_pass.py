"""The conventional first pass (ROI cross-correlation of the unremapped
patterns, the method section 3 compares demons with) and the mean angular
error of each fit, on the GPU through the C ABI, against the FP64 oracle.
Needs an MI355X; run with -m gpu.

Bars:
  * integer shift of a pattern of period N (every test ROI a circular shift of
    the reference ROI, no window): q1 = s to 1e-4 px (FP32), as the oracle's
    exact case;
  * q1 on generated pairs of 0-2 deg: |dq1| <= 2e-3 px against the oracle's
    FP64 correlation of its own FP64-normalised patterns (the stage XCF bar
    plus the normalisation's rounding);
  * F_first and its mean angular error from the GPU's own q1: the oracle's
    Eq. (3) solve on the same shifts to 1e-9, the error to 1e-12 rad (both
    FP64);
  * second pass from the same R_finite: |dF| <= 1e-6, mean angular error
    to 1e-7 rad (q2 agree to ~1e-5 px, 1e-7 rad at Z* = 179 px).
"""
import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    from paper_1907_05993_amd import ebsd
    ebsd.lib()
    return ebsd


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def tiled_pair(N, tiles, shift, seed):
    block = ndi.gaussian_filter(np.random.default_rng(seed).normal(size=(N, N)), 1.5, mode="wrap")
    ref = np.tile(block, (tiles, tiles)).astype(np.float32)
    return ref, np.roll(ref, (shift[1], shift[0]), axis=(0, 1))


def test_xcf_first_pass_integer_shift(E, orc):
    shifts = [(3, -2), (-5, 0), (0, 7), (9, 4)]
    refs, tests = zip(*[tiled_pair(32, 4, s, seed=60 + i) for i, s in enumerate(shifts)])
    print("XCF first pass, integer shifts of period-32 patterns at 128 px", flush=True)
    reg = E.Registrar(E.Params(levels=3, iters=(10, 10, 10), roi_size=32, window=0, second_pass=0,
                               first_pass=1))
    g = reg.register(cuda(np.stack(refs)), cuda(np.stack(tests)))
    torch.cuda.synchronize()
    assert "field" not in g
    q1 = g["q1"].cpu().numpy()
    for i, s in enumerate(shifts):
        d = np.abs(q1[i] - np.array(s, np.float32)).max()
        print(f"  shift {s}: max |q1 - s| {d:.1e}")
        assert d <= 1e-4
    np.testing.assert_allclose(g["peak_height"].cpu().numpy(), 1.0, atol=1e-5)
    assert not g["iters"].cpu().numpy().any()
    assert not g["status"].cpu().numpy().any()
    np.testing.assert_array_equal(g["F"].cpu().numpy(), g["F_first"].cpu().numpy())
    np.testing.assert_array_equal(g["mae"].cpu().numpy(), g["mae_first"].cpu().numpy())
    assert g["mae_first"].cpu().numpy().max() < 1e-6


@pytest.mark.parametrize("roi,H", [(64, 256), (32, 128), (256, 1024)])
def test_xcf_first_pass_parity(E, orc, roi, H):
    from paper_1907_05993_amd import synth as S
    specs = [S.make_spec(7, i, H, H, mis_deg=(0.0, 2.0)) for i in range(4)]
    refs, tests = S.render_batch(specs)
    print(f"XCF first pass + second pass, 4 pairs of {H} px, 0-2 deg, ROIs of {roi}", flush=True)
    gp = E.Params(levels=3, iters=(15, 15, 15), roi_size=roi, first_pass=1)
    op = orc.make_params(levels=3, iters=15, roi_size=roi, n_roi=20, first_pass=1)
    g = E.Registrar(gp).register(cuda(refs), cuda(tests), want_field=False)
    torch.cuda.synchronize()
    o = orc.register_batch(refs, tests, op, want_field=False)
    q1 = g["q1"].cpu().numpy()
    dq1 = np.abs(q1 - o["q1"]).max()
    print("  max |dq1| %.2e px" % dq1)
    assert dq1 <= 2e-3
    assert not g["iters"].cpu().numpy().any()
    # the first fit from the GPU's own shifts
    cx, cy, _, _, _ = orc.roi_layout(H, H, op)
    pcs = orc.pc_pixels(H, H, op)
    F1 = g["F_first"].cpu().numpy()
    m1 = g["mae_first"].cpu().numpy()
    for i in range(len(specs)):
        Fo, _ = orc.solve_F(q1[i], cx, cy, pcs)
        assert np.abs(F1[i] - Fo).max() <= 1e-9
        assert abs(m1[i] - orc.mae(q1[i], F1[i], cx, cy, pcs)) <= 1e-12
    # second pass from the same R_finite
    o2 = orc.register_batch(refs, tests, op, rfin=g["R_finite"].cpu().numpy(), want_field=False)
    dF = np.abs(g["F"].cpu().numpy() - o2["F"]).max()
    dm = np.abs(g["mae"].cpu().numpy() - o2["mae"]).max()
    fmt = {"float_kind": lambda x: "%.1e" % x}
    print("  from the GPU's R_finite: max |dF| %.2e, max |d mae| %.2e rad; mae first %s, last %s rad"
          % (dF, dm, np.array2string(m1, formatter=fmt), np.array2string(o2["mae"], formatter=fmt)))
    assert dF <= 1e-6
    assert dm <= 1e-7
    assert np.array_equal(g["status"].cpu().numpy().astype(np.uint32), o2["status"])


def test_demons_first_pass_mae_parity(E, orc):
    """The mean angular errors of the default path (demons first pass): the
    first from the GPU's own q1 and F_first, the last from a common R_finite."""
    from paper_1907_05993_amd import synth as S
    specs = S.workload_specs("batch_256", n=4)
    refs, tests = S.render_batch(specs)
    gp = E.Params(levels=3, iters=(15, 15, 15), roi_size=64)
    op = orc.make_params(levels=3, iters=15, roi_size=64, n_roi=20)
    print("demons first pass, 4 pairs of 256: mean angular errors", flush=True)
    g = E.Registrar(gp).register(cuda(refs), cuda(tests), want_field=False)
    torch.cuda.synchronize()
    cx, cy, _, _, _ = orc.roi_layout(256, 256, op)
    pcs = orc.pc_pixels(256, 256, op)
    q1 = g["q1"].cpu().numpy()
    F1 = g["F_first"].cpu().numpy()
    m1 = g["mae_first"].cpu().numpy()
    for i in range(4):
        assert abs(m1[i] - orc.mae(q1[i], F1[i], cx, cy, pcs)) <= 1e-12
    o2 = orc.register_batch(refs, tests, op, rfin=g["R_finite"].cpu().numpy(), want_field=False)
    dm = np.abs(g["mae"].cpu().numpy() - o2["mae"]).max()
    print("  max |d mae| from a common R_finite %.2e rad" % dm)
    assert dm <= 1e-7
    # without the second pass the last fit is the first
    g0 = E.Registrar(E.Params(levels=3, iters=(15, 15, 15), roi_size=64, second_pass=0)).register(
        cuda(refs), cuda(tests), want_field=False)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(g0["mae"].cpu().numpy(), g0["mae_first"].cpu().numpy())

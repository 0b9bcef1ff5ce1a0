"""Stage parity: each HIP kernel (through the C ABI) against the FP64 oracle on
the same seeded inputs.  Needs an MI355X; run with -m gpu.

Tolerances follow from FP32 arithmetic on O(1) normalised intensities:
a few ulp of 1 for pointwise stages, 1e-5 px for one demons step (the
reciprocal is the hardware one, relative error ~1e-7 on |du| <= 0.5),
1e-3 px for a sub-pixel XCF peak of random textures (FP32 FFT round-off
divided by the peak curvature), exact integer peaks.
"""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    from paper_1907_05993_amd import ebsd
    ebsd.lib()
    assert torch.cuda.is_available()
    return ebsd


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def rng(s):
    return np.random.default_rng(s)


def test_stage_normalize(E, orc):
    from paper_1907_05993_amd import synth as S
    ref, test = S.render_pair(S.make_spec(11, 0, 128, 96, exact_angle=3.0, strain=1e-3))
    x = np.stack([ref, test])
    out, flags = E.stage_normalize(cuda(x))
    out = out.cpu().numpy()
    for i in range(2):
        o, st = orc.normalize(x[i])
        assert st == 0 and flags[i].item() == 0
        np.testing.assert_allclose(out[i], o, atol=2e-6)


def test_stage_normalize_flags(E, orc):
    x = np.ones((3, 32, 32), np.float32)
    x[1] = rng(1).normal(size=(32, 32))
    x[2, 5, 5] = np.inf
    out, flags = E.stage_normalize(cuda(x))
    assert flags.tolist() == [orc.DEGENERATE_INPUT, 0, orc.NONFINITE_INPUT]
    o = out.cpu().numpy()
    assert not o[0].any() and not o[2].any()


@pytest.mark.parametrize("shape", [(3, 64, 64), (2, 36, 20), (1, 256, 128)])
def test_stage_restrict(E, orc, shape):
    x = rng(2).normal(size=shape).astype(np.float32)
    out = E.stage_restrict(cuda(x)).cpu().numpy()
    for i in range(shape[0]):
        np.testing.assert_allclose(out[i], orc.restrict(x[i].astype(np.float64)), atol=1e-6)


@pytest.mark.parametrize("shape,sigma", [((2, 64, 64), 1.0), ((1, 40, 100), 1.0), ((2, 33, 70), 0.5),
                                         ((1, 128, 128), 1.3), ((1, 17, 64), 0.0), ((1, 256, 64), 1.0),
                                         ((2, 64, 256), 1.0), ((1, 40, 300), 1.0), ((1, 20, 260), 0.5)])
def test_stage_demons_iter(E, orc, shape, sigma):
    n, H, W = shape
    base = ndi.gaussian_filter(rng(3).normal(size=(H + 8, W + 8)), 1.5)
    R = base[4:4 + H, 4:4 + W]
    T = ndi.shift(base, (0.6, -0.9), order=1, mode="nearest")[4:4 + H, 4:4 + W]
    R = np.stack([R] * n).astype(np.float32)
    T = np.stack([T + 0.01 * k for k in range(n)]).astype(np.float32)
    u = rng(4).normal(scale=0.8, size=(n, 2, H, W)).astype(np.float32)
    un, rms = E.stage_demons_iter(cuda(R), cuda(T), cuda(u), sigma)
    un = un.cpu().numpy()
    rms = rms.cpu().numpy()
    for i in range(n):
        o, r = orc.demons_iter(R[i].astype(np.float64), T[i].astype(np.float64),
                               u[i].astype(np.float64), sigma)
        np.testing.assert_allclose(un[i], o, atol=1e-5)
        assert abs(rms[i] - r) <= 1e-5 * max(1.0, r)


def test_stage_demons_identical_images_exact(E):
    R = ndi.gaussian_filter(rng(5).normal(size=(1, 64, 80)), (0, 2, 2)).astype(np.float32)
    un, rms = E.stage_demons_iter(cuda(R), cuda(R), torch.zeros(1, 2, 64, 80, device="cuda"), 1.0)
    assert not un.any().item() and rms.item() == 0.0


@pytest.mark.parametrize("sigma", [0.0, 1.0])
def test_stage_demons_ramp_trajectory_closed_form(E, sigma):
    """R(x) = x, T(x) = x - s through the stage kernels: restriction, 3 coarse
    steps, prolongation, 4 fine steps.  Away from the borders the field is
    uniform (smoothing keeps it so) and follows the scalar recurrences of
    Eq. (1) for a linear pattern, U += 4 a / (4 + a^2) on the coarse level
    (full-resolution px, slope 2) and U += a / (1 + a^2) on the fine one,
    a = s - U; no oracle involved.  FP32 bar 1e-4 px (intensities up to 127)."""
    s, k1, k0, H, W = 6.0, 3, 4, 16, 128
    x = np.tile(np.arange(W, dtype=np.float32), (1, H, 1))
    R, T = cuda(x), cuda(x - np.float32(s))
    R1, T1 = E.stage_restrict(R), E.stage_restrict(T)
    u = torch.zeros(1, 2, H // 2, W // 2, device="cuda")
    for _ in range(k1):
        u, _ = E.stage_demons_iter(R1, T1, u, sigma)
    u = E.stage_prolong(u)
    for _ in range(k0):
        u, _ = E.stage_demons_iter(R, T, u, sigma)
    U = 0.0
    for _ in range(k1):
        a = s - U
        U += 4.0 * a / (4.0 + a * a)
    for _ in range(k0):
        a = s - U
        U += a / (1.0 + a * a)
    f = u.cpu().numpy()[0].astype(np.float64)
    lo, hi = (8, 112) if sigma == 0 else (24, 100)  # border effects spread 3 columns per smoothed step
    print("closed form U = %.6f; GPU interior min %.6f max %.6f" % (U, f[0][:, lo:hi].min(), f[0][:, lo:hi].max()))
    np.testing.assert_allclose(f[0][:, lo:hi], U, rtol=0, atol=1e-4)
    assert np.abs(f[1]).max() <= 1e-6


@pytest.mark.parametrize("hw", [(8, 8), (16, 32), (64, 64), (5, 7)])
def test_stage_prolong(E, orc, hw):
    h, w = hw
    u = rng(6).normal(size=(2, 2, h, w)).astype(np.float32)
    out = E.stage_prolong(cuda(u)).cpu().numpy()
    for i in range(2):
        np.testing.assert_allclose(out[i], orc.prolong(u[i].astype(np.float64)), atol=2e-6)


@pytest.mark.parametrize("N", [32, 64, 128, 256])
def test_stage_xcf_random_textures(E, orc, N):
    n = 6
    A = np.empty((n, N, N), np.float32)
    B = np.empty((n, N, N), np.float32)
    for i in range(n):
        big = ndi.gaussian_filter(rng(10 + i).normal(size=(N + 16, N + 16)), 2.0)
        s = rng(20 + i).uniform(-3, 3, size=2)
        A[i] = big[8:8 + N, 8:8 + N]
        B[i] = ndi.shift(big, (s[1], s[0]), order=3, mode="nearest")[8:8 + N, 8:8 + N]
    for window in (1, 0):
        q, ph = E.stage_xcf(cuda(A), cuda(B), window)
        q = q.cpu().numpy()
        ph = ph.cpu().numpy()
        for i in range(n):
            qo, pho, _ = orc.xcf(A[i].astype(np.float64), B[i].astype(np.float64), window)
            np.testing.assert_allclose(q[i], qo, atol=1e-3)
            assert abs(ph[i] - pho) < 1e-5


@pytest.mark.parametrize("N", [32, 64, 128, 256])
def test_stage_xcf_integer_shift_and_identical(E, N):
    A = ndi.gaussian_filter(rng(30).normal(size=(N, N)), 1.5, mode="wrap").astype(np.float32)
    shifts = [(0, 0), (3, -5), (-N // 4, N // 4 - 1), (7, 2)]
    As = np.stack([A] * len(shifts))
    Bs = np.stack([np.roll(A, shift=(s[1], s[0]), axis=(0, 1)) for s in shifts])
    q, ph = E.stage_xcf(cuda(As), cuda(Bs), 0)
    np.testing.assert_allclose(q.cpu().numpy(), np.array(shifts, np.float64), atol=1e-4)
    assert abs(ph[0].item() - 1.0) < 1e-5


def test_stage_xcf_256_more_rois_than_workgroups(E, orc):
    """ROIs of 256 x 256 go through global scratch, one slot per workgroup; with
    more ROIs than workgroups (600 > 512) a workgroup reuses its slot for a
    second ROI.  Sampled ROIs against the oracle (first and second round of
    the slots), and every ROI against the same ROI correlated alone."""
    N, n = 256, 600
    print(f"case: XCF N=256, {n} ROIs", flush=True)
    base = ndi.gaussian_filter(rng(40).normal(size=(N + 32, N + 32)), (1.5, 3.0))
    A = np.empty((n, N, N), np.float32)
    B = np.empty((n, N, N), np.float32)
    sh = rng(41).uniform(-6, 6, size=(n, 2))
    off = rng(42).integers(0, 32, size=(n, 2))
    for i in range(n):
        big = np.roll(base, shift=(int(off[i, 0]), int(off[i, 1])), axis=(0, 1))
        A[i] = big[16:16 + N, 16:16 + N]
        B[i] = ndi.shift(big, (sh[i, 1], sh[i, 0]), order=3, mode="wrap")[16:16 + N, 16:16 + N]
    q, ph = E.stage_xcf(cuda(A), cuda(B), 1)
    q, ph = q.cpu().numpy(), ph.cpu().numpy()
    for i in (0, 1, 255, 511, 512, 513, 599):
        qo, pho, _ = orc.xcf(A[i].astype(np.float64), B[i].astype(np.float64), 1)
        np.testing.assert_allclose(q[i], qo, atol=1e-3)
        assert abs(ph[i] - pho) < 1e-5
    for i in (3, 300, 512, 599):
        q1, ph1 = E.stage_xcf(cuda(A[i:i + 1]), cuda(B[i:i + 1]), 1)
        assert np.array_equal(q1.cpu().numpy()[0], q[i]) and ph1.item() == ph[i]


def test_stage_solve(E, orc):
    from scipy.spatial.transform import Rotation
    p = orc.make_params(n_roi=20, roi_size=64)
    cx, cy, _, _, _ = orc.roi_layout(256, 256, p)
    pcs = (127.5, 127.5, 179.2)
    Fs = []
    qs = []
    for k in range(8):
        eps = rng(40 + k).uniform(-2e-3, 2e-3, size=(3, 3))
        eps = 0.5 * (eps + eps.T)
        F = (np.eye(3) + eps) @ Rotation.from_rotvec(rng(50 + k).normal(scale=0.08, size=3)).as_matrix()
        r = np.stack([cx - pcs[0], cy - pcs[1], np.full_like(cx, pcs[2])])
        v = F @ r
        q = np.stack([pcs[0] + pcs[2] * v[0] / v[2] - cx, pcs[1] + pcs[2] * v[1] / v[2] - cy], 1)
        q = q + rng(60 + k).normal(scale=0.05, size=q.shape)
        Fs.append(F)
        qs.append(q.astype(np.float32))
    qs = np.stack(qs)
    F, R, st = E.stage_solve(cuda(qs), cx, cy, pcs)
    F = F.cpu().numpy()
    R = R.cpu().numpy()
    for k in range(8):
        Fo, sto = orc.solve_F(qs[k].astype(np.float64), cx, cy, pcs)
        np.testing.assert_allclose(F[k], Fo, atol=1e-11)
        np.testing.assert_allclose(R[k], orc.polar(Fo), atol=1e-11)
        assert st[k].item() == sto


@pytest.mark.parametrize("n_roi,roi,size", [(5, 64, 256), (101, 32, 256), (256, 32, 512)])
def test_stage_solve_roi_counts(E, orc, n_roi, roi, size):
    """The solve (one wavefront per shift set, sums over the ROIs on its lanes)
    at the fewest ROIs the entry accepts, more ROIs than lanes, and the most it
    accepts; plus an exact identity (zero shifts) and a shift set the fit
    cannot explain (one ROI moved by 1e6 px), against the oracle's F and status."""
    from scipy.spatial.transform import Rotation
    p = orc.make_params(n_roi=n_roi, roi_size=roi)
    cx, cy, _, _, bad = orc.roi_layout(size, size, p)
    assert not bad
    pcs = (0.5 * size - 0.5, 0.5 * size - 0.5, 0.7 * size)
    qs = []
    for k in range(6):
        eps = rng(140 + k).uniform(-2e-3, 2e-3, size=(3, 3))
        eps = 0.5 * (eps + eps.T)
        F = (np.eye(3) + eps) @ Rotation.from_rotvec(rng(150 + k).normal(scale=0.08, size=3)).as_matrix()
        r = np.stack([cx - pcs[0], cy - pcs[1], np.full_like(cx, pcs[2])])
        v = F @ r
        q = np.stack([pcs[0] + pcs[2] * v[0] / v[2] - cx, pcs[1] + pcs[2] * v[1] / v[2] - cy], 1)
        qs.append((q + rng(160 + k).normal(scale=0.05, size=q.shape)).astype(np.float32))
    qs.append(np.zeros((n_roi, 2), np.float32))
    far = qs[0].copy()
    far[0, 0] = 1e6
    qs.append(far)
    qs = np.stack(qs)
    F, R, st = E.stage_solve(cuda(qs), cx, cy, pcs)
    F, R, st = F.cpu().numpy(), R.cpu().numpy(), st.cpu().numpy()
    for k in range(7):
        Fo, sto = orc.solve_F(qs[k].astype(np.float64), cx, cy, pcs)
        assert st[k].item() == sto == 0, k
        np.testing.assert_allclose(F[k], Fo, atol=1e-11)
        np.testing.assert_allclose(R[k], orc.polar(Fo), atol=1e-11)
    np.testing.assert_allclose(F[6], np.eye(3), atol=1e-13)
    # the 1e6 px outlier: both sides flag the fit (the values of F differ, both meaningless)
    _, sto = orc.solve_F(qs[7].astype(np.float64), cx, cy, pcs)
    assert sto == E.SOLVE_ILLCOND and st[7].item() & E.SOLVE_ILLCOND


def test_teacher_forced_full_depth(E, orc):
    """150 GPU iterations at 256^2 (level 0 of a real 10-degree pair, field
    started from the oracle's prolonged level-1 field); every 15th step the
    GPU's step from its own state is compared with the oracle's step from that
    same state.  Proves per-step parity across the whole depth, independently
    of the iteration's sensitivity to round-off."""
    from paper_1907_05993_amd import synth as S
    spec = S.make_spec(6, 3, 256, 256, exact_angle=10.0, strain=2e-3)
    ref, test = S.render_pair(spec)
    Rn, _ = orc.normalize(ref)
    Tn, _ = orc.normalize(test)
    p = orc.make_params(levels=2, iters=150, sigma=1.0)
    # coarse start: oracle demons on levels 1..2 only (prolonged to level 0)
    R1, T1 = orc.restrict(Rn), orc.restrict(Tn)
    f1, _, _ = orc.demons(R1, T1, orc.make_params(levels=2, iters=150, sigma=1.0))
    u0 = orc.prolong(f1)
    R = cuda(Rn[None])
    T = cuda(Tn[None])
    u = cuda(u0[None])
    Rf = Rn.astype(np.float32).astype(np.float64)
    Tf = Tn.astype(np.float32).astype(np.float64)
    worst = 0.0
    for k in range(150):
        un, rms = E.stage_demons_iter(R, T, u, 1.0)
        if k % 15 == 0 or k == 149:
            ug = u[0].cpu().numpy().astype(np.float64)
            o, r = orc.demons_iter(Rf, Tf, ug, 1.0)
            d = np.abs(un[0].cpu().numpy() - o).max()
            worst = max(worst, d)
            assert d <= 1e-4, (k, d)
        u = un
    print("teacher-forced worst per-step |du| difference: %.2e px" % worst)
